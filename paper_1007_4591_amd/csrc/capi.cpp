// C-ABI of the library: argument checks, error mapping, tree lifetime.
// No C++ exception crosses this boundary.
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>

#include "common.h"

namespace bemfmm {

static thread_local std::string g_err;

void set_error(const std::string &msg) { g_err = msg; }

Tree::~Tree() {
  fmm_free(*this);
  lpb_free(*this);
  if (ev_init) {
    for (auto &e : ev) (void)hipEventDestroy(e);
    (void)hipEventDestroy(ev_fork);
    (void)hipEventDestroy(ev_join);
    (void)hipStreamDestroy(side_stream);
  }
  magic = 0;
}

Tree *check_tree(const bemfmm_tree *t) {
  Tree *T = reinterpret_cast<Tree *>(const_cast<bemfmm_tree *>(t));
  if (!T || T->magic != 0x5eedbe11) BF_THROW(BEMFMM_ESTATE, "NULL or destroyed tree");
  return T;
}

// Makes the tree's device current for the duration of an entry point and
// restores the caller's device afterwards.
struct DeviceScope {
  int prev = -1, want = 0;
  explicit DeviceScope(const Tree &T) : want(T.device) {
    HIP_OK(hipGetDevice(&prev));
    if (prev != want) HIP_OK(hipSetDevice(want));
  }
  ~DeviceScope() {
    if (prev >= 0 && prev != want) (void)hipSetDevice(prev);
  }
  DeviceScope(const DeviceScope &) = delete;
  DeviceScope &operator=(const DeviceScope &) = delete;
};

template <class F>
static int guard(F &&f) {
  g_err.clear();
  try {
    f();
    return BEMFMM_OK;
  } catch (const Error &e) {
    g_err = e.msg;
    return e.code;
  } catch (const std::bad_alloc &) {
    g_err = "host allocation failed";
    return BEMFMM_ENOMEM;
  } catch (const std::exception &e) {
    g_err = e.what();
    return BEMFMM_EDEVICE;
  }
}

static void need(bool ok, const char *msg) {
  if (!ok) BF_THROW(BEMFMM_EINVAL, msg);
}


}  // namespace bemfmm

using namespace bemfmm;

extern "C" {

int bemfmm_build_tree(const double *verts, int64_t nv, const int32_t *tris, int64_t nt, const double *charge_pos,
                      int64_t nq, const bemfmm_params *params, void *stream, bemfmm_tree **out) {
  return guard([&] {
    need(out != nullptr, "out is NULL");
    *out = nullptr;
    need(params != nullptr, "params is NULL");
    need(nt > 0 && nv > 0, "empty mesh");
    need(nt < (int64_t)1 << 30 && nq < (int64_t)1 << 30, "too many panels or charges (int32 indices)");
    need(verts && tris, "verts/tris are NULL");
    need(nq == 0 || charge_pos, "charge_pos is NULL");
    need(nq >= 0, "nq < 0");
    const bemfmm_params &P = *params;
    need(P.p >= 1 && P.p <= 11, "p outside 1..11");
    need(P.ncrit >= 1, "ncrit < 1");
    need(P.mac == BEMFMM_MAC_THETA || P.mac == BEMFMM_MAC_ADJACENT, "unknown MAC");
    need(P.mac == BEMFMM_MAC_ADJACENT || (P.theta >= 0.3 && P.theta <= 1.0), "theta outside [0.3, 1]");
    need(P.eps_in > 0 && P.eps_out > 0 && std::isfinite(P.eps_in) && std::isfinite(P.eps_out),
         "permittivities must be positive");
    need(std::isfinite(P.near_quad) && P.near_quad >= 0.0 && P.near_quad <= 16.0, "near_quad outside [0, 16]");
    Tree *T = new Tree();
    try {
      HIP_OK(hipGetDevice(&T->device));
      T->prm = P;
      build_tree(*T, verts, nv, tris, nt, charge_pos, nq, (hipStream_t)stream);
    } catch (...) {
      delete T;
      throw;
    }
    *out = reinterpret_cast<bemfmm_tree *>(T);
  });
}

int bemfmm_set_charges(bemfmm_tree *tree, const double *charge_pos, void *stream) {
  return guard([&] {
    Tree *T = check_tree(tree);
    DeviceScope dev_scope(*T);
    need(T->Q == 0 || charge_pos, "charge_pos is NULL");
    set_charges(*T, charge_pos, (hipStream_t)stream);
  });
}

int bemfmm_set_charges_noalloc(bemfmm_tree *tree, const double *charge_pos, void *stream) {
  return guard([&] {
    Tree *T = check_tree(tree);
    DeviceScope dev_scope(*T);
    need(T->Q == 0 || charge_pos, "charge_pos is NULL");
    set_charges_noalloc(*T, charge_pos, (hipStream_t)stream);
  });
}

static void need_kappa(const Tree &T, double kappa) {
  need(std::isfinite(kappa) && kappa > 0.0, "kappa must be positive");
  need(kappa * T.side <= 400.0, "kappa times the root cube side exceeds 400");
}

int bemfmm_lpb_matvec(bemfmm_tree *tree, double kappa, const double *uv, double *y, void *stream) {
  return guard([&] {
    Tree *T = check_tree(tree);
    DeviceScope dev_scope(*T);
    need_kappa(*T, kappa);
    need(uv && y, "uv/y are NULL");
    lpb_matvec(*T, kappa, uv, y, (hipStream_t)stream);
  });
}

int bemfmm_lpb_solve(bemfmm_tree *tree, const double *q, double kappa, double *uv, double tol, int maxit,
                     int restart, bemfmm_solve_info *info, void *stream) {
  return guard([&] {
    Tree *T = check_tree(tree);
    DeviceScope dev_scope(*T);
    need_kappa(*T, kappa);
    need(uv != nullptr && (T->Q == 0 || q != nullptr), "q/uv are NULL");
    need(tol > 0 && maxit >= 1, "tol must be > 0 and maxit >= 1");
    lpb_solve(*T, q, kappa, uv, tol, maxit, restart, info, (hipStream_t)stream);
  });
}

int bemfmm_lpb_energy(bemfmm_tree *tree, const double *q, const double *uv, double *dG_host, void *stream) {
  return guard([&] {
    Tree *T = check_tree(tree);
    DeviceScope dev_scope(*T);
    need(dG_host != nullptr && uv != nullptr && (T->Q == 0 || q != nullptr), "q/uv/dG are NULL");
    *dG_host = lpb_energy(*T, q, uv, (hipStream_t)stream);
  });
}

int bemfmm_tree_destroy(bemfmm_tree *tree) {
  return guard([&] {
    Tree *T = check_tree(tree);
    DeviceScope dev_scope(*T);
    (void)hipDeviceSynchronize();
    delete T;
  });
}

int bemfmm_tree_get_info(const bemfmm_tree *tree, bemfmm_tree_info *info) {
  return guard([&] {
    Tree *T = check_tree(tree);
    DeviceScope dev_scope(*T);
    need(info != nullptr, "info is NULL");
    bemfmm_tree_info I{};
    I.n_panels = T->N;
    I.n_charges = T->Q;
    I.leaf_level = T->L;
    I.n_cells = T->ncell_tot;
    I.n_leaves = T->ncell[T->L];
    I.n_near_pairs = T->n_near_leaf;
    I.n_far_pairs = T->nfar;
    I.n_nearquad_pairs = T->n_nq;
    I.n_m2l_panel_pairs = T->m2l[0].n;
    I.n_offsets = T->tab ? T->tab->noff() : 0;
    I.p2p_pairs_panels = T->p2p_pairs_pp;
    for (int d = 0; d < 3; ++d) I.lo[d] = T->lo[d];
    I.side = T->side;
    *info = I;
  });
}

int bemfmm_fmm_matvec(bemfmm_tree *tree, int op, int precision, const double *x, double *y, void *stream) {
  return guard([&] {
    Tree *T = check_tree(tree);
    DeviceScope dev_scope(*T);
    need(op >= BEMFMM_OP_A && op <= BEMFMM_OP_CT, "unknown operator");
    need(precision >= BEMFMM_FP64 && precision <= BEMFMM_FP32_REFINED, "unknown precision");
    need(x && y, "x/y are NULL");
    op_apply(*T, op, precision, x, y, (hipStream_t)stream);
  });
}

int bemfmm_solve_bem(bemfmm_tree *tree, const double *q, double *x, double tol, int maxit, int restart,
                     int precision, bemfmm_solve_info *info, void *stream) {
  return guard([&] {
    Tree *T = check_tree(tree);
    DeviceScope dev_scope(*T);
    need(precision >= BEMFMM_FP64 && precision <= BEMFMM_FP32_REFINED, "unknown precision");
    need(x != nullptr && (T->Q == 0 || q != nullptr), "q/x are NULL");
    need(tol > 0 && maxit >= 1, "tol must be > 0 and maxit >= 1");
    solve_bem(*T, q, x, tol, maxit, restart, precision, info, (hipStream_t)stream);
  });
}

int bemfmm_bibee_energy(bemfmm_tree *tree, const double *q, int kind, int precision, double *dG_host,
                        void *stream) {
  return guard([&] {
    Tree *T = check_tree(tree);
    DeviceScope dev_scope(*T);
    need(kind == BEMFMM_BIBEE_CFA || kind == BEMFMM_BIBEE_P || kind == BEMFMM_BIBEE_PLUS_HALF, "unknown BIBEE kind");
    need(precision >= BEMFMM_FP64 && precision <= BEMFMM_FP32_REFINED, "unknown precision");
    need(dG_host != nullptr && (T->Q == 0 || q != nullptr), "q/dG are NULL");
    *dG_host = bibee(*T, q, kind, precision, (hipStream_t)stream);
  });
}

int bemfmm_solvation_energy(bemfmm_tree *tree, const double *q, const double *x, int precision, double *dG_host,
                            void *stream) {
  return guard([&] {
    Tree *T = check_tree(tree);
    DeviceScope dev_scope(*T);
    need(dG_host != nullptr && x != nullptr && (T->Q == 0 || q != nullptr), "q/x/dG are NULL");
    *dG_host = energy(*T, q, x, precision, (hipStream_t)stream);
  });
}

int bemfmm_adjoint_grad(bemfmm_tree *tree, const double *q, const double *x, double tol, int maxit, int restart,
                        int precision, double *dG_dq, double *dG_dpos, bemfmm_solve_info *info, void *stream) {
  return guard([&] {
    Tree *T = check_tree(tree);
    DeviceScope dev_scope(*T);
    need(x != nullptr && (T->Q == 0 || q != nullptr), "q/x are NULL");
    need(tol > 0 && maxit >= 1, "tol must be > 0 and maxit >= 1");
    adjoint(*T, q, x, tol, maxit, restart, precision, dG_dq, dG_dpos, info, (hipStream_t)stream);
  });
}

int bemfmm_binding_energy(bemfmm_tree *complex_tree, const double *q_complex, bemfmm_tree *protein_tree,
                          const double *q_protein, bemfmm_tree *inhibitor_tree, const double *q_inhibitor,
                          int method, int precision, double tol, int maxit, int restart, double *dG_host,
                          void *stream) {
  return guard([&] {
    Tree *T[3] = {check_tree(complex_tree), check_tree(protein_tree), check_tree(inhibitor_tree)};
    const double *q[3] = {q_complex, q_protein, q_inhibitor};
    need(dG_host != nullptr, "dG is NULL");
    need(method >= BEMFMM_ENERGY_BEM && method <= BEMFMM_ENERGY_BIBEE_PLUS_HALF, "unknown energy method");
    need(precision >= BEMFMM_FP64 && precision <= BEMFMM_FP32_REFINED, "unknown precision");
    need(method != BEMFMM_ENERGY_BEM || (tol > 0 && maxit >= 1), "tol must be > 0 and maxit >= 1");
    for (int k = 0; k < 3; ++k) {
      need(T[k]->Q == 0 || q[k] != nullptr, "charges are NULL");
      need(T[k]->device == T[0]->device, "the three trees must live on one device");
    }
    DeviceScope dev_scope(*T[0]);
    double e[3];
    for (int k = 0; k < 3; ++k)
      e[k] = molecule_energy(*T[k], q[k], method, precision, tol, maxit, restart, (hipStream_t)stream);
    dG_host[0] = e[0] - e[1] - e[2];
    dG_host[1] = e[0];
    dG_host[2] = e[1];
    dG_host[3] = e[2];
  });
}

const char *bemfmm_last_error(void) { return g_err.c_str(); }

int bemfmm_release_cache(void) {
  return guard([&] { dev_cache_release(); });
}

int bemfmm_tree_export(const bemfmm_tree *tree, int32_t *panel_perm, int32_t *charge_perm, uint32_t *panel_key,
                       uint32_t *charge_key, uint32_t *cell_key, int32_t *cell_level, int32_t *cell_range,
                       int32_t *cell_parent, int32_t *near_ptr, int32_t *near_idx, int32_t *far_pairs) {
  return guard([&] {
    Tree *T = check_tree(tree);
    DeviceScope dev_scope(*T);
    const int L = T->L;
    auto d2h = [&](void *dst, const void *src, size_t bytes) {
      if (dst && bytes) HIP_OK(hipMemcpy(dst, src, bytes, hipMemcpyDeviceToHost));
    };
    d2h(panel_perm, T->pperm.p, T->N * 4);
    d2h(panel_key, T->pkey.p, T->N * 4);
    d2h(charge_perm, T->qperm.p, T->Q * 4);
    d2h(charge_key, T->qkey.p, T->Q * 4);
    d2h(cell_key, T->ckey.p, T->ncell_tot * 4);
    d2h(cell_level, T->clevel.p, T->ncell_tot * 4);
    d2h(cell_range, T->crange.p, T->ncell_tot * 16);
    d2h(cell_parent, T->cparent.p, T->ncell_tot * 4);
    d2h(near_ptr, T->near_ptr.p + T->near_ptr_off[L], ((size_t)T->ncell[L] + 1) * 4);
    d2h(near_idx, T->near_idx.p + T->near_off[L], T->n_near_leaf * 4);
    if (far_pairs && T->nfar) {
      std::vector<int2> ts(T->nfar);
      d2h(ts.data(), T->far_ts.p, T->nfar * sizeof(int2));
      std::vector<int32_t> lev(T->ncell_tot);
      for (int l = 0; l <= L; ++l)
        for (int64_t i = T->coff[l]; i < T->coff[l + 1]; ++i) lev[i] = l;
      for (int64_t k = 0; k < T->nfar; ++k) {
        const int l = lev[ts[k].x];
        far_pairs[3 * k] = l;
        far_pairs[3 * k + 1] = ts[k].x - (int32_t)T->coff[l];
        far_pairs[3 * k + 2] = ts[k].y - (int32_t)T->coff[l];
      }
    }
  });
}

int bemfmm_debug_expansions(bemfmm_tree *tree, int precision, int which, double *out_host) {
  return guard([&] {
    Tree *T = check_tree(tree);
    DeviceScope dev_scope(*T);
    need(out_host != nullptr, "out is NULL");
    HIP_OK(hipDeviceSynchronize());
    debug_expansions(*T, precision, which, out_host, nullptr);
  });
}

int bemfmm_debug_record(bemfmm_tree *tree, int enable) {
  return guard([&] {
    Tree *T = check_tree(tree);
    T->debug_record = enable != 0;
  });
}

int bemfmm_debug_fields(bemfmm_tree *tree, int precision, double *near_host, double *far_host) {
  return guard([&] {
    Tree *T = check_tree(tree);
    DeviceScope dev_scope(*T);
    HIP_OK(hipDeviceSynchronize());
    debug_fields(*T, precision, near_host, far_host, nullptr);
  });
}

int bemfmm_profile(bemfmm_tree *tree, int enable, int reset) {
  return guard([&] {
    Tree *T = check_tree(tree);
    DeviceScope dev_scope(*T);
    T->prof = enable != 0;
    if (reset)
      for (auto &k : T->prof_ms)
        for (auto &pr : k)
          for (auto &v : pr) v = 0;
    if (reset)
      for (auto &k : T->prof_cnt)
        for (auto &pr : k)
          for (auto &v : pr) v = 0;
  });
}

int bemfmm_profile_select(bemfmm_tree *tree, int op, int precision) {
  return guard([&] {
    Tree *T = check_tree(tree);
    DeviceScope dev_scope(*T);
    need(op >= -1 && op < 6, "op must be -1 or a BEMFMM_OP_* value");
    need(precision == -1 || precision == BEMFMM_FP64 || precision == BEMFMM_FP32,
         "precision must be -1, BEMFMM_FP64 or BEMFMM_FP32");
    T->prof_op = op;
    T->prof_sel_prec = precision == -1 ? -1 : (precision == BEMFMM_FP64 ? 0 : 1);
  });
}

int bemfmm_profile_get(bemfmm_tree *tree, const char *stage, double *ms_host, int64_t *count_host) {
  return guard([&] {
    Tree *T = check_tree(tree);
    DeviceScope dev_scope(*T);
    need(stage != nullptr, "stage is NULL");
    static const char *names[7] = {"p2m", "m2m", "m2l", "l2l", "p2p", "other", "l2p"};
    // "name" (every product) or "name/op/precision" (one operator, FP64 = 0 or FP32 = 1)
    const std::string sname(stage);
    const size_t slash = sname.find('/');
    const std::string base = sname.substr(0, slash);
    int k = -1;
    for (int i = 0; i < 7; ++i)
      if (base == names[i]) k = i;
    need(k >= 0, "unknown stage");
    int op = -1, prec = -1;
    if (slash != std::string::npos) {
      need(std::sscanf(sname.c_str() + slash, "/%d/%d", &op, &prec) == 2 && op >= 0 && op < 6 &&
               (prec == 0 || prec == 1),
           "stage filter must be name/op/precision with op 0..5 and precision 0 or 1");
    }
    double ms = 0;
    int64_t cnt = 0;
    for (int kind = 0; kind < 7; ++kind)
      for (int pr = 0; pr < 2; ++pr) {
        if (op >= 0 && (kind != op || pr != prec)) continue;
        ms += T->prof_ms[kind][pr][k];
        cnt += T->prof_cnt[kind][pr][k];
      }
    if (ms_host) *ms_host = ms;
    if (count_host) *count_host = cnt;
  });
}

}  // extern "C"
