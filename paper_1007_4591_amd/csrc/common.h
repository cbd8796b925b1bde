// Internal declarations of the bemfmm library (gfx950 / MI355X).
//
// Layout in HBM (all library-owned, allocated at tree build):
//   * panels and charges are kept in Morton order; every per-point array
//     below is indexed by the sorted position;
//   * positions are stored relative to the centre of the point's leaf cell
//     (FP32 and FP64 copies), so FP32 differences inside the near field do
//     not lose digits to the absolute coordinate;
//   * cells of all levels live in one global array, level by level, each
//     level in increasing Morton prefix;
//   * expansions are [cells x PS] (PS = p^2 rounded up to a multiple of 16,
//     zero padded), one array per precision.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cstddef>
#include <functional>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "../../include/bemfmm.h"

namespace bemfmm {

constexpr int KEY_BITS = 10;  // bits per axis of the Morton keys (30-bit keys)
constexpr int LMAX = KEY_BITS;
constexpr int PMAX = 12;
// expansion order with kernels specialised at compile time (the order the
// method is run at, Section 4); other orders take the generic kernels
constexpr int P_FIXED = 10;
// points of the upward pass where the near field can fork to the second stream
enum ForkAt { FORK_START = 0, FORK_AFTER_P2M = 1, FORK_AFTER_M2M = 2, FORK_AFTER_M2L = 3 };
// M2L work tiles: 4 waves x RT row tiles of 16 pairs
constexpr int M2L_RT32 = 4, M2L_RT64 = 2;
constexpr int M2L_ROWS32 = 4 * M2L_RT32 * 16, M2L_ROWS64 = 4 * M2L_RT64 * 16;
// row tiles per wave of the persistent FP32 M2L (a tile list tile is split into
// units of 4 * M2L_PERS_RT * 16 rows)
constexpr int M2L_PERS_RT = 2;
constexpr int LEVEL_RT = 1, LEVEL_ROWS = 4 * LEVEL_RT * 16;  // per-level M2M and L2L tiles
constexpr double PI = 3.14159265358979323846;
constexpr double K_COULOMB = 332.06;

struct Error {
  int code;
  std::string msg;
};

void set_error(const std::string &msg);

#define BF_THROW(code_, msg_)                                                     \
  do {                                                                            \
    throw ::bemfmm::Error{(code_), std::string(msg_)};                            \
  } while (0)

#define HIP_OK(expr)                                                              \
  do {                                                                            \
    hipError_t e_ = (expr);                                                       \
    if (e_ != hipSuccess)                                                         \
      BF_THROW(e_ == hipErrorOutOfMemory ? BEMFMM_ENOMEM : BEMFMM_EDEVICE,        \
               std::string(#expr) + ": " + hipGetErrorString(e_) + " (" __FILE__ ")"); \
  } while (0)

#define LAUNCH_OK() HIP_OK(hipGetLastError())

// Caching device allocator (alloc.cpp): blocks freed by one tree are reused
// by the next build of a similar size instead of going back to the driver.
void *dev_alloc(size_t bytes);
void dev_free(void *p) noexcept;
void dev_cache_release();

// Owning device buffer.
template <class T>
struct DBuf {
  T *p = nullptr;
  size_t n = 0;
  DBuf() = default;
  DBuf(const DBuf &) = delete;
  DBuf &operator=(const DBuf &) = delete;
  ~DBuf() { release(); }
  void release() {
    if (p) dev_free(p);
    p = nullptr;
    n = 0;
  }
  void alloc(size_t count) {
    if (count == n && p) return;
    release();
    if (count == 0) return;
    p = static_cast<T *>(dev_alloc(count * sizeof(T)));
    n = count;
  }
  // grow only
  void reserve(size_t count) {
    if (count > n) alloc(count);
  }
  void zero(hipStream_t s) {
    if (p) HIP_OK(hipMemsetAsync(p, 0, n * sizeof(T), s));
  }
  T *get() const { return p; }
};

inline int cdiv(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }
inline int pad16(int v) { return (v + 15) / 16 * 16; }

// Packed index of Re(n, m) (m >= 0) / Im(n, m) (m >= 1) in a p^2 vector.
__host__ __device__ inline int idx_re(int n, int m) { return m == 0 ? n * n : n * n + 2 * m - 1; }
__host__ __device__ inline int idx_im(int n, int m) { return n * n + 2 * m; }

// Storage order of every expansion row (multipole, local, and the rows of
// the M2L, M2M and L2L products).  A row of ps = pad16(p^2) reals is four
// blocks of ps/4; coefficient k (the packed index above) goes to place
// k div 4 of block k mod 4, so every block holds at most r4 = ceil(p^2/4)
// coefficients and the rest of it is zero.  The MFMA products take one block
// per lane group along K, so the k-steps from r4 on would multiply zeros
// only and are skipped; and a k-step takes consecutive coefficients (4 for
// FP32 and FP64 MFMA, 32 for bf16), of neighbouring degrees and so of
// similar size, which keeps the sums inside one instruction close to exact.
__host__ __device__ inline int coef_r4(int p) { return (p * p + 3) / 4; }
__host__ __device__ inline int coef_pos(int k, int p, int ps) { return (k & 3) * (ps / 4) + (k >> 2); }
// inverse of coef_pos: the coefficient stored at place i, or -1 (padding)
__host__ __device__ inline int coef_at(int i, int p, int ps) {
  const int b = i / (ps / 4), o = i - b * (ps / 4);
  const int k = 4 * o + b;
  return k < p * p ? k : -1;
}
// k-steps of an MFMA product over rows of NT column tiles: the largest r4 of
// the orders whose rows have NT tiles (pad16(p^2) = 16 NT)
constexpr int kk_used(int NT) {
  return NT == 1 ? 4 : NT == 2 ? 7 : NT == 3 ? 9 : NT == 4 ? 16 : NT == 6 ? 21 : NT == 7 ? 25 : NT == 8 ? 31 : NT * 4;
}

// ---------------------------------------------------------------- tables

// FP64 translation operators for order p and a MAC (host-built, cached).
struct Tables {
  int p = 0, ps = 0;
  double theta = 0;
  int mac = 0;
  int R = 0;                       // offsets lie in [-R, R]^3
  std::vector<int> offset_id;      // (2R+1)^3 -> compact id or -1
  std::vector<int> offsets;        // compact id -> (ox, oy, oz)
  std::vector<double> m2l;         // [noff][ps][ps] (row = output, col = input)
  std::vector<double> m2m;         // [8][ps][ps]  child octant -> parent
  std::vector<double> l2l;         // [8][ps][ps]  parent -> child octant
  int noff() const { return (int)offsets.size() / 3; }
};

const Tables &get_tables(int p, double theta, int mac);
bool mac_far_host(int ox, int oy, int oz, double theta, int mac);

// ---------------------------------------------------------------- tree

struct PrecBufs;  // per-precision FMM buffers (fmm.hip)
struct LpbState;  // screened-kernel state of a tree (yukawa.hip)

struct Tree {
  int magic = 0x5eedbe11;
  int device = 0;
  bemfmm_params prm{};
  int p = 10, ps = 112;
  int64_t N = 0, Q = 0;
  int L = 0;
  double lo[3] = {0, 0, 0};
  double side = 1;
  std::vector<int> ncell;       // per level
  std::vector<int64_t> coff;    // per level offset into global cell arrays (size L+2)
  int64_t ncell_tot = 0;

  // user-order geometry (FP64)
  DBuf<double> c, nrm, area;  // 3N, 3N, N
  DBuf<double> pverts;        // 9N: the three vertices of each panel (caller order)
  DBuf<double> qpos;          // 3Q user-order charge positions (current)

  // Morton order
  DBuf<int32_t> pperm, qperm;     // sorted -> user
  DBuf<int32_t> pinv, qinv;       // user -> sorted
  DBuf<uint32_t> pkey, qkey;      // sorted keys
  DBuf<int32_t> pleaf, qleaf;     // leaf (level-L local) index of each sorted point

  // sorted point data, leaf-relative
  DBuf<float4> p32pos, p32nrm;    // (rx, ry, rz, area), (nx, ny, nz, 0)
  DBuf<double4> p64pos, p64nrm;
  DBuf<float4> q32pos;            // (rx, ry, rz, 0)
  DBuf<double4> q64pos;

  // cells (global over levels)
  DBuf<uint32_t> ckey;    // level prefix
  DBuf<int32_t> clevel;
  DBuf<int4> crange;      // panel begin, end, charge begin, end
  DBuf<int32_t> cparent;  // global index (-1 root)
  DBuf<int2> cchild;      // global child range [b, e)
  DBuf<int32_t> cxyz;     // packed integer coords x | y << 10 | z << 20

  // lists
  std::vector<int64_t> near_off;     // per level offsets into near_idx (levels 0..L), size L+2
  DBuf<int32_t> near_ptr;            // per level CSR, concatenated: [sum (ncell_l + 1)]
  std::vector<int64_t> near_ptr_off; // per level offset into near_ptr
  DBuf<int32_t> near_idx;            // level-local source cells
  int64_t n_near_leaf = 0;

  std::vector<int64_t> far_off;      // per level offsets into far pairs (size L+2)
  int64_t nfar = 0;
  DBuf<int2> far_ts;                 // (target, source) level-local, target-major per level
  DBuf<int32_t> far_ptr;             // per-level target CSR into far pairs (global pair index), [ncell_tot + 1]
  // M2L work lists, one per (source kind, target kind): 0 panels -> panels,
  // 1 charges -> panels, 2 panels -> charges.  Only pairs whose source cell
  // holds sources and whose target cell holds targets of that kind are kept;
  // they are sorted by translation offset (all levels together).
  struct M2LList {
    DBuf<int32_t> src;               // source cell (global index) of each kept pair, offset-sorted
                                     // (= M2L output row order)
    DBuf<int32_t> dest;              // output row of each kept pair: rows are in pair order
                                     // (level, target, source), so a cell's rows are contiguous
    DBuf<int32_t> kptr;              // [cells + 1] first output row of each cell
    DBuf<int32_t> group_off;         // per offset group: compact offset id
    DBuf<int32_t> group_end;         // per group: end row
    DBuf<int32_t> tile_group, tile_row;      // FP32 tiles of M2L_ROWS32 rows
    DBuf<int32_t> tile_group64, tile_row64;  // FP64 tiles of M2L_ROWS64 rows
    int64_t n = 0, ngroups = 0, ntiles = 0, ntiles64 = 0;
  } m2l[3];
  int64_t p2p_pairs_pp = 0;

  // translation tables on the device, shared by every tree with the same
  // (device, p, MAC) and kept until the process ends
  const Tables *tab = nullptr;
  const float *t_m2l32 = nullptr;   // [noff][PS/4 kk][PS/16 ct][64 lanes], MFMA B-operand order
  const double *t_m2l64 = nullptr;  // same layout
  // the M2L operators of order P_FIXED as three bf16 parts each (bit
  // patterns), in the B-operand order of the split-bf16 M2L; null for other
  // orders
  const uint16_t *t_m2lbf = nullptr;
  // M2M and L2L: [8 octants][PS/4 kk][PS/16 ct][64 lanes], MFMA B-operand order
  const float *t_m2m32 = nullptr, *t_l2l32 = nullptr;
  const double *t_m2m64 = nullptr, *t_l2l64 = nullptr;

  // L2L and M2M as batched MFMA products, per level l >= 3: rows are the
  // level's cells grouped by octant (the operators depend on the octant
  // only); src = parent cell (L2L input), self = the cell (M2M input), both
  // global indices; dest = cell index within the level.  Tiles of level l
  // are [t0[l], t1[l]) in both precisions.
  struct L2LList {
    DBuf<int32_t> src, self, dest, group_off, group_end;
    // tiles of 64 rows (4 waves x one row tile of 16): the per-level products
    // are small, so short tiles give more workgroups and shorter MFMA chains
    DBuf<int32_t> tile_group, tile_row;
    std::vector<int64_t> t0, t1;
    int64_t max_cells = 0;
  } l2lw;

  // near quadrature (params.near_quad = nu > 0): per sorted panel, the close
  // source panels (|c_t - c_j| < nu rho_j) as a CSR of caller indices, with
  // 4 pi (K'_tj exact - K'_tj one-point) in FP64, for A; and the transposed
  // lists for A^T (K'_it; the product divides by the area of t), added to the
  // near field
  DBuf<int32_t> nq_ptr, nq_idx, nqT_ptr, nqT_idx;
  DBuf<double> nq_coef, nqT_coef;
  int64_t n_nq = 0, n_nqT = 0;

  // P2P work decomposition: (leaf, first sorted index, count, lane groups)
  // per chunk of at most 64 targets of one leaf
  DBuf<int4> chunk_p, chunk_q;
  int64_t nchunk_p = 0, nchunk_q = 0;

  PrecBufs *pb32 = nullptr, *pb64 = nullptr;
  LpbState *lpb = nullptr;  // screened-kernel tables, lists and buffers (yukawa.hip)

  // persistent FP64 work vectors of the solvers, by purpose (grow only)
  std::map<std::string, std::unique_ptr<DBuf<double>>> work;
  double *buf(const std::string &name, size_t n) {
    auto &b = work[name];
    if (!b) b.reset(new DBuf<double>());
    b->reserve(std::max<size_t>(n, 1));
    return b->p;
  }

  // second stream for the near field (default priority) and its fork/join
  // events; stage profiling events
  hipStream_t side_stream = nullptr;
  bool concurrent = true;        // near field on the second stream
  bool m2l_persistent = true;    // FP32 M2L: persistent workgroups (else one tile per workgroup)
  bool m2l_split = true;         // persistent FP32 M2L of order P_FIXED on split-bf16 MFMA (else FP32 MFMA)
  int fork_at = -1;              // where the near field forks: a ForkAt value, -1 = per precision
  int n_cu = 256;                // compute units of the device
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  bool prof = false;
  int prof_op = -1, prof_sel_prec = -1;  // record only this operator / precision (-1: any)
  bool prof_now = false;                  // the product being run is recorded
  // stage times per [product kind: the six operators, then any other][FP64, FP32][stage]
  double prof_ms[7][2][7] = {};
  int64_t prof_cnt[7][2][7] = {};
  bool prof_pending[7] = {false, false, false, false, false, false, false};
  int prof_kind = 6, prof_prec = 0;  // product being timed
  hipEvent_t ev[14] = {};
  bool ev_init = false;

  int last_op32 = -1, last_op64 = -1;
  bool debug_record = false;  // products also write their near and far parts (bemfmm_debug_fields)

  ~Tree();
};

Tree *check_tree(const bemfmm_tree *t);

// tree_build.hip
void build_tree(Tree &T, const double *verts, int64_t nv, const int32_t *tris, int64_t nt,
                const double *qpos, int64_t nq, hipStream_t s);
void build_nearquad(Tree &T, const double *verts, const int32_t *tris, hipStream_t s);
void set_charges(Tree &T, const double *qpos, hipStream_t s);
void set_charges_noalloc(Tree &T, const double *qpos, hipStream_t s);
int64_t noalloc_max_charges();
void upload_tables(Tree &T, hipStream_t s);

// primitives (tree_build.hip)
void exclusive_scan_i32(const int32_t *in, int32_t *out, int64_t n, hipStream_t s, int32_t *total_host);
void radix_sort_u32(uint32_t *keys, int32_t *vals, int64_t n, int bits, hipStream_t s);

// fmm.hip
enum SrcKind { SRC_PANEL_MONO = 0, SRC_PANEL_DIP = 1, SRC_PANEL_MONODIP = 2, SRC_CHARGE_MONO = 3 };
enum TgtKind { TGT_PANEL = 0, TGT_CHARGE = 1 };
enum OutKind { OUT_POT = 0, OUT_NGRAD = 1, OUT_POTGRAD = 2 };

struct FmmRequest {
  int src;          // SrcKind
  int tgt;          // TgtKind
  int out;          // OutKind
  const double *wmono;  // user-order monopole weights (panels: multiplied by area inside) or NULL
  const double *wdip;   // user-order dipole strengths (along panel normals) or NULL
  bool mono_area;       // panel monopoles: weight = area * wmono
  // epilogue: y[user] = alpha * xin[user] + beta * (area_scale ? a : 1) * field / (4 pi)
  const double *xin;
  double alpha, beta;
  bool area_scale;
  double *y;            // OUT_POT/NGRAD: [n_targets]; OUT_POTGRAD: [n_targets*4] (pot, gx, gy, gz)
  bool accumulate;      // y += instead of y =
  int op = -1;          // BEMFMM_OP_* this request implements (-1: another product), for stage timing
  bool far_only = false;  // skip the near field (the caller adds its own direct sums)
};

void fmm_apply(Tree &T, int precision, const FmmRequest &rq, hipStream_t s);
void fmm_free(Tree &T);
void debug_expansions(Tree &T, int precision, int which, double *out_host, hipStream_t s);
void debug_fields(Tree &T, int precision, double *near_host, double *far_host, hipStream_t s);

// solve.hip
void op_apply(Tree &T, int op, int precision, const double *x, double *y, hipStream_t s);
void solve_bem(Tree &T, const double *q, double *x, double tol, int maxit, int restart, int precision,
               bemfmm_solve_info *info, hipStream_t s);
double energy(Tree &T, const double *q, const double *x, int precision, hipStream_t s);
double bibee(Tree &T, const double *q, int kind, int precision, hipStream_t s);
// solvation energy of one tree by the full BEM solve or a BIBEE variant (bemfmm_energy_method)
double molecule_energy(Tree &T, const double *q, int method, int precision, double tol, int maxit, int restart,
                       hipStream_t s);
void adjoint(Tree &T, const double *q, const double *x, double tol, int maxit, int restart, int precision,
             double *dq, double *dpos, bemfmm_solve_info *info, hipStream_t s);
double dot_d(Tree &T, const double *a, const double *b, int64_t n, hipStream_t s);
// GMRES(restart) from x = 0 on any operator of vectors of length n; returns the iterations
int gmres_apply(Tree &T, const std::function<void(const double *, double *)> &A, int64_t n, const double *b,
                double *x, double tol, int maxit, int restart, hipStream_t s);

// FP64 building blocks of the FMM shared with the screened-kernel (Yukawa)
// far field of yukawa.hip: the batched per-level MFMA product (M2M when m2m,
// else L2L) with a given octant table, the parents' sums of M2M rows, the
// offset-grouped MFMA M2L over a work list with a given operator table, and
// the downward pass of one level without leaf evaluation coefficients.
void level_product64(Tree &T, int l, const int32_t *src, const double *table, const double *in, double *out,
                     bool m2m, hipStream_t s);
void m2m_sum64(Tree &T, int l, const double *rows, double *M, hipStream_t s);
void m2l_tiles64(const Tree::M2LList &ML, int ps, const double *table, const double *M, double *out, hipStream_t s);
void downward64(Tree &T, int l, const double *l2l_rows, const int32_t *kptr, const double *m2l_rows, double *Lx,
                hipStream_t s);

// linearised Poisson-Boltzmann (yukawa.hip)
void lpb_free(Tree &T);
void lpb_matvec(Tree &T, double kappa, const double *uv, double *y, hipStream_t s);
void lpb_solve(Tree &T, const double *q, double kappa, double *uv, double tol, int maxit, int restart,
               bemfmm_solve_info *info, hipStream_t s);
double lpb_energy(Tree &T, const double *q, const double *uv, hipStream_t s);

// profiling helpers (fmm.hip)
enum Stage { ST_P2M = 0, ST_M2M = 1, ST_M2L = 2, ST_L2L = 3, ST_P2P = 4, ST_OTHER = 5, ST_L2P = 6 };
void prof_begin(Tree &T, int stage, hipStream_t s);
void prof_end(Tree &T, int stage, hipStream_t s);

}  // namespace bemfmm
