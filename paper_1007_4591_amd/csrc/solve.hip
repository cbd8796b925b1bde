// Krylov solve, energies, BIBEE and the adjoint (Sections 2.1 and 2.2).
//
// All vectors are FP64 device arrays in the caller's order.  GMRES keeps its
// Krylov basis in HBM and orthogonalises with classical Gram-Schmidt applied
// twice (two batched passes over the basis per step instead of k sequential
// ones); the small Hessenberg least-squares problem and its Givens rotations
// live on the host in FP64.  Reductions are two-stage with a fixed order, so
// repeated runs give identical bits.
//
// FP32_REFINED: iterative refinement -- the residual r = b - A x is taken with
// the FP64 FMM operator, the correction A d = r is solved by GMRES around the
// FP32 FMM operator to a relative tolerance eta, and x += d.
#include <algorithm>
#include <chrono>
#include <cmath>

#include <functional>

#include "common.h"

namespace bemfmm {

namespace {

constexpr int RB = 256;  // reduction block

__device__ inline double block_sum(double v) {
  __shared__ double sh[RB];
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int w = RB / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  double r = sh[0];
  __syncthreads();
  return r;
}

// partial[i * nb + b] = sum over block b's rows of V_i[r] * w[r]
__global__ void __launch_bounds__(RB) k_dots(const double *__restrict__ V, int64_t ld, const double *__restrict__ w,
                                             int64_t n, int nb, double *__restrict__ partial) {
  const int b = blockIdx.x, i = blockIdx.y;
  const double *v = V + (size_t)i * ld;
  const int64_t per = (n + nb - 1) / nb;
  const int64_t r0 = (int64_t)b * per, r1 = min(n, r0 + per);
  double s = 0.0;
  for (int64_t r = r0 + threadIdx.x; r < r1; r += RB) s += v[r] * w[r];
  s = block_sum(s);
  if (threadIdx.x == 0) partial[(size_t)i * nb + b] = s;
}

// out[i] = sum_b partial[i * nb + b]  (+ out[i] if accumulate)
__global__ void __launch_bounds__(RB) k_reduce(const double *__restrict__ partial, int nb, double *__restrict__ out,
                                               int accumulate) {
  const int i = blockIdx.x;
  double s = 0.0;
  for (int b = threadIdx.x; b < nb; b += RB) s += partial[(size_t)i * nb + b];
  s = block_sum(s);
  if (threadIdx.x == 0) out[i] = accumulate ? out[i] + s : s;
}

// w[r] -= sum_{i < k} h[i] V_i[r]
__global__ void k_orth_update(double *__restrict__ w, const double *__restrict__ V, int64_t ld, int k,
                              const double *__restrict__ h, int64_t n) {
  int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  double acc = 0.0;
  for (int i = 0; i < k; ++i) acc += h[i] * V[(size_t)i * ld + r];
  w[r] -= acc;
}

// x[r] += sum_{i < k} y[i] V_i[r]
__global__ void k_combine_basis(double *__restrict__ x, const double *__restrict__ V, int64_t ld, int k,
                                const double *__restrict__ y, int64_t n) {
  int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  double acc = 0.0;
  for (int i = 0; i < k; ++i) acc += y[i] * V[(size_t)i * ld + r];
  x[r] += acc;
}

__global__ void k_scale(double *__restrict__ y, const double *__restrict__ x, double a, int64_t n) {
  int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r < n) y[r] = a * x[r];
}

// y = x / s[0] (s on device)
__global__ void k_div(double *__restrict__ y, const double *__restrict__ x, const double *__restrict__ s, int64_t n) {
  int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r < n) y[r] = x[r] / s[0];
}

__global__ void k_sub(double *__restrict__ r_, const double *__restrict__ b, const double *__restrict__ ax, int64_t n) {
  int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r < n) r_[r] = b[r] - ax[r];
}

__global__ void k_axpy(double *__restrict__ y, const double *__restrict__ x, double a, int64_t n) {
  int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r < n) y[r] += a * x[r];
}

__global__ void k_sqrt_inplace(double *v) { v[0] = sqrt(v[0]); }

// dG/dq = kappa * phi;  dG/dpos = kappa * q * grad  from [Q x 4] = (phi, gx, gy, gz)
__global__ void k_adjoint_out(const double *__restrict__ pg, const double *__restrict__ q, int64_t Q, double kappa,
                              double *__restrict__ dq, double *__restrict__ dpos) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= Q) return;
  if (dq) dq[i] = kappa * pg[4 * i];
  if (dpos) {
    const double s = kappa * q[i];
    dpos[3 * i] = s * pg[4 * i + 1];
    dpos[3 * i + 1] = s * pg[4 * i + 2];
    dpos[3 * i + 2] = s * pg[4 * i + 3];
  }
}

// reduction scratch (device): partial sums and one result slot
// Each call site passes its own tag, so nested users never share (and
// never reallocate) the same scratch.
struct Ws {
  double *partial = nullptr, *h = nullptr;
  size_t cap = 0;
  Ws(Tree &T, size_t nvec, const char *tag, int64_t nlen = 0) {
    cap = (size_t)std::max(1, std::min(512, (int)((T.N + 4 * 256 - 1) / (4 * 256)))) * std::max<size_t>(nvec, 1);
    const int64_t nmax = std::max<int64_t>(std::max<int64_t>(T.N, T.Q), nlen);
    cap = std::max(cap, (size_t)std::max(1, std::min(512, (int)((nmax + 1023) / 1024))) * std::max<size_t>(nvec, 1));
    partial = T.buf(std::string("wsp_") + tag, cap);
    h = T.buf(std::string("wsh_") + tag, 4);
  }
};

int nblocks_for(int64_t n) { return std::max(1, std::min(512, cdiv(n, 4 * RB))); }

// out_dev[i] = <V_i, w>, i < k (device result)
void dots(Ws &ws, const double *V, int64_t ld, int k, const double *w, int64_t n, double *out_dev, int accumulate,
          hipStream_t s) {
  const int nb = nblocks_for(n);
  if ((size_t)nb * std::max(k, 1) > ws.cap) BF_THROW(BEMFMM_EDEVICE, "reduction scratch too small");
  k_dots<<<dim3(nb, k), RB, 0, s>>>(V, ld, w, n, nb, ws.partial);
  LAUNCH_OK();
  k_reduce<<<k, RB, 0, s>>>(ws.partial, nb, out_dev, accumulate);
  LAUNCH_OK();
}

double dot_host(Ws &ws, const double *a, const double *b, int64_t n, hipStream_t s) {
  dots(ws, a, n, 1, b, n, ws.h, 0, s);
  double v = 0.0;
  HIP_OK(hipMemcpyAsync(&v, ws.h, 8, hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  return v;
}

struct GmresOut {
  int iters = 0;
  double est = 0.0;  // Givens residual estimate relative to |b|
};

// GMRES(m) from x = 0 on the operator A (vectors of length n): stops when
// the Givens estimate |g_{k+1}| <= tol |b| or after maxit steps.
GmresOut gmres_fn(Tree &T, const std::function<void(const double *, double *)> &A, int64_t n, const double *b,
                  double *x, double tol, int maxit, int restart, hipStream_t s) {
  const int m = std::max(1, std::min(restart > 0 ? restart : 30, maxit > 0 ? maxit : 1));
  Ws ws(T, m + 2, "gmres", n);
  struct { double *p; } V{T.buf("gm_V", (size_t)(m + 1) * n)}, w{T.buf("gm_w", n)}, hd{T.buf("gm_hd", 2 * (m + 2))},
      yv{T.buf("gm_y", m + 1)}, r{T.buf("gm_r", n)}, ax{T.buf("gm_ax", n)};
  HIP_OK(hipMemsetAsync(x, 0, n * 8, s));
  GmresOut out;
  const double bnorm = std::sqrt(dot_host(ws, b, b, n, s));
  if (bnorm == 0.0) return out;
  HIP_OK(hipMemcpyAsync(r.p, b, n * 8, hipMemcpyDeviceToDevice, s));
  double beta = bnorm;
  const int TB = 256;
  std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), hh(m + 2), y(m), h1(m + 1), h2(m + 2);
  bool first = true;
  while (out.iters < maxit) {
    if (!first) {
      A(x, ax.p);
      k_sub<<<cdiv(n, TB), TB, 0, s>>>(r.p, b, ax.p, n);
      LAUNCH_OK();
      beta = std::sqrt(dot_host(ws, r.p, r.p, n, s));
    }
    first = false;
    out.est = beta / bnorm;
    if (out.est <= tol) break;
    k_scale<<<cdiv(n, TB), TB, 0, s>>>(V.p, r.p, 1.0 / beta, n);
    LAUNCH_OK();
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    int k = 0;
    for (; k < m && out.iters < maxit; ++k) {
      double *vk = V.p + (size_t)k * n, *vn = V.p + (size_t)(k + 1) * n;
      A(vk, w.p);
      // classical Gram-Schmidt, twice
      dots(ws, V.p, n, k + 1, w.p, n, hd.p, 0, s);
      k_orth_update<<<cdiv(n, TB), TB, 0, s>>>(w.p, V.p, n, k + 1, hd.p, n);
      LAUNCH_OK();
      dots(ws, V.p, n, k + 1, w.p, n, hd.p + (m + 2), 0, s);
      k_orth_update<<<cdiv(n, TB), TB, 0, s>>>(w.p, V.p, n, k + 1, hd.p + (m + 2), n);
      LAUNCH_OK();
      dots(ws, w.p, n, 1, w.p, n, hd.p + (m + 2) + (k + 1), 0, s);
      HIP_OK(hipMemcpyAsync(h1.data(), hd.p, (k + 1) * 8, hipMemcpyDeviceToHost, s));
      HIP_OK(hipMemcpyAsync(h2.data(), hd.p + (m + 2), (k + 2) * 8, hipMemcpyDeviceToHost, s));
      HIP_OK(hipStreamSynchronize(s));
      for (int i = 0; i <= k; ++i) H[(size_t)i * m + k] = h1[i] + h2[i];
      const double hn = std::sqrt(std::max(0.0, h2[k + 1]));
      H[(size_t)(k + 1) * m + k] = hn;
      if (hn > 0.0) {
        k_scale<<<cdiv(n, TB), TB, 0, s>>>(vn, w.p, 1.0 / hn, n);
        LAUNCH_OK();
      }
      for (int i = 0; i < k; ++i) {
        const double a0 = H[(size_t)i * m + k], a1 = H[(size_t)(i + 1) * m + k];
        H[(size_t)i * m + k] = cs[i] * a0 + sn[i] * a1;
        H[(size_t)(i + 1) * m + k] = -sn[i] * a0 + cs[i] * a1;
      }
      const double a0 = H[(size_t)k * m + k], a1 = H[(size_t)(k + 1) * m + k];
      const double den = std::sqrt(a0 * a0 + a1 * a1);
      cs[k] = den > 0.0 ? a0 / den : 1.0;
      sn[k] = den > 0.0 ? a1 / den : 0.0;
      H[(size_t)k * m + k] = den;
      H[(size_t)(k + 1) * m + k] = 0.0;
      g[k + 1] = -sn[k] * g[k];
      g[k] = cs[k] * g[k];
      ++out.iters;
      out.est = std::fabs(g[k + 1]) / bnorm;
      if (out.est <= tol || hn == 0.0) {
        ++k;
        break;
      }
    }
    for (int i = k - 1; i >= 0; --i) {
      double acc = g[i];
      for (int j = i + 1; j < k; ++j) acc -= H[(size_t)i * m + j] * y[j];
      y[i] = acc / H[(size_t)i * m + i];
    }
    if (k > 0) {
      HIP_OK(hipMemcpyAsync(yv.p, y.data(), k * 8, hipMemcpyHostToDevice, s));
      k_combine_basis<<<cdiv(n, TB), TB, 0, s>>>(x, V.p, n, k, yv.p, n);
      LAUNCH_OK();
      HIP_OK(hipStreamSynchronize(s));
    }
    if (out.est <= tol) break;
  }
  HIP_OK(hipStreamSynchronize(s));
  return out;
}

GmresOut gmres(Tree &T, int op, int prec, const double *b, double *x, double tol, int maxit, int restart,
               hipStream_t s) {
  return gmres_fn(
      T, [&](const double *v, double *w) { op_apply(T, op, prec, v, w, s); }, T.N, b, x, tol, maxit, restart, s);
}

double rel_residual64(Tree &T, int op, const double *b, const double *x, double bnorm, hipStream_t s) {
  Ws ws(T, 1, "resid");
  const int64_t n = T.N;
  double *tmp = T.buf("res_tmp", n);
  op_apply(T, op, BEMFMM_FP64, x, tmp, s);
  k_sub<<<cdiv(n, 256), 256, 0, s>>>(tmp, b, tmp, n);
  LAUNCH_OK();
  return std::sqrt(dot_host(ws, tmp, tmp, n, s)) / bnorm;
}

// Solve op x = b (op = A or A^T) at the requested precision; fills info.
void solve_op(Tree &T, int op, const double *b, double *x, double tol, int maxit, int restart, int precision,
              bemfmm_solve_info *info, hipStream_t s) {
  const int64_t n = T.N;
  Ws ws(T, 1, "solve");
  const double bnorm = std::sqrt(dot_host(ws, b, b, n, s));
  bemfmm_solve_info inf{};
  inf.outer_iters = 1;
  if (bnorm == 0.0) {
    HIP_OK(hipMemsetAsync(x, 0, n * 8, s));
    HIP_OK(hipStreamSynchronize(s));
    inf.converged = 1;
    if (info) *info = inf;
    return;
  }
  if (precision != BEMFMM_FP32_REFINED) {
    GmresOut g = gmres(T, op, precision, b, x, tol, maxit, restart, s);
    inf.iters = g.iters;
    inf.rel_residual = rel_residual64(T, op, b, x, bnorm, s);
    inf.converged = inf.rel_residual <= tol;
    if (info) *info = inf;
    return;
  }
  // iterative refinement: FP64 residual, FP32-operator correction
  struct { double *p; } r{T.buf("ir_r", n)}, d{T.buf("ir_d", n)}, tmp{T.buf("ir_tmp", n)};
  HIP_OK(hipMemsetAsync(x, 0, n * 8, s));
  HIP_OK(hipMemcpyAsync(r.p, b, n * 8, hipMemcpyDeviceToDevice, s));
  double rn = bnorm;
  // The FP32 and FP64 FMM operators of one tree differ by rounding only
  // (about 6e-8 relative at p = 10), so the inner solve can go to 2e-7 and
  // one refinement step usually reaches a 1e-6 FP64 residual.
  const double eta_min = 2e-7;
  inf.outer_iters = 0;
  const int max_outer = 20;
  while (rn / bnorm > tol && inf.iters < maxit && inf.outer_iters < max_outer) {
    const double eta = std::max(0.5 * tol * bnorm / rn, eta_min);
    GmresOut g = gmres(T, op, BEMFMM_FP32, r.p, d.p, std::min(eta, 0.5), maxit - inf.iters, restart, s);
    inf.iters += g.iters;
    ++inf.outer_iters;
    k_axpy<<<cdiv(n, 256), 256, 0, s>>>(x, d.p, 1.0, n);
    LAUNCH_OK();
    op_apply(T, op, BEMFMM_FP64, x, tmp.p, s);
    k_sub<<<cdiv(n, 256), 256, 0, s>>>(r.p, b, tmp.p, n);
    LAUNCH_OK();
    rn = std::sqrt(dot_host(ws, r.p, r.p, n, s));
    if (g.iters == 0) break;
  }
  inf.rel_residual = rn / bnorm;
  inf.converged = inf.rel_residual <= tol;
  if (info) *info = inf;
}

}  // namespace

void op_apply(Tree &T, int op, int precision, const double *x, double *y, hipStream_t s) {
  const double f = 1.0 - T.prm.eps_in / T.prm.eps_out;
  const int prec = (precision == BEMFMM_FP64) ? BEMFMM_FP64 : BEMFMM_FP32;
  FmmRequest r{};
  r.y = y;
  switch (op) {
    case BEMFMM_OP_A:  // (1 - f/2) x - f K' x
      r = FmmRequest{SRC_PANEL_MONO, TGT_PANEL, OUT_NGRAD, x, nullptr, true, x, 1.0 - 0.5 * f, -f, false, y, false};
      break;
    case BEMFMM_OP_AT:  // (1 - f/2) x - f a_i DL(x)(c_i)
      r = FmmRequest{SRC_PANEL_DIP, TGT_PANEL, OUT_POT, nullptr, x, false, x, 1.0 - 0.5 * f, -f, true, y, false};
      break;
    case BEMFMM_OP_B:  // normal field of charges x at the panels
      r = FmmRequest{SRC_CHARGE_MONO, TGT_PANEL, OUT_NGRAD, x, nullptr, false, nullptr, 0.0, 1.0, false, y, false};
      break;
    case BEMFMM_OP_BT:  // DL(x) at the charges
      r = FmmRequest{SRC_PANEL_DIP, TGT_CHARGE, OUT_POT, nullptr, x, false, nullptr, 0.0, 1.0, false, y, false};
      break;
    case BEMFMM_OP_C:  // SL(a x) at the charges
      r = FmmRequest{SRC_PANEL_MONO, TGT_CHARGE, OUT_POT, x, nullptr, true, nullptr, 0.0, 1.0, false, y, false};
      break;
    case BEMFMM_OP_CT:  // a_j * potential of the charges x at the panels
      r = FmmRequest{SRC_CHARGE_MONO, TGT_PANEL, OUT_POT, x, nullptr, false, nullptr, 0.0, 1.0, true, y, false};
      break;
    default:
      BF_THROW(BEMFMM_EINVAL, "unknown operator");
  }
  r.op = op;
  const bool to_charges = (op == BEMFMM_OP_BT || op == BEMFMM_OP_C);
  const bool from_charges = (op == BEMFMM_OP_B || op == BEMFMM_OP_CT);
  if ((to_charges || from_charges) && T.Q == 0) {
    if (!to_charges) HIP_OK(hipMemsetAsync(y, 0, T.N * 8, s));
    return;
  }
  fmm_apply(T, prec, r, s);
}

double dot_d(Tree &T, const double *a, const double *b, int64_t n, hipStream_t s) {
  Ws ws(T, 1, "dot", n);
  return dot_host(ws, a, b, n, s);
}

int gmres_apply(Tree &T, const std::function<void(const double *, double *)> &A, int64_t n, const double *b,
                double *x, double tol, int maxit, int restart, hipStream_t s) {
  return gmres_fn(T, A, n, b, x, tol, maxit, restart, s).iters;
}

void solve_bem(Tree &T, const double *q, double *x, double tol, int maxit, int restart, int precision,
               bemfmm_solve_info *info, hipStream_t s) {
  auto t0 = std::chrono::steady_clock::now();
  const int64_t n = T.N;
  const double f = 1.0 - T.prm.eps_in / T.prm.eps_out;
  struct { double *p; } b{T.buf("sv_b", n)};
  // right-hand side f E with E = B q (FP64 operator unless plain FP32)
  op_apply(T, BEMFMM_OP_B, precision == BEMFMM_FP32 ? BEMFMM_FP32 : BEMFMM_FP64, q, b.p, s);
  k_scale<<<cdiv(n, 256), 256, 0, s>>>(b.p, b.p, f, n);
  LAUNCH_OK();
  bemfmm_solve_info inf{};
  solve_op(T, BEMFMM_OP_A, b.p, x, tol, maxit, restart, precision, &inf, s);
  HIP_OK(hipStreamSynchronize(s));
  inf.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (info) *info = inf;
  if (!inf.converged) BF_THROW(BEMFMM_ENOCONV, "GMRES did not reach the tolerance within maxit");
}

double energy(Tree &T, const double *q, const double *x, int precision, hipStream_t s) {
  if (T.Q == 0) return 0.0;
  struct { double *p; } phi{T.buf("en_phi", T.Q)};
  op_apply(T, BEMFMM_OP_C, precision, x, phi.p, s);
  const double kappa = 2.0 * PI * K_COULOMB / T.prm.eps_in;
  return kappa * dot_d(T, q, phi.p, T.Q, s);
}

double bibee(Tree &T, const double *q, int kind, int precision, hipStream_t s) {
  const int64_t n = T.N;
  const double f = 1.0 - T.prm.eps_in / T.prm.eps_out;
  struct { double *p; } xh{T.buf("bb_x", n)};
  op_apply(T, BEMFMM_OP_B, precision, q, xh.p, s);
  // K' replaced by -1/2 (CFA), 0 (P) or +1/2 times the identity, with the
  // interior jump +1/2 kept: x (1 - f (lambda + 1/2)) = f E
  const double scale = (kind == BEMFMM_BIBEE_P) ? f / (1.0 - 0.5 * f) : (kind == BEMFMM_BIBEE_PLUS_HALF) ? f / (1.0 - f) : f;
  k_scale<<<cdiv(n, 256), 256, 0, s>>>(xh.p, xh.p, scale, n);
  LAUNCH_OK();
  return energy(T, q, xh.p, precision, s);
}

double molecule_energy(Tree &T, const double *q, int method, int precision, double tol, int maxit, int restart,
                       hipStream_t s) {
  if (method == BEMFMM_ENERGY_BEM) {
    double *x = T.buf("me_x", T.N);
    solve_bem(T, q, x, tol, maxit, restart, precision, nullptr, s);
    return energy(T, q, x, precision == BEMFMM_FP32 ? BEMFMM_FP32 : BEMFMM_FP64, s);
  }
  const int kind = method == BEMFMM_ENERGY_BIBEE_CFA ? BEMFMM_BIBEE_CFA
                   : method == BEMFMM_ENERGY_BIBEE_P ? BEMFMM_BIBEE_P
                                                     : BEMFMM_BIBEE_PLUS_HALF;
  return bibee(T, q, kind, precision, s);
}

void adjoint(Tree &T, const double *q, const double *x, double tol, int maxit, int restart, int precision,
             double *dq, double *dpos, bemfmm_solve_info *info, hipStream_t s) {
  auto t0 = std::chrono::steady_clock::now();
  const int64_t n = T.N, Q = T.Q;
  const double f = 1.0 - T.prm.eps_in / T.prm.eps_out;
  const double kappa = 2.0 * PI * K_COULOMB / T.prm.eps_in;
  bemfmm_solve_info inf{};
  if (Q == 0) {
    if (info) *info = inf;
    return;
  }
  struct { double *p; } ct{T.buf("ad_ct", n)}, y{T.buf("ad_y", n)}, fy{T.buf("ad_fy", n)}, pg{T.buf("ad_pg", 4 * Q)};
  // A^T y = C^T q
  op_apply(T, BEMFMM_OP_CT, precision == BEMFMM_FP32 ? BEMFMM_FP32 : BEMFMM_FP64, q, ct.p, s);
  solve_op(T, BEMFMM_OP_AT, ct.p, y.p, tol, maxit, restart, precision, &inf, s);
  // phi(r) = SL(a x) + f DL(y) and its gradient at the charges, one FMM
  k_scale<<<cdiv(n, 256), 256, 0, s>>>(fy.p, y.p, f, n);
  LAUNCH_OK();
  FmmRequest r{SRC_PANEL_MONODIP, TGT_CHARGE, OUT_POTGRAD, x, fy.p, true, nullptr, 0.0, 1.0, false, pg.p, false};
  fmm_apply(T, precision == BEMFMM_FP64 ? BEMFMM_FP64 : (precision == BEMFMM_FP32 ? BEMFMM_FP32 : BEMFMM_FP64), r,
            s);
  k_adjoint_out<<<cdiv(Q, 256), 256, 0, s>>>(pg.p, q, Q, kappa, dq, dpos);
  LAUNCH_OK();
  HIP_OK(hipStreamSynchronize(s));
  inf.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (info) *info = inf;
  if (!inf.converged) BF_THROW(BEMFMM_ENOCONV, "adjoint GMRES did not reach the tolerance within maxit");
}

}  // namespace bemfmm
