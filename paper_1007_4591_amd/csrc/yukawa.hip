// Screened-Coulomb (Yukawa) FMM and the linearised Poisson-Boltzmann BEM
// operator (Section 2.1: the screened solvent, lap phi = kappa^2 phi outside
// the molecule, is the model the method is being extended to; Section 5
// names it as the next step).
//
// Formulation.  Unknowns u = phi and v = d phi / dn on the interior side of
// the surface, collocated at the panel centroids, one point per panel.  With
// G0 = 1/(4 pi r), Gk = exp(-kappa r)/(4 pi r), h = G0 - Gk,
// eps = eps_out/eps_in, the interior Green identity plus eps times the
// exterior one, and the sum of their normal derivatives, give
//   (1+eps)/2 u + (K0 - eps Kk) u - (V0 - Vk) v = S
//   (1+1/eps)/2 v - (K0' - Kk'/eps) v + (D0 - Dk) u = dS/dn,
// S = sum_k q_k G0(x, r_k)/eps_in (V single layer, K double layer, K' its
// adjoint, D the normal derivative of the double layer).  The product is
// split as the FMM splits every sum:
//   * far field of the Laplace part: the existing FMM with monopoles a v and
//     dipoles -a u (P0 = SL0(a v) - DL0(a u), potential and gradient);
//   * far field of the screened part: this file's FMM with monopoles a v and
//     dipoles -eps a u (Pk, potential and normal derivative);
//   * near field of both kernels together, pair by pair in FP64, with the
//     difference kernels h, h', h'' formed directly;
//   * self terms: 0 for the double-layer kinds (flat panels), and the exact
//     integrals over the panel of h and of -h'(R)/R (polar integration about
//     the centroid, 32-point Gauss-Legendre per edge).
//   y_u = (1+eps)/2 u - P0 + Pk + near_u - Vself v
//   y_v = (1+1/eps)/2 v - n.grad P0 + n.grad Pk / eps + near_v + Dself u
// The energy is 2 pi K q^T phi_reac with phi_reac = SL0(a v) - DL0(a u) at
// the charges (the Laplace FMM with charge targets).
//
// Expansions of the screened kernel.  With Y_nm the real orthonormal
// spherical harmonics (packed index n^2 for m = 0, n^2 + 2m - 1 and n^2 + 2m
// for the cos and sin parts), and i_n, k_n the modified spherical Bessel
// functions normalised so that i_0(x) = sinh(x)/x and k_0(x) = exp(-x)/x,
//   exp(-kappa|x - y|) / (4 pi |x - y|) = kappa sum_nm i_n(kappa r<) k_n(kappa r>) Y_nm(x^) Y_nm(y^).
// A cell's multipole expansion is kappa sum M_nm k_n(kappa rho) Y_nm with
// M_nm = sum_j w_j i_n(kappa rho_j) Y_nm(rho_j^) (and the derivative of that
// along a dipole's direction), its local expansion sum L_nm i_n(kappa rho) Y_nm.
// i_n(kappa rho) Y_nm = g_n(rho^2) R_nm, where R_nm = rho^n Y_nm is a
// polynomial (Cartesian recurrence below) and
// g_n(s) = kappa^n / (2n+1)!! sum_k (kappa^2 s / 2)^k / (k! (2n+3)(2n+5)...(2n+2k+1))
// is entire, so P2M and L2P need no Bessel functions at all.
//
// Translation operators depend on kappa times the cell side, so there is
// one set per level.  Each is the truncated operator itself, built on the
// GPU by projection: the source basis function is evaluated on a sphere
// about the target centre and projected on the target basis with a
// Gauss-Legendre (in cos theta) by trapezoidal (in phi) rule of 32 x 64
// nodes, exact for products of band limit below 64.  The rest of the
// far field (batched M2M and L2L, offset-grouped M2L, downward sums) runs on
// the same MFMA kernels as the Laplace FMM, with the per-level tables; the
// M2L work list is the Laplace one regrouped by (level, offset).  FP64 only.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <functional>
#include <mutex>
#include <vector>

#include "common.h"

namespace bemfmm {

// one translation operator to build by projection
struct YkTask {
  double cx, cy, cz;  // centre of the source basis function, relative to the projection centre
  double rho0;        // radius of the projection sphere
  int irregular;      // source basis: kappa k_n(kappa r) Y_nm (1) or i_n(kappa r) Y_nm (0)
  int multipole;      // target basis: kappa k_n Y_nm (1) or i_n Y_nm (0)
  int slot;           // output operator
  int pad;
};

namespace {

constexpr int YQ_T = 32, YQ_P = 64, YQ_N = YQ_T * YQ_P;  // projection rule
constexpr int YQ_CHUNK = 64;                              // quadrature points per LDS chunk
constexpr int YK_THREADS = 1024;                          // projection workgroup
constexpr int YK_ACC = 16;                                // projection outputs per thread (p <= 11: 121^2 / 1024 < 15)
constexpr int SELF_GL = 32;                               // Gauss-Legendre points per edge, self integrals

__constant__ double c_ya[PMAX][PMAX];  // Q_n^m = a z Q_{n-1}^m - b rho^2 Q_{n-2}^m (normalised)
__constant__ double c_yb[PMAX][PMAX];
__constant__ double c_yd[PMAX];        // Q_m^m = d_m (x + i y)^m
__constant__ double c_gl_x[SELF_GL], c_gl_w[SELF_GL];

// Gauss-Legendre nodes and weights on [-1, 1] (Newton on P_n from the
// Chebyshev guesses)
void gauss_legendre(int n, std::vector<double> &x, std::vector<double> &w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    double z = std::cos(PI * (i + 0.75) / (n + 0.5)), dp = 0.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      const double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    double p0 = 1.0, p1 = z;
    for (int k = 2; k <= n; ++k) {
      const double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    dp = n * (z * p1 - p0) / (z * z - 1.0);
    x[i] = z;
    w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

// normalisation of the real harmonics: sqrt((2n+1)/(4 pi) (n-m)!/(n+m)!), times sqrt 2 for m > 0
double ynorm(int n, int m) {
  double r = (2 * n + 1) / (4.0 * PI);
  for (int k = n - m + 1; k <= n + m; ++k) r /= k;
  return std::sqrt(r) * (m > 0 ? std::sqrt(2.0) : 1.0);
}

void set_yk_constants() {
  static std::mutex mu;
  static std::vector<int> done;
  int dev = 0;
  HIP_OK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> g(mu);
  if (std::find(done.begin(), done.end(), dev) != done.end()) return;
  double a[PMAX][PMAX] = {}, b[PMAX][PMAX] = {}, d[PMAX] = {};
  for (int m = 0; m < PMAX; ++m) {
    double df = 1.0;
    for (int k = 2 * m - 1; k > 0; k -= 2) df *= k;
    d[m] = ynorm(m, m) * df;
    for (int n = m + 1; n < PMAX; ++n) {
      a[n][m] = ynorm(n, m) / ynorm(n - 1, m) * (2 * n - 1) / double(n - m);
      b[n][m] = (n >= m + 2) ? ynorm(n, m) / ynorm(n - 2, m) * (n + m - 1) / double(n - m) : 0.0;
    }
  }
  std::vector<double> gx, gw;
  gauss_legendre(SELF_GL, gx, gw);
  HIP_OK(hipMemcpyToSymbol(HIP_SYMBOL(c_ya), a, sizeof(a)));
  HIP_OK(hipMemcpyToSymbol(HIP_SYMBOL(c_yb), b, sizeof(b)));
  HIP_OK(hipMemcpyToSymbol(HIP_SYMBOL(c_yd), d, sizeof(d)));
  HIP_OK(hipMemcpyToSymbol(HIP_SYMBOL(c_gl_x), gx.data(), SELF_GL * sizeof(double)));
  HIP_OK(hipMemcpyToSymbol(HIP_SYMBOL(c_gl_w), gw.data(), SELF_GL * sizeof(double)));
  done.push_back(dev);
}

// R_nm = rho^n Y_nm at (x, y, z) for n < p; with DER also the derivative
// along (dx, dy, dz).  term(k, n, value, derivative) for each packed index k.
template <bool DER, class F>
__device__ inline void yk_solid(int p, double x, double y, double z, double dx, double dy, double dz, F &&term) {
  const double r2 = x * x + y * y + z * z;
  const double dr2 = DER ? 2.0 * (x * dx + y * dy + z * dz) : 0.0;
  double wr = 1.0, wi = 0.0, dwr = 0.0, dwi = 0.0;  // (x + i y)^m
  for (int m = 0; m < p; ++m) {
    if (m > 0) {
      const double nr = wr * x - wi * y, ni = wr * y + wi * x;
      if (DER) {
        const double ndr = dwr * x + wr * dx - dwi * y - wi * dy;
        const double ndi = dwr * y + wr * dy + dwi * x + wi * dx;
        dwr = ndr;
        dwi = ndi;
      }
      wr = nr;
      wi = ni;
    }
    double cr = c_yd[m] * wr, ci = c_yd[m] * wi, dcr = DER ? c_yd[m] * dwr : 0.0, dci = DER ? c_yd[m] * dwi : 0.0;
    double pr = 0.0, pi = 0.0, dpr = 0.0, dpi = 0.0;  // degree n - 1
    for (int n = m; n < p; ++n) {
      if (n > m) {
        const double a = c_ya[n][m], b = c_yb[n][m];
        const double nr = a * z * cr - b * r2 * pr, ni = a * z * ci - b * r2 * pi;
        double ndr = 0.0, ndi = 0.0;
        if (DER) {
          ndr = a * (dz * cr + z * dcr) - b * (dr2 * pr + r2 * dpr);
          ndi = a * (dz * ci + z * dci) - b * (dr2 * pi + r2 * dpi);
        }
        pr = cr;
        pi = ci;
        dpr = dcr;
        dpi = dci;
        cr = nr;
        ci = ni;
        dcr = ndr;
        dci = ndi;
      }
      if (m == 0) {
        term(n * n, n, cr, dcr);
      } else {
        term(n * n + 2 * m - 1, n, cr, dcr);
        term(n * n + 2 * m, n, ci, dci);
      }
    }
  }
}

// g_n(s) and dg_n/ds at s = rho^2, n < p
__device__ inline void yk_g(int p, double kappa, double s, double *g, double *gp) {
  const double hk = 0.5 * kappa * kappa;
  double pref = 1.0;
  for (int n = 0; n < p; ++n) {
    if (n > 0) pref *= kappa / (2 * n + 1);
    double t = 1.0, sum = 1.0, dsum = 0.0;
    for (int k = 1; k < 400; ++k) {
      const double f = hk / (2 * n + 2 * k + 1);
      dsum += t * f;  // k c_k s^(k-1) = t_(k-1) f
      t *= f * s / k;
      sum += t;
      if (t <= 1e-18 * sum && t * f <= 1e-18 * dsum * s + 1e-300) break;
    }
    g[n] = pref * sum;
    gp[n] = pref * dsum;
  }
}

// k_n(x) for n < p (k_0 = exp(-x)/x), upward recurrence (stable for k)
__device__ inline void yk_khat(int p, double x, double *k) {
  const double e = exp(-x);
  k[0] = e / x;
  if (p > 1) k[1] = e * (x + 1.0) / (x * x);
  for (int n = 1; n + 1 < p; ++n) k[n + 1] = k[n - 1] + (2 * n + 1) / x * k[n];
}

// One translation operator per workgroup of 1024 threads: T[o][i] =
// (1 / target radial factor at rho0) * sum over the nodes of
// w_q Y_o(u_q) B_i(rho0 u_q - C), written in the MFMA B-operand order of the
// M2L kernel (padding places are left as the caller zeroed them).  Per chunk
// of 64 nodes, 64 threads evaluate the source basis at their node and 64 the
// weighted target harmonics (radial factors through LDS); then thread t
// accumulates column t % p^2 for up to 16 rows.
__global__ void __launch_bounds__(YK_THREADS) k_yk_project(int p, int ps, double kappa, const YkTask *__restrict__ tasks,
                                                           const double4 *__restrict__ quad,
                                                           double *__restrict__ tables) {
  extern __shared__ double smem[];
  const int np2 = p * p;
  double *Bv = smem;                      // [YQ_CHUNK][np2] source basis at the nodes
  double *Wv = Bv + YQ_CHUNK * np2;       // [YQ_CHUNK][np2] w_q Y_o(u_q)
  double *rad = Wv + YQ_CHUNK * np2;      // [YQ_CHUNK][PMAX] radial factors
  double *aux = rad + YQ_CHUNK * PMAX;    // [YQ_CHUNK][PMAX] work space
  double *norm = aux + YQ_CHUNK * PMAX;   // [PMAX] 1 / target radial factor at rho0
  const YkTask tk = tasks[blockIdx.x];
  const int tid = threadIdx.x;
  const int ngroups = YK_THREADS / np2, rows = (np2 + ngroups - 1) / ngroups;
  const int col = tid % np2, grp = tid / np2;
  const bool mine = grp < ngroups;
  if (tid == 0) {
    if (tk.multipole) {
      yk_khat(p, kappa * tk.rho0, aux);
      for (int n = 0; n < p; ++n) norm[n] = 1.0 / (kappa * aux[n]);
    } else {
      yk_g(p, kappa, tk.rho0 * tk.rho0, aux, aux + PMAX);
      double rp = 1.0;
      for (int n = 0; n < p; ++n) {
        norm[n] = 1.0 / (aux[n] * rp);
        rp *= tk.rho0;
      }
    }
  }
  __syncthreads();
  double acc[YK_ACC];
#pragma unroll
  for (int k = 0; k < YK_ACC; ++k) acc[k] = 0.0;
  for (int c0 = 0; c0 < YQ_N; c0 += YQ_CHUNK) {
    if (tid < YQ_CHUNK) {
      const double4 u = quad[c0 + tid];
      const double x = tk.rho0 * u.x - tk.cx, y = tk.rho0 * u.y - tk.cy, z = tk.rho0 * u.z - tk.cz;
      const double r2 = x * x + y * y + z * z;
      double *rd = rad + tid * PMAX, *ax = aux + tid * PMAX;
      if (tk.irregular) {
        const double r = sqrt(r2);
        yk_khat(p, kappa * r, ax);
        double rp = 1.0;  // r^-n
        for (int n = 0; n < p; ++n) {
          rd[n] = kappa * ax[n] * rp;
          rp /= r;
        }
      } else {
        double gp[PMAX];
        yk_g(p, kappa, r2, rd, gp);
      }
      double *row = Bv + tid * np2;
      yk_solid<false>(p, x, y, z, 0.0, 0.0, 0.0, [&](int k, int n, double v, double) { row[k] = rd[n] * v; });
    } else if (tid < 2 * YQ_CHUNK) {
      const int q = tid - YQ_CHUNK;
      const double4 u = quad[c0 + q];
      double *row = Wv + q * np2;
      yk_solid<false>(p, u.x, u.y, u.z, 0.0, 0.0, 0.0, [&](int k, int, double v, double) { row[k] = u.w * v; });
    }
    __syncthreads();
    if (mine) {
      for (int q = 0; q < YQ_CHUNK; ++q) {
        const double b = Bv[q * np2 + col];
        const double *w = Wv + q * np2 + grp * rows;
#pragma unroll
        for (int k = 0; k < YK_ACC; ++k)
          if (k < rows && grp * rows + k < np2) acc[k] += w[k] * b;
      }
    }
    __syncthreads();
  }
  if (!mine) return;
  const int KK = ps / 4, NT = ps / 16;
  const int pi = coef_pos(col, p, ps);
  const int gq = pi / KK, kk = pi - gq * KK;
#pragma unroll
  for (int k = 0; k < YK_ACC; ++k) {
    const int o = grp * rows + k;
    if (k < rows && o < np2) {
      int no = 0;
      while ((no + 1) * (no + 1) <= o) ++no;
      const int po = coef_pos(o, p, ps);
      const int ct = po / 16, lo = po - ct * 16;
      const size_t at = (((size_t)tk.slot * KK + kk) * NT + ct) * 64 + gq * 16 + lo;
      tables[at] = acc[k] * norm[no];
    }
  }
}

// P2M of the screened kernel at the leaves: one wave per leaf, each lane
// sums its sources into its own LDS row, then the 64 rows are added in lane
// order.  w = (monopole weight, dipole weight along the panel normal).
__global__ void __launch_bounds__(64) k_yk_p2m(int p, int ps, const int4 *__restrict__ leaf_range,
                                               const double4 *__restrict__ pos, const double4 *__restrict__ nrm,
                                               const double2 *__restrict__ w, double kappa, double *__restrict__ M) {
  extern __shared__ double part[];  // [64][np2]
  const int np2 = p * p, lane = threadIdx.x;
  const int4 rg = leaf_range[blockIdx.x];
  double *mine = part + lane * np2;
  for (int k = 0; k < np2; ++k) mine[k] = 0.0;
  for (int j = rg.x + lane; j < rg.y; j += 64) {
    const double4 r = pos[j], n4 = nrm[j];
    const double2 ww = w[j];
    double g[PMAX], gp[PMAX];
    yk_g(p, kappa, r.x * r.x + r.y * r.y + r.z * r.z, g, gp);
    const double nd = n4.x * r.x + n4.y * r.y + n4.z * r.z;
    yk_solid<true>(p, r.x, r.y, r.z, n4.x, n4.y, n4.z, [&](int k, int n, double v, double dv) {
      mine[k] += ww.x * g[n] * v + ww.y * (2.0 * gp[n] * nd * v + g[n] * dv);
    });
  }
  __syncthreads();
  double *row = M + (size_t)blockIdx.x * ps;
  for (int i = lane; i < ps; i += 64) {
    const int k = coef_at(i, p, ps);
    double s = 0.0;
    if (k >= 0)
      for (int l = 0; l < 64; ++l) s += part[l * np2 + k];
    row[i] = s;
  }
}

// L2P of the screened kernel at every panel: potential and normal derivative
__global__ void k_yk_l2p(int p, int ps, int64_t N, const int32_t *__restrict__ pleaf, const double4 *__restrict__ pos,
                         const double4 *__restrict__ nrm, const double *__restrict__ Lleaf, double kappa,
                         double2 *__restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N) return;
  const double *Lr = Lleaf + (size_t)pleaf[t] * ps;
  const double4 r = pos[t], n4 = nrm[t];
  double g[PMAX], gp[PMAX];
  yk_g(p, kappa, r.x * r.x + r.y * r.y + r.z * r.z, g, gp);
  const double nd = n4.x * r.x + n4.y * r.y + n4.z * r.z;
  double phi = 0.0, dphi = 0.0;
  yk_solid<true>(p, r.x, r.y, r.z, n4.x, n4.y, n4.z, [&](int k, int n, double v, double dv) {
    const double c = Lr[coef_pos(k, p, ps)];
    phi += c * g[n] * v;
    dphi += c * (2.0 * gp[n] * nd * v + g[n] * dv);
  });
  out[t] = make_double2(phi, dphi);
}

// e^{-x} for 0 <= x <= 745 (the near field's kappa r).  With k the integer
// nearest to 64 x / ln 2, k = 64 n + j (0 <= j < 64) and r = x - k ln 2 / 64
// (|r| <= ln 2 / 128), e^{-x} = 2^{-n} 2^{-j/64} e^{-r}: 2^{-j/64} comes from
// a table (tab, 64 entries in LDS) and e^{-r} from its Taylor polynomial of
// degree 5, whose remainder is below 3.4e-17 relative.  r is reduced with
// ln 2 / 64 split in two: the leading part has 32 significant bits, so k
// times it is exact for every k below 2^21 and so is its difference with x;
// the result is within 2 ulp of e^{-x}.
__device__ __forceinline__ double exp_neg(double x, const double *tab) {
  constexpr double C_HI = 0x1.62e42fee00000p-7, C_LO = 0x1.a39ef35793c76p-39;  // ln 2 / 64 = C_HI + C_LO
  const double k = __builtin_rint(x * (64.0 / 0.69314718055994530942));
  const double r = __builtin_fma(-k, C_LO, __builtin_fma(-k, C_HI, x));
  double q = __builtin_fma(r, -1.0 / 120.0, 1.0 / 24.0);
  q = __builtin_fma(q, r, -1.0 / 6.0);
  q = __builtin_fma(q, r, 0.5);
  q = __builtin_fma(q, r, -1.0);
  q = __builtin_fma(q, r, 1.0);
  const int ki = (int)k;
  return __builtin_ldexp(tab[ki & 63] * q, -(ki >> 6));
}

// Near field of both kernels together (sorted order): for target t and every
// panel j != t of its near leaves,
//   near_u += a_j ((dG0/dn_j - eps dGk/dn_j) u_j - h v_j)
//   near_v += a_j (d2h/dn_t dn_j u_j - (dG0/dn_t - dGk/dn_t / eps) v_j).
// With d = x_t - x_j, r = |d|, E = e^{-kappa r}, A = E (1 + kappa r),
// B = E (kappa r)^2, p_t = n_t . d, p_j = n_j . d, and every kernel taken
// without its factor 1/(4 pi) (applied to the sums at the end):
//   dG0/dn_j - eps dGk/dn_j     = (1 - eps A) p_j / r^3
//   h                           = (1 - E) / r
//   d2h/dn_t dn_j               = -((3 - 3A - B) p_t p_j / r^2 + (A - 1) n_t . n_j) / r^3
//   dG0/dn_t - dGk/dn_t / eps   = (A / eps - 1) p_t / r^3
// (h' = (A - 1)/r^2 and h'' = (2 - 2A - B)/r^3 are differences of the two
// kernels' derivatives; their relative rounding grows as 1/(kappa r)^2, far
// below the product's truncation error at the distances of a near field).
// The sources arrive weighted by their areas, (a_j u_j, a_j v_j).  One wave
// per chunk of at most 64 targets of one leaf (the Laplace near field's
// chunks): a chunk of n targets splits each near leaf's sources over
// G = 64 / n lane groups, strided; with one group the source index is
// uniform over the wave and the source records come through the scalar
// cache.  The G partial sums are added in group order through LDS.
__device__ __forceinline__ void lpb_pair(double tx, double ty, double tz, double ntx, double nty, double ntz, double4 cj,
                                         double4 nj, double2 w, double kappa, double eps, double ieps,
                                         const double *tab, double &su, double &sv) {
  const double dx = tx - cj.x, dy = ty - cj.y, dz = tz - cj.z;
  const double r2 = dx * dx + dy * dy + dz * dz;
  // 1/sqrt(r2): the hardware estimate and one Newton step for x^(-1/2)
  const double y0 = __builtin_amdgcn_rsq(r2);
  const double ir = __builtin_fma(0.5 * y0, __builtin_fma(-r2 * y0, y0, 1.0), y0);
  const double kr = kappa * (r2 * ir);
  const double E = exp_neg(kr, tab);
  const double A = __builtin_fma(kr, E, E);
  const double Bk = E * kr * kr;
  const double ir2 = ir * ir;
  const double pt = ntx * dx + nty * dy + ntz * dz;
  const double pj = nj.x * dx + nj.y * dy + nj.z * dz;
  const double nn = ntx * nj.x + nty * nj.y + ntz * nj.z;
  su = __builtin_fma(ir, __builtin_fma(__builtin_fma(-eps, A, 1.0) * ir2 * pj, w.x, -(1.0 - E) * w.y), su);
  const double t1 = __builtin_fma(__builtin_fma(-3.0, A, 3.0) - Bk, pt * pj * ir2, (A - 1.0) * nn);
  sv = __builtin_fma(-ir * ir2, __builtin_fma(t1, w.x, __builtin_fma(A, ieps, -1.0) * pt * w.y), sv);
}

__global__ void __launch_bounds__(64) k_lpb_near(const int4 *__restrict__ chunks, const double4 *__restrict__ ca,
                                                 const double4 *__restrict__ nrm, const double2 *__restrict__ uvs,
                                                 const int4 *__restrict__ leaf_range,
                                                 const int32_t *__restrict__ near_ptr,
                                                 const int32_t *__restrict__ near_idx, double kappa, double eps,
                                                 double2 *__restrict__ out) {
  __shared__ double2 red[64];
  __shared__ double tab[64];
  const int4 ch = chunks[blockIdx.x];
  const int leaf = ch.x, count = ch.z, G = ch.w;
  const int lane = threadIdx.x;
  tab[lane] = exp2(-lane / 64.0);
  __syncthreads();
  const int g = lane / count, tl = lane - g * count;
  const bool active = g < G;
  const int ti = ch.y + (active ? tl : 0);
  const double4 ct = ca[ti], nt = nrm[ti];
  const double ieps = 1.0 / eps;
  double su = 0.0, sv = 0.0;
  for (int e = near_ptr[leaf]; e < near_ptr[leaf + 1]; ++e) {
    const int4 rg = leaf_range[near_idx[e]];
    if (G == 1) {
      for (int j = rg.x; j < rg.y; ++j) {
        const double4 cj = ca[j], nj = nrm[j];
        const double2 w = uvs[j];
        if (j != ti) lpb_pair(ct.x, ct.y, ct.z, nt.x, nt.y, nt.z, cj, nj, w, kappa, eps, ieps, tab, su, sv);
      }
    } else if (active) {
      for (int j = rg.x + g; j < rg.y; j += G) {
        if (j == ti) continue;
        lpb_pair(ct.x, ct.y, ct.z, nt.x, nt.y, nt.z, ca[j], nrm[j], uvs[j], kappa, eps, ieps, tab, su, sv);
      }
    }
  }
  const double q4 = 1.0 / (4.0 * PI);
  if (G == 1) {
    if (active) out[ti] = make_double2(q4 * su, q4 * sv);
    return;
  }
  red[lane] = make_double2(su, sv);
  __syncthreads();
  if (g == 0 && active) {
    for (int k = 1; k < G; ++k) {
      const double2 o = red[k * count + tl];
      su += o.x;
      sv += o.y;
    }
    out[ti] = make_double2(q4 * su, q4 * sv);
  }
}

// self integrals over each panel (caller order) of h(R) and -h'(R)/R,
// R = |x - c|, by polar integration about the centroid:
//   int_T f dA = sum over edges of int F(P / cos t) dt, F(rho) = int_0^rho f(s) s ds
__global__ void k_lpb_self(int64_t N, const double *__restrict__ pv, const double *__restrict__ c, double kappa,
                           double *__restrict__ sv, double *__restrict__ sd) {
  const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= N) return;
  const double q4 = 1.0 / (4.0 * PI);
  const double cx = c[3 * u], cy = c[3 * u + 1], cz = c[3 * u + 2];
  double iv = 0.0, id = 0.0;
  for (int e = 0; e < 3; ++e) {
    const double *a = pv + 9 * u + 3 * e, *b = pv + 9 * u + 3 * ((e + 1) % 3);
    double tx = b[0] - a[0], ty = b[1] - a[1], tz = b[2] - a[2];
    const double tl = sqrt(tx * tx + ty * ty + tz * tz);
    tx /= tl;
    ty /= tl;
    tz /= tl;
    const double sa = (cx - a[0]) * tx + (cy - a[1]) * ty + (cz - a[2]) * tz;
    const double fx = a[0] + sa * tx, fy = a[1] + sa * ty, fz = a[2] + sa * tz;  // foot on the edge line
    const double P = sqrt((cx - fx) * (cx - fx) + (cy - fy) * (cy - fy) + (cz - fz) * (cz - fz));
    const double ta = atan2((a[0] - fx) * tx + (a[1] - fy) * ty + (a[2] - fz) * tz, P);
    const double tb = atan2((b[0] - fx) * tx + (b[1] - fy) * ty + (b[2] - fz) * tz, P);
    const double mid = 0.5 * (ta + tb), half = 0.5 * (tb - ta);
    for (int k = 0; k < SELF_GL; ++k) {
      const double rho = P / cos(mid + half * c_gl_x[k]);
      const double em = expm1(-kappa * rho);
      iv += half * c_gl_w[k] * q4 * (rho + em / kappa);
      id += half * c_gl_w[k] * q4 * (kappa + em / rho);
    }
  }
  sv[u] = iv;
  sd[u] = id;
}

// sorted copies of the panel data and this product's weights: the screened
// expansions' (a v, -eps a u), the near field's area-weighted (a u, a v), and
// the Laplace dipole weights -a u (caller order)
__global__ void k_lpb_pack(int64_t N, const int32_t *__restrict__ perm, const double *__restrict__ c,
                           const double *__restrict__ area, const double *__restrict__ uv, double eps,
                           double4 *__restrict__ ca, double2 *__restrict__ w, double2 *__restrict__ uvs,
                           double *__restrict__ wd0) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N) return;
  const int64_t u = perm[t];
  const double a = area[u], uu = uv[u], vv = uv[N + u];
  if (ca) ca[t] = make_double4(c[3 * u], c[3 * u + 1], c[3 * u + 2], a);
  w[t] = make_double2(a * vv, -eps * a * uu);
  uvs[t] = make_double2(a * uu, a * vv);
  wd0[u] = -a * uu;
}

__global__ void k_lpb_combine(int64_t N, const int32_t *__restrict__ perm, const double *__restrict__ uv,
                              const double *__restrict__ lap4, const double *__restrict__ nrm,
                              const double2 *__restrict__ yk, const double2 *__restrict__ nr,
                              const double *__restrict__ sv, const double *__restrict__ sd, double eps,
                              double *__restrict__ y) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N) return;
  const int64_t u = perm[t];
  const double uu = uv[u], vv = uv[N + u];
  const double2 k = yk ? yk[t] : make_double2(0.0, 0.0), n = nr[t];
  const double ngrad0 = nrm[3 * u] * lap4[4 * u + 1] + nrm[3 * u + 1] * lap4[4 * u + 2] + nrm[3 * u + 2] * lap4[4 * u + 3];
  y[u] = 0.5 * (1.0 + eps) * uu - lap4[4 * u] + k.x + n.x - sv[u] * vv;
  y[N + u] = 0.5 * (1.0 + 1.0 / eps) * vv - ngrad0 + k.y / eps + n.y + sd[u] * uu;
}

__global__ void k_lpb_rhs_scale(double *__restrict__ b, int64_t n, double s) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] *= s;
}

__global__ void k_sub2(double *__restrict__ r, const double *__restrict__ b, const double *__restrict__ a, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) r[i] = b[i] - a[i];
}

}  // namespace

struct LpbState {
  double kappa = -1.0;
  bool ready = false;
  int noff = 0, nlev = 0;           // M2L levels 2..L
  int64_t m2m_base = 0, l2l_base = 0, nslots = 0;
  DBuf<double> tables;              // [nslots][ps * ps], MFMA B-operand order
  Tree::M2LList list;               // panel -> panel M2L pairs grouped by (level, offset)
  DBuf<double> M, Lx, m2l_out, rows;
  DBuf<double4> ca;                 // sorted (centroid, area)
  DBuf<double2> w, uvs, yk, nr;    // uvs: sorted (a u, a v)
  DBuf<double> lap4, wd0, sv, sd, b, r;
  DBuf<double4> quad;
  DBuf<YkTask> tasks;
};

void lpb_free(Tree &T) {
  delete T.lpb;
  T.lpb = nullptr;
}

namespace {

// the Laplace panel -> panel M2L list regrouped by (level, offset): group
// key (level - 2) * noff + offset is the operator's slot in the tables
void build_level_list(Tree &T, LpbState &S, hipStream_t s) {
  const Tree::M2LList &ML = T.m2l[0];
  const int64_t n = ML.n, G = ML.ngroups;
  Tree::M2LList &Y = S.list;
  Y.n = n;
  if (n == 0) return;
  std::vector<int32_t> src(n), dest(n), goff(G), gend(G), lev(T.ncell_tot);
  HIP_OK(hipMemcpyAsync(src.data(), ML.src.p, n * 4, hipMemcpyDeviceToHost, s));
  HIP_OK(hipMemcpyAsync(dest.data(), ML.dest.p, n * 4, hipMemcpyDeviceToHost, s));
  HIP_OK(hipMemcpyAsync(goff.data(), ML.group_off.p, G * 4, hipMemcpyDeviceToHost, s));
  HIP_OK(hipMemcpyAsync(gend.data(), ML.group_end.p, G * 4, hipMemcpyDeviceToHost, s));
  HIP_OK(hipMemcpyAsync(lev.data(), T.clevel.p, T.ncell_tot * 4, hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  const int64_t nkeys = (int64_t)S.nlev * S.noff;
  std::vector<int32_t> key(n);
  std::vector<int64_t> cnt(nkeys + 1, 0);
  for (int64_t g = 0, r = 0; g < G; ++g)
    for (; r < gend[g]; ++r) {
      const int l = lev[src[r]];
      if (l < 2 || l - 2 >= S.nlev) BF_THROW(BEMFMM_EDEVICE, "screened M2L: pair outside levels 2..L");
      key[r] = (l - 2) * S.noff + goff[g];
      ++cnt[key[r] + 1];
    }
  for (int64_t k = 0; k < nkeys; ++k) cnt[k + 1] += cnt[k];
  std::vector<int32_t> ysrc(n), ydest(n), at(cnt.begin(), cnt.end() - 1);
  std::vector<int32_t> ykey(n);
  for (int64_t r = 0; r < n; ++r) {  // stable counting sort by key
    const int64_t k = at[key[r]]++;
    ysrc[k] = src[r];
    ydest[k] = dest[r];
    ykey[k] = key[r];
  }
  std::vector<int32_t> yoff, yend, tg, tr;
  for (int64_t r = 0; r < n;) {
    int64_t e = r;
    while (e < n && ykey[e] == ykey[r]) ++e;
    const int32_t g = (int32_t)yoff.size();
    yoff.push_back(ykey[r]);
    yend.push_back((int32_t)e);
    for (int64_t x = r; x < e; x += M2L_ROWS64) {
      tg.push_back(g);
      tr.push_back((int32_t)x);
    }
    r = e;
  }
  auto up = [&](DBuf<int32_t> &d, const std::vector<int32_t> &h) {
    d.alloc(std::max<size_t>(h.size(), 1));
    if (!h.empty()) HIP_OK(hipMemcpyAsync(d.p, h.data(), h.size() * 4, hipMemcpyHostToDevice, s));
  };
  up(Y.src, ysrc);
  up(Y.dest, ydest);
  up(Y.group_off, yoff);
  up(Y.group_end, yend);
  up(Y.tile_group64, tg);
  up(Y.tile_row64, tr);
  Y.ngroups = (int64_t)yoff.size();
  Y.ntiles64 = (int64_t)tg.size();
  HIP_OK(hipStreamSynchronize(s));  // host vectors go out of scope
}

void lpb_setup(Tree &T, double kappa, hipStream_t s) {
  set_yk_constants();
  if (!T.lpb) T.lpb = new LpbState();
  LpbState &S = *T.lpb;
  const int ps = T.ps, L = T.L;
  const int64_t N = T.N;
  if (!S.ready) {
    S.noff = T.tab ? T.tab->noff() : 0;
    S.nlev = std::max(0, L - 1);
    build_level_list(T, S, s);
    S.M.alloc((size_t)T.ncell_tot * ps);
    S.Lx.alloc((size_t)T.ncell_tot * ps);
    S.m2l_out.alloc((size_t)std::max<int64_t>(S.list.n, 1) * ps);
    S.rows.alloc((size_t)std::max<int64_t>(T.l2lw.max_cells, 1) * ps);
    S.M.zero(s);
    S.Lx.zero(s);
    S.ca.alloc(N);
    S.w.alloc(N);
    S.uvs.alloc(N);
    S.yk.alloc(N);
    S.nr.alloc(N);
    S.lap4.alloc(4 * N);
    S.wd0.alloc(N);
    S.sv.alloc(N);
    S.sd.alloc(N);
    // projection nodes: Gauss-Legendre in cos theta x trapezoidal in phi
    std::vector<double> x, wq;
    gauss_legendre(YQ_T, x, wq);
    std::vector<double4> q(YQ_N);
    for (int i = 0; i < YQ_T; ++i) {
      const double st = std::sqrt(std::max(0.0, 1.0 - x[i] * x[i]));
      for (int j = 0; j < YQ_P; ++j) {
        const double ph = 2.0 * PI * j / YQ_P;
        q[i * YQ_P + j] = make_double4(st * std::cos(ph), st * std::sin(ph), x[i], wq[i] * 2.0 * PI / YQ_P);
      }
    }
    // dynamic LDS beyond 64 KB is allowed once per kernel, here
    HIP_OK(hipFuncSetAttribute((const void *)k_yk_p2m, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)((size_t)64 * T.p * T.p * sizeof(double))));
    HIP_OK(hipFuncSetAttribute((const void *)k_yk_project, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)(((size_t)2 * YQ_CHUNK * T.p * T.p + 2 * YQ_CHUNK * PMAX + PMAX) * sizeof(double))));
    S.quad.alloc(YQ_N);
    HIP_OK(hipMemcpyAsync(S.quad.p, q.data(), YQ_N * sizeof(double4), hipMemcpyHostToDevice, s));
    HIP_OK(hipStreamSynchronize(s));
    S.ready = true;
  }
  if (S.kappa == kappa) return;
  // per-level translation operators
  std::vector<YkTask> tk;
  auto side = [&](int l) { return T.side / double(1 << l); };
  for (int l = 2; l <= L; ++l)
    for (int o = 0; o < S.noff; ++o) {
      const double sl = side(l);
      // an M2L offset is source cell minus target cell
      tk.push_back(YkTask{T.tab->offsets[3 * o] * sl, T.tab->offsets[3 * o + 1] * sl, T.tab->offsets[3 * o + 2] * sl,
                          0.9 * sl, 1, 0, (l - 2) * S.noff + o, 0});
    }
  S.m2m_base = (int64_t)S.nlev * S.noff;
  S.l2l_base = S.m2m_base + (int64_t)std::max(0, L - 2) * 8;
  for (int l = 3; l <= L; ++l)
    for (int oct = 0; oct < 8; ++oct) {
      const double sc = side(l);
      const double dx = (((oct >> 2) & 1) ? 0.5 : -0.5) * sc, dy = (((oct >> 1) & 1) ? 0.5 : -0.5) * sc,
                   dz = ((oct & 1) ? 0.5 : -0.5) * sc;
      // M2M: the child's multipole basis about the parent centre
      tk.push_back(YkTask{dx, dy, dz, 1.5 * side(l - 1), 1, 1, (int)(S.m2m_base + (l - 3) * 8 + oct), 0});
      // L2L: the parent's local basis about the child centre
      tk.push_back(YkTask{-dx, -dy, -dz, 0.5 * sc, 0, 0, (int)(S.l2l_base + (l - 3) * 8 + oct), 0});
    }
  S.nslots = S.l2l_base + (int64_t)std::max(0, L - 2) * 8;
  S.tables.alloc((size_t)std::max<int64_t>(S.nslots, 1) * ps * ps);
  S.tables.zero(s);
  if (!tk.empty()) {
    S.tasks.alloc(tk.size());
    HIP_OK(hipMemcpyAsync(S.tasks.p, tk.data(), tk.size() * sizeof(YkTask), hipMemcpyHostToDevice, s));
    const size_t shm = ((size_t)2 * YQ_CHUNK * T.p * T.p + 2 * YQ_CHUNK * PMAX + PMAX) * sizeof(double);
    k_yk_project<<<(unsigned)tk.size(), YK_THREADS, shm, s>>>(T.p, ps, kappa, S.tasks.p, S.quad.p, S.tables.p);
    LAUNCH_OK();
  }
  k_lpb_self<<<cdiv(N, 256), 256, 0, s>>>(N, T.pverts.p, T.c.p, kappa, S.sv.p, S.sd.p);
  LAUNCH_OK();
  HIP_OK(hipStreamSynchronize(s));
  S.kappa = kappa;
}

// far field of the screened kernel at the panels (sorted): S.yk
void yukawa_far(Tree &T, LpbState &S, double kappa, hipStream_t s) {
  const int L = T.L, p = T.p, ps = T.ps;
  const int64_t CL = T.ncell[L];
  double *M = S.M.p, *Lx = S.Lx.p;
  const size_t shm = (size_t)64 * p * p * sizeof(double);
  k_yk_p2m<<<(unsigned)CL, 64, shm, s>>>(p, ps, T.crange.p + T.coff[L], T.p64pos.p, T.p64nrm.p, S.w.p, kappa,
                                         M + (size_t)T.coff[L] * ps);
  LAUNCH_OK();
  const double *tab = S.tables.p;
  for (int l = L; l >= 3; --l) {
    level_product64(T, l, T.l2lw.self.p, tab + (size_t)(S.m2m_base + (l - 3) * 8) * ps * ps, M, S.rows.p, true, s);
    m2m_sum64(T, l, S.rows.p, M, s);
  }
  m2l_tiles64(S.list, ps, tab, M, S.m2l_out.p, s);
  for (int l = 2; l <= L; ++l) {
    if (l > 2)
      level_product64(T, l, T.l2lw.src.p, tab + (size_t)(S.l2l_base + (l - 3) * 8) * ps * ps, Lx, S.rows.p, false, s);
    downward64(T, l, S.rows.p, T.m2l[0].kptr.p, S.m2l_out.p, Lx, s);
  }
  k_yk_l2p<<<cdiv(T.N, 128), 128, 0, s>>>(p, ps, T.N, T.pleaf.p, T.p64pos.p, T.p64nrm.p,
                                          Lx + (size_t)T.coff[L] * ps, kappa, S.yk.p);
  LAUNCH_OK();
}

}  // namespace

void lpb_matvec(Tree &T, double kappa, const double *uv, double *y, hipStream_t s) {
  lpb_setup(T, kappa, s);
  LpbState &S = *T.lpb;
  const int64_t N = T.N;
  const double eps = T.prm.eps_out / T.prm.eps_in;
  const int TB = 256;
  k_lpb_pack<<<cdiv(N, TB), TB, 0, s>>>(N, T.pperm.p, T.c.p, T.area.p, uv, eps, S.ca.p, S.w.p, S.uvs.p, S.wd0.p);
  LAUNCH_OK();
  // Laplace far field: P0 = SL0(a v) - DL0(a u), potential and gradient
  FmmRequest rq{SRC_PANEL_MONODIP, TGT_PANEL, OUT_POTGRAD, uv + N, S.wd0.p, true, nullptr, 0.0, 1.0, false,
                S.lap4.p, false};
  rq.far_only = true;
  fmm_apply(T, BEMFMM_FP64, rq, s);
  const bool far = T.L >= 2 && S.list.n > 0;
  if (far) yukawa_far(T, S, kappa, s);
  const int L = T.L;
  if (T.nchunk_p > 0) {
    k_lpb_near<<<(unsigned)T.nchunk_p, 64, 0, s>>>(T.chunk_p.p, S.ca.p, T.p64nrm.p, S.uvs.p, T.crange.p + T.coff[L],
                                                   T.near_ptr.p + T.near_ptr_off[L], T.near_idx.p + T.near_off[L],
                                                   kappa, eps, S.nr.p);
    LAUNCH_OK();
  }
  k_lpb_combine<<<cdiv(N, TB), TB, 0, s>>>(N, T.pperm.p, uv, S.lap4.p, T.nrm.p, far ? S.yk.p : nullptr, S.nr.p,
                                           S.sv.p, S.sd.p, eps, y);
  LAUNCH_OK();
}

void lpb_solve(Tree &T, const double *q, double kappa, double *uv, double tol, int maxit, int restart,
               bemfmm_solve_info *info, hipStream_t s) {
  auto t0 = std::chrono::steady_clock::now();
  lpb_setup(T, kappa, s);
  LpbState &S = *T.lpb;
  const int64_t N = T.N;
  S.b.alloc(2 * N);
  S.r.alloc(2 * N);
  // right-hand side [S; dS/dn]: the charges' potential and normal field over eps_in
  if (T.Q > 0) {
    FmmRequest r1{SRC_CHARGE_MONO, TGT_PANEL, OUT_POT, q, nullptr, false, nullptr, 0.0, 1.0 / T.prm.eps_in, false,
                  S.b.p, false};
    fmm_apply(T, BEMFMM_FP64, r1, s);
    FmmRequest r2{SRC_CHARGE_MONO, TGT_PANEL, OUT_NGRAD, q, nullptr, false, nullptr, 0.0, 1.0 / T.prm.eps_in, false,
                  S.b.p + N, false};
    fmm_apply(T, BEMFMM_FP64, r2, s);
  } else {
    HIP_OK(hipMemsetAsync(S.b.p, 0, 2 * N * sizeof(double), s));
  }
  auto A = [&](const double *v, double *w) { lpb_matvec(T, kappa, v, w, s); };
  bemfmm_solve_info inf{};
  inf.outer_iters = 1;
  const double bn = std::sqrt(dot_d(T, S.b.p, S.b.p, 2 * N, s));
  inf.iters = gmres_apply(T, A, 2 * N, S.b.p, uv, tol, maxit, restart, s);
  if (bn > 0.0) {
    A(uv, S.r.p);
    k_sub2<<<cdiv(2 * N, 256), 256, 0, s>>>(S.r.p, S.b.p, S.r.p, 2 * N);
    LAUNCH_OK();
    inf.rel_residual = std::sqrt(dot_d(T, S.r.p, S.r.p, 2 * N, s)) / bn;
  }
  inf.converged = inf.rel_residual <= tol;
  HIP_OK(hipStreamSynchronize(s));
  inf.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (info) *info = inf;
  if (!inf.converged) BF_THROW(BEMFMM_ENOCONV, "GMRES did not reach the tolerance within maxit");
}

double lpb_energy(Tree &T, const double *q, const double *uv, hipStream_t s) {
  if (T.Q == 0) return 0.0;
  if (!T.lpb) T.lpb = new LpbState();
  LpbState &S = *T.lpb;
  const int64_t N = T.N;
  S.wd0.alloc(N);
  S.r.alloc(std::max<int64_t>(2 * N, T.Q));
  S.w.alloc(N);
  S.uvs.alloc(N);
  // dipole weights -a u (the packing's sorted outputs are not needed here)
  k_lpb_pack<<<cdiv(N, 256), 256, 0, s>>>(N, T.pperm.p, T.c.p, T.area.p, uv, 1.0, nullptr, S.w.p, S.uvs.p, S.wd0.p);
  LAUNCH_OK();
  FmmRequest rq{SRC_PANEL_MONODIP, TGT_CHARGE, OUT_POT, uv + N, S.wd0.p, true, nullptr, 0.0, 1.0, false, S.r.p, false};
  fmm_apply(T, BEMFMM_FP64, rq, s);
  return 2.0 * PI * K_COULOMB * dot_d(T, q, S.r.p, T.Q, s);
}

}  // namespace bemfmm
