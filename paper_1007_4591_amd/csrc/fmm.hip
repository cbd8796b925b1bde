// Fast-multipole evaluation (Section 2.3) on gfx950.  One product runs
//   pack sources -> P2M (leaves) -> M2M (levels L..3 to their parents,
//   batched MFMA products per level and octant) -> M2L (all levels, grouped
//   by translation offset, dense contractions on MFMA) -> downward pass
//   (batched MFMA L2L + ordered sum of the M2L results, levels 2..L, and the
//   leaves' evaluation coefficients) -> L2P fused with the operator's final
//   combination,
// while the P2P near field runs on a second stream and is joined before L2P.
//
// Every stage is templated on the working precision (float or double); the
// FP32 path uses v_mfma_f32_16x16x4f32 (M2M, L2L, M2L at other orders),
// v_mfma_f32_16x16x32_bf16 on operands split into three bf16 parts (M2L at
// the compile-time order) and v_rsq_f32, the FP64 path
// v_mfma_f64_16x16x4f64 and a refined FP64 reciprocal square root.
// Accumulation orders are fixed (no floating-point atomics), so results are
// reproducible run to run.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <mutex>
#include <set>
#include <type_traits>

#include "common.h"

namespace bemfmm {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

template <class R> struct V4;
template <> struct V4<float> { using T = float4; };
template <> struct V4<double> { using T = double4; };

struct PrecBufs {
  int prec = 0;  // 0 = FP64, 1 = FP32
  DBuf<char> src_pos, src_dip;  // real4 [max(N, Q)]
  DBuf<char> M, L;              // real [ncell_tot * ps]
  DBuf<char> m2l_out;           // real [nfar * ps]
  DBuf<char> l2l_out;           // real [cells of the largest level * ps]
  DBuf<char> E;                 // real [nleaf * 4 * ps]
  DBuf<double> dbg_near, dbg_far;  // sorted-order raw fields (only while debug recording is on)
  bool dbg_valid = false;          // the last product recorded them
  DBuf<double> near_out;           // near field per target (sorted order)
  int last_tgt = 0;
  bool have = false;
};

namespace {

__constant__ float c_rec1_f[PMAX + 1][PMAX + 1];  // (2n-1)/(n^2-m^2)
__constant__ float c_rec2_f[PMAX + 1][PMAX + 1];  // 1/(n^2-m^2)
__constant__ double c_rec1_d[PMAX + 1][PMAX + 1];
__constant__ double c_rec2_d[PMAX + 1][PMAX + 1];
__constant__ float c_half_inv_m_f[PMAX + 1];      // 1/(2m)
__constant__ double c_half_inv_m_d[PMAX + 1];

template <class R> __device__ inline R rec1(int n, int m);
template <> __device__ inline float rec1<float>(int n, int m) { return c_rec1_f[n][m]; }
template <> __device__ inline double rec1<double>(int n, int m) { return c_rec1_d[n][m]; }
template <class R> __device__ inline R rec2(int n, int m);
template <> __device__ inline float rec2<float>(int n, int m) { return c_rec2_f[n][m]; }
template <> __device__ inline double rec2<double>(int n, int m) { return c_rec2_d[n][m]; }
template <class R> __device__ inline R hinv(int m);
template <> __device__ inline float hinv<float>(int m) { return c_half_inv_m_f[m]; }
template <> __device__ inline double hinv<double>(int m) { return c_half_inv_m_d[m]; }

__device__ inline float rsq(float x) { return __builtin_amdgcn_rsqf(x); }
// 1/sqrt(x) in FP64: the hardware estimate refined by one Newton step for
// x^(-1/2), y <- y + y (1 - x y^2) / 2.  Arguments are positive: the only
// zero (the excluded self pair) is discarded by index after the call.
__device__ inline double rsq(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  const double e = __builtin_fma(-x * y, y, 1.0);
  return __builtin_fma(0.5 * y, e, y);
}

// Regular solid harmonics R_n^m(x, y, z) for 0 <= m <= n < p, generated in
// m-major order by the recurrences documented with the host tables; calls
// f(n, m, Re, Im) once per pair.
template <class R, class F>
__device__ inline void regular_harmonics(int p, R x, R y, R z, F &&f) {
  const R r2 = x * x + y * y + z * z;
  R dr = R(1), di = R(0);
  for (int m = 0; m < p; ++m) {
    if (m > 0) {
      const R c = -hinv<R>(m);
      const R nr = c * (x * dr - y * di);
      const R ni = c * (x * di + y * dr);
      dr = nr;
      di = ni;
    }
    f(m, m, dr, di);
    if (m + 1 < p) {
      R pr = dr, pi = di;
      R qr = z * dr, qi = z * di;
      f(m + 1, m, qr, qi);
      for (int n = m + 2; n < p; ++n) {
        const R a = rec1<R>(n, m) * z, b = rec2<R>(n, m) * r2;
        const R nr = a * qr - b * pr;
        const R ni = a * qi - b * pi;
        f(n, m, nr, ni);
        pr = qr;
        pi = qi;
        qr = nr;
        qi = ni;
      }
    }
  }
}

// The same recurrences for an order P fixed at compile time: the loops
// unroll completely, the recurrence coefficients fold to constants (computed
// in FP64 and rounded to R, as the host tables are), and f receives constant
// (n, m), so callers can keep one register per coefficient.
template <int P, class R, class F>
__device__ __forceinline__ void regular_harmonics_fixed(R x, R y, R z, F &&f) {
  const R r2 = x * x + y * y + z * z;
  R dr = R(1), di = R(0);
#pragma unroll
  for (int m = 0; m < P; ++m) {
    if (m > 0) {
      const R c = -R(1.0 / (2.0 * m));
      const R nr = c * (x * dr - y * di);
      const R ni = c * (x * di + y * dr);
      dr = nr;
      di = ni;
    }
    f(m, m, dr, di);
    if (m + 1 < P) {
      R pr = dr, pi = di;
      R qr = z * dr, qi = z * di;
      f(m + 1, m, qr, qi);
#pragma unroll
      for (int n = m + 2; n < P; ++n) {
        const double den = double(n * n - m * m);
        const R a = R((2.0 * n - 1.0) / den) * z, b = R(1.0 / den) * r2;
        const R nr = a * qr - b * pr;
        const R ni = a * qi - b * pi;
        f(n, m, nr, ni);
        pr = qr;
        pi = qi;
        qr = nr;
        qi = ni;
      }
    }
  }
}

__device__ inline void xyz_of(int32_t v, int &x, int &y, int &z) {
  x = v & 1023;
  y = (v >> 10) & 1023;
  z = (v >> 20) & 1023;
}

// ------------------------------------------------------------ pack sources

// src_pos[i] = (rx, ry, rz, w) in sorted order; src_dip[i] = d * n (moment)
template <class R>
__global__ void k_pack_panels(int64_t N, const int32_t *__restrict__ perm, const typename V4<R>::T *__restrict__ pos,
                              const typename V4<R>::T *__restrict__ nrm, const double *__restrict__ area,
                              const double *__restrict__ wmono, int mono_area, const double *__restrict__ wdip,
                              typename V4<R>::T *__restrict__ out_pos, typename V4<R>::T *__restrict__ out_dip) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const int64_t u = perm[i];
  typename V4<R>::T p = pos[i];
  R w = R(0);
  if (wmono) {
    double wd = wmono[u];
    if (mono_area) wd *= area[u];
    w = (R)wd;
  }
  typename V4<R>::T o;
  o.x = p.x;
  o.y = p.y;
  o.z = p.z;
  o.w = w;
  out_pos[i] = o;
  if (wdip) {
    typename V4<R>::T n = nrm[i];
    R d = (R)wdip[u];
    typename V4<R>::T m;
    m.x = d * n.x;
    m.y = d * n.y;
    m.z = d * n.z;
    m.w = R(0);
    out_dip[i] = m;
  }
}

template <class R>
__global__ void k_pack_charges(int64_t Q, const int32_t *__restrict__ perm, const typename V4<R>::T *__restrict__ pos,
                               const double *__restrict__ q, typename V4<R>::T *__restrict__ out_pos) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= Q) return;
  typename V4<R>::T p = pos[i];
  p.w = (R)q[perm[i]];
  out_pos[i] = p;
}

// -------------------------------------------------------------------- P2M

// One wave per leaf: each lane accumulates its sources' contributions in a
// private LDS row (stride ps + 1 avoids bank conflicts), then lanes sum the
// columns in lane order.  Monopoles add w conj(R_n^m(rho)); dipoles add
// mu . grad conj(R_n^m) = mu_z conj(R_{n-1}^m) + (mu_x + i mu_y)/2 conj(R_{n-1}^{m+1})
//                        - (mu_x - i mu_y)/2 conj(R_{n-1}^{m-1}),
// with R_{n-1}^{-1} = -conj(R_{n-1}^1); rho and mu are in units of the leaf side.
template <class R, bool MONO, bool DIP>
__global__ void __launch_bounds__(64) k_p2m(int p, int ps, int64_t C, const int4 *__restrict__ range, int charges,
                                            const typename V4<R>::T *__restrict__ src,
                                            const typename V4<R>::T *__restrict__ dip, R inv_s,
                                            R *__restrict__ M) {
  extern __shared__ char smem_raw[];
  R *row = reinterpret_cast<R *>(smem_raw);
  const int lane = threadIdx.x;
  const int stride = ps + 1;
  const int64_t c = blockIdx.x;
  if (c >= C) return;
  R *my = row + lane * stride;
  for (int k = 0; k < ps; ++k) my[k] = R(0);
  const int4 rg = range[c];
  const int b = charges ? rg.z : rg.x, e = charges ? rg.w : rg.y;
  for (int j0 = b; j0 < e; j0 += 64) {
    const int j = j0 + lane;
    if (j < e) {
      const typename V4<R>::T sp = src[j];
      const R x = sp.x * inv_s, y = sp.y * inv_s, z = sp.z * inv_s;
      const R w = sp.w;
      R mx = R(0), myy = R(0), mz = R(0);
      if (DIP) {
        const typename V4<R>::T mo = dip[j];
        mx = mo.x * inv_s;
        myy = mo.y * inv_s;
        mz = mo.z * inv_s;
      }
      regular_harmonics<R>(p, x, y, z, [&](int n, int m, R re, R im) {
        if (MONO) {
          my[idx_re(n, m)] += w * re;
          if (m > 0) my[idx_im(n, m)] -= w * im;
        }
        if (DIP && n <= p - 2) {
          const int no = n + 1;
          my[idx_re(no, m)] += mz * re;
          if (m > 0) my[idx_im(no, m)] -= mz * im;
          if (m >= 1) {
            const R hr = R(0.5) * (mx * re + myy * im);
            if (m == 1) {
              my[idx_re(no, 0)] += hr + hr;
            } else {
              my[idx_re(no, m - 1)] += hr;
              my[idx_im(no, m - 1)] += R(0.5) * (myy * re - mx * im);
            }
          }
          my[idx_re(no, m + 1)] -= R(0.5) * (mx * re - myy * im);
          my[idx_im(no, m + 1)] += R(0.5) * (mx * im + myy * re);
        }
      });
    }
  }
  __syncthreads();
  R *out = M + c * ps;
  for (int i = lane; i < ps; i += 64) {
    const int k = coef_at(i, p, ps);
    R acc = R(0);
    if (k >= 0)
      for (int l = 0; l < 64; ++l) acc += row[l * stride + k];
    out[i] = acc;
  }
}

// P2M for an order P fixed at compile time.  Same arithmetic and order as
// k_p2m (each lane sums its own sources, then the lanes are added in lane
// order), but a lane's partial expansion lives in registers while it sweeps
// its sources; LDS is used once, to add the 64 partial rows column by column.
template <int P, class R, bool MONO, bool DIP>
__global__ void __launch_bounds__(64) k_p2m_fixed(int ps, int64_t C, const int4 *__restrict__ range, int charges,
                                                  const typename V4<R>::T *__restrict__ src,
                                                  const typename V4<R>::T *__restrict__ dip, R inv_s,
                                                  R *__restrict__ M) {
  constexpr int NC = P * P;
  __shared__ R part[64][NC + 1];
  const int lane = threadIdx.x;
  const int64_t c = blockIdx.x;
  if (c >= C) return;
  R acc[NC];
#pragma unroll
  for (int k = 0; k < NC; ++k) acc[k] = R(0);
  const int4 rg = range[c];
  const int b = charges ? rg.z : rg.x, e = charges ? rg.w : rg.y;
  for (int j = b + lane; j < e; j += 64) {
    const typename V4<R>::T sp = src[j];
    const R x = sp.x * inv_s, y = sp.y * inv_s, z = sp.z * inv_s;
    const R w = sp.w;
    R mx = R(0), myy = R(0), mz = R(0);
    if (DIP) {
      const typename V4<R>::T mo = dip[j];
      mx = mo.x * inv_s;
      myy = mo.y * inv_s;
      mz = mo.z * inv_s;
    }
    regular_harmonics_fixed<P, R>(x, y, z, [&](int n, int m, R re, R im) {
      if (MONO) {
        acc[idx_re(n, m)] += w * re;
        if (m > 0) acc[idx_im(n, m)] -= w * im;
      }
      if (DIP && n <= P - 2) {
        const int no = n + 1;
        acc[idx_re(no, m)] += mz * re;
        if (m > 0) acc[idx_im(no, m)] -= mz * im;
        if (m >= 1) {
          const R hr = R(0.5) * (mx * re + myy * im);
          if (m == 1) {
            acc[idx_re(no, 0)] += hr + hr;
          } else {
            acc[idx_re(no, m - 1)] += hr;
            acc[idx_im(no, m - 1)] += R(0.5) * (myy * re - mx * im);
          }
        }
        acc[idx_re(no, m + 1)] -= R(0.5) * (mx * re - myy * im);
        acc[idx_im(no, m + 1)] += R(0.5) * (mx * im + myy * re);
      }
    });
  }
#pragma unroll
  for (int k = 0; k < NC; ++k) part[lane][k] = acc[k];
  __syncthreads();
  R *out = M + c * ps;
  for (int i = lane; i < ps; i += 64) {
    const int k = coef_at(i, P, ps);
    R t = R(0);
    if (k >= 0)
      for (int l = 0; l < 64; ++l) t += part[l][k];
    out[i] = t;
  }
}

// -------------------------------------------------------------------- M2M

// M2M, second half: the multipole expansion of every cell of level l - 1 is
// the sum of its children's translated expansions (rows of the batched M2M
// product of level l, one per child), added in child order.
template <class R>
__global__ void k_m2m_sum(int ps, int64_t cp0, int64_t CP, int64_t cl0, const int2 *__restrict__ child,
                          const R *__restrict__ rows, R *__restrict__ M) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= CP * ps) return;
  const int64_t P = i / ps;
  const int k = (int)(i - P * ps);
  const int2 ch = child[cp0 + P];  // global child range
  R acc = R(0);
  for (int c = ch.x; c < ch.y; ++c) acc += rows[(size_t)(c - cl0) * ps + k];
  M[(size_t)(cp0 + P) * ps + k] = acc;
}

// -------------------------------------------------------------------- M2L

// Workgroups are dispatched to the 8 XCDs of the chip in turn, and each XCD
// has its own L2.  This maps launch order to work order so that XCD x runs
// the x-th contiguous eighth of the work items: neighbouring chunks (which
// share most of their near-field sources) then meet in the same L2.
__device__ __forceinline__ int xcd_block(int bid, int n) {
  constexpr int NX = 8;
  const int q = n / NX, r = n - q * NX;
  const int x = bid % NX, k = bid / NX;
  return x < r ? x * (q + 1) + k : r * (q + 1) + (x - r) * q + k;
}

// Offset-grouped dense M2L on MFMA.  A work tile is 4 waves x RT x 16
// consecutive pairs of one offset group (pairs are sorted by offset, all
// levels together: the scaled operator depends on the offset only).  Each
// wave computes, for RT row tiles of 16 pairs,
//   D[16 x 16*NT] += A[16 x 4] * B[4 x 16*NT]   for every k-step,
// A = gathered source expansions (held in registers for the whole tile),
// B = T_o^T read once per k-step and reused by the RT row tiles.  The K
// dimension is permuted so that each lane reads a contiguous quarter of its
// source row: at k-step kk, lane group g = lane/16 supplies input g*KK + kk
// (the B table is stored in that order).  Rows past the end of the group
// repeat its last row (MFMA rows are independent; they are not stored).
// The same kernel runs the batched per-level M2M and L2L products (one
// octant operator per group); USE only names the instance (0: M2L, 1: L2L,
// 2: M2M) so that profiles tell them apart.
// Registers are budgeted for two waves per SIMD so that one wave's gather
// overlaps the other's MFMA work.  With BLDS the four waves of a tile share
// the operator through LDS instead of each reading it from L2.
// Each result row goes to dest[row]: for M2L its place in pair order
// (level, target, source), so that the downward pass reads a cell's rows as
// one contiguous run; for M2M and L2L the cell's index within its level.
// Output layouts (checked on the device): FP32 16x16x4 puts
// D[4*(lane/16) + q][lane%16] in register q; FP64 16x16x4 puts
// D[lane/16 + 4*q][lane%16] in register q.
template <class R, int NT, int RT, bool BLDS, int USE>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
k_m2l(const int32_t *__restrict__ tile_group, const int32_t *__restrict__ tile_row,
      const int32_t *__restrict__ group_off, const int32_t *__restrict__ group_end, const int32_t *__restrict__ src,
      const int32_t *__restrict__ dest, const R *__restrict__ Tsw, const R *__restrict__ M, R *__restrict__ out) {
  constexpr bool F64 = sizeof(R) == 8;
  constexpr int W = 16 / sizeof(R);
  constexpr int PS = NT * 16;
  constexpr int KK = PS / 4;
  constexpr int TB = KK * NT * 64;  // reals of one offset's operator
  using V16 = typename std::conditional<F64, double2, float4>::type;
  using Acc = typename std::conditional<F64, f64x4, f32x4>::type;
  __shared__ V16 Bs[BLDS ? TB / W : 1];
  __shared__ int Ds[BLDS ? 4 * 16 * RT : 1];
  const int tile = xcd_block(blockIdx.x, gridDim.x);  // tiles of one group share an L2
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = tile_group[tile];
  const int end = group_end[g];
  const int row0 = tile_row[tile] + wave * (16 * RT);
  const bool active = row0 < end;
  if (!BLDS && !active) return;
  const int off = group_off[g];
  const int i = lane & 15, kq = lane >> 4;
  int sr[RT];
#pragma unroll
  for (int rt = 0; rt < RT; ++rt) sr[rt] = src[min(row0 + rt * 16 + i, end - 1)];
  // output rows of the rows this lane stores (-1 past the end); with BLDS
  // they are staged in LDS with the operator
  int dr[RT][4];
  if constexpr (!BLDS) {
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int rr = row0 + rt * 16 + (F64 ? kq + 4 * q : 4 * kq + q);
        dr[rt][q] = rr < end ? dest[rr] : -1;
      }
  }
  R a[RT][KK];
#pragma unroll
  for (int rt = 0; rt < RT; ++rt) {
    const V16 *Ms = reinterpret_cast<const V16 *>(M + (size_t)sr[rt] * PS + kq * KK);
#pragma unroll
    for (int v = 0; v < KK / W; ++v) {
      const V16 t = Ms[v];
      if constexpr (F64) {
        a[rt][2 * v] = t.x;
        a[rt][2 * v + 1] = t.y;
      } else {
        a[rt][4 * v] = t.x;
        a[rt][4 * v + 1] = t.y;
        a[rt][4 * v + 2] = t.z;
        a[rt][4 * v + 3] = t.w;
      }
    }
  }
  const R *B;
  if constexpr (BLDS) {
    const V16 *Bg = reinterpret_cast<const V16 *>(Tsw + (size_t)off * TB);
    for (int v = threadIdx.x; v < TB / W; v += 256) Bs[v] = Bg[v];
    for (int v = threadIdx.x; v < 4 * 16 * RT; v += 256) {
      const int rr = tile_row[tile] + v;
      Ds[v] = rr < end ? dest[rr] : -1;
    }
    __syncthreads();
    if (!active) return;
    B = reinterpret_cast<const R *>(Bs) + lane;
  } else {
    B = Tsw + (size_t)off * TB + lane;
  }
  Acc acc[RT][NT];
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int ct = 0; ct < NT; ++ct) acc[rt][ct] = Acc{0, 0, 0, 0};
#pragma unroll
  for (int kk = 0; kk < kk_used(NT); ++kk) {
#pragma unroll
    for (int ct = 0; ct < NT; ++ct) {
      const R b = B[(kk * NT + ct) * 64];
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) {
        if constexpr (F64)
          acc[rt][ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[rt][kk], b, acc[rt][ct], 0, 0, 0);
        else
          acc[rt][ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[rt][kk], b, acc[rt][ct], 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int d = BLDS ? Ds[wave * 16 * RT + rt * 16 + (F64 ? kq + 4 * q : 4 * kq + q)] : dr[rt][q];
      if (d >= 0) {
        R *o = out + (size_t)d * PS + i;
#pragma unroll
        for (int ct = 0; ct < NT; ++ct) o[ct * 16] = acc[rt][ct][q];
      }
    }
}

// Persistent FP32 M2L.  A workgroup (4 waves, one per SIMD) walks a
// contiguous range of work units; the ranges are XCD-aware, so the ranges of
// one XCD are adjacent and consecutive units mostly share their offset group.
// A unit is one part of a tile of the tile list (M2L_ROWS32 rows): 4 waves x
// RT x 16 rows.  The operator is reloaded into LDS only when the offset group
// changes.  Two workgroups share a CU and drift out of step, so one's loads
// overlap the other's MFMA work.
// Per unit, the source rows of the next unit are requested right after the
// products and before this unit's results are stored, so the latency of the
// gather runs alongside that of the stores instead of after it.  The results
// go out through a per-wave LDS staging area, 16 rows at a time, so that each
// lane stores 16 contiguous bytes of a row (RT x PS / 4 stores per wave and
// unit instead of RT x 4 x NT).  RT = 2 keeps the accumulators, the
// prefetched rows and the staging within 256 registers.  The arithmetic per
// row is that of k_m2l (same operand layouts, same K order), so results are
// identical.
template <int NT, int RT>
__device__ __forceinline__ void m2l_tiles(const int32_t *__restrict__ tile_group,
                                          const int32_t *__restrict__ tile_row,
                                          const int32_t *__restrict__ group_off,
                                          const int32_t *__restrict__ group_end,
                                          const int32_t *__restrict__ src, const int32_t *__restrict__ dest,
                                          const float *__restrict__ Tsw, const float *__restrict__ M,
                                          float *__restrict__ out, int ntiles, float4 *Bs, float *Ts) {
  constexpr int PS = NT * 16;
  constexpr int KK = PS / 4;
  constexpr int TB4 = KK * NT * 16;          // float4 per operator
  constexpr int UROWS = 4 * RT * 16;         // rows per unit
  static_assert(M2L_ROWS32 % UROWS == 0, "a tile splits into whole units");
  constexpr int SUB = M2L_ROWS32 / UROWS;    // units per tile
  constexpr int TS = PS + 4;                 // staging row stride (floats, 16-byte aligned)
  constexpr int F4 = PS / 4;                 // float4 per result row
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int i16 = lane & 15, kq = lane >> 4;
  const int nwg = gridDim.x;
  const int wg = xcd_block(blockIdx.x, nwg);
  const int64_t nunits = (int64_t)ntiles * SUB;
  const int u0 = (int)(nunits * wg / nwg), u1 = (int)(nunits * (wg + 1) / nwg);
  if (u0 >= u1) return;  // uniform over the workgroup
  float *Tw = Ts + wave * 16 * TS;

  struct UnitIn {
    int g, end, row0;
  };
  auto unit_in = [&](int u) {
    UnitIn s;
    const int t = u / SUB;
    s.g = tile_group[t];
    s.end = group_end[s.g];
    s.row0 = tile_row[t] + (u - t * SUB) * UROWS + wave * (16 * RT);
    return s;
  };
  // lane (i16, kq) supplies row i16 of a row tile, inputs kq*KK .. kq*KK+KK-1
  auto load_rows = [&](const UnitIn &s, float (&a)[RT][KK]) {
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
      const int sr = src[min(s.row0 + rt * 16 + i16, s.end - 1)];
      const float4 *Ms = reinterpret_cast<const float4 *>(M + (size_t)sr * PS + kq * KK);
#pragma unroll
      for (int v = 0; v < KK / 4; ++v) {
        const float4 q = Ms[v];
        a[rt][4 * v] = q.x;
        a[rt][4 * v + 1] = q.y;
        a[rt][4 * v + 2] = q.z;
        a[rt][4 * v + 3] = q.w;
      }
    }
  };
  // lane (i16, .) holds the destination of row i16 of each row tile
  auto load_dest = [&](const UnitIn &s, int (&d)[RT]) {
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) d[rt] = dest[min(s.row0 + rt * 16 + i16, s.end - 1)];
  };
  auto stage_b = [&](int g) {
    const float4 *Bg = reinterpret_cast<const float4 *>(Tsw) + (size_t)group_off[g] * TB4;
    for (int v = threadIdx.x; v < TB4; v += 256) Bs[v] = Bg[v];
  };

  float a[RT][KK];
  int d[RT];
  UnitIn cur = unit_in(u0);
  stage_b(cur.g);
  load_rows(cur, a);
  load_dest(cur, d);
  __syncthreads();
  for (int u = u0; u < u1; ++u) {
    const bool work = cur.row0 < cur.end;  // uniform over the wave
    f32x4 acc[RT][NT];
    if (work) {
#pragma unroll
      for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int ct = 0; ct < NT; ++ct) acc[rt][ct] = f32x4{0.f, 0.f, 0.f, 0.f};
      const float *B = reinterpret_cast<const float *>(Bs) + lane;
#pragma unroll
      for (int kk = 0; kk < kk_used(NT); ++kk) {
#pragma unroll
        for (int ct = 0; ct < NT; ++ct) {
          const float b = B[(kk * NT + ct) * 64];
#pragma unroll
          for (int rt = 0; rt < RT; ++rt)
            acc[rt][ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[rt][kk], b, acc[rt][ct], 0, 0, 0);
        }
      }
    }
    const bool more = u + 1 < u1;
    UnitIn nxt = cur;
    int dn[RT];
    if (more) {
      nxt = unit_in(u + 1);
      load_rows(nxt, a);
      load_dest(nxt, dn);
    }
    __asm__ volatile("" ::: "memory");  // keep the prefetch ahead of the stores
    if (work) {
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) {
        // MFMA output: register q of lane (i16, kq) is row 4 kq + q, column
        // ct * 16 + i16 of column tile ct
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
          for (int ct = 0; ct < NT; ++ct) Tw[(4 * kq + q) * TS + ct * 16 + i16] = acc[rt][ct][q];
        __builtin_amdgcn_wave_barrier();
        // 16 rows x F4 float4, 64 lanes at a time (16 F4 = 64 NT: whole passes)
#pragma unroll
        for (int v = 0; v < NT; ++v) {
          const int f = lane + 64 * v;
          const int row = f / F4, c4 = f - row * F4;
          const int dr = __shfl(d[rt], row);
          const float4 val = *reinterpret_cast<const float4 *>(Tw + row * TS + 4 * c4);
          if (cur.row0 + rt * 16 + row < cur.end) *reinterpret_cast<float4 *>(out + (size_t)dr * PS + 4 * c4) = val;
        }
        __builtin_amdgcn_wave_barrier();
      }
    }
    if (more) {
      if (group_off[nxt.g] != group_off[cur.g]) {
        __syncthreads();  // every wave is done with the current operator
        stage_b(nxt.g);
        __syncthreads();
      }
      cur = nxt;
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) d[rt] = dn[rt];
    }
  }
}

template <int NT, int RT>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(NT <= 7 ? 2 : 1)))
k_m2l_pers(const int32_t *__restrict__ tile_group, const int32_t *__restrict__ tile_row,
           const int32_t *__restrict__ group_off, const int32_t *__restrict__ group_end,
           const int32_t *__restrict__ src, const int32_t *__restrict__ dest, const float *__restrict__ Tsw,
           const float *__restrict__ M, float *__restrict__ out, int ntiles) {
  __shared__ float4 Bs[NT * 4 * NT * 16];
  __shared__ float Ts[4 * 16 * (NT * 16 + 4)];
  m2l_tiles<NT, RT>(tile_group, tile_row, group_off, group_end, src, dest, Tsw, M, out, ntiles, Bs, Ts);
}

// Persistent FP32 M2L on the bf16 matrix cores, for the expansion order with
// compile-time kernels.  A bf16 step (16x16x32) covers 8x the K of an FP32
// step (16x16x4) in about half the issue time.  Each FP32 multipole value x
// is split in registers into three bf16 parts, rounding to nearest at each
// step, so that x = x1 + x2 + x3 exactly (|x2| <= 2^-8 |x|, |x3| <= 2^-16 |x|);
// each operator value y is split the same way on the host from its FP64
// value.  The product keeps the six part products x_i y_j with i + j <= 4,
// each exact in the FP32 accumulator; what is left out, with the rounding of
// the operator's split, is below 2^-22 |x y|, the size of FP32 rounding.
// The rows therefore agree with the FP32 MFMA kernels to rounding, not
// bitwise, and are themselves deterministic.
//
// K layout.  Lane group g = lane / 16 owns block g of the stored row (places
// g KK .. g KK + RB - 1, its RB coefficients; in the interleaved storage
// order a full sub-step j covers the packed coefficients 32 j .. 32 j + 31,
// of neighbouring degrees, so the products one instruction sums are of
// similar size and its truncating sum loses little).  Full steps:
// for sub-step j < RB / 8 and each of the six part pairs, slot e of lane
// group g is input place g KK + 8 j + e.  The last R = RB % 8 inputs of
// every block, for all six pairs, share ceil(6 R / 8) remainder steps: slot
// 8 s + e holds pair (8 s + e) / R at input 8 (RB / 8) + (8 s + e) % R, and
// the slots past 6 R are zero.  The host table holds, per offset and column
// tile, the B operand of every step in that order (parts 1, 2, 3 of each full
// sub-step, then the remainder steps).
//
// Work order is that of k_m2l_pers, with one workgroup of 8 waves per CU:
// the split operator takes 70 KB of LDS at p = 10 and the store staging
// 52 KB, so two workgroups do not fit.  A result row holds the coefficients
// in packed order (100 reals at p = 10), without the padding places of the
// stored layout; the downward pass reads it so.  A wave takes RT row tiles of 16
// pairs per unit; the sub-steps run in order, each splitting its 8 inputs
// just before its products, so that few parts are live at once.  The next
// unit's rows are requested after the products and before the stores.
__device__ __forceinline__ void split3(f32x2 x, bf16x2 &h1, bf16x2 &h2, bf16x2 &h3) {
  h1 = __builtin_convertvector(x, bf16x2);
  const f32x2 r1 = x - __builtin_convertvector(h1, f32x2);
  h2 = __builtin_convertvector(r1, bf16x2);
  const f32x2 r2 = r1 - __builtin_convertvector(h2, f32x2);
  h3 = __builtin_convertvector(r2, bf16x2);
}

// Sizes of the split-bf16 M2L for rows of NT column tiles and RB real
// coefficients per lane-group block.
template <int NT, int RB>
struct M2LBf {
  static constexpr int PS = NT * 16, KK = PS / 4;
  static constexpr int J = RB / 8, R = RB % 8, NRS = (6 * R + 7) / 8, NBLK = 3 * J + NRS;
  static constexpr int NW = 8;                 // waves per workgroup
  static constexpr int TBV = NT * NBLK * 64;   // bf16x8 per operator
  static constexpr int CS = 4 * RB;            // reals per result row (compact: no padding places)
  static constexpr int TS = CS + 4;            // staging row stride (floats, 16-byte aligned)
};

template <int NT, int RB, int RT>
__device__ __forceinline__ void m2l_bf_units(const int32_t *__restrict__ tile_group,
                                             const int32_t *__restrict__ tile_row,
                                             const int32_t *__restrict__ group_off,
                                             const int32_t *__restrict__ group_end,
                                             const int32_t *__restrict__ src, const int32_t *__restrict__ dest,
                                             const bf16x8 *__restrict__ Tbf, const float *__restrict__ M,
                                             float *__restrict__ out, int ntiles, bf16x8 *Bs, float *Ts) {
  using C = M2LBf<NT, RB>;
  constexpr int PS = C::PS, KK = C::KK, J = C::J, R = C::R, NRS = C::NRS, NBLK = C::NBLK, NW = C::NW;
  constexpr int TBV = C::TBV, TS = C::TS, CS = C::CS;
  static_assert(CS % 4 == 0, "compact rows of whole float4");
  constexpr int UROWS = NW * RT * 16;
  static_assert(M2L_ROWS32 % UROWS == 0, "a tile splits into whole units");
  constexpr int SUB = M2L_ROWS32 / UROWS;  // units per tile
  static_assert(RB <= KK && J >= 1, "at least one full sub-step per block");
  constexpr int F4 = CS / 4;           // float4 per result row
  constexpr int NV4 = RB / 4;          // float4 loads per block, then RB % 4 scalars
  // part of x in each of the six products (the host table pairs each with
  // its part of y)
  constexpr int PA[6] = {1, 1, 2, 1, 2, 3};
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int i16 = lane & 15, kq = lane >> 4;
  const int nwg = gridDim.x;
  const int wg = xcd_block(blockIdx.x, nwg);
  const int64_t nunits = (int64_t)ntiles * SUB;
  const int u0 = (int)(nunits * wg / nwg), u1 = (int)(nunits * (wg + 1) / nwg);
  if (u0 >= u1) return;  // uniform over the workgroup
  float *Tw = Ts + wave * 16 * TS;

  struct UnitIn {
    int g, end, row0;
  };
  auto unit_in = [&](int u) {
    UnitIn v;
    const int t = u / SUB;
    v.g = tile_group[t];
    v.end = group_end[v.g];
    v.row0 = tile_row[t] + (u - t * SUB) * UROWS + wave * (16 * RT);
    return v;
  };
  // lane (i16, kq) loads the RB real coefficients of block kq of row i16
  auto load_rows = [&](const UnitIn &v, float (&a)[RT][RB]) {
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
      const int sr = src[min(v.row0 + rt * 16 + i16, v.end - 1)];
      const float *Mr = M + (size_t)sr * PS + kq * KK;
      const float4 *M4 = reinterpret_cast<const float4 *>(Mr);
#pragma unroll
      for (int q = 0; q < NV4; ++q) {
        const float4 t = M4[q];
        a[rt][4 * q] = t.x;
        a[rt][4 * q + 1] = t.y;
        a[rt][4 * q + 2] = t.z;
        a[rt][4 * q + 3] = t.w;
      }
#pragma unroll
      for (int q = 4 * NV4; q < RB; ++q) a[rt][q] = Mr[q];
    }
  };
  auto load_dest = [&](const UnitIn &v, int (&d)[RT]) {
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) d[rt] = dest[min(v.row0 + rt * 16 + i16, v.end - 1)];
  };
  auto stage_b = [&](int g) {
    const bf16x8 *Bg = Tbf + (size_t)group_off[g] * TBV;
    for (int v = threadIdx.x; v < TBV; v += 64 * NW) Bs[v] = Bg[v];
  };

  float a[RT][RB];
  int d[RT];
  UnitIn cur = unit_in(u0);
  stage_b(cur.g);
  load_rows(cur, a);
  load_dest(cur, d);
  __syncthreads();
  for (int u = u0; u < u1; ++u) {
    const bool work = cur.row0 < cur.end;  // uniform over the wave
    f32x4 acc[RT][NT];
    if (work) {
#pragma unroll
      for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int ct = 0; ct < NT; ++ct) acc[rt][ct] = f32x4{0.f, 0.f, 0.f, 0.f};
      const bf16x8 *B = Bs + lane;
      // full sub-steps: the parts of inputs 8j .. 8j+7, split just before use
#pragma unroll
      for (int j = 0; j < J; ++j) {
        bf16x8 A1[RT], A2[RT], A3[RT];
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
          for (int e = 0; e < 8; e += 2) {
            bf16x2 h1, h2, h3;
            split3(f32x2{a[rt][8 * j + e], a[rt][8 * j + e + 1]}, h1, h2, h3);
            A1[rt][e] = h1[0], A1[rt][e + 1] = h1[1];
            A2[rt][e] = h2[0], A2[rt][e + 1] = h2[1];
            A3[rt][e] = h3[0], A3[rt][e + 1] = h3[1];
          }
#pragma unroll
        for (int ct = 0; ct < NT; ++ct) {
          const bf16x8 b1 = B[(ct * NBLK + 3 * j) * 64];
          const bf16x8 b2 = B[(ct * NBLK + 3 * j + 1) * 64];
          const bf16x8 b3 = B[(ct * NBLK + 3 * j + 2) * 64];
#pragma unroll
          for (int rt = 0; rt < RT; ++rt) {
            f32x4 c = acc[rt][ct];
            c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A1[rt], b3, c, 0, 0, 0);
            c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A2[rt], b2, c, 0, 0, 0);
            c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A3[rt], b1, c, 0, 0, 0);
            c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A1[rt], b2, c, 0, 0, 0);
            c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A2[rt], b1, c, 0, 0, 0);
            c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A1[rt], b1, c, 0, 0, 0);
            acc[rt][ct] = c;
          }
        }
      }
      // remainder steps: the last R inputs of the block, all six products
      if constexpr (NRS > 0) {
        bf16x8 AR[RT][NRS];
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) {
          __bf16 q1[R + 1], q2[R + 1], q3[R + 1];
#pragma unroll
          for (int i = 0; i < R; i += 2) {
            bf16x2 h1, h2, h3;
            split3(f32x2{a[rt][8 * J + i], i + 1 < R ? a[rt][8 * J + i + 1] : 0.f}, h1, h2, h3);
            q1[i] = h1[0], q1[i + 1] = h1[1];
            q2[i] = h2[0], q2[i + 1] = h2[1];
            q3[i] = h3[0], q3[i + 1] = h3[1];
          }
#pragma unroll
          for (int sr = 0; sr < NRS; ++sr)
#pragma unroll
            for (int e = 0; e < 8; ++e) {
              const int gs = 8 * sr + e;
              if (gs < 6 * R) {
                const int idx = gs % R, pa = PA[gs / R];
                AR[rt][sr][e] = pa == 1 ? q1[idx] : pa == 2 ? q2[idx] : q3[idx];
              } else {
                AR[rt][sr][e] = (__bf16)0.f;
              }
            }
        }
#pragma unroll
        for (int ct = 0; ct < NT; ++ct)
#pragma unroll
          for (int sr = 0; sr < NRS; ++sr) {
            const bf16x8 br = B[(ct * NBLK + 3 * J + sr) * 64];
#pragma unroll
            for (int rt = 0; rt < RT; ++rt)
              acc[rt][ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(AR[rt][sr], br, acc[rt][ct], 0, 0, 0);
          }
      }
    }
    const bool more = u + 1 < u1;
    UnitIn nxt = cur;
    int dn[RT];
    if (more) {
      nxt = unit_in(u + 1);
      load_rows(nxt, a);
      load_dest(nxt, dn);
    }
    __asm__ volatile("" ::: "memory");  // keep the prefetch ahead of the stores
    if (work) {
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) {
        // MFMA output: register q of lane (i16, kq) is row 4 kq + q, column
        // ct * 16 + i16 of column tile ct, the coefficient stored at that
        // place; it goes to its compact place, its packed index
        // (4 * offset + block), and the padding places are left out
        // (the lane index is passed through an empty asm so that the
        // compiler computes the places here instead of holding all of them
        // in registers for the whole loop)
        int il = i16;
        __asm__ volatile("" : "+v"(il));
#pragma unroll
        for (int ct = 0; ct < NT; ++ct) {
          const int pl = ct * 16 + il, blk = pl / KK, o = pl - blk * KK;
          if (o < RB) {
#pragma unroll
            for (int q = 0; q < 4; ++q) Tw[(4 * kq + q) * TS + 4 * o + blk] = acc[rt][ct][q];
          }
        }
        __builtin_amdgcn_wave_barrier();
        // 16 rows x F4 float4, 64 lanes at a time
        constexpr int NPASS = (16 * F4 + 63) / 64;
#pragma unroll
        for (int v = 0; v < NPASS; ++v) {
          const int f = min(lane + 64 * v, 16 * F4 - 1);
          const int row = f / F4, c4 = f - row * F4;
          const int dr = __shfl(d[rt], row);
          const float4 val = *reinterpret_cast<const float4 *>(Tw + row * TS + 4 * c4);
          if (lane + 64 * v < 16 * F4 && cur.row0 + rt * 16 + row < cur.end)
            *reinterpret_cast<float4 *>(out + (size_t)dr * CS + 4 * c4) = val;
        }
        __builtin_amdgcn_wave_barrier();
      }
    }
    if (more) {
      if (group_off[nxt.g] != group_off[cur.g]) {
        __syncthreads();  // every wave is done with the current operator
        stage_b(nxt.g);
        __syncthreads();
      }
      cur = nxt;
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) d[rt] = dn[rt];
    }
  }
}

// The kernel: one row tile per wave, so that a wave needs at most 128
// registers and four near-field waves per SIMD (56 registers each) can be
// resident beside the two M2L waves, which leave the matrix cores idle for
// most of the launch while they wait on memory.  The LDS is dynamic (set at
// launch) so that the compiler holds the register budget of four waves per
// SIMD, which a static 128 KB would tell it it cannot reach.
template <int NT, int RB>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4)))
k_m2l_bf(const int32_t *__restrict__ tile_group, const int32_t *__restrict__ tile_row,
         const int32_t *__restrict__ group_off, const int32_t *__restrict__ group_end,
         const int32_t *__restrict__ src, const int32_t *__restrict__ dest, const bf16x8 *__restrict__ Tbf,
         const float *__restrict__ M, float *__restrict__ out, int ntiles) {
  using C = M2LBf<NT, RB>;
  extern __shared__ bf16x8 dyn_lds[];
  bf16x8 *Bs = dyn_lds;                                   // C::TBV operator entries
  float *Ts = reinterpret_cast<float *>(dyn_lds + C::TBV);  // store staging
  m2l_bf_units<NT, RB, 1>(tile_group, tile_row, group_off, group_end, src, dest, Tbf, M, out, ntiles, Bs, Ts);
}
constexpr int NT_FIXED = (P_FIXED * P_FIXED + 15) / 16, RB_FIXED = (P_FIXED * P_FIXED + 3) / 4;
constexpr int M2L_BF_LDS = M2LBf<NT_FIXED, RB_FIXED>::TBV * 16 + M2LBf<NT_FIXED, RB_FIXED>::NW * 16 *
                                                                   M2LBf<NT_FIXED, RB_FIXED>::TS * 4;
static_assert(M2LBf<NT_FIXED, RB_FIXED>::CS == P_FIXED * P_FIXED, "compact rows hold the p^2 coefficients");

// Persistent FP64 M2L, for large pair counts (on small ones one tile per
// workgroup is faster).  The FP64 operator (100 KB at p = 10) leaves room in
// LDS for one workgroup per CU, so the workgroup has 8 waves (two per SIMD,
// each with RT = 2 row tiles: 256 rows per tile, the FP32 tile lists) and
// walks a contiguous, XCD-aware range of tiles, reloading the operator only
// when the offset group changes.  Per tile the arithmetic is that of
// k_m2l<double, NT, 2, false, 0> (same operands, same K order), so results
// are identical; the operator is read from LDS instead of from L2 at every
// k-step.
template <int NT>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2)))
k_m2l_pers64(const int32_t *__restrict__ tile_group, const int32_t *__restrict__ tile_row,
             const int32_t *__restrict__ group_off, const int32_t *__restrict__ group_end,
             const int32_t *__restrict__ src, const int32_t *__restrict__ dest, const double *__restrict__ Tsw,
             const double *__restrict__ M, double *__restrict__ out, int ntiles) {
  constexpr int RT = 2, NW = 8;
  constexpr int PS = NT * 16;
  constexpr int KK = PS / 4;
  constexpr int TB2 = KK * NT * 32;  // double2 per operator
  __shared__ double2 Bs[TB2];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int i16 = lane & 15, kq = lane >> 4;
  const int nwg = gridDim.x;
  const int wg = xcd_block(blockIdx.x, nwg);
  const int t0 = (int)((int64_t)ntiles * wg / nwg), t1 = (int)((int64_t)ntiles * (wg + 1) / nwg);
  if (t0 >= t1) return;  // uniform over the workgroup

  struct TileIn {
    int g, end, row0;
  };
  auto tile_in = [&](int t) {
    TileIn v;
    v.g = tile_group[t];
    v.end = group_end[v.g];
    v.row0 = tile_row[t] + wave * (16 * RT);
    return v;
  };
  auto stage_b = [&](int g) {
    const double2 *Bg = reinterpret_cast<const double2 *>(Tsw) + (size_t)group_off[g] * TB2;
    for (int v = threadIdx.x; v < TB2; v += 64 * NW) Bs[v] = Bg[v];
  };

  double a[RT][KK];
  int d[RT][4];
  TileIn cur = tile_in(t0);
  stage_b(cur.g);
  __syncthreads();
  for (int t = t0; t < t1; ++t) {
    if (t > t0) {
      const TileIn nxt = tile_in(t);
      if (group_off[nxt.g] != group_off[cur.g]) {
        __syncthreads();  // every wave is done with the current operator
        stage_b(nxt.g);
        __syncthreads();
      }
      cur = nxt;
    }
    // gather: a lane loads the K slice of its lane group of row i16 of each
    // row tile, and the destinations of the rows it stores
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
      const int sr = src[min(cur.row0 + rt * 16 + i16, cur.end - 1)];
      const double2 *Ms = reinterpret_cast<const double2 *>(M + (size_t)sr * PS + kq * KK);
#pragma unroll
      for (int v = 0; v < KK / 2; ++v) {
        const double2 q = Ms[v];
        a[rt][2 * v] = q.x;
        a[rt][2 * v + 1] = q.y;
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) d[rt][q] = dest[min(cur.row0 + rt * 16 + kq + 4 * q, cur.end - 1)];
    }
    if (cur.row0 >= cur.end) continue;
    f64x4 acc[RT][NT];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int ct = 0; ct < NT; ++ct) acc[rt][ct] = f64x4{0.0, 0.0, 0.0, 0.0};
    const double *B = reinterpret_cast<const double *>(Bs) + lane;
#pragma unroll
    for (int kk = 0; kk < kk_used(NT); ++kk) {
#pragma unroll
      for (int ct = 0; ct < NT; ++ct) {
        const double b = B[(kk * NT + ct) * 64];
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
          acc[rt][ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[rt][kk], b, acc[rt][ct], 0, 0, 0);
      }
    }
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (cur.row0 + rt * 16 + kq + 4 * q < cur.end) {
          double *o = out + (size_t)d[rt][q] * PS + i16;
#pragma unroll
          for (int ct = 0; ct < NT; ++ct) o[ct * 16] = acc[rt][ct][q];
        }
  }
}

// ----------------------------------------------------------- downward pass

template <class R> struct VecT;
template <> struct VecT<float> { using T = float4; static constexpr int W = 4; };
template <> struct VecT<double> { using T = double2; static constexpr int W = 2; };

// One wave per cell of level l: L = L2L(parent) + sum of the cell's M2L
// results.  The cell's result rows are one contiguous run (kptr), read with
// vector loads: a row of rs reals takes rs/W lanes, so several rows are
// read per step by lane groups, U rows in flight per group; every lane keeps
// a compensated sum, and the groups are added in group order; the L2L term
// (a batched MFMA product per level, l2l[cell of the level][ps]) is added
// last.  Rows are either in the stored layout (rs = ps) or compact (the
// split-bf16 M2L: rs = p^2 coefficients in packed order, no padding places),
// whose sums go to their places.  At the leaf level the kernel also writes
// the evaluation coefficients E[leaf][4][ps] of the potential and of its
// gradient (see L2P).
template <class R>
__global__ void __launch_bounds__(256) k_downward(int p, int ps, int rs, int compact, int64_t c0, int64_t C,
                                                  int with_parent, const R *__restrict__ l2l,
                                                  const int32_t *__restrict__ kptr, const R *__restrict__ m2l,
                                                  R *__restrict__ Lx, int leaf, R inv_s, R *__restrict__ E) {
  using VT = typename VecT<R>::T;
  constexpr int W = VecT<R>::W;
  constexpr int U = 8;
  extern __shared__ char smem_raw[];
  const int nthr = blockDim.x;                // 64 or 256
  R *Ls = reinterpret_cast<R *>(smem_raw);     // [ps]
  R *part = Ls + ps;                          // [nthr * W] group partials
  const int64_t c = c0 + blockIdx.x;
  if (blockIdx.x >= C) return;
  const int lane = threadIdx.x;
  const int np2 = p * p;
  const int lpr = rs / W;                     // lanes per row
  // rows per step, from the stored row length whatever the row format, so
  // that every coefficient is summed over the same rows in the same order
  // from compact and from stored rows
  const int groups = nthr / (ps / W);
  const int grp = lane / lpr, k4 = lane - grp * lpr;
  const bool act = grp < groups;
  R s[W], comp[W];
#pragma unroll
  for (int w = 0; w < W; ++w) s[w] = comp[w] = R(0);
  const int b = kptr[c], e = kptr[c + 1];
  if (act) {
    const VT *rows = reinterpret_cast<const VT *>(m2l) + k4;
    int q = b + grp;
    for (; q + (U - 1) * groups < e; q += U * groups) {
      VT v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) v[u] = rows[(size_t)(q + u * groups) * lpr];
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int w = 0; w < W; ++w) {
          const R y = reinterpret_cast<const R *>(&v[u])[w] - comp[w];
          const R t = s[w] + y;
          comp[w] = (t - s[w]) - y;
          s[w] = t;
        }
    }
    for (; q < e; q += groups) {
      const VT v = rows[(size_t)q * lpr];
#pragma unroll
      for (int w = 0; w < W; ++w) {
        const R y = reinterpret_cast<const R *>(&v)[w] - comp[w];
        const R t = s[w] + y;
        comp[w] = (t - s[w]) - y;
        s[w] = t;
      }
    }
  }
#pragma unroll
  for (int w = 0; w < W; ++w) part[lane * W + w] = s[w];
  if (compact)
    for (int k = lane; k < ps; k += nthr) Ls[k] = R(0);  // the padding places
  __syncthreads();
  // group totals in group order -> Ls[place of k]
  for (int k = lane; k < rs; k += nthr) {
    const int kk = k / W, w = k - kk * W;
    R acc = part[kk * W + w], cc = R(0);
    for (int h = 1; h < groups; ++h) {
      const R y = part[(h * lpr + kk) * W + w] - cc;
      const R t = acc + y;
      cc = (t - acc) - y;
      acc = t;
    }
    Ls[compact ? coef_pos(k, p, ps) : k] = acc;
  }
  __syncthreads();
  if (with_parent) {
    const R *Lc = l2l + (size_t)blockIdx.x * ps;
    for (int k = lane; k < ps; k += nthr) Ls[k] += Lc[k];
  }
  __syncthreads();
  R *out = Lx + (size_t)c * ps;
  for (int k = lane; k < ps; k += nthr) out[k] = Ls[k];
  if (!leaf) return;
  // evaluation coefficients of the leaf (scaled to physical units):
  // phi(x) = sum_k E0[k] * Rpacked_k(rho), grad phi = sum_k E{x,y,z}[k] * Rpacked_k(rho)
  R *Ec = E + (size_t)blockIdx.x * 4 * ps;
  const R inv_s2 = inv_s * inv_s;
  for (int k = lane; k < ps; k += nthr) {
    Ec[k] = R(0);
    Ec[ps + k] = R(0);
    Ec[2 * ps + k] = R(0);
    Ec[3 * ps + k] = R(0);
  }
  __syncthreads();
  auto Lre = [&](int n, int m) -> R {  // Re L_n^m for any m
    if (n >= p || m > n || -m > n) return R(0);
    if (m >= 0) return Ls[coef_pos(idx_re(n, m), p, ps)];
    return ((-m) & 1) ? -Ls[coef_pos(idx_re(n, -m), p, ps)] : Ls[coef_pos(idx_re(n, -m), p, ps)];
  };
  auto Lim = [&](int n, int m) -> R {
    if (n >= p || m > n || -m > n || m == 0) return R(0);
    if (m > 0) return Ls[coef_pos(idx_im(n, m), p, ps)];
    // L^{-m} = (-1)^m conj(L^m)
    return ((-m) & 1) ? Ls[coef_pos(idx_im(n, -m), p, ps)] : -Ls[coef_pos(idx_im(n, -m), p, ps)];
  };
  for (int k = lane; k < np2; k += nthr) {
    int n = 0;
    while ((n + 1) * (n + 1) <= k) ++n;
    const int rem = k - n * n;
    const int m = (rem + 1) / 2;
    const bool im = (rem > 0) && ((rem & 1) == 0);
    const R two = (m > 0) ? R(2) : R(1);
    Ec[k] = im ? (-R(2) * Lim(n, m) * inv_s) : (two * Lre(n, m) * inv_s);
    if (n <= p - 2) {
      // G_z = L_{n+1}^m; G_x = (L_{n+1}^{m-1} - L_{n+1}^{m+1})/2; G_y = -i (L_{n+1}^{m+1} + L_{n+1}^{m-1})/2
      const R gzr = Lre(n + 1, m), gzi = Lim(n + 1, m);
      const R gxr = R(0.5) * (Lre(n + 1, m - 1) - Lre(n + 1, m + 1));
      const R gxi = R(0.5) * (Lim(n + 1, m - 1) - Lim(n + 1, m + 1));
      const R sr = R(0.5) * (Lre(n + 1, m + 1) + Lre(n + 1, m - 1));
      const R si = R(0.5) * (Lim(n + 1, m + 1) + Lim(n + 1, m - 1));
      const R gyr = si, gyi = -sr;  // -i (sr + i si)
      if (im) {
        Ec[ps + k] = -R(2) * gxi * inv_s2;
        Ec[2 * ps + k] = -R(2) * gyi * inv_s2;
        Ec[3 * ps + k] = -R(2) * gzi * inv_s2;
      } else {
        Ec[ps + k] = two * gxr * inv_s2;
        Ec[2 * ps + k] = two * gyr * inv_s2;
        Ec[3 * ps + k] = two * gzr * inv_s2;
      }
    }
  }
}

// -------------------------------------------------------------- P2P + L2P

// One source-target pair.  Monopole: lp += w/r, (lx,ly,lz) += w d/r^3 (=
// -grad).  Dipole m: lp += m.d/r^3, (lx,ly,lz) += 3 (m.d) d/r^5 - m/r^3 (=
// -grad).  d = target - source, ri = 1/r (0 for the excluded self pair).
template <class R, int SRC, int OUT>
__device__ __forceinline__ void pair_eval(const typename V4<R>::T &s4, const typename V4<R>::T &m4, R dx, R dy, R dz,
                                          R ri, R &lp, R &lx, R &ly, R &lz) {
  if (SRC == SRC_PANEL_MONO || SRC == SRC_CHARGE_MONO) {
    const R wr = s4.w * ri;
    if (OUT == OUT_POT || OUT == OUT_POTGRAD) lp += wr;
    if (OUT != OUT_POT) {
      const R t = wr * ri * ri;
      lx += t * dx;
      ly += t * dy;
      lz += t * dz;
    }
  } else {
    const R ri2 = ri * ri;
    const R ri3 = ri2 * ri;
    const R md = m4.x * dx + m4.y * dy + m4.z * dz;
    R t = R(0), pot = md * ri3;
    if (SRC == SRC_PANEL_MONODIP) {
      const R wr = s4.w * ri;
      pot += wr;
      t = wr * ri2;
    }
    if (OUT == OUT_POT || OUT == OUT_POTGRAD) lp += pot;
    if (OUT != OUT_POT) {
      t += R(3) * md * ri3 * ri2;
      lx += t * dx - m4.x * ri3;
      ly += t * dy - m4.y * ri3;
      lz += t * dz - m4.z * ri3;
    }
  }
}



// 1/r^3 in FP64 from r^2 without forming 1/r: with y0 the hardware estimate
// of r^-1/2 and e = 1 - r^2 y0^2, the Newton-corrected 1/r^3 is
// y0^3 (1 + 3e/2) to first order in e, one multiply fewer than correcting
// 1/r and cubing it.
__device__ __forceinline__ double inv_r3(double r2) {
  const double y0 = __builtin_amdgcn_rsq(r2);
  const double y2 = y0 * y0;
  const double e = __builtin_fma(-r2, y2, 1.0);
  const double y3 = y2 * y0;
  return __builtin_fma(1.5 * y3, e, y3);
}

// A pair from r^2; `skip` marks the excluded self pair (its terms are zero).
// In FP64 the pairs that need only 1/r^3 take it from inv_r3: monopole
// sources with the normal derivative (the A and B products) and dipole
// sources with the potential (the A^T product).
template <class R, int SRC, int OUT>
__device__ __forceinline__ void pair_eval_r2(const typename V4<R>::T &s4, const typename V4<R>::T &m4, R dx, R dy,
                                             R dz, R r2, bool skip, R &lp, R &lx, R &ly, R &lz) {
  constexpr bool F64 = std::is_same<R, double>::value;
  if constexpr (F64 && (SRC == SRC_PANEL_MONO || SRC == SRC_CHARGE_MONO) && OUT == OUT_NGRAD) {
    const double t = skip ? 0.0 : s4.w * inv_r3(r2);
    lx += t * dx;
    ly += t * dy;
    lz += t * dz;
  } else if constexpr (F64 && SRC == SRC_PANEL_DIP && OUT == OUT_POT) {
    const double ri3 = skip ? 0.0 : inv_r3(r2);
    lp += (m4.x * dx + m4.y * dy + m4.z * dz) * ri3;
  } else {
    const R ri = skip ? R(0) : rsq(r2);
    pair_eval<R, SRC, OUT>(s4, m4, dx, dy, dz, ri, lp, lx, ly, lz);
  }
}

template <class R, int SRC, int OUT>
__device__ __forceinline__ void pair_accumulate(const typename V4<R>::T &s4, const typename V4<R>::T *sdip, int j,
                                                R dx, R dy, R dz, R r2, bool skip, R &lp, R &lx, R &ly, R &lz) {
  typename V4<R>::T m4{};
  if (SRC == SRC_PANEL_DIP || SRC == SRC_PANEL_MONODIP) m4 = sdip[j];
  pair_eval_r2<R, SRC, OUT>(s4, m4, dx, dy, dz, r2, skip, lp, lx, ly, lz);
}

// Near quadrature: near_out[t] += sum over the close pairs of t, in list
// order, of coef * x[caller index] (FP64; 4 pi times the exact-minus-point
// difference of K' or of K'^T, see the tree's nq lists).  For A^T the sum is
// divided by the target's area as the product stores it (the combine
// multiplies the near field by that same area).
template <class R>
__global__ void k_nq_apply(int64_t n, const int32_t *__restrict__ ptr, const int32_t *__restrict__ idx,
                           const double *__restrict__ coef, const double *__restrict__ x,
                           const typename V4<R>::T *__restrict__ tgt_pos, double *__restrict__ near_out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  double acc = 0.0;
  for (int k = ptr[t]; k < ptr[t + 1]; ++k) acc += coef[k] * x[idx[k]];
  if (tgt_pos) acc /= (double)tgt_pos[t].w;
  near_out[t] += acc;
}

struct P2PArgs {
  int p, ps;
  const int4 *chunks;        // (leaf, first target, count, lane groups) per chunk
  const int4 *leaf_range;    // level-L ranges
  const int32_t *leaf_xyz;
  const int32_t *near_ptr, *near_idx;  // level-L CSR
  const void *tgt_pos;       // real4 (rx, ry, rz, area) [targets]
  const void *tgt_nrm;       // real4 [panels] (NGRAD)
  const void *src_pos;       // real4 (rx, ry, rz, w)
  const void *src_dip;       // real4 (mx, my, mz, 0)
  const void *E;             // real [nleaf][4][ps]
  const int32_t *tperm;      // sorted target -> caller index
  double sL;
  const double *xin;
  double alpha, beta;        // beta already includes 1/(4 pi)
  int area_scale;
  int accumulate;
  double *y;
  double *dbg_near, *dbg_far;  // sorted order, may be NULL
  double *near_out;            // near field per target, sorted order ([n] or [4n])
};

// Near field (P2P).  One wave per chunk of up to 64 targets of one leaf.  A
// chunk of n targets uses G = 64 / n lane groups: lane l works on target
// l % n and on every G-th source of each near leaf (starting at l / n), so
// small leaves still fill the wave; with one group the source index is
// uniform and the records come through the scalar cache.  Each lane sums
// one source leaf in plain arithmetic, adds the leaf total to a compensated
// (Kahan) accumulator, and the G partial results are added in group order
// through LDS.  The per-target result (potential, normal derivative, or
// potential and -gradient) goes to near_out in sorted order, in FP64.
template <class R, int SRC, int TGT, int OUT>
__global__ void __launch_bounds__(64) k_p2p_near(P2PArgs a) {
  using R4 = typename V4<R>::T;
  // staged source records during the sweep, group partials after it (the
  // two never live at once: 64 real4 = 4 x 64 reals)
  __shared__ R4 src_s[64];
  __shared__ R4 dip_s[(SRC == SRC_PANEL_DIP || SRC == SRC_PANEL_MONODIP) ? 64 : 1];
  R(*red)[64] = reinterpret_cast<R(*)[64]>(src_s);
  // (leaf, first target, count, groups); chunks are in Morton order
  const int4 ch = a.chunks[xcd_block(blockIdx.x, gridDim.x)];
  const int leaf = ch.x, count = ch.z, G = ch.w;
  const int lane = threadIdx.x;
  const int g = lane / count, tl = lane - g * count;
  const bool active = g < G;
  const int ti = ch.y + tl;
  const R4 *tpos = reinterpret_cast<const R4 *>(a.tgt_pos);
  const R4 *spos = reinterpret_cast<const R4 *>(a.src_pos);
  const R4 *sdip = reinterpret_cast<const R4 *>(a.src_dip);
  const R4 tp = tpos[ti];
  const R tx = tp.x, ty = tp.y, tz = tp.z;
  // ---- near field: direct sum over the near leaves, compensated per leaf
  R sp = R(0), cp = R(0), sx = R(0), cx = R(0), sy = R(0), cy = R(0), sz = R(0), cz = R(0);
  int txi, tyi, tzi;
  xyz_of(a.leaf_xyz[leaf], txi, tyi, tzi);
  const R sL = (R)a.sL;
  const int e0 = a.near_ptr[leaf], e1 = a.near_ptr[leaf + 1];
  for (int e = e0; e < e1; ++e) {
    const int sl = a.near_idx[e];
    const int4 sr = a.leaf_range[sl];
    const int sb = (SRC == SRC_CHARGE_MONO) ? sr.z : sr.x;
    const int se = (SRC == SRC_CHARGE_MONO) ? sr.w : sr.y;
    if (sb == se) continue;
    int sxi, syi, szi;
    xyz_of(a.leaf_xyz[sl], sxi, syi, szi);
    // target relative to the source leaf centre
    const R ux = tx + R(txi - sxi) * sL, uy = ty + R(tyi - syi) * sL, uz = tz + R(tzi - szi) * sL;
    R lp = R(0), lx = R(0), ly = R(0), lz = R(0);
    const bool self = (SRC != SRC_CHARGE_MONO) && (TGT == TGT_PANEL) && (sl == leaf);
    if (G == 1) {
      // one lane group: the source index is uniform across the wave, so the
      // source records come through the scalar cache
      if (self) {
        for (int j = sb; j < se; ++j) {
          const R4 s4 = spos[j];
          const R dx = ux - s4.x, dy = uy - s4.y, dz = uz - s4.z;
          const R r2 = dx * dx + dy * dy + dz * dz;
          // K'_ii = 0: the self panel is skipped by index
          pair_accumulate<R, SRC, OUT>(s4, sdip, j, dx, dy, dz, r2, j == ti, lp, lx, ly, lz);
        }
      } else {
        // software pipelined: the records of the next PF sources are
        // requested before the current PF are evaluated, so the wait for
        // the scalar loads falls after the arithmetic
        constexpr int PF = 4;
        constexpr bool DIPS = SRC == SRC_PANEL_DIP || SRC == SRC_PANEL_MONODIP;
        int j = sb;
        if (se - sb >= 2 * PF) {
          R4 cs[PF], cm[PF];
#pragma unroll
          for (int u = 0; u < PF; ++u) {
            cs[u] = spos[j + u];
            if (DIPS) cm[u] = sdip[j + u];
          }
          for (; j + 2 * PF <= se; j += PF) {
            R4 ns[PF], nm[PF];
#pragma unroll
            for (int u = 0; u < PF; ++u) {
              ns[u] = spos[j + PF + u];
              if (DIPS) nm[u] = sdip[j + PF + u];
            }
#pragma unroll
            for (int u = 0; u < PF; ++u) {
              const R dx = ux - cs[u].x, dy = uy - cs[u].y, dz = uz - cs[u].z;
              const R r2 = dx * dx + dy * dy + dz * dz;
              pair_eval_r2<R, SRC, OUT>(cs[u], cm[u], dx, dy, dz, r2, false, lp, lx, ly, lz);
            }
#pragma unroll
            for (int u = 0; u < PF; ++u) {
              cs[u] = ns[u];
              if (DIPS) cm[u] = nm[u];
            }
          }
#pragma unroll
          for (int u = 0; u < PF; ++u) {
            const R dx = ux - cs[u].x, dy = uy - cs[u].y, dz = uz - cs[u].z;
            const R r2 = dx * dx + dy * dy + dz * dz;
            pair_eval_r2<R, SRC, OUT>(cs[u], cm[u], dx, dy, dz, r2, false, lp, lx, ly, lz);
          }
          j += PF;
        }
        for (; j < se; ++j) {
          const R4 s4 = spos[j];
          const R dx = ux - s4.x, dy = uy - s4.y, dz = uz - s4.z;
          const R r2 = dx * dx + dy * dy + dz * dz;
          pair_accumulate<R, SRC, OUT>(s4, sdip, j, dx, dy, dz, r2, false, lp, lx, ly, lz);
        }
      }
    } else {
      // several lane groups: the source leaf is staged in LDS, 64 records at
      // a time, with one coalesced load; every lane group then reads its own
      // sources there (a group's lanes read the same record: a broadcast)
      constexpr bool DIPS = SRC == SRC_PANEL_DIP || SRC == SRC_PANEL_MONODIP;
      for (int base = sb; base < se; base += 64) {
        const int cnt = min(64, se - base);
        __syncthreads();  // the previous records are no longer read
        if (lane < cnt) {
          src_s[lane] = spos[base + lane];
          if (DIPS) dip_s[lane] = sdip[base + lane];
        }
        __syncthreads();
        if (!active) continue;
        if (self) {
          for (int jj = g; jj < cnt; jj += G) {
            const R4 s4 = src_s[jj];
            const R dx = ux - s4.x, dy = uy - s4.y, dz = uz - s4.z;
            const R r2 = dx * dx + dy * dy + dz * dz;
            pair_eval_r2<R, SRC, OUT>(s4, DIPS ? dip_s[jj] : s4, dx, dy, dz, r2, base + jj == ti, lp, lx, ly, lz);
          }
        } else {
#pragma unroll 4
          for (int jj = g; jj < cnt; jj += G) {
            const R4 s4 = src_s[jj];
            const R dx = ux - s4.x, dy = uy - s4.y, dz = uz - s4.z;
            const R r2 = dx * dx + dy * dy + dz * dz;
            pair_eval_r2<R, SRC, OUT>(s4, DIPS ? dip_s[jj] : s4, dx, dy, dz, r2, false, lp, lx, ly, lz);
          }
        }
      }
    }
    // Kahan accumulation of the per-leaf partial sums
    {
      R y_ = lp - cp, t_ = sp + y_;
      cp = (t_ - sp) - y_;
      sp = t_;
      y_ = lx - cx; t_ = sx + y_; cx = (t_ - sx) - y_; sx = t_;
      y_ = ly - cy; t_ = sy + y_; cy = (t_ - sy) - y_; sy = t_;
      y_ = lz - cz; t_ = sz + y_; cz = (t_ - sz) - y_; sz = t_;
    }
  }
  // ---- combine the G lane groups in group order
  if (G > 1) {
    __syncthreads();  // the last staged records are no longer read
    red[0][lane] = sp;
    red[1][lane] = sx;
    red[2][lane] = sy;
    red[3][lane] = sz;
    __syncthreads();
    if (g == 0) {
      R s0 = red[0][tl], c0 = R(0), s1 = red[1][tl], c1 = R(0), s2 = red[2][tl], c2 = R(0), s3 = red[3][tl],
        c3 = R(0);
      for (int h = 1; h < G; ++h) {
        const int k = h * count + tl;
        R y_ = red[0][k] - c0, t_ = s0 + y_; c0 = (t_ - s0) - y_; s0 = t_;
        y_ = red[1][k] - c1; t_ = s1 + y_; c1 = (t_ - s1) - y_; s1 = t_;
        y_ = red[2][k] - c2; t_ = s2 + y_; c2 = (t_ - s2) - y_; s2 = t_;
        y_ = red[3][k] - c3; t_ = s3 + y_; c3 = (t_ - s3) - y_; s3 = t_;
      }
      sp = s0;
      sx = s1;
      sy = s2;
      sz = s3;
    }
  }
  if (g != 0) return;
  if (OUT == OUT_POT) {
    a.near_out[ti] = (double)sp;
  } else if (OUT == OUT_NGRAD) {
    const R4 nn = reinterpret_cast<const R4 *>(a.tgt_nrm)[ti];
    a.near_out[ti] = -((double)nn.x * sx + (double)nn.y * sy + (double)nn.z * sz);
  } else {
    a.near_out[4 * (size_t)ti] = (double)sp;
    a.near_out[4 * (size_t)ti + 1] = -(double)sx;
    a.near_out[4 * (size_t)ti + 2] = -(double)sy;
    a.near_out[4 * (size_t)ti + 3] = -(double)sz;
  }
}

// Far field (L2P from the leaf's evaluation coefficients, read through the
// scalar cache) plus the near field, combined into the operator's output in
// the caller's order: y = alpha x + beta (area) field.
// P > 0: the order fixed at compile time (P == a.p), so the harmonics unroll
// and the coefficient loads are at constant offsets; P = 0: any order.
template <class R, int TGT, int OUT, int P>
__global__ void __launch_bounds__(64) k_l2p_combine(P2PArgs a) {
  using R4 = typename V4<R>::T;
  const int4 ch = a.chunks[blockIdx.x];
  const int leaf = ch.x, count = ch.z;
  const int tl = threadIdx.x;
  if (tl >= count) return;
  const int ti = ch.y + tl;
  const R4 tp = reinterpret_cast<const R4 *>(a.tgt_pos)[ti];
  const R *E = reinterpret_cast<const R *>(a.E) + (size_t)leaf * 4 * a.ps;
  const R inv_s = R(1.0 / a.sL);
  R fp = R(0), fgx = R(0), fgy = R(0), fgz = R(0);
  {
    const R x = tp.x * inv_s, y = tp.y * inv_s, z = tp.z * inv_s;
    const int p = P > 0 ? P : a.p;
    auto term = [&](int n, int m, R re, R im) {
      const int kr = idx_re(n, m);
      if (OUT != OUT_NGRAD) {
        fp += E[kr] * re;
        if (m > 0) fp += E[idx_im(n, m)] * im;
      }
      if (OUT != OUT_POT && n <= p - 2) {
        fgx += E[a.ps + kr] * re;
        fgy += E[2 * a.ps + kr] * re;
        fgz += E[3 * a.ps + kr] * re;
        if (m > 0) {
          const int ki = idx_im(n, m);
          fgx += E[a.ps + ki] * im;
          fgy += E[2 * a.ps + ki] * im;
          fgz += E[3 * a.ps + ki] * im;
        }
      }
    };
    if constexpr (P > 0)
      regular_harmonics_fixed<P, R>(x, y, z, term);
    else
      regular_harmonics<R>(p, x, y, z, term);
  }
  const int64_t u = a.tperm[ti];
  double res[4], near_v, far_v;
  int nres = 1;
  // near_out is NULL for a far-field-only product
  const double *no = a.near_out;
  if (OUT == OUT_POT) {
    near_v = no ? no[ti] : 0.0;
    far_v = (double)fp;
    res[0] = near_v + far_v;
  } else if (OUT == OUT_NGRAD) {
    const R4 nn = reinterpret_cast<const R4 *>(a.tgt_nrm)[ti];
    near_v = no ? no[ti] : 0.0;
    far_v = (double)nn.x * fgx + (double)nn.y * fgy + (double)nn.z * fgz;
    res[0] = near_v + far_v;
  } else {
    near_v = no ? no[4 * (size_t)ti] : 0.0;
    far_v = (double)fp;
    res[0] = near_v + far_v;
    res[1] = (no ? no[4 * (size_t)ti + 1] : 0.0) + (double)fgx;
    res[2] = (no ? no[4 * (size_t)ti + 2] : 0.0) + (double)fgy;
    res[3] = (no ? no[4 * (size_t)ti + 3] : 0.0) + (double)fgz;
    nres = 4;
  }
  if (a.dbg_near) {
    a.dbg_near[ti] = near_v;
    a.dbg_far[ti] = far_v;
  }
  double scale = a.beta;
  if (a.area_scale) scale *= (double)tp.w;
  if (nres == 1) {
    double v = scale * res[0];
    if (a.xin) v += a.alpha * a.xin[u];
    if (a.accumulate) v += a.y[u];
    a.y[u] = v;
  } else {
    for (int k = 0; k < 4; ++k) {
      double v = scale * res[k];
      if (a.accumulate) v += a.y[4 * u + k];
      a.y[4 * u + k] = v;
    }
  }
}

// Uploads the recurrence coefficients to the current device's constant
// memory, once per device (constant memory is per device).
void set_rec_constants() {
  static std::mutex mu;
  static std::set<int> done;
  int dev = 0;
  HIP_OK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(mu);
  if (done.count(dev)) return;
  float r1f[PMAX + 1][PMAX + 1] = {}, r2f[PMAX + 1][PMAX + 1] = {}, hf[PMAX + 1] = {};
  double r1d[PMAX + 1][PMAX + 1] = {}, r2d[PMAX + 1][PMAX + 1] = {}, hd[PMAX + 1] = {};
  for (int n = 0; n <= PMAX; ++n)
    for (int m = 0; m <= PMAX; ++m)
      if (n > m) {
        double den = double(n * n - m * m);
        r1d[n][m] = (2.0 * n - 1.0) / den;
        r2d[n][m] = 1.0 / den;
        r1f[n][m] = (float)r1d[n][m];
        r2f[n][m] = (float)r2d[n][m];
      }
  for (int m = 1; m <= PMAX; ++m) {
    hd[m] = 1.0 / (2.0 * m);
    hf[m] = (float)hd[m];
  }
  HIP_OK(hipMemcpyToSymbol(HIP_SYMBOL(c_rec1_f), r1f, sizeof(r1f)));
  HIP_OK(hipMemcpyToSymbol(HIP_SYMBOL(c_rec2_f), r2f, sizeof(r2f)));
  HIP_OK(hipMemcpyToSymbol(HIP_SYMBOL(c_rec1_d), r1d, sizeof(r1d)));
  HIP_OK(hipMemcpyToSymbol(HIP_SYMBOL(c_rec2_d), r2d, sizeof(r2d)));
  HIP_OK(hipMemcpyToSymbol(HIP_SYMBOL(c_half_inv_m_f), hf, sizeof(hf)));
  HIP_OK(hipMemcpyToSymbol(HIP_SYMBOL(c_half_inv_m_d), hd, sizeof(hd)));
  done.insert(dev);
}

}  // namespace

// ---------------------------------------------------------------- driver

// Stage timing: events are recorded on the stream that runs the stage and
// read after the product has finished, so profiling does not serialise the
// two streams.
void prof_begin(Tree &T, int stage, hipStream_t s) {
  if (!T.prof_now) return;
  HIP_OK(hipEventRecord(T.ev[2 * stage], s));
}

void prof_end(Tree &T, int stage, hipStream_t s) {
  if (!T.prof_now) return;
  HIP_OK(hipEventRecord(T.ev[2 * stage + 1], s));
  T.prof_pending[stage] = true;
}

static void prof_collect(Tree &T) {
  if (!T.prof_now) return;
  for (int st = 0; st < 7; ++st) {
    if (!T.prof_pending[st]) continue;
    HIP_OK(hipEventSynchronize(T.ev[2 * st + 1]));
    float ms = 0.f;
    HIP_OK(hipEventElapsedTime(&ms, T.ev[2 * st], T.ev[2 * st + 1]));
    T.prof_ms[T.prof_kind][T.prof_prec][st] += ms;
    T.prof_cnt[T.prof_kind][T.prof_prec][st] += 1;
    T.prof_pending[st] = false;
  }
}

static PrecBufs &bufs(Tree &T, int prec, hipStream_t s) {
  PrecBufs *&pb = (prec == BEMFMM_FP64) ? T.pb64 : T.pb32;
  if (!pb) {
    pb = new PrecBufs();
    const size_t rs = (prec == BEMFMM_FP64) ? 8 : 4;
    const int64_t npts = std::max<int64_t>(std::max(T.N, T.Q), 1);
    pb->src_pos.alloc(npts * 4 * rs);
    pb->src_dip.alloc(npts * 4 * rs);
    pb->M.alloc((size_t)T.ncell_tot * T.ps * rs);
    pb->L.alloc((size_t)T.ncell_tot * T.ps * rs);
    pb->m2l_out.alloc((size_t)std::max<int64_t>(T.nfar, 1) * T.ps * rs);
    pb->l2l_out.alloc((size_t)std::max<int64_t>(T.l2lw.max_cells, 1) * T.ps * rs);
    pb->E.alloc((size_t)T.ncell[T.L] * 4 * T.ps * rs);
    pb->near_out.alloc(4 * npts);
    pb->M.zero(s);
    pb->L.zero(s);
    pb->E.zero(s);
    pb->src_dip.zero(s);
    pb->prec = prec;
  }
  return *pb;
}

template <class R>
static void launch_p2m(Tree &T, PrecBufs &B, int src, hipStream_t s) {
  using R4 = typename V4<R>::T;
  const int L = T.L, ps = T.ps;
  const int64_t CL = T.ncell[L];
  const double sL = T.side / double(1 << L);
  const size_t shm = (size_t)64 * (ps + 1) * sizeof(R);
  const R4 *spos = reinterpret_cast<const R4 *>(B.src_pos.p);
  const R4 *sdip = reinterpret_cast<const R4 *>(B.src_dip.p);
  R *M = reinterpret_cast<R *>(B.M.p) + (size_t)T.coff[L] * ps;
  const int4 *rg = T.crange.p + T.coff[L];
  const R inv = R(1.0 / sL);
  if (T.p == P_FIXED) {
    switch (src) {
      case SRC_PANEL_MONO:
        k_p2m_fixed<P_FIXED, R, true, false><<<CL, 64, 0, s>>>(ps, CL, rg, 0, spos, sdip, inv, M);
        break;
      case SRC_CHARGE_MONO:
        k_p2m_fixed<P_FIXED, R, true, false><<<CL, 64, 0, s>>>(ps, CL, rg, 1, spos, sdip, inv, M);
        break;
      case SRC_PANEL_DIP:
        k_p2m_fixed<P_FIXED, R, false, true><<<CL, 64, 0, s>>>(ps, CL, rg, 0, spos, sdip, inv, M);
        break;
      default:
        k_p2m_fixed<P_FIXED, R, true, true><<<CL, 64, 0, s>>>(ps, CL, rg, 0, spos, sdip, inv, M);
        break;
    }
    LAUNCH_OK();
    return;
  }
  switch (src) {
    case SRC_PANEL_MONO:
      k_p2m<R, true, false><<<CL, 64, shm, s>>>(T.p, ps, CL, rg, 0, spos, sdip, inv, M);
      break;
    case SRC_CHARGE_MONO:
      k_p2m<R, true, false><<<CL, 64, shm, s>>>(T.p, ps, CL, rg, 1, spos, sdip, inv, M);
      break;
    case SRC_PANEL_DIP:
      k_p2m<R, false, true><<<CL, 64, shm, s>>>(T.p, ps, CL, rg, 0, spos, sdip, inv, M);
      break;
    default:
      k_p2m<R, true, true><<<CL, 64, shm, s>>>(T.p, ps, CL, rg, 0, spos, sdip, inv, M);
      break;
  }
  LAUNCH_OK();
}

// Batched per-level product on the MFMA kernel: for every cell c of level
// l (l >= 3), out[c - coff[l]] = S_oct(c) in[src[c]], with the per-octant
// operator table S (M2M: src = the cell, L2L: src = its parent).
template <class R, int USE>
static void level_product(Tree &T, int l, const int32_t *src, const void *table, const R *in, R *out,
                          hipStream_t s) {
  const bool f64 = std::is_same<R, double>::value;
  const Tree::L2LList &LW = T.l2lw;
  const int64_t t0 = LW.t0[l], t1 = LW.t1[l];
  if (t1 <= t0) return;
  const dim3 grid((unsigned)(t1 - t0));
#define LEVEL_CASE(nt)                                                                                          \
  case nt:                                                                                                      \
    if (f64)                                                                                                    \
      k_m2l<double, nt, LEVEL_RT, false, USE><<<grid, 256, 0, s>>>(                                             \
          LW.tile_group.p + t0, LW.tile_row.p + t0, LW.group_off.p, LW.group_end.p, src, LW.dest.p,             \
          reinterpret_cast<const double *>(table), reinterpret_cast<const double *>(in),                        \
          reinterpret_cast<double *>(out));                                                                     \
    else                                                                                                        \
      k_m2l<float, nt, LEVEL_RT, true, USE><<<grid, 256, 0, s>>>(                                               \
          LW.tile_group.p + t0, LW.tile_row.p + t0, LW.group_off.p, LW.group_end.p, src, LW.dest.p,             \
          reinterpret_cast<const float *>(table), reinterpret_cast<const float *>(in),                          \
          reinterpret_cast<float *>(out));                                                                      \
    break;
  switch (T.ps / 16) {
    LEVEL_CASE(1)
    LEVEL_CASE(2)
    LEVEL_CASE(3)
    LEVEL_CASE(4)
    LEVEL_CASE(5)
    LEVEL_CASE(6)
    LEVEL_CASE(7)
    LEVEL_CASE(8)
    default:
      BF_THROW(BEMFMM_EINVAL, "unsupported expansion order");
  }
#undef LEVEL_CASE
  LAUNCH_OK();
}

template <class R>
static void run_fmm(Tree &T, PrecBufs &B, const FmmRequest &rq, hipStream_t s) {
  using R4 = typename V4<R>::T;
  set_rec_constants();
  const bool f64 = std::is_same<R, double>::value;
  const int L = T.L, p = T.p, ps = T.ps;
  const int TB = 256;
  const double sL = T.side / double(1 << L);
  const bool src_charges = rq.src == SRC_CHARGE_MONO;
  R4 *spos = reinterpret_cast<R4 *>(B.src_pos.p);
  R4 *sdip = reinterpret_cast<R4 *>(B.src_dip.p);
  R *M = reinterpret_cast<R *>(B.M.p);
  R *Lx = reinterpret_cast<R *>(B.L.p);
  R *m2l = reinterpret_cast<R *>(B.m2l_out.p);
  R *E = reinterpret_cast<R *>(B.E.p);

  prof_begin(T, ST_OTHER, s);
  if (src_charges) {
    if (T.Q > 0) {
      k_pack_charges<R><<<cdiv(T.Q, TB), TB, 0, s>>>(
          T.Q, T.qperm.p, reinterpret_cast<const R4 *>(f64 ? (void *)T.q64pos.p : (void *)T.q32pos.p), rq.wmono, spos);
      LAUNCH_OK();
    }
  } else {
    k_pack_panels<R><<<cdiv(T.N, TB), TB, 0, s>>>(
        T.N, T.pperm.p, reinterpret_cast<const R4 *>(f64 ? (void *)T.p64pos.p : (void *)T.p32pos.p),
        reinterpret_cast<const R4 *>(f64 ? (void *)T.p64nrm.p : (void *)T.p32nrm.p), T.area.p, rq.wmono,
        rq.mono_area ? 1 : 0, rq.wdip, spos, sdip);
    LAUNCH_OK();
  }
  prof_end(T, ST_OTHER, s);
  P2PArgs a{};
  a.p = p;
  a.ps = ps;
  const bool tgt_ch = rq.tgt == TGT_CHARGE;
  a.chunks = tgt_ch ? T.chunk_q.p : T.chunk_p.p;
  const int64_t nchunks = tgt_ch ? T.nchunk_q : T.nchunk_p;
  a.leaf_range = T.crange.p + T.coff[L];
  a.leaf_xyz = T.cxyz.p + T.coff[L];
  a.near_ptr = T.near_ptr.p + T.near_ptr_off[L];
  a.near_idx = T.near_idx.p + T.near_off[L];
  a.tgt_pos = tgt_ch ? (f64 ? (const void *)T.q64pos.p : (const void *)T.q32pos.p)
                     : (f64 ? (const void *)T.p64pos.p : (const void *)T.p32pos.p);
  a.tgt_nrm = f64 ? (const void *)T.p64nrm.p : (const void *)T.p32nrm.p;
  a.src_pos = spos;
  a.src_dip = sdip;
  a.E = E;
  a.tperm = tgt_ch ? T.qperm.p : T.pperm.p;
  a.sL = sL;
  a.xin = rq.xin;
  a.alpha = rq.alpha;
  a.beta = rq.beta / (4.0 * PI);
  a.area_scale = rq.area_scale ? 1 : 0;
  a.accumulate = rq.accumulate ? 1 : 0;
  a.y = rq.y;
  // near and far parts are written only while the caller records them
  if (T.debug_record) {
    const int64_t npts = std::max<int64_t>(std::max(T.N, T.Q), 1);
    B.dbg_near.reserve(npts);
    B.dbg_far.reserve(npts);
  }
  a.dbg_near = T.debug_record ? B.dbg_near.p : nullptr;
  a.dbg_far = T.debug_record ? B.dbg_far.p : nullptr;
  B.dbg_valid = T.debug_record;
  a.near_out = rq.far_only ? nullptr : B.near_out.p;
  B.last_tgt = rq.tgt;
  // The near field runs on the second stream, forked from the caller's
  // stream at a point of the upward pass and joined before L2P.  It forks
  // after P2M, except for an M2L large enough to keep persistent workgroups
  // busy for a while (at least 32 tiles of 256 pairs per CU; 8 for the
  // split-bf16 M2L, whose waves leave room for near-field waves): that M2L
  // runs persistent (in FP64 too) and the fork comes after M2M, so that the
  // M2L workgroups are resident before near-field waves fill the chip, and
  // the near field takes the rest.  Smaller M2L runs one tile per workgroup
  // in FP64.
  const hipStream_t ss = T.concurrent ? T.side_stream : s;
  const int combo = src_charges ? 1 : (rq.tgt == TGT_CHARGE ? 2 : 0);
  const Tree::M2LList &ML = T.m2l[combo];
  const bool far = (L >= 2) && T.nfar > 0;
  const bool big_m2l = T.m2l_persistent && ML.ntiles >= 32 * (int64_t)T.n_cu;
  // The split-bf16 M2L runs the panel-to-panel products (A, A^T), where it
  // agrees with the FP32 MFMA kernel to about 1e-9.  Products from or to
  // charges keep the FP32 MFMA kernel: their FP32 sums are more sensitive
  // (an energy sums them over the charges), and they are a small part of a
  // solve.  It leaves registers for near-field waves beside it, so it gains
  // from going first from 8 tiles per CU on (the others from 32).
  const bool split_m2l =
      !f64 && combo == 0 && T.m2l_persistent && T.m2l_split && T.p == P_FIXED && T.t_m2lbf;
  const bool m2l_first = split_m2l ? ML.ntiles >= 8 * (int64_t)T.n_cu : big_m2l;
  // M2L result rows without the padding places (read so by the downward pass)
  const bool compact_rows = split_m2l;
  const int fork_at = !far ? FORK_START : T.fork_at >= 0 ? T.fork_at : (m2l_first ? FORK_AFTER_M2M : FORK_AFTER_P2M);
  auto fork_near = [&]() {
    if (rq.far_only) return;
    HIP_OK(hipEventRecord(T.ev_fork, s));
    if (nchunks > 0) {
      HIP_OK(hipStreamWaitEvent(ss, T.ev_fork, 0));
      const P2PArgs &ap = a;
      const unsigned nb = (unsigned)nchunks;
      prof_begin(T, ST_P2P, ss);
#define P2P_CALL(S, Tg, O) k_p2p_near<R, S, Tg, O><<<nb, 64, 0, ss>>>(ap)
      if (!tgt_ch) {
        if (rq.src == SRC_PANEL_MONO && rq.out == OUT_NGRAD) P2P_CALL(SRC_PANEL_MONO, TGT_PANEL, OUT_NGRAD);
        else if (rq.src == SRC_PANEL_DIP && rq.out == OUT_POT) P2P_CALL(SRC_PANEL_DIP, TGT_PANEL, OUT_POT);
        else if (rq.src == SRC_CHARGE_MONO && rq.out == OUT_NGRAD) P2P_CALL(SRC_CHARGE_MONO, TGT_PANEL, OUT_NGRAD);
        else if (rq.src == SRC_CHARGE_MONO && rq.out == OUT_POT) P2P_CALL(SRC_CHARGE_MONO, TGT_PANEL, OUT_POT);
        else BF_THROW(BEMFMM_EINVAL, "unsupported FMM request (panel targets)");
      } else {
        if (rq.src == SRC_PANEL_MONO && rq.out == OUT_POT) P2P_CALL(SRC_PANEL_MONO, TGT_CHARGE, OUT_POT);
        else if (rq.src == SRC_PANEL_DIP && rq.out == OUT_POT) P2P_CALL(SRC_PANEL_DIP, TGT_CHARGE, OUT_POT);
        else if (rq.src == SRC_PANEL_MONODIP && rq.out == OUT_POTGRAD) P2P_CALL(SRC_PANEL_MONODIP, TGT_CHARGE, OUT_POTGRAD);
        else if (rq.src == SRC_PANEL_MONODIP && rq.out == OUT_POT) P2P_CALL(SRC_PANEL_MONODIP, TGT_CHARGE, OUT_POT);
        else BF_THROW(BEMFMM_EINVAL, "unsupported FMM request (charge targets)");
      }
#undef P2P_CALL
      LAUNCH_OK();
      if (T.n_nq > 0 && (rq.op == BEMFMM_OP_A || rq.op == BEMFMM_OP_AT)) {
        const bool tr = rq.op == BEMFMM_OP_AT;
        k_nq_apply<R><<<cdiv(T.N, 256), 256, 0, ss>>>(
            T.N, tr ? T.nqT_ptr.p : T.nq_ptr.p, tr ? T.nqT_idx.p : T.nq_idx.p, tr ? T.nqT_coef.p : T.nq_coef.p,
            tr ? rq.wdip : rq.wmono, tr ? reinterpret_cast<const R4 *>(a.tgt_pos) : nullptr, B.near_out.p);
        LAUNCH_OK();
      }
      prof_end(T, ST_P2P, ss);
      HIP_OK(hipEventRecord(T.ev_join, ss));
    }
  };
  if (fork_at == FORK_START) fork_near();

  if (far) {
    prof_begin(T, ST_P2M, s);
    launch_p2m<R>(T, B, rq.src, s);
    prof_end(T, ST_P2M, s);
    if (fork_at == FORK_AFTER_P2M) fork_near();
    // M2M, parents of levels L-1 .. 2: a batched MFMA product per child level
    // (one row per child), then each parent adds its children's rows
    prof_begin(T, ST_M2M, s);
    const void *Sm = f64 ? (const void *)T.t_m2m64 : (const void *)T.t_m2m32;
    R *rows = reinterpret_cast<R *>(B.l2l_out.p);
    for (int l = L; l >= 3; --l) {
      level_product<R, 2>(T, l, T.l2lw.self.p, Sm, M, rows, s);
      const int64_t CP = T.ncell[l - 1];
      k_m2m_sum<R><<<cdiv(CP * ps, TB), TB, 0, s>>>(ps, T.coff[l - 1], CP, T.coff[l], T.cchild.p, rows, M);
      LAUNCH_OK();
    }
    prof_end(T, ST_M2M, s);
    if (fork_at == FORK_AFTER_M2M) fork_near();
  }
  if (far) {
    // M2L, every level in one launch
    prof_begin(T, ST_M2L, s);
    const int NT = ps / 16;
    if (ML.n > 0) {
#define M2L_CASE(nt)                                                                                           \
  case nt:                                                                                                     \
    if (f64 && big_m2l)                                                                                        \
      k_m2l_pers64<nt><<<dim3((unsigned)std::min<int64_t>(ML.ntiles, T.n_cu)), 512, 0, s>>>(                    \
          ML.tile_group.p, ML.tile_row.p, ML.group_off.p, ML.group_end.p, ML.src.p, ML.dest.p, T.t_m2l64,      \
          reinterpret_cast<const double *>(M), reinterpret_cast<double *>(m2l), (int)ML.ntiles);               \
    else if (f64)                                                                                              \
      k_m2l<double, nt, M2L_RT64, false, 0><<<dim3((unsigned)ML.ntiles64), 256, 0, s>>>(                         \
          ML.tile_group64.p, ML.tile_row64.p, ML.group_off.p, ML.group_end.p, ML.src.p, ML.dest.p, T.t_m2l64,             \
          reinterpret_cast<const double *>(M), reinterpret_cast<double *>(m2l));                               \
    else if (T.m2l_persistent)                                                                                  \
      k_m2l_pers<nt, M2L_PERS_RT><<<dim3((unsigned)std::min<int64_t>(ML.ntiles * (M2L_ROWS32 / (64 * M2L_PERS_RT)), \
                                                                   2 * T.n_cu)), 256, 0, s>>>(                 \
          ML.tile_group.p, ML.tile_row.p, ML.group_off.p, ML.group_end.p, ML.src.p, ML.dest.p, T.t_m2l32,      \
          reinterpret_cast<const float *>(M), reinterpret_cast<float *>(m2l), (int)ML.ntiles);                 \
    else                                                                                                       \
      k_m2l<float, nt, M2L_RT32, true, 0><<<dim3((unsigned)ML.ntiles), 256, 0, s>>>(                              \
          ML.tile_group.p, ML.tile_row.p, ML.group_off.p, ML.group_end.p, ML.src.p, ML.dest.p, T.t_m2l32,                 \
          reinterpret_cast<const float *>(M), reinterpret_cast<float *>(m2l));                                 \
    break;
      if (split_m2l) {
        k_m2l_bf<NT_FIXED, RB_FIXED>
            <<<dim3((unsigned)std::min<int64_t>(ML.ntiles * (M2L_ROWS32 / (8 * 16)), T.n_cu)), 512, M2L_BF_LDS, s>>>(
                ML.tile_group.p, ML.tile_row.p, ML.group_off.p, ML.group_end.p, ML.src.p, ML.dest.p,
                reinterpret_cast<const bf16x8 *>(T.t_m2lbf), reinterpret_cast<const float *>(M),
                reinterpret_cast<float *>(m2l), (int)ML.ntiles);
      } else switch (NT) {
        M2L_CASE(1)
        M2L_CASE(2)
        M2L_CASE(3)
        M2L_CASE(4)
        M2L_CASE(5)
        M2L_CASE(6)
        M2L_CASE(7)
        M2L_CASE(8)
        default:
          BF_THROW(BEMFMM_EINVAL, "unsupported expansion order");
      }
#undef M2L_CASE
      LAUNCH_OK();
    }
    prof_end(T, ST_M2L, s);
    if (fork_at == FORK_AFTER_M2L) fork_near();
    // downward pass, levels 2 .. L
    prof_begin(T, ST_L2L, s);
    const Tree::L2LList &LW = T.l2lw;
    R *l2l = reinterpret_cast<R *>(B.l2l_out.p);
    for (int l = 2; l <= L; ++l) {
      const bool leaf = (l == L);
      if (l > 2) {
        // L2L of every cell of level l from its parent's final expansion
        level_product<R, 1>(T, l, LW.src.p, f64 ? (const void *)T.t_l2l64 : (const void *)T.t_l2l32, Lx, l2l, s);
      }
      // levels with few cells (long interaction lists, too few waves to hide
      // the load latency) take four waves per cell
      const int nthr = T.ncell[l] < 4 * T.n_cu * 8 ? 256 : 64;
      const size_t shm2 = (size_t)(ps + nthr * VecT<R>::W) * sizeof(R);
      k_downward<R><<<T.ncell[l], nthr, shm2, s>>>(p, ps, compact_rows ? p * p : ps, compact_rows ? 1 : 0, T.coff[l],
                                                   T.ncell[l], l > 2 ? 1 : 0, l2l, ML.kptr.p,
                                                   m2l, Lx, leaf ? 1 : 0, R(1.0 / sL), E);
      LAUNCH_OK();
    }
    prof_end(T, ST_L2L, s);
  } else {
    B.E.zero(s);
  }

  // far field + near field -> output, after the join
  if (nchunks > 0) {
    if (!rq.far_only) HIP_OK(hipStreamWaitEvent(s, T.ev_join, 0));
    prof_begin(T, ST_L2P, s);
#define L2P_CALL(Tg, O)                                                 \
  do {                                                                  \
    if (p == P_FIXED)                                                   \
      k_l2p_combine<R, Tg, O, P_FIXED><<<nchunks, 64, 0, s>>>(a);       \
    else                                                                \
      k_l2p_combine<R, Tg, O, 0><<<nchunks, 64, 0, s>>>(a);             \
  } while (0)
    if (!tgt_ch) {
      if (rq.out == OUT_NGRAD) L2P_CALL(TGT_PANEL, OUT_NGRAD);
      else if (rq.out == OUT_POTGRAD) L2P_CALL(TGT_PANEL, OUT_POTGRAD);
      else L2P_CALL(TGT_PANEL, OUT_POT);
    } else {
      if (rq.out == OUT_POTGRAD) L2P_CALL(TGT_CHARGE, OUT_POTGRAD);
      else L2P_CALL(TGT_CHARGE, OUT_POT);
    }
#undef L2P_CALL
    LAUNCH_OK();
    prof_end(T, ST_L2P, s);
  }
  B.have = true;
  prof_collect(T);
}

void fmm_apply(Tree &T, int precision, const FmmRequest &rq, hipStream_t s) {
  const int prec = (precision == BEMFMM_FP64) ? BEMFMM_FP64 : BEMFMM_FP32;
  if (rq.tgt == TGT_CHARGE && T.Q == 0) return;
  PrecBufs &B = bufs(T, prec, s);
  if (!T.ev_init) {
    for (auto &e : T.ev) HIP_OK(hipEventCreate(&e));
    HIP_OK(hipEventCreateWithFlags(&T.ev_fork, hipEventDisableTiming));
    HIP_OK(hipEventCreateWithFlags(&T.ev_join, hipEventDisableTiming));
    HIP_OK(hipStreamCreateWithFlags(&T.side_stream, hipStreamNonBlocking));  // default priority
    T.ev_init = true;
    if (const char *e = getenv("BEMFMM_CONCURRENT_P2P")) T.concurrent = atoi(e) != 0;
    if (const char *e = getenv("BEMFMM_M2L_PERSISTENT")) T.m2l_persistent = atoi(e) != 0;
    if (const char *e = getenv("BEMFMM_M2L_SPLIT")) T.m2l_split = atoi(e) != 0;
    // the split-bf16 M2L takes more dynamic LDS than the default limit
    HIP_OK(hipFuncSetAttribute((const void *)k_m2l_bf<NT_FIXED, RB_FIXED>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               M2L_BF_LDS));
    if (const char *e = getenv("BEMFMM_FORK_AT")) T.fork_at = std::min(std::max(atoi(e), -1), (int)FORK_AFTER_M2L);
    int dev = 0;
    HIP_OK(hipGetDevice(&dev));
    HIP_OK(hipDeviceGetAttribute(&T.n_cu, hipDeviceAttributeMultiprocessorCount, dev));
  }
  T.prof_kind = (rq.op >= 0 && rq.op < 6) ? rq.op : 6;
  T.prof_prec = prec == BEMFMM_FP64 ? 0 : 1;
  T.prof_now = T.prof && (T.prof_op < 0 || T.prof_op == rq.op) && (T.prof_sel_prec < 0 || T.prof_sel_prec == T.prof_prec);
  if (prec == BEMFMM_FP64)
    run_fmm<double>(T, B, rq, s);
  else
    run_fmm<float>(T, B, rq, s);
}

void level_product64(Tree &T, int l, const int32_t *src, const double *table, const double *in, double *out,
                     bool m2m, hipStream_t s) {
  if (m2m)
    level_product<double, 2>(T, l, src, table, in, out, s);
  else
    level_product<double, 1>(T, l, src, table, in, out, s);
}

void m2m_sum64(Tree &T, int l, const double *rows, double *M, hipStream_t s) {
  const int64_t CP = T.ncell[l - 1];
  k_m2m_sum<double><<<cdiv(CP * T.ps, 256), 256, 0, s>>>(T.ps, T.coff[l - 1], CP, T.coff[l], T.cchild.p, rows, M);
  LAUNCH_OK();
}

void m2l_tiles64(const Tree::M2LList &ML, int ps, const double *table, const double *M, double *out, hipStream_t s) {
  if (ML.ntiles64 <= 0) return;
  const dim3 grid((unsigned)ML.ntiles64);
#define M2L64_CASE(nt)                                                                                      \
  case nt:                                                                                                  \
    k_m2l<double, nt, M2L_RT64, false, 0><<<grid, 256, 0, s>>>(ML.tile_group64.p, ML.tile_row64.p,         \
                                                                ML.group_off.p, ML.group_end.p, ML.src.p,  \
                                                                ML.dest.p, table, M, out);                 \
    break;
  switch (ps / 16) {
    M2L64_CASE(1)
    M2L64_CASE(2)
    M2L64_CASE(3)
    M2L64_CASE(4)
    M2L64_CASE(5)
    M2L64_CASE(6)
    M2L64_CASE(7)
    M2L64_CASE(8)
    default:
      BF_THROW(BEMFMM_EINVAL, "unsupported expansion order");
  }
#undef M2L64_CASE
  LAUNCH_OK();
}

void downward64(Tree &T, int l, const double *l2l_rows, const int32_t *kptr, const double *m2l_rows, double *Lx,
                hipStream_t s) {
  const int ps = T.ps;
  const int nthr = T.ncell[l] < 4 * T.n_cu * 8 ? 256 : 64;
  const size_t shm = (size_t)(ps + nthr * VecT<double>::W) * sizeof(double);
  k_downward<double><<<T.ncell[l], nthr, shm, s>>>(T.p, ps, ps, 0, T.coff[l], T.ncell[l], l > 2 ? 1 : 0, l2l_rows, kptr,
                                                   m2l_rows, Lx, 0, 1.0, nullptr);
  LAUNCH_OK();
}

void fmm_free(Tree &T) {
  delete T.pb32;
  delete T.pb64;
  T.pb32 = T.pb64 = nullptr;
}

void debug_expansions(Tree &T, int precision, int which, double *out_host, hipStream_t s) {
  PrecBufs *B = (precision == BEMFMM_FP64) ? T.pb64 : T.pb32;
  if (!B || !B->have) BF_THROW(BEMFMM_ESTATE, "no matvec has run at this precision");
  const size_t n = (size_t)T.ncell_tot * T.ps;
  const int np2 = T.p * T.p;
  std::vector<double> full(n);
  const DBuf<char> &src = which ? B->L : B->M;
  if (B->prec == BEMFMM_FP64) {
    HIP_OK(hipMemcpyAsync(full.data(), src.p, n * 8, hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
  } else {
    std::vector<float> f(n);
    HIP_OK(hipMemcpyAsync(f.data(), src.p, n * 4, hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    for (size_t i = 0; i < n; ++i) full[i] = f[i];
  }
  for (int64_t c = 0; c < T.ncell_tot; ++c)
    for (int k = 0; k < np2; ++k) out_host[(size_t)c * np2 + k] = full[(size_t)c * T.ps + coef_pos(k, T.p, T.ps)];
}

void debug_fields(Tree &T, int precision, double *near_host, double *far_host, hipStream_t s) {
  PrecBufs *B = (precision == BEMFMM_FP64) ? T.pb64 : T.pb32;
  if (!B || !B->have) BF_THROW(BEMFMM_ESTATE, "no matvec has run at this precision");
  if (!B->dbg_valid) BF_THROW(BEMFMM_ESTATE, "the last product at this precision ran without bemfmm_debug_record");
  const int64_t nt = (B->last_tgt == TGT_CHARGE) ? T.Q : T.N;
  std::vector<double> ns(nt), fs(nt);
  std::vector<int32_t> perm(nt);
  HIP_OK(hipMemcpyAsync(ns.data(), B->dbg_near.p, nt * 8, hipMemcpyDeviceToHost, s));
  HIP_OK(hipMemcpyAsync(fs.data(), B->dbg_far.p, nt * 8, hipMemcpyDeviceToHost, s));
  HIP_OK(hipMemcpyAsync(perm.data(), (B->last_tgt == TGT_CHARGE) ? T.qperm.p : T.pperm.p, nt * 4,
                        hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  const double k4 = 1.0 / (4.0 * PI);
  for (int64_t i = 0; i < nt; ++i) {
    if (near_host) near_host[perm[i]] = ns[i] * k4;
    if (far_host) far_host[perm[i]] = fs[i] * k4;
  }
}

}  // namespace bemfmm
