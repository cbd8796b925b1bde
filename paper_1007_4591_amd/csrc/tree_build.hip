// Octree construction on the GPU (Section 2.3 hierarchy, Section 3.1 Morton
// ordering; the paper built these on the host, here every pass is a HIP
// kernel over HBM-resident arrays and the host only reads counts).
//
// Passes: panel geometry -> bounding cube (exact min/max) -> 30-bit Morton
// keys -> stable LSD radix sort (8-bit digits, one wave per 1024-key tile,
// ballot-based stable ranking) -> leaf level from per-level distinct-cell
// counts -> cells of every level (union of panel and charge prefixes) ->
// near/far lists top down (children of the parent's near cells, MAC test) ->
// M2L pairs sorted by translation offset.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>

#include "common.h"

// Device memory of the allocation-free bemfmm_set_charges_noalloc: one error
// word, then the staged leaf-relative FP32 and FP64 charge positions.  Every
// device the library runs on holds its own copy until the process ends; host
// code reaches it only through the address hipGetSymbolAddress returns for
// the current device (the array's name is not a device address on the host).
static __device__ __align__(256) unsigned char scratch[BEMFMM_NOALLOC_SCRATCH_BYTES];

namespace bemfmm {

namespace {

constexpr int SCAN_BLOCK = 256;
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = SCAN_BLOCK * SCAN_ITEMS;

// ------------------------------------------------------------------ scan

__device__ inline int32_t block_exclusive_scan(int32_t v, int32_t *total) {
  __shared__ int32_t wsum[SCAN_BLOCK / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  int32_t x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    int32_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) wsum[wid] = x;
  __syncthreads();
  int32_t base = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < SCAN_BLOCK / 64; ++w) {
    if (w < wid) base += wsum[w];
    tot += wsum[w];
  }
  __syncthreads();
  *total = tot;
  return base + x - v;
}

__global__ void __launch_bounds__(SCAN_BLOCK) k_scan_reduce(const int32_t *__restrict__ in, int64_t n,
                                                            int32_t *__restrict__ sums) {
  int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
  int32_t s = 0;
#pragma unroll
  for (int k = 0; k < SCAN_ITEMS; ++k)
    if (base + k < n) s += in[base + k];
  int32_t tot;
  (void)block_exclusive_scan(s, &tot);
  if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// `in` and `out` may alias (each thread reads its items before writing them);
// the last block also writes the scan's total to `total` when non-NULL
__global__ void __launch_bounds__(SCAN_BLOCK) k_scan_apply(const int32_t *in, int64_t n, const int32_t *offs,
                                                           int32_t *out, int32_t *total) {
  int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
  int32_t v[SCAN_ITEMS];
  int32_t s = 0;
#pragma unroll
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    v[k] = (base + k < n) ? in[base + k] : 0;
    s += v[k];
  }
  int32_t tot;
  const int32_t off = offs ? offs[blockIdx.x] : 0;
  int32_t run = block_exclusive_scan(s, &tot) + off;
#pragma unroll
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    if (base + k < n) out[base + k] = run;
    run += v[k];
  }
  if (total && threadIdx.x == 0 && blockIdx.x == gridDim.x - 1) *total = off + tot;
}

}  // namespace

// Exclusive prefix sum of n int32 values (out may alias in); the total is
// returned through total_host when non-NULL (one stream synchronisation).
// One launch when n fits one block; otherwise block sums, their scan (one
// launch up to 2048 blocks) and the apply pass.  Without a total nothing
// waits: temporary buffers go back to the caching allocator, which
// synchronises before it reuses them.
void exclusive_scan_i32(const int32_t *in, int32_t *out, int64_t n, hipStream_t s, int32_t *total_host) {
  if (n <= 0) {
    if (total_host) *total_host = 0;
    return;
  }
  const int nb = cdiv(n, SCAN_TILE);
  DBuf<int32_t> sums, sums_scan;
  if (nb > 1 || total_host) sums.alloc(nb + 1);  // block sums, then the total
  int32_t *tot_dev = total_host ? sums.p + nb : nullptr;
  if (nb > 1) {
    k_scan_reduce<<<nb, SCAN_BLOCK, 0, s>>>(in, n, sums.p);
    LAUNCH_OK();
    sums_scan.alloc(nb);
    exclusive_scan_i32(sums.p, sums_scan.p, nb, s, nullptr);
  }
  k_scan_apply<<<nb, SCAN_BLOCK, 0, s>>>(in, n, nb > 1 ? sums_scan.p : nullptr, out, tot_dev);
  LAUNCH_OK();
  if (total_host) {
    HIP_OK(hipMemcpyAsync(total_host, tot_dev, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
  }
}

namespace {

// ------------------------------------------------------------ radix sort

constexpr int RADIX_ITEMS = 16;
constexpr int RADIX_TILE = 64 * RADIX_ITEMS;

__global__ void __launch_bounds__(64) k_radix_hist(const uint32_t *__restrict__ keys, int64_t n, int shift,
                                                   int32_t *__restrict__ hist, int ntiles) {
  __shared__ int32_t cnt[256];
  for (int d = threadIdx.x; d < 256; d += 64) cnt[d] = 0;
  __syncthreads();
  int64_t base = (int64_t)blockIdx.x * RADIX_TILE;
  for (int it = 0; it < RADIX_ITEMS; ++it) {
    int64_t i = base + it * 64 + threadIdx.x;
    if (i < n) atomicAdd(&cnt[(keys[i] >> shift) & 255u], 1);
  }
  __syncthreads();
  for (int d = threadIdx.x; d < 256; d += 64) hist[(int64_t)d * ntiles + blockIdx.x] = cnt[d];
}

__global__ void __launch_bounds__(64) k_radix_scatter(const uint32_t *__restrict__ kin,
                                                      const int32_t *__restrict__ vin, uint32_t *__restrict__ kout,
                                                      int32_t *__restrict__ vout, int64_t n, int shift,
                                                      const int32_t *__restrict__ offs, int ntiles) {
  __shared__ int32_t base_d[256];
  for (int d = threadIdx.x; d < 256; d += 64) base_d[d] = offs[(int64_t)d * ntiles + blockIdx.x];
  __syncthreads();
  const int lane = threadIdx.x;
  const uint64_t lt = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
  int64_t base = (int64_t)blockIdx.x * RADIX_TILE;
  for (int it = 0; it < RADIX_ITEMS; ++it) {
    int64_t i = base + it * 64 + lane;
    bool valid = i < n;
    uint32_t k = valid ? kin[i] : 0u;
    int32_t v = valid ? vin[i] : 0;
    uint32_t d = (k >> shift) & 255u;
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      bool bit = (d >> b) & 1u;
      uint64_t bb = __ballot(valid && bit);
      peers &= bit ? bb : ~bb;
    }
    int rank = __popcll(peers & lt);
    int pos = valid ? base_d[d] + rank : 0;
    __syncthreads();
    if (valid && rank == 0) base_d[d] += __popcll(peers);
    __syncthreads();
    if (valid) {
      kout[pos] = k;
      vout[pos] = v;
    }
  }
}

}  // namespace

// Stable LSD radix sort of (key, value) pairs on the low `bits` key bits.
void radix_sort_u32(uint32_t *keys, int32_t *vals, int64_t n, int bits, hipStream_t s) {
  if (n <= 1 || bits <= 0) return;
  int ntiles = cdiv(n, RADIX_TILE);
  DBuf<uint32_t> k2;
  DBuf<int32_t> v2, hist;
  k2.alloc(n);
  v2.alloc(n);
  hist.alloc((size_t)256 * ntiles);
  uint32_t *ka = keys, *kb = k2.p;
  int32_t *va = vals, *vb = v2.p;
  int passes = (bits + 7) / 8;
  for (int ps = 0; ps < passes; ++ps) {
    int shift = 8 * ps;
    k_radix_hist<<<ntiles, 64, 0, s>>>(ka, n, shift, hist.p, ntiles);
    LAUNCH_OK();
    exclusive_scan_i32(hist.p, hist.p, (int64_t)256 * ntiles, s, nullptr);
    k_radix_scatter<<<ntiles, 64, 0, s>>>(ka, va, kb, vb, n, shift, hist.p, ntiles);
    LAUNCH_OK();
    std::swap(ka, kb);
    std::swap(va, vb);
  }
  if (ka != keys) {
    HIP_OK(hipMemcpyAsync(keys, ka, n * sizeof(uint32_t), hipMemcpyDeviceToDevice, s));
    HIP_OK(hipMemcpyAsync(vals, va, n * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
  }
}

namespace {

// -------------------------------------------------------------- geometry

// Centroid, outward normal and area of each triangle (flat panels with one
// centroid quadrature point, Section 2.1).  Built without FP contraction so
// the FP64 values are reproducible bit for bit.
#pragma clang fp contract(off)
__global__ void k_geometry(const double *__restrict__ V, int64_t nv, const int32_t *__restrict__ tri, int64_t nt,
                           double *__restrict__ c, double *__restrict__ nrm, double *__restrict__ a,
                           int *__restrict__ err) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nt) return;
  int32_t i0 = tri[3 * i], i1 = tri[3 * i + 1], i2 = tri[3 * i + 2];
  if (i0 < 0 || i1 < 0 || i2 < 0 || i0 >= nv || i1 >= nv || i2 >= nv) {
    atomicOr(err, 1);
    c[3 * i] = c[3 * i + 1] = c[3 * i + 2] = 0.0;
    nrm[3 * i] = nrm[3 * i + 1] = nrm[3 * i + 2] = 0.0;
    a[i] = 0.0;
    return;
  }
  const double *v0 = V + 3 * (int64_t)i0, *v1 = V + 3 * (int64_t)i1, *v2 = V + 3 * (int64_t)i2;
  double e1[3], e2[3];
  for (int d = 0; d < 3; ++d) {
    c[3 * i + d] = (v0[d] + v1[d] + v2[d]) / 3.0;
    e1[d] = v1[d] - v0[d];
    e2[d] = v2[d] - v0[d];
  }
  double m0 = e1[1] * e2[2] - e1[2] * e2[1];
  double m1 = e1[2] * e2[0] - e1[0] * e2[2];
  double m2 = e1[0] * e2[1] - e1[1] * e2[0];
  double len = sqrt(m0 * m0 + m1 * m1 + m2 * m2);
  if (!(len > 0.0) || !isfinite(len) || !isfinite(c[3 * i] + c[3 * i + 1] + c[3 * i + 2])) {
    atomicOr(err, 2);
    a[i] = 0.0;
    nrm[3 * i] = nrm[3 * i + 1] = nrm[3 * i + 2] = 0.0;
    return;
  }
  a[i] = 0.5 * len;
  nrm[3 * i] = m0 / len;
  nrm[3 * i + 1] = m1 / len;
  nrm[3 * i + 2] = m2 / len;
}

// the three vertices of each panel, caller order (9 doubles per panel)
__global__ void k_panel_verts(const double *__restrict__ verts, const int32_t *__restrict__ tris, int64_t nt,
                              double *__restrict__ pv) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nt) return;
  for (int k = 0; k < 3; ++k) {
    const int64_t v = tris[3 * i + k];
    for (int d = 0; d < 3; ++d) pv[9 * i + 3 * k + d] = verts[3 * v + d];
  }
}

__global__ void k_check_points(const double *__restrict__ x, int64_t n, int *__restrict__ err) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (!isfinite(x[3 * i] + x[3 * i + 1] + x[3 * i + 2])) atomicOr(err, 4);
}

// exact per-block min/max of two point sets -> part[block][6]
__global__ void __launch_bounds__(256) k_minmax(const double *__restrict__ a, int64_t na,
                                                const double *__restrict__ b, int64_t nb,
                                                double *__restrict__ part) {
  __shared__ double sh[6][256];
  double mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
  int64_t ntot = na + nb;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < ntot; i += (int64_t)gridDim.x * blockDim.x) {
    const double *p = (i < na) ? a + 3 * i : b + 3 * (i - na);
    for (int d = 0; d < 3; ++d) {
      mn[d] = fmin(mn[d], p[d]);
      mx[d] = fmax(mx[d], p[d]);
    }
  }
  for (int d = 0; d < 3; ++d) {
    sh[d][threadIdx.x] = mn[d];
    sh[3 + d][threadIdx.x] = mx[d];
  }
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int d = 0; d < 3; ++d) {
        sh[d][threadIdx.x] = fmin(sh[d][threadIdx.x], sh[d][threadIdx.x + w]);
        sh[3 + d][threadIdx.x] = fmax(sh[3 + d][threadIdx.x], sh[3 + d][threadIdx.x + w]);
      }
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int d = 0; d < 6; ++d) part[blockIdx.x * 6 + d] = sh[d][0];
}

__device__ inline uint32_t spread3(uint32_t v) {  // 10 bits -> every third bit
  v &= 0x3ffu;
  v = (v | (v << 16)) & 0x030000FFu;
  v = (v | (v << 8)) & 0x0300F00Fu;
  v = (v | (v << 4)) & 0x030C30C3u;
  v = (v | (v << 2)) & 0x09249249u;
  return v;
}

__device__ inline uint32_t compact3(uint32_t v) {
  v &= 0x09249249u;
  v = (v | (v >> 2)) & 0x030C30C3u;
  v = (v | (v >> 4)) & 0x0300F00Fu;
  v = (v | (v >> 8)) & 0x030000FFu;
  v = (v | (v >> 16)) & 0x000003FFu;
  return v;
}

__device__ inline uint32_t quant(double x, double lo, double inv) {
  double t = floor((x - lo) * inv);
  t = fmin(fmax(t, 0.0), 1023.0);
  return (uint32_t)t;
}

__global__ void k_morton(const double *__restrict__ x, int64_t n, double lox, double loy, double loz, double inv,
                         uint32_t *__restrict__ key, int32_t *__restrict__ idx) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint32_t kx = quant(x[3 * i], lox, inv), ky = quant(x[3 * i + 1], loy, inv), kz = quant(x[3 * i + 2], loz, inv);
  key[i] = (spread3(kx) << 2) | (spread3(ky) << 1) | spread3(kz);
  idx[i] = (int32_t)i;
}
#pragma clang fp contract(on)

// count of adjacent sorted keys whose first differing level is l (1..10)
__global__ void k_level_hist(const uint32_t *__restrict__ key, int64_t n, unsigned long long *__restrict__ hist) {
  __shared__ unsigned int h[LMAX + 1];
  if (threadIdx.x <= LMAX) h[threadIdx.x] = 0;
  __syncthreads();
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x + 1; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    uint32_t d = key[i] ^ key[i - 1];
    if (d) {
      int hb = 31 - __clz((int)d);
      int lmin = LMAX - hb / 3;
      atomicAdd(&h[lmin], 1u);
    }
  }
  __syncthreads();
  if (threadIdx.x <= LMAX && h[threadIdx.x]) atomicAdd(&hist[threadIdx.x], (unsigned long long)h[threadIdx.x]);
}

__global__ void k_flags_unique(const uint32_t *__restrict__ key, int64_t n, int shift, int32_t *__restrict__ flag) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  flag[i] = (i == 0 || (key[i] >> shift) != (key[i - 1] >> shift)) ? 1 : 0;
}

__global__ void k_compact_unique(const uint32_t *__restrict__ key, int64_t n, int shift,
                                 const int32_t *__restrict__ flag, const int32_t *__restrict__ pos,
                                 uint32_t *__restrict__ out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (flag[i]) out[pos[i]] = key[i] >> shift;
}

__device__ inline int64_t lower_bound_sh(const uint32_t *a, int64_t n, int shift, uint32_t v) {
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    int64_t mid = (lo + hi) >> 1;
    if ((a[mid] >> shift) < v) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// leaf cells: ranges by binary search in the sorted point keys
__global__ void k_leaf_cells(const uint32_t *__restrict__ U, int64_t C, const uint32_t *__restrict__ pk, int64_t N,
                             const uint32_t *__restrict__ qk, int64_t Q, int shift, int4 *__restrict__ range) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= C) return;
  uint32_t v = U[i];
  int4 r;
  r.x = (int)lower_bound_sh(pk, N, shift, v);
  r.y = (int)lower_bound_sh(pk, N, shift, v + 1);
  r.z = (int)lower_bound_sh(qk, Q, shift, v);
  r.w = (int)lower_bound_sh(qk, Q, shift, v + 1);
  range[i] = r;
}

// parents of level-l cells: flags where the parent prefix changes
__global__ void k_parent_flags(const uint32_t *__restrict__ U, int64_t C, int32_t *__restrict__ flag) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= C) return;
  flag[i] = (i == 0 || (U[i] >> 3) != (U[i - 1] >> 3)) ? 1 : 0;
}

// build level l-1 from level l (C cells): keys, child ranges, point ranges,
// and the parent index of each level-l cell (level-local)
__global__ void k_make_parents(const uint32_t *__restrict__ U, const int4 *__restrict__ range, int64_t C,
                               const int32_t *__restrict__ flag, const int32_t *__restrict__ pos, int32_t Cp,
                               uint32_t *__restrict__ Up, int2 *__restrict__ child, int4 *__restrict__ rangep,
                               int32_t *__restrict__ parent) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= C) return;
  int32_t pi = pos[i] + flag[i] - 1;
  parent[i] = pi;
  bool last = (i == C - 1) || flag[i + 1];
  if (flag[i]) {
    Up[pi] = U[i] >> 3;
    child[pi].x = (int)i;
    rangep[pi].x = range[i].x;
    rangep[pi].z = range[i].z;
  }
  if (last) {
    child[pi].y = (int)(i + 1);
    rangep[pi].y = range[i].y;
    rangep[pi].w = range[i].w;
  }
  (void)Cp;
}

// global cell arrays: packed integer coordinates from the prefix
__global__ void k_cell_xyz(const uint32_t *__restrict__ key, int64_t n, int32_t *__restrict__ xyz) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint32_t k = key[i];
  uint32_t x = compact3(k >> 2), y = compact3(k >> 1), z = compact3(k);
  xyz[i] = (int32_t)(x | (y << 10) | (z << 20));
}

__device__ inline void unpack_xyz(int32_t v, int &x, int &y, int &z) {
  x = v & 1023;
  y = (v >> 10) & 1023;
  z = (v >> 20) & 1023;
}

__device__ inline bool mac_far_dev(int ox, int oy, int oz, double theta2, int mac) {
  if (mac == BEMFMM_MAC_ADJACENT) return max(abs(ox), max(abs(oy), abs(oz))) > 1;
  double d2 = (double)(ox * ox + oy * oy + oz * oz);
  return 3.0 < theta2 * d2;
}

// Lists at level l (l >= 1): candidates are the children of the near cells
// of the target's parent; the MAC splits them into near and far.  Pass 1
// counts (fill == 0), pass 2 writes.
// Inclusive prefix sum over the 64 lanes of a wave.
__device__ __forceinline__ int wave_incl_scan(int v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int u = __shfl_up(v, d, 64);
    if (lane >= d) v += u;
  }
  return v;
}

// Near and far lists of the cells of level l (level-local index t), one wave
// per cell.  The candidates are the children of the parent's near cells, in
// increasing order (the parent's near list is increasing, and child ranges
// are increasing and disjoint).  Lane k takes the k-th parent-near entry of
// each run of 64 and classifies its children (at most 8); a prefix sum over
// the lanes gives each lane its place, so both lists keep candidate order.
// fill = 0 counts, fill = 1 writes at near_ptr / far_ptr.
__global__ void __launch_bounds__(64) k_lists(int32_t C, int64_t cl, int64_t cpl, const int32_t *__restrict__ parent_g,
                                              const int32_t *__restrict__ xyz, const int2 *__restrict__ child,
                                              const int32_t *__restrict__ pnear_ptr,
                                              const int32_t *__restrict__ pnear_idx, double theta2, int mac,
                                              int fill, int32_t *__restrict__ near_cnt, int32_t *__restrict__ far_cnt,
                                              const int32_t *__restrict__ near_ptr, int32_t *__restrict__ near_idx,
                                              const int32_t *__restrict__ far_ptr, int2 *__restrict__ far_ts) {
  const int32_t t = blockIdx.x;
  if (t >= C) return;
  const int lane = threadIdx.x;
  int tx, ty, tz;
  unpack_xyz(xyz[cl + t], tx, ty, tz);
  const int32_t P = parent_g[cl + t] - (int32_t)cpl;  // level-local parent
  int32_t nn = 0, nf = 0;                              // running totals (uniform)
  const int32_t nbase = fill ? near_ptr[t] : 0;
  const int32_t fbase = fill ? far_ptr[t] : 0;
  const int32_t e0 = pnear_ptr[P], e1 = pnear_ptr[P + 1];
  for (int32_t eb = e0; eb < e1; eb += 64) {
    const int32_t e = eb + lane;
    int my_n = 0, my_f = 0;
    unsigned farmask = 0;
    int2 ch = make_int2(0, 0);
    if (e < e1) {
      ch = child[cpl + pnear_idx[e]];  // global child range
      for (int32_t sg = ch.x; sg < ch.y; ++sg) {
        int sx, sy, sz;
        unpack_xyz(xyz[sg], sx, sy, sz);
        if (mac_far_dev(sx - tx, sy - ty, sz - tz, theta2, mac)) {
          farmask |= 1u << (sg - ch.x);
          ++my_f;
        } else {
          ++my_n;
        }
      }
    }
    const int in_n = wave_incl_scan(my_n), in_f = wave_incl_scan(my_f);
    if (fill && e < e1) {
      int32_t on = nbase + nn + in_n - my_n, of = fbase + nf + in_f - my_f;
      for (int32_t sg = ch.x; sg < ch.y; ++sg) {
        if (farmask & (1u << (sg - ch.x)))
          far_ts[of++] = make_int2((int)(cl + t), (int)sg);
        else
          near_idx[on++] = sg - (int32_t)cl;
      }
    }
    nn += __shfl(in_n, 63, 64);
    nf += __shfl(in_f, 63, 64);
  }
  if (!fill && lane == 0) {
    near_cnt[t] = nn;
    far_cnt[t] = nf;
  }
}

__global__ void k_offset_keys(const int2 *__restrict__ ts, int64_t n, const int32_t *__restrict__ xyz,
                              const int32_t *__restrict__ offset_id, int R, uint32_t *__restrict__ key,
                              int32_t *__restrict__ idx, int *__restrict__ err) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int tx, ty, tz, sx, sy, sz;
  unpack_xyz(xyz[ts[i].x], tx, ty, tz);
  unpack_xyz(xyz[ts[i].y], sx, sy, sz);
  int ox = sx - tx, oy = sy - ty, oz = sz - tz;
  int W = 2 * R + 1;
  int id = -1;
  if (abs(ox) <= R && abs(oy) <= R && abs(oz) <= R) id = offset_id[((ox + R) * W + (oy + R)) * W + (oz + R)];
  if (id < 0) {
    atomicOr(err, 8);
    id = 0;
  }
  key[i] = (uint32_t)id;
  idx[i] = (int32_t)i;
}

// *p = v (a small constant without a host copy)
__global__ void k_set_i32(int32_t *p, int32_t v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

__global__ void k_group_flags(const uint32_t *__restrict__ key, int64_t n, int32_t *__restrict__ flag) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  flag[i] = (i == 0 || key[i] != key[i - 1]) ? 1 : 0;
}

__global__ void k_group_make(const uint32_t *__restrict__ key, int64_t n, const int32_t *__restrict__ flag,
                             const int32_t *__restrict__ pos, int32_t *__restrict__ goff, int32_t *__restrict__ gbeg,
                             int32_t *__restrict__ gend) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int32_t g = pos[i] + flag[i] - 1;
  if (flag[i]) {
    goff[g] = (int32_t)key[i];
    gbeg[g] = (int32_t)i;
  }
  if (i == n - 1 || flag[i + 1]) gend[g] = (int32_t)(i + 1);
}

__global__ void k_group_tiles(const int32_t *__restrict__ gbeg, const int32_t *__restrict__ gend, int64_t G,
                              int rows, int32_t *__restrict__ ntile) {
  int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= G) return;
  ntile[g] = (gend[g] - gbeg[g] + rows - 1) / rows;
}

__global__ void k_tile_list(const int32_t *__restrict__ gbeg, const int32_t *__restrict__ gend, int64_t G,
                            int rows, const int32_t *__restrict__ tpos, int32_t *__restrict__ tile_group,
                            int32_t *__restrict__ tile_row) {
  int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= G) return;
  int32_t b = gbeg[g], e = gend[g];
  int32_t t0 = tpos[g];
  for (int32_t r = b, k = 0; r < e; r += rows, ++k) {
    tile_group[t0 + k] = (int32_t)g;
    tile_row[t0 + k] = r;
  }
}

// keep a sorted M2L pair if its source cell has sources and its target cell
// targets of the list's kinds (0 panels->panels, 1 charges->panels,
// 2 panels->charges)
// what each cell holds: bit 0 panels, bit 1 charges
__global__ void k_cell_kinds(const int4 *__restrict__ crange, int64_t n, uint8_t *__restrict__ kind) {
  int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  const int4 r = crange[c];
  kind[c] = (uint8_t)((r.y > r.x ? 1 : 0) | (r.w > r.z ? 2 : 0));
}

// a far pair is kept in list `combo` if its source cell has sources and its
// target cell targets of the list's kinds (0 panels -> panels, 1 charges ->
// panels, 2 panels -> charges)
__device__ inline bool combo_keep(uint8_t kt, uint8_t ks, int combo) {
  return combo == 0 ? ((ks & 1) && (kt & 1)) : (combo == 1 ? ((ks & 2) && (kt & 1)) : ((ks & 1) && (kt & 2)));
}

// the far pairs in offset order (one gather through the sort's permutation)
__global__ void k_gather_pairs(const int32_t *__restrict__ order, const int2 *__restrict__ ts, int64_t n,
                               int2 *__restrict__ ts_sorted) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) ts_sorted[i] = ts[order[i]];
}

// keep flags of one list, in the order of `ts` (offset order or pair order)
__global__ void k_combo_flags(const int2 *__restrict__ ts, const uint8_t *__restrict__ kind, int64_t n, int combo,
                              int32_t *__restrict__ flag) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int2 p = ts[i];
  flag[i] = combo_keep(kind[p.x], kind[p.y], combo) ? 1 : 0;
}

__global__ void k_combo_compact(const int32_t *__restrict__ order, const uint32_t *__restrict__ key,
                                const int32_t *__restrict__ flag, const int32_t *__restrict__ pos, int64_t n,
                                const int2 *__restrict__ ts_sorted, const int32_t *__restrict__ pos_t,
                                int32_t *__restrict__ src_k, uint32_t *__restrict__ key_k,
                                int32_t *__restrict__ dest_k) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (!flag[i]) return;
  src_k[pos[i]] = ts_sorted[i].y;
  key_k[pos[i]] = key[i];
  dest_k[pos[i]] = pos_t[order[i]];
}


// first kept row of every cell (CSR over all cells, rows in pair order)
__global__ void k_kept_ptr(const int32_t *__restrict__ far_ptr, const int32_t *__restrict__ pos_t, int64_t n1,
                           int32_t *__restrict__ kptr) {
  int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c < n1) kptr[c] = pos_t[far_ptr[c]];
}

__global__ void k_far_ptr(const int32_t *__restrict__ cnt_scan, int32_t C, int64_t cl, int64_t foff,
                          int32_t *__restrict__ far_ptr) {
  int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= C) return;
  far_ptr[cl + t] = (int32_t)(foff + cnt_scan[t]);
}

__global__ void k_fill_leaf(const int4 *__restrict__ range, int64_t C, int32_t *__restrict__ pleaf,
                            int32_t *__restrict__ qleaf) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= C) return;
  int4 r = range[t];
  for (int i = r.x; i < r.y; ++i) pleaf[i] = (int32_t)t;
  for (int i = r.z; i < r.w; ++i) qleaf[i] = (int32_t)t;
}

__global__ void k_inverse_perm(const int32_t *__restrict__ perm, int64_t n, int32_t *__restrict__ inv) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  inv[perm[i]] = (int32_t)i;
}

__device__ inline void cell_centre(int32_t xyz, double lox, double loy, double loz, double s, double &X,
                                   double &Y, double &Z) {
  int x, y, z;
  unpack_xyz(xyz, x, y, z);
  X = lox + (x + 0.5) * s;
  Y = loy + (y + 0.5) * s;
  Z = loz + (z + 0.5) * s;
}

// sorted panel data relative to the leaf centre
__global__ void k_gather_panels(const int32_t *__restrict__ perm, const int32_t *__restrict__ leaf, int64_t N,
                                const int32_t *__restrict__ xyzL, double lox, double loy, double loz, double sL,
                                const double *__restrict__ c, const double *__restrict__ nrm,
                                const double *__restrict__ a, float4 *__restrict__ p32, float4 *__restrict__ n32,
                                double4 *__restrict__ p64, double4 *__restrict__ n64) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  int64_t u = perm[i];
  double X, Y, Z;
  cell_centre(xyzL[leaf[i]], lox, loy, loz, sL, X, Y, Z);
  double rx = c[3 * u] - X, ry = c[3 * u + 1] - Y, rz = c[3 * u + 2] - Z;
  double nx = nrm[3 * u], ny = nrm[3 * u + 1], nz = nrm[3 * u + 2], ar = a[u];
  p64[i] = make_double4(rx, ry, rz, ar);
  n64[i] = make_double4(nx, ny, nz, 0.0);
  p32[i] = make_float4((float)rx, (float)ry, (float)rz, (float)ar);
  n32[i] = make_float4((float)nx, (float)ny, (float)nz, 0.0f);
}

__global__ void k_gather_charges(const int32_t *__restrict__ perm, const int32_t *__restrict__ leaf, int64_t Q,
                                 const int32_t *__restrict__ xyzL, double lox, double loy, double loz, double sL,
                                 const double *__restrict__ x, float4 *__restrict__ q32, double4 *__restrict__ q64,
                                 double maxrel, int *__restrict__ err) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= Q) return;
  int64_t u = perm[i];
  double X, Y, Z;
  cell_centre(xyzL[leaf[i]], lox, loy, loz, sL, X, Y, Z);
  double rx = x[3 * u] - X, ry = x[3 * u + 1] - Y, rz = x[3 * u + 2] - Z;
  if (!(fabs(rx) <= maxrel && fabs(ry) <= maxrel && fabs(rz) <= maxrel)) atomicOr(err, 16);
  q64[i] = make_double4(rx, ry, rz, 0.0);
  q32[i] = make_float4((float)rx, (float)ry, (float)rz, 0.0f);
}

__global__ void k_p2p_pairs(const int4 *__restrict__ range, int64_t C, const int32_t *__restrict__ near_ptr,
                            const int32_t *__restrict__ near_idx, unsigned long long *__restrict__ out) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  unsigned long long s = 0;
  if (t < C) {
    int4 rt = range[t];
    unsigned long long nt = (unsigned long long)(rt.y - rt.x);
    for (int e = near_ptr[t]; e < near_ptr[t + 1]; ++e) {
      int4 rs = range[near_idx[e]];
      s += nt * (unsigned long long)(rs.y - rs.x);
    }
  }
  if (s) atomicAdd(out, s);
}

template <class T>
void copy_d2d(T *dst, const T *src, size_t n, hipStream_t s) {
  if (n) HIP_OK(hipMemcpyAsync(dst, src, n * sizeof(T), hipMemcpyDeviceToDevice, s));
}

int read_err(DBuf<int> &e, hipStream_t s) {
  int h = 0;
  HIP_OK(hipMemcpyAsync(&h, e.p, sizeof(int), hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  return h;
}

}  // namespace

namespace {
struct DevTables {
  DBuf<float> m2l32, m2m32, l2l32;
  DBuf<double> m2l64, m2m64, l2l64;
  DBuf<uint16_t> m2lbf;
};

// bf16 nearest to f (ties to even), as its bit pattern; the tables hold
// finite values only
uint16_t bf16_bits(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
double bf16_value(uint16_t h) {
  const uint32_t u = (uint32_t)h << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}
}  // namespace

// Work lists of the batched L2L and M2M products: per level l >= 3, the
// level's cells grouped by octant, cut into MFMA tiles.  Built on the host from the
// cell keys and parents (a few tens of thousands of cells).
static void build_l2l_lists(Tree &T, hipStream_t s) {
  Tree::L2LList &W = T.l2lw;
  const int L = T.L;
  W.t0.assign(L + 2, 0);
  W.t1.assign(L + 2, 0);
  W.max_cells = 0;
  if (L < 3) return;
  std::vector<uint32_t> key(T.ncell_tot);
  std::vector<int32_t> par(T.ncell_tot);
  HIP_OK(hipMemcpyAsync(key.data(), T.ckey.p, T.ncell_tot * 4, hipMemcpyDeviceToHost, s));
  HIP_OK(hipMemcpyAsync(par.data(), T.cparent.p, T.ncell_tot * 4, hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  std::vector<int32_t> src, self, dest, goff, gend, tg, tr;
  for (int l = 3; l <= L; ++l) {
    W.t0[l] = (int64_t)tg.size();
    const int64_t c0 = T.coff[l], c1 = c0 + T.ncell[l];
    // the level's cells bucketed by octant, each bucket in cell order
    int64_t cnt[9] = {0};
    for (int64_t c = c0; c < c1; ++c) ++cnt[(key[c] & 7u) + 1];
    for (int o = 0; o < 8; ++o) cnt[o + 1] += cnt[o];
    const size_t base = src.size();
    src.resize(base + (c1 - c0));
    self.resize(base + (c1 - c0));
    dest.resize(base + (c1 - c0));
    {
      int64_t at[8];
      for (int o = 0; o < 8; ++o) at[o] = cnt[o];
      for (int64_t c = c0; c < c1; ++c) {
        const size_t k = base + at[key[c] & 7u]++;
        src[k] = par[c];
        self[k] = (int32_t)c;
        dest[k] = (int32_t)(c - c0);
      }
    }
    for (uint32_t o = 0; o < 8; ++o) {
      const int32_t b = (int32_t)(base + cnt[o]);
      const int32_t e = (int32_t)(base + cnt[o + 1]);
      if (e == b) continue;
      const int32_t g = (int32_t)goff.size();
      goff.push_back((int32_t)o);
      gend.push_back(e);
      for (int32_t r = b; r < e; r += LEVEL_ROWS) {
        tg.push_back(g);
        tr.push_back(r);
      }
    }
    W.t1[l] = (int64_t)tg.size();
    W.max_cells = std::max<int64_t>(W.max_cells, T.ncell[l]);
  }
  auto up = [&](DBuf<int32_t> &d, const std::vector<int32_t> &h) {
    d.alloc(std::max<size_t>(h.size(), 1));
    if (!h.empty()) HIP_OK(hipMemcpyAsync(d.p, h.data(), h.size() * 4, hipMemcpyHostToDevice, s));
  };
  up(W.src, src);
  up(W.self, self);
  up(W.dest, dest);
  up(W.group_off, goff);
  up(W.group_end, gend);
  up(W.tile_group, tg);
  up(W.tile_row, tr);
  HIP_OK(hipStreamSynchronize(s));  // host vectors go out of scope
}

// Device copies of the translation operators, built once per (device, p,
// MAC) and shared by all trees.
void upload_tables(Tree &T, hipStream_t s) {
  static std::mutex mu;
  static std::map<std::tuple<int, int, double, int>, DevTables *> cache;
  std::lock_guard<std::mutex> lk(mu);
  const Tables &tb = *T.tab;
  auto key = std::make_tuple(T.device, tb.p, tb.theta, tb.mac);
  DevTables *D = nullptr;
  auto it = cache.find(key);
  if (it != cache.end()) {
    D = it->second;
  } else {
    D = new DevTables();
    const int ps = T.ps, noff = tb.noff();
    const int KK = ps / 4, NT = ps / 16;
    // MFMA-swizzled M2L: for k-step kk and column tile ct, lane l holds
    // B[k][j] = T[out][in] for the coefficients stored at places
    // ct*16 + l%16 (out) and (l/16)*KK + kk (in), zero at padding places
    const int p = T.p;
    std::vector<float> sw32((size_t)noff * KK * NT * 64);
    std::vector<double> sw64(sw32.size());
    for (int o = 0; o < noff; ++o) {
      const double *Tm = tb.m2l.data() + (size_t)o * ps * ps;
      for (int kk = 0; kk < KK; ++kk)
        for (int ct = 0; ct < NT; ++ct)
          for (int l = 0; l < 64; ++l) {
            const int out = coef_at(ct * 16 + (l % 16), p, ps), in = coef_at((l / 16) * KK + kk, p, ps);
            const double v = (out >= 0 && in >= 0) ? Tm[(size_t)out * ps + in] : 0.0;
            size_t at = (((size_t)o * KK + kk) * NT + ct) * 64 + l;
            sw64[at] = v;
            sw32[at] = (float)v;
          }
    }
    D->m2l32.alloc(sw32.size());
    D->m2l64.alloc(sw64.size());
    HIP_OK(hipMemcpyAsync(D->m2l32.p, sw32.data(), sw32.size() * 4, hipMemcpyHostToDevice, s));
    HIP_OK(hipMemcpyAsync(D->m2l64.p, sw64.data(), sw64.size() * 8, hipMemcpyHostToDevice, s));
    // The M2L operators of order P_FIXED for the split-bf16 kernel: each
    // value y as three bf16 parts, each the nearest to what the previous
    // ones leave (y1 + y2 + y3 within about 2^-24 |y|).  Per offset and
    // column tile, NBLK B operands of 64 lanes x 8 slots: for each full
    // sub-step j, parts 1, 2, 3 of inputs 8j .. 8j+7 of the lane's block;
    // then the remainder steps, whose slot 8s+e holds, for product
    // t = (8s+e) / R, part PB[t] of input 8J + (8s+e) % R, and zero past the
    // six products.  PB pairs with the multipole parts {1,1,2,1,2,3}.
    std::vector<uint16_t> sbf;
    if (p == P_FIXED) {
      const int RB = coef_r4(p), J = RB / 8, R = RB % 8, NRS = (6 * R + 7) / 8, NBLK = 3 * J + NRS;
      static const int PB[6] = {1, 2, 1, 3, 2, 1};
      sbf.assign((size_t)noff * NT * NBLK * 64 * 8, 0);
      for (int o = 0; o < noff; ++o) {
        const double *Tm = tb.m2l.data() + (size_t)o * ps * ps;
        for (int ct = 0; ct < NT; ++ct)
          for (int blk = 0; blk < NBLK; ++blk)
            for (int l = 0; l < 64; ++l)
              for (int e = 0; e < 8; ++e) {
                int part, idx;
                if (blk < 3 * J) {
                  part = blk % 3 + 1;
                  idx = 8 * (blk / 3) + e;
                } else {
                  const int gs = 8 * (blk - 3 * J) + e;
                  if (gs >= 6 * R) continue;
                  part = PB[gs / R];
                  idx = 8 * J + gs % R;
                }
                const int out = coef_at(ct * 16 + (l % 16), p, ps), in = coef_at((l / 16) * KK + idx, p, ps);
                if (out < 0 || in < 0) continue;
                double r = Tm[(size_t)out * ps + in];
                uint16_t h[3];
                for (int i = 0; i < 3; ++i) {
                  h[i] = bf16_bits((float)r);
                  r -= bf16_value(h[i]);
                }
                sbf[((((size_t)o * NT + ct) * NBLK + blk) * 64 + l) * 8 + e] = h[part - 1];
              }
      }
      D->m2lbf.alloc(sbf.size());
      HIP_OK(hipMemcpyAsync(D->m2lbf.p, sbf.data(), sbf.size() * 2, hipMemcpyHostToDevice, s));
    }
    // M2M and L2L in the MFMA B-operand order of the M2L tables, one per
    // octant (the batched per-level products reuse the M2L kernel)
    std::vector<double> a((size_t)8 * KK * NT * 64), b(a.size());
    for (int o = 0; o < 8; ++o)
      for (int kk = 0; kk < KK; ++kk)
        for (int ct = 0; ct < NT; ++ct)
          for (int l = 0; l < 64; ++l) {
            const int out = coef_at(ct * 16 + (l % 16), p, ps), in = coef_at((l / 16) * KK + kk, p, ps);
            const size_t at = (((size_t)o * KK + kk) * NT + ct) * 64 + l;
            const bool real = out >= 0 && in >= 0;
            a[at] = real ? tb.m2m[((size_t)o * ps + out) * ps + in] : 0.0;
            b[at] = real ? tb.l2l[((size_t)o * ps + out) * ps + in] : 0.0;
          }
    std::vector<float> a32(a.size()), b32(b.size());
    for (size_t i = 0; i < a.size(); ++i) a32[i] = (float)a[i];
    for (size_t i = 0; i < b.size(); ++i) b32[i] = (float)b[i];
    D->m2m32.alloc(a32.size());
    D->l2l32.alloc(b32.size());
    D->m2m64.alloc(a.size());
    D->l2l64.alloc(b.size());
    HIP_OK(hipMemcpyAsync(D->m2m32.p, a32.data(), a32.size() * 4, hipMemcpyHostToDevice, s));
    HIP_OK(hipMemcpyAsync(D->l2l32.p, b32.data(), b32.size() * 4, hipMemcpyHostToDevice, s));
    HIP_OK(hipMemcpyAsync(D->m2m64.p, a.data(), a.size() * 8, hipMemcpyHostToDevice, s));
    HIP_OK(hipMemcpyAsync(D->l2l64.p, b.data(), b.size() * 8, hipMemcpyHostToDevice, s));
    HIP_OK(hipStreamSynchronize(s));
    cache[key] = D;
  }
  T.t_m2l32 = D->m2l32.p;
  T.t_m2l64 = D->m2l64.p;
  T.t_m2lbf = D->m2lbf.p;
  T.t_m2m32 = D->m2m32.p;
  T.t_l2l32 = D->l2l32.p;
  T.t_m2m64 = D->m2m64.p;
  T.t_l2l64 = D->l2l64.p;
}

void build_tree(Tree &T, const double *verts, int64_t nv, const int32_t *tris, int64_t nt, const double *qpos,
                int64_t nq, hipStream_t s) {
  const int TB = 256;
  T.N = nt;
  T.Q = nq;
  T.p = T.prm.p;
  T.ps = pad16(T.p * T.p);
  T.c.alloc(3 * nt);
  T.nrm.alloc(3 * nt);
  T.area.alloc(nt);
  T.qpos.alloc(3 * std::max<int64_t>(nq, 1));
  DBuf<int> err;
  err.alloc(1);
  err.zero(s);
  k_geometry<<<cdiv(nt, TB), TB, 0, s>>>(verts, nv, tris, nt, T.c.p, T.nrm.p, T.area.p, err.p);
  LAUNCH_OK();
  if (nq > 0) {
    HIP_OK(hipMemcpyAsync(T.qpos.p, qpos, 3 * nq * sizeof(double), hipMemcpyDeviceToDevice, s));
    k_check_points<<<cdiv(nq, TB), TB, 0, s>>>(T.qpos.p, nq, err.p);
    LAUNCH_OK();
  }
  int e = read_err(err, s);
  if (e & 1) BF_THROW(BEMFMM_EINVAL, "triangle vertex index out of range");
  if (e & 2) BF_THROW(BEMFMM_EINVAL, "degenerate (zero-area) or non-finite triangle");
  if (e & 4) BF_THROW(BEMFMM_EINVAL, "non-finite charge position");
  T.pverts.alloc(9 * nt);
  k_panel_verts<<<cdiv(nt, TB), TB, 0, s>>>(verts, tris, nt, T.pverts.p);
  LAUNCH_OK();

  // bounding cube (exact min / max)
  {
    int nb = std::min(1024, std::max(1, cdiv(nt + nq, TB)));
    DBuf<double> part;
    part.alloc((size_t)nb * 6);
    k_minmax<<<nb, TB, 0, s>>>(T.c.p, nt, T.qpos.p, nq, part.p);
    LAUNCH_OK();
    std::vector<double> h((size_t)nb * 6);
    HIP_OK(hipMemcpyAsync(h.data(), part.p, h.size() * 8, hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    double mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int b = 0; b < nb; ++b)
      for (int d = 0; d < 3; ++d) {
        mn[d] = std::min(mn[d], h[b * 6 + d]);
        mx[d] = std::max(mx[d], h[b * 6 + 3 + d]);
      }
    double ext = std::max(mx[0] - mn[0], std::max(mx[1] - mn[1], mx[2] - mn[2]));
    if (ext == 0.0) ext = 1.0;
    for (int d = 0; d < 3; ++d) T.lo[d] = mn[d];
    T.side = ext * (1.0 + std::ldexp(1.0, -20));
  }
  const double inv = 1024.0 / T.side;

  // keys and sort
  T.pkey.alloc(nt);
  T.pperm.alloc(nt);
  k_morton<<<cdiv(nt, TB), TB, 0, s>>>(T.c.p, nt, T.lo[0], T.lo[1], T.lo[2], inv, T.pkey.p, T.pperm.p);
  LAUNCH_OK();
  radix_sort_u32(T.pkey.p, T.pperm.p, nt, 3 * KEY_BITS, s);
  T.qkey.alloc(std::max<int64_t>(nq, 1));
  T.qperm.alloc(std::max<int64_t>(nq, 1));
  if (nq > 0) {
    k_morton<<<cdiv(nq, TB), TB, 0, s>>>(T.qpos.p, nq, T.lo[0], T.lo[1], T.lo[2], inv, T.qkey.p, T.qperm.p);
    LAUNCH_OK();
    radix_sort_u32(T.qkey.p, T.qperm.p, nq, 3 * KEY_BITS, s);
  }

  // leaf level: the level whose mean panel occupancy m_l = N / c_l is
  // closest to ncrit on a log scale, between the first level with m_l <=
  // ncrit and the one above it (exact integer test N^2 < ncrit^2 c_{l-1} c_l)
  {
    DBuf<unsigned long long> hist;
    hist.alloc(LMAX + 1);
    hist.zero(s);
    int nb = std::min(1024, std::max(1, cdiv(nt, TB)));
    k_level_hist<<<nb, TB, 0, s>>>(T.pkey.p, nt, hist.p);
    LAUNCH_OK();
    unsigned long long h[LMAX + 1];
    HIP_OK(hipMemcpyAsync(h, hist.p, sizeof(h), hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    int64_t distinct = 1, prev = 1;
    T.L = LMAX;
    const __int128 nc = T.prm.ncrit;
    for (int l = 0; l <= LMAX; ++l) {
      distinct += (int64_t)h[l];
      if (nt <= (int64_t)T.prm.ncrit * distinct) {
        T.L = l;
        if (l > 0 && (__int128)nt * nt < nc * nc * prev * distinct) T.L = l - 1;
        break;
      }
      prev = distinct;
    }
  }
  const int L = T.L;

  // leaf cells: union of panel and charge leaf prefixes
  std::vector<DBuf<uint32_t>> Ukey(L + 1);
  std::vector<DBuf<int4>> Urange(L + 1);
  std::vector<DBuf<int32_t>> Upar(L + 1);
  std::vector<DBuf<int2>> Uchild(L + 1);
  T.ncell.assign(L + 1, 0);
  {
    const int shift = 3 * (LMAX - L);
    int32_t cp = 0, cq = 0;
    DBuf<uint32_t> cat;
    DBuf<int32_t> pflag, ppos;
    pflag.alloc(nt);
    ppos.alloc(nt);
    k_flags_unique<<<cdiv(nt, TB), TB, 0, s>>>(T.pkey.p, nt, shift, pflag.p);
    LAUNCH_OK();
    exclusive_scan_i32(pflag.p, ppos.p, nt, s, &cp);
    DBuf<int32_t> qflag, qpos_;
    if (nq > 0) {
      qflag.alloc(nq);
      qpos_.alloc(nq);
      k_flags_unique<<<cdiv(nq, TB), TB, 0, s>>>(T.qkey.p, nq, shift, qflag.p);
      LAUNCH_OK();
      exclusive_scan_i32(qflag.p, qpos_.p, nq, s, &cq);
    }
    cat.alloc((size_t)cp + cq);
    k_compact_unique<<<cdiv(nt, TB), TB, 0, s>>>(T.pkey.p, nt, shift, pflag.p, ppos.p, cat.p);
    LAUNCH_OK();
    if (nq > 0) {
      k_compact_unique<<<cdiv(nq, TB), TB, 0, s>>>(T.qkey.p, nq, 0 + shift, qflag.p, qpos_.p, cat.p + cp);
      LAUNCH_OK();
    }
    int64_t ncat = (int64_t)cp + cq;
    DBuf<int32_t> dummy;
    dummy.alloc(ncat);
    HIP_OK(hipMemsetAsync(dummy.p, 0, ncat * sizeof(int32_t), s));
    radix_sort_u32(cat.p, dummy.p, ncat, std::max(1, 3 * L), s);
    DBuf<int32_t> uf, up;
    uf.alloc(ncat);
    up.alloc(ncat);
    k_flags_unique<<<cdiv(ncat, TB), TB, 0, s>>>(cat.p, ncat, 0, uf.p);
    LAUNCH_OK();
    int32_t C = 0;
    exclusive_scan_i32(uf.p, up.p, ncat, s, &C);
    Ukey[L].alloc(C);
    k_compact_unique<<<cdiv(ncat, TB), TB, 0, s>>>(cat.p, ncat, 0, uf.p, up.p, Ukey[L].p);
    LAUNCH_OK();
    Urange[L].alloc(C);
    k_leaf_cells<<<cdiv(C, TB), TB, 0, s>>>(Ukey[L].p, C, T.pkey.p, nt, T.qkey.p, nq, shift, Urange[L].p);
    LAUNCH_OK();
    T.ncell[L] = C;
    Uchild[L].alloc(C);
    HIP_OK(hipMemsetAsync(Uchild[L].p, 0, C * sizeof(int2), s));
  }
  // upper levels
  for (int l = L; l >= 1; --l) {
    int64_t C = T.ncell[l];
    DBuf<int32_t> flag, pos;
    flag.alloc(C);
    pos.alloc(C);
    k_parent_flags<<<cdiv(C, TB), TB, 0, s>>>(Ukey[l].p, C, flag.p);
    LAUNCH_OK();
    int32_t Cp = 0;
    exclusive_scan_i32(flag.p, pos.p, C, s, &Cp);
    Ukey[l - 1].alloc(Cp);
    Urange[l - 1].alloc(Cp);
    Uchild[l - 1].alloc(Cp);
    Upar[l].alloc(C);
    k_make_parents<<<cdiv(C, TB), TB, 0, s>>>(Ukey[l].p, Urange[l].p, C, flag.p, pos.p, Cp, Ukey[l - 1].p,
                                              Uchild[l - 1].p, Urange[l - 1].p, Upar[l].p);
    LAUNCH_OK();
    T.ncell[l - 1] = Cp;
  }
  if (T.ncell[0] != 1) BF_THROW(BEMFMM_EDEVICE, "tree build: root level has more than one cell");
  Upar[0].alloc(1);
  HIP_OK(hipMemsetAsync(Upar[0].p, 0xff, sizeof(int32_t), s));  // -1

  // global cell arrays
  T.coff.assign(L + 2, 0);
  for (int l = 0; l <= L; ++l) T.coff[l + 1] = T.coff[l] + T.ncell[l];
  T.ncell_tot = T.coff[L + 1];
  const int64_t CT = T.ncell_tot;
  T.ckey.alloc(CT);
  T.clevel.alloc(CT);
  T.crange.alloc(CT);
  T.cparent.alloc(CT);
  T.cchild.alloc(CT);
  T.cxyz.alloc(CT);
  {
    std::vector<int32_t> lev(CT);
    for (int l = 0; l <= L; ++l)
      for (int64_t i = T.coff[l]; i < T.coff[l + 1]; ++i) lev[i] = l;
    HIP_OK(hipMemcpyAsync(T.clevel.p, lev.data(), CT * 4, hipMemcpyHostToDevice, s));
    HIP_OK(hipStreamSynchronize(s));
  }
  for (int l = 0; l <= L; ++l) {
    int64_t C = T.ncell[l], o = T.coff[l];
    copy_d2d(T.ckey.p + o, Ukey[l].p, C, s);
    copy_d2d(T.crange.p + o, Urange[l].p, C, s);
    copy_d2d(T.cchild.p + o, Uchild[l].p, C, s);
    copy_d2d(T.cparent.p + o, Upar[l].p, C, s);
  }
  // convert level-local parent / child indices to global ones on the host
  // side of a small pass (counts are per level)
  {
    std::vector<int32_t> par(CT);
    std::vector<int2> ch(CT);
    HIP_OK(hipMemcpyAsync(par.data(), T.cparent.p, CT * 4, hipMemcpyDeviceToHost, s));
    HIP_OK(hipMemcpyAsync(ch.data(), T.cchild.p, CT * sizeof(int2), hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    for (int l = 0; l <= L; ++l)
      for (int64_t i = T.coff[l]; i < T.coff[l + 1]; ++i) {
        if (l > 0) par[i] += (int32_t)T.coff[l - 1];
        if (l < L) {
          ch[i].x += (int32_t)T.coff[l + 1];
          ch[i].y += (int32_t)T.coff[l + 1];
        } else {
          ch[i].x = ch[i].y = 0;
        }
      }
    par[0] = -1;
    HIP_OK(hipMemcpyAsync(T.cparent.p, par.data(), CT * 4, hipMemcpyHostToDevice, s));
    HIP_OK(hipMemcpyAsync(T.cchild.p, ch.data(), CT * sizeof(int2), hipMemcpyHostToDevice, s));
    HIP_OK(hipStreamSynchronize(s));
  }
  k_cell_xyz<<<cdiv(CT, TB), TB, 0, s>>>(T.ckey.p, CT, T.cxyz.p);
  LAUNCH_OK();

  // tables for this (p, MAC)
  T.tab = &get_tables(T.p, T.prm.theta, T.prm.mac);
  upload_tables(T, s);
  DBuf<int32_t> offid;
  offid.alloc(T.tab->offset_id.size());
  HIP_OK(hipMemcpyAsync(offid.p, T.tab->offset_id.data(), T.tab->offset_id.size() * 4, hipMemcpyHostToDevice, s));

  // lists, top down
  const double theta2 = T.prm.theta * T.prm.theta;
  T.near_off.assign(L + 2, 0);
  T.near_ptr_off.assign(L + 2, 0);
  for (int l = 0; l <= L; ++l) T.near_ptr_off[l + 1] = T.near_ptr_off[l] + T.ncell[l] + 1;
  std::vector<DBuf<int32_t>> nptr(L + 1), nidx(L + 1);
  std::vector<DBuf<int2>> fts(L + 1);
  std::vector<int64_t> nfar_l(L + 1, 0), nnear_l(L + 1, 0);
  std::vector<DBuf<int32_t>> fptr_l(L + 1);
  nptr[0].alloc(2);
  nidx[0].alloc(1);
  // the root is near itself: nptr[0] = {0, 1}, nidx[0] = {0}
  k_set_i32<<<1, 1, 0, s>>>(nptr[0].p, 0);
  k_set_i32<<<1, 1, 0, s>>>(nptr[0].p + 1, 1);
  k_set_i32<<<1, 1, 0, s>>>(nidx[0].p, 0);
  LAUNCH_OK();
  nnear_l[0] = 1;
  for (int l = 1; l <= L; ++l) {
    int32_t C = T.ncell[l];
    if (C == 0) BF_THROW(BEMFMM_EDEVICE, "tree build: empty level");
    DBuf<int32_t> ncnt, fcnt;
    ncnt.alloc(C + 1);
    fcnt.alloc(C + 1);
    k_lists<<<C, 64, 0, s>>>(C, T.coff[l], T.coff[l - 1], T.cparent.p, T.cxyz.p, T.cchild.p, nptr[l - 1].p,
                                        nidx[l - 1].p, theta2, T.prm.mac, 0, ncnt.p, fcnt.p, nullptr, nullptr,
                                        nullptr, nullptr);
    LAUNCH_OK();
    HIP_OK(hipMemsetAsync(ncnt.p + C, 0, 4, s));
    HIP_OK(hipMemsetAsync(fcnt.p + C, 0, 4, s));
    nptr[l].alloc(C + 1);
    fptr_l[l].alloc(C + 1);
    int32_t nn = 0, nf = 0;
    exclusive_scan_i32(ncnt.p, nptr[l].p, C + 1, s, &nn);
    exclusive_scan_i32(fcnt.p, fptr_l[l].p, C + 1, s, &nf);
    nidx[l].alloc(std::max<int32_t>(nn, 1));
    fts[l].alloc(std::max<int32_t>(nf, 1));
    k_lists<<<C, 64, 0, s>>>(C, T.coff[l], T.coff[l - 1], T.cparent.p, T.cxyz.p, T.cchild.p, nptr[l - 1].p,
                                        nidx[l - 1].p, theta2, T.prm.mac, 1, nullptr, nullptr, nptr[l].p, nidx[l].p,
                                        fptr_l[l].p, fts[l].p);
    LAUNCH_OK();
    nnear_l[l] = nn;
    nfar_l[l] = nf;
  }
  // concatenate near lists
  for (int l = 0; l <= L; ++l) T.near_off[l + 1] = T.near_off[l] + nnear_l[l];
  T.near_ptr.alloc(T.near_ptr_off[L + 1]);
  T.near_idx.alloc(std::max<int64_t>(T.near_off[L + 1], 1));
  for (int l = 0; l <= L; ++l) {
    copy_d2d(T.near_ptr.p + T.near_ptr_off[l], nptr[l].p, (size_t)T.ncell[l] + 1, s);
    copy_d2d(T.near_idx.p + T.near_off[l], nidx[l].p, (size_t)nnear_l[l], s);
  }
  T.n_near_leaf = nnear_l[L];
  // far pairs, global cell indices, target-major per level
  T.far_off.assign(L + 2, 0);
  for (int l = 0; l <= L; ++l) T.far_off[l + 1] = T.far_off[l] + nfar_l[l];
  T.nfar = T.far_off[L + 1];
  T.far_ts.alloc(std::max<int64_t>(T.nfar, 1));
  T.far_ptr.alloc(CT + 1);
  HIP_OK(hipMemsetAsync(T.far_ptr.p, 0, (CT + 1) * 4, s));
  for (int l = 1; l <= L; ++l) {
    copy_d2d(T.far_ts.p + T.far_off[l], fts[l].p, (size_t)nfar_l[l], s);
    k_far_ptr<<<cdiv(T.ncell[l], TB), TB, 0, s>>>(fptr_l[l].p, T.ncell[l], T.coff[l], T.far_off[l], T.far_ptr.p);
    LAUNCH_OK();
  }
  k_set_i32<<<1, 1, 0, s>>>(T.far_ptr.p + CT, (int32_t)T.nfar);
  LAUNCH_OK();

  // M2L pairs sorted by translation offset (all levels together: the scaled
  // operator depends on the offset only), then one filtered list per
  // (source kind, target kind)
  if (T.nfar > 0) {
    const int64_t nf = T.nfar;
    DBuf<uint32_t> key;
    DBuf<int32_t> order;
    key.alloc(nf);
    order.alloc(nf);
    err.zero(s);
    k_offset_keys<<<cdiv(nf, TB), TB, 0, s>>>(T.far_ts.p, nf, T.cxyz.p, offid.p, T.tab->R, key.p, order.p, err.p);
    LAUNCH_OK();
    if (read_err(err, s) & 8) BF_THROW(BEMFMM_EDEVICE, "tree build: M2L offset outside the operator table");
    int nbits = 1;
    while ((1 << nbits) < T.tab->noff()) ++nbits;
    radix_sort_u32(key.p, order.p, nf, nbits, s);
    DBuf<int32_t> flag, pos, flag_t, pos_t;
    DBuf<uint32_t> ckeyc;
    DBuf<uint8_t> kind;
    DBuf<int2> ts_sorted;
    flag.alloc(nf);
    pos.alloc(nf);
    flag_t.alloc(nf + 1);
    pos_t.alloc(nf + 1);
    ckeyc.alloc(nf);
    kind.alloc(T.ncell_tot);
    ts_sorted.alloc(nf);
    k_cell_kinds<<<cdiv(T.ncell_tot, TB), TB, 0, s>>>(T.crange.p, T.ncell_tot, kind.p);
    LAUNCH_OK();
    k_gather_pairs<<<cdiv(nf, TB), TB, 0, s>>>(order.p, T.far_ts.p, nf, ts_sorted.p);
    LAUNCH_OK();
    const int64_t CT1 = T.ncell_tot + 1;
    for (int combo = 0; combo < 3; ++combo) {
      Tree::M2LList &ML = T.m2l[combo];
      k_combo_flags<<<cdiv(nf, TB), TB, 0, s>>>(ts_sorted.p, kind.p, nf, combo, flag.p);
      LAUNCH_OK();
      int32_t nk = 0;
      exclusive_scan_i32(flag.p, pos.p, nf, s, &nk);
      ML.n = nk;
      // output rows in pair order: a cell's rows are contiguous (the same
      // flags, taken in pair order)
      k_combo_flags<<<cdiv(nf, TB), TB, 0, s>>>(T.far_ts.p, kind.p, nf, combo, flag_t.p);
      LAUNCH_OK();
      HIP_OK(hipMemsetAsync(flag_t.p + nf, 0, 4, s));
      exclusive_scan_i32(flag_t.p, pos_t.p, nf + 1, s, nullptr);
      ML.kptr.alloc(CT1);
      k_kept_ptr<<<cdiv(CT1, TB), TB, 0, s>>>(T.far_ptr.p, pos_t.p, CT1, ML.kptr.p);
      LAUNCH_OK();
      ML.src.alloc(std::max<int32_t>(nk, 1));
      ML.dest.alloc(std::max<int32_t>(nk, 1));
      k_combo_compact<<<cdiv(nf, TB), TB, 0, s>>>(order.p, key.p, flag.p, pos.p, nf, ts_sorted.p, pos_t.p, ML.src.p,
                                                  ckeyc.p, ML.dest.p);
      LAUNCH_OK();
      if (nk == 0) continue;
      DBuf<int32_t> gflag, gpos, gbeg;
      gflag.alloc(nk);
      gpos.alloc(nk);
      k_group_flags<<<cdiv(nk, TB), TB, 0, s>>>(ckeyc.p, nk, gflag.p);
      LAUNCH_OK();
      int32_t G = 0;
      exclusive_scan_i32(gflag.p, gpos.p, nk, s, &G);
      ML.group_off.alloc(G);
      ML.group_end.alloc(G);
      gbeg.alloc(G);
      k_group_make<<<cdiv(nk, TB), TB, 0, s>>>(ckeyc.p, nk, gflag.p, gpos.p, ML.group_off.p, gbeg.p, ML.group_end.p);
      LAUNCH_OK();
      ML.ngroups = G;
      for (int pass = 0; pass < 2; ++pass) {
        const int ROWS = pass == 0 ? M2L_ROWS32 : M2L_ROWS64;
        DBuf<int32_t> ntile, tpos;
        ntile.alloc(G + 1);
        tpos.alloc(G + 1);
        k_group_tiles<<<cdiv(G, TB), TB, 0, s>>>(gbeg.p, ML.group_end.p, G, ROWS, ntile.p);
        LAUNCH_OK();
        HIP_OK(hipMemsetAsync(ntile.p + G, 0, 4, s));
        int32_t ntiles = 0;
        exclusive_scan_i32(ntile.p, tpos.p, G + 1, s, &ntiles);
        DBuf<int32_t> &tg = pass == 0 ? ML.tile_group : ML.tile_group64;
        DBuf<int32_t> &tr = pass == 0 ? ML.tile_row : ML.tile_row64;
        tg.alloc(ntiles);
        tr.alloc(ntiles);
        k_tile_list<<<cdiv(G, TB), TB, 0, s>>>(gbeg.p, ML.group_end.p, G, ROWS, tpos.p, tg.p, tr.p);
        LAUNCH_OK();
        (pass == 0 ? ML.ntiles : ML.ntiles64) = ntiles;
      }
    }
  }

  build_l2l_lists(T, s);

  // leaf membership, inverse permutations, sorted point data
  const int64_t CL = T.ncell[L];
  T.pleaf.alloc(nt);
  T.qleaf.alloc(std::max<int64_t>(nq, 1));
  k_fill_leaf<<<cdiv(CL, TB), TB, 0, s>>>(T.crange.p + T.coff[L], CL, T.pleaf.p, T.qleaf.p);
  LAUNCH_OK();
  T.pinv.alloc(nt);
  k_inverse_perm<<<cdiv(nt, TB), TB, 0, s>>>(T.pperm.p, nt, T.pinv.p);
  LAUNCH_OK();
  T.qinv.alloc(std::max<int64_t>(nq, 1));
  if (nq > 0) {
    k_inverse_perm<<<cdiv(nq, TB), TB, 0, s>>>(T.qperm.p, nq, T.qinv.p);
    LAUNCH_OK();
  }
  const double sL = T.side / double(1 << L);
  T.p32pos.alloc(nt);
  T.p32nrm.alloc(nt);
  T.p64pos.alloc(nt);
  T.p64nrm.alloc(nt);
  k_gather_panels<<<cdiv(nt, TB), TB, 0, s>>>(T.pperm.p, T.pleaf.p, nt, T.cxyz.p + T.coff[L], T.lo[0], T.lo[1],
                                              T.lo[2], sL, T.c.p, T.nrm.p, T.area.p, T.p32pos.p, T.p32nrm.p,
                                              T.p64pos.p, T.p64nrm.p);
  LAUNCH_OK();
  T.q32pos.alloc(std::max<int64_t>(nq, 1));
  T.q64pos.alloc(std::max<int64_t>(nq, 1));
  if (nq > 0) {
    err.zero(s);
    k_gather_charges<<<cdiv(nq, TB), TB, 0, s>>>(T.qperm.p, T.qleaf.p, nq, T.cxyz.p + T.coff[L], T.lo[0], T.lo[1],
                                                 T.lo[2], sL, T.qpos.p, T.q32pos.p, T.q64pos.p, 0.5 * sL * (1 + 1e-9),
                                                 err.p);
    LAUNCH_OK();
    if (read_err(err, s) & 16) BF_THROW(BEMFMM_EDEVICE, "tree build: a charge lies outside its leaf cell");
  }
  // work estimate: P2P panel pairs
  {
    DBuf<unsigned long long> acc;
    acc.alloc(1);
    acc.zero(s);
    k_p2p_pairs<<<cdiv(CL, TB), TB, 0, s>>>(T.crange.p + T.coff[L], CL, T.near_ptr.p + T.near_ptr_off[L],
                                            T.near_idx.p + T.near_off[L], acc.p);
    LAUNCH_OK();
    unsigned long long h = 0;
    HIP_OK(hipMemcpyAsync(&h, acc.p, 8, hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    T.p2p_pairs_pp = (int64_t)h;
  }
  // P2P chunks: at most 64 targets of one leaf per wave; a chunk of n < 64
  // targets splits the sources over 64 / n lane groups
  {
    std::vector<int4> rg(CL);
    HIP_OK(hipMemcpyAsync(rg.data(), T.crange.p + T.coff[L], CL * sizeof(int4), hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    std::vector<int4> cp, cq;
    auto add = [](std::vector<int4> &v, int leaf, int b, int e) {
      for (int x = b; x < e; x += 64) {
        const int n = std::min(64, e - x);
        v.push_back(make_int4(leaf, x, n, 64 / n));
      }
    };
    for (int64_t t = 0; t < CL; ++t) {
      add(cp, (int)t, rg[t].x, rg[t].y);
      add(cq, (int)t, rg[t].z, rg[t].w);
    }
    T.nchunk_p = (int64_t)cp.size();
    T.nchunk_q = (int64_t)cq.size();
    T.chunk_p.alloc(std::max<size_t>(cp.size(), 1));
    T.chunk_q.alloc(std::max<size_t>(cq.size(), 1));
    if (!cp.empty())
      HIP_OK(hipMemcpyAsync(T.chunk_p.p, cp.data(), cp.size() * sizeof(int4), hipMemcpyHostToDevice, s));
    if (!cq.empty())
      HIP_OK(hipMemcpyAsync(T.chunk_q.p, cq.data(), cq.size() * sizeof(int4), hipMemcpyHostToDevice, s));
  }
  if (T.prm.near_quad > 0.0) build_nearquad(T, verts, tris, s);
  HIP_OK(hipStreamSynchronize(s));
}

namespace {

// ----------------------------------------------------- near quadrature
// (Section 2.1, discretisation paragraph: for flat panels the integrals can
// be taken analytically.)  For a flat triangle T (vertices counter-clockwise
// about its unit normal n) and a point r off its edges,
//   grad_r of the integral over T of 1/|r - r'| dA' = - sum_e f_e m_e - W n,
// with, per edge e from a to b: t = (b - a)/|b - a|, m = t x n (in-plane,
// outward), f_e = asinh(s_b/d) - asinh(s_a/d) the integral of 1/|r - r'|
// along the edge (s = (vertex - r).t, d the distance of r to the edge line),
// and W the solid angle of T at r (Van Oosterom and Strackee's closed form),
// positive on the side n points to and 0 in the plane of T.
__device__ void tri_grad_exact(const double *__restrict__ verts, const int32_t *__restrict__ tri, const double r[3],
                               double g[3]) {
  double v[3][3];
  for (int k = 0; k < 3; ++k)
    for (int d = 0; d < 3; ++d) v[k][d] = verts[3 * (int64_t)tri[k] + d];
  const double e1[3] = {v[1][0] - v[0][0], v[1][1] - v[0][1], v[1][2] - v[0][2]};
  const double e2[3] = {v[2][0] - v[0][0], v[2][1] - v[0][1], v[2][2] - v[0][2]};
  double n[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
  const double nl = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
  for (int d = 0; d < 3; ++d) n[d] /= nl;
  g[0] = g[1] = g[2] = 0.0;
  for (int e = 0; e < 3; ++e) {
    const double *a = v[e], *b = v[(e + 1) % 3];
    double t[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
    const double tl = sqrt(t[0] * t[0] + t[1] * t[1] + t[2] * t[2]);
    for (int d = 0; d < 3; ++d) t[d] /= tl;
    const double m[3] = {t[1] * n[2] - t[2] * n[1], t[2] * n[0] - t[0] * n[2], t[0] * n[1] - t[1] * n[0]};
    const double ar[3] = {a[0] - r[0], a[1] - r[1], a[2] - r[2]};
    const double br[3] = {b[0] - r[0], b[1] - r[1], b[2] - r[2]};
    const double sa = ar[0] * t[0] + ar[1] * t[1] + ar[2] * t[2];
    const double sb = br[0] * t[0] + br[1] * t[1] + br[2] * t[2];
    const double d2 = fmax(ar[0] * ar[0] + ar[1] * ar[1] + ar[2] * ar[2] - sa * sa, 0.0);
    double f;
    if (d2 > 1e-28 * fmax(sa * sa, sb * sb)) {
      const double d = sqrt(d2);
      f = asinh(sb / d) - asinh(sa / d);
    } else {  // on the edge's line, outside the segment
      f = copysign(log(fabs(sb) / fabs(sa)), sb);
    }
    for (int d = 0; d < 3; ++d) g[d] -= f * m[d];
  }
  double R[3][3], l[3];
  for (int k = 0; k < 3; ++k) {
    for (int d = 0; d < 3; ++d) R[k][d] = v[k][d] - r[d];
    l[k] = sqrt(R[k][0] * R[k][0] + R[k][1] * R[k][1] + R[k][2] * R[k][2]);
  }
  const double c23[3] = {R[1][1] * R[2][2] - R[1][2] * R[2][1], R[1][2] * R[2][0] - R[1][0] * R[2][2],
                         R[1][0] * R[2][1] - R[1][1] * R[2][0]};
  // the triple product of v_k - r is negative on the side n points to (the
  // counter-clockwise vertices turn clockwise seen from there)
  const double num = -(R[0][0] * c23[0] + R[0][1] * c23[1] + R[0][2] * c23[2]);
  auto dot3 = [](const double *x, const double *y) { return x[0] * y[0] + x[1] * y[1] + x[2] * y[2]; };
  const double den = l[0] * l[1] * l[2] + dot3(R[0], R[1]) * l[2] + dot3(R[0], R[2]) * l[1] + dot3(R[1], R[2]) * l[0];
  const double W = (fabs(num) <= 1e-15 * l[0] * l[1] * l[2]) ? 0.0 : 2.0 * atan2(num, den);
  for (int d = 0; d < 3; ++d) g[d] -= W * n[d];
}

// sorted-order centroid and circumradius (largest centroid-vertex distance)
__global__ void k_nq_points(const int32_t *__restrict__ perm, int64_t N, const double *__restrict__ c,
                            const double *__restrict__ verts, const int32_t *__restrict__ tris,
                            double4 *__restrict__ cr, double *__restrict__ bmax) {
  __shared__ double sh[256];
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double rho = 0.0;
  if (i < N) {
    const int64_t u = perm[i];
    const double X = c[3 * u], Y = c[3 * u + 1], Z = c[3 * u + 2];
    for (int k = 0; k < 3; ++k) {
      const int64_t vk = tris[3 * u + k];
      const double dx = verts[3 * vk] - X, dy = verts[3 * vk + 1] - Y, dz = verts[3 * vk + 2] - Z;
      rho = fmax(rho, sqrt(dx * dx + dy * dy + dz * dz));
    }
    cr[i] = make_double4(X, Y, Z, rho);
  }
  sh[threadIdx.x] = rho;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) bmax[blockIdx.x] = sh[0];
}

// Close panel pairs of every sorted target panel, over its near leaves in
// list order and the sources of each leaf in sorted order.  TRANSPOSE = 0
// (A): the pairs (t, j) with |c_t - c_j| < nu rho_j, j != t; each stores the
// source's caller index and 4 pi (K'_tj exact - K'_tj one-point).
// TRANSPOSE = 1 (A^T): the pairs (i, t) with |c_i - c_t| < nu rho_t, i != t;
// each stores i's caller index and the same difference for K'_it (the
// product divides by the area of t).  FILL = 0 only counts.
template <int TRANSPOSE, int FILL>
__global__ void k_nq_pairs(int64_t N, const double4 *__restrict__ cr, const int32_t *__restrict__ pleaf,
                           const int4 *__restrict__ leaf_range, const int32_t *__restrict__ leaf_xyz,
                           const int32_t *__restrict__ near_ptr, const int32_t *__restrict__ near_idx, double lox,
                           double loy, double loz, double sL, double nu, double reach,
                           const int32_t *__restrict__ perm, const double *__restrict__ nrm,
                           const double *__restrict__ area, const double *__restrict__ verts,
                           const int32_t *__restrict__ tris, int32_t *__restrict__ cnt,
                           const int32_t *__restrict__ ptr, int32_t *__restrict__ idx, double *__restrict__ coef) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N) return;
  const double4 ct = cr[t];
  const int leaf = pleaf[t];
  int32_t k = FILL ? ptr[t] : 0;
  const int64_t ut = perm[t];
  for (int e = near_ptr[leaf]; e < near_ptr[leaf + 1]; ++e) {
    const int sl = near_idx[e];
    // skip a leaf whose box lies farther than the largest radius
    double X, Y, Z;
    cell_centre(leaf_xyz[sl], lox, loy, loz, sL, X, Y, Z);
    const double gx = fmax(fabs(ct.x - X) - 0.5 * sL, 0.0), gy = fmax(fabs(ct.y - Y) - 0.5 * sL, 0.0),
                 gz = fmax(fabs(ct.z - Z) - 0.5 * sL, 0.0);
    if (gx * gx + gy * gy + gz * gz >= reach * reach) continue;
    const int4 rg = leaf_range[sl];
    for (int j = rg.x; j < rg.y; ++j) {
      if (j == t) continue;
      const double4 cj = cr[j];
      const double dx = ct.x - cj.x, dy = ct.y - cj.y, dz = ct.z - cj.z;
      const double r2 = dx * dx + dy * dy + dz * dz;
      const double lim = nu * (TRANSPOSE ? ct.w : cj.w);
      if (!(r2 < lim * lim)) continue;
      if (FILL) {
        const int64_t uj = perm[j];
        // pair (target i, source panel s) of K'
        const int64_t ui = TRANSPOSE ? uj : ut, us = TRANSPOSE ? ut : uj;
        const double ri[3] = {TRANSPOSE ? cj.x : ct.x, TRANSPOSE ? cj.y : ct.y, TRANSPOSE ? cj.z : ct.z};
        double g[3];
        tri_grad_exact(verts, tris + 3 * us, ri, g);
        const double ni[3] = {nrm[3 * ui], nrm[3 * ui + 1], nrm[3 * ui + 2]};
        // 4 pi K' exact = n_i . g;  4 pi K' one-point = -a_s n_i . (c_i - c_s) / r^3
        const double sgn = TRANSPOSE ? -1.0 : 1.0;  // c_i - c_s = sgn (c_t - c_j)
        const double ndot = sgn * (ni[0] * dx + ni[1] * dy + ni[2] * dz);
        const double inv_r = 1.0 / sqrt(r2);
        const double d4 = (ni[0] * g[0] + ni[1] * g[1] + ni[2] * g[2]) + area[us] * ndot * inv_r * inv_r * inv_r;
        idx[k] = (int32_t)uj;
        coef[k] = d4;
      }
      ++k;
    }
  }
  if (!FILL) cnt[t] = k;
}

__global__ void k_sum_i32_to_u64(const int32_t *__restrict__ v, int64_t n, unsigned long long *__restrict__ out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  unsigned long long x = (i < n) ? (unsigned long long)v[i] : 0ull;
  for (int o = 32; o > 0; o >>= 1) x += __shfl_down(x, o, 64);
  if ((threadIdx.x & 63) == 0 && x) atomicAdd(out, x);
}

__global__ void k_zero_i32(int *p) { *p = 0; }

int read_err_ptr(const int *e, hipStream_t s) {
  int h = 0;
  HIP_OK(hipMemcpyAsync(&h, e, sizeof(int), hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  return h;
}

// Device address of `scratch` per device, taken once per device with that
// device current (the caller's DeviceScope makes the tree's device current).
constexpr int SCRATCH_MAX_DEVICES = 64;
std::mutex scratch_mu;
void *scratch_dev[SCRATCH_MAX_DEVICES] = {};

unsigned char *scratch_ptr() {
  int dev = 0;
  HIP_OK(hipGetDevice(&dev));
  if (dev < 0 || dev >= SCRATCH_MAX_DEVICES) BF_THROW(BEMFMM_EDEVICE, "device index beyond the scratch table");
  std::lock_guard<std::mutex> g(scratch_mu);
  if (!scratch_dev[dev]) {
    void *p = nullptr;
    HIP_OK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) BF_THROW(BEMFMM_EDEVICE, "hipGetSymbolAddress returned no address for the scratch array");
    scratch_dev[dev] = p;
  }
  return static_cast<unsigned char *>(scratch_dev[dev]);
}

}  // namespace

// Smallest gap between two leaf boxes that are not in each other's near
// list, in leaf sides: far pairs are M2L offsets at the leaf level or pairs
// whose ancestors were far, whose gap in leaf sides is larger still.
static double far_gap_leaf_sides(const Tables &tb) {
  double g = 1e300;
  for (int c = 0; c < tb.noff(); ++c) {
    double s2 = 0.0;
    for (int d = 0; d < 3; ++d) {
      const double a = std::max(std::abs(tb.offsets[3 * c + d]) - 1, 0);
      s2 += a * a;
    }
    g = std::min(g, std::sqrt(s2));
  }
  return g;
}

void build_nearquad(Tree &T, const double *verts, const int32_t *tris, hipStream_t s) {
  const int TB = 256;
  const int64_t N = T.N;
  const int L = T.L;
  const double nu = T.prm.near_quad;
  const double sL = T.side / double(1 << L);
  DBuf<double4> cr;
  cr.alloc(N);
  const int nb = cdiv(N, TB);
  DBuf<double> bmax;
  bmax.alloc(nb);
  k_nq_points<<<nb, TB, 0, s>>>(T.pperm.p, N, T.c.p, verts, tris, cr.p, bmax.p);
  LAUNCH_OK();
  std::vector<double> hb(nb);
  HIP_OK(hipMemcpyAsync(hb.data(), bmax.p, nb * sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  const double rho_max = *std::max_element(hb.begin(), hb.end());
  const double reach = nu * rho_max;
  // every close pair must lie in the near field, where the correction is
  // applied to the direct sum
  const double gap = (L >= 2 && T.tab) ? far_gap_leaf_sides(*T.tab) * sL : 1e300;
  if (!(reach < gap))
    BF_THROW(BEMFMM_EINVAL, "near_quad radius (" + std::to_string(reach) + ") reaches beyond the near field (" +
                                std::to_string(gap) + "): lower near_quad or raise ncrit");
  const int4 *lr = T.crange.p + T.coff[L];
  const int32_t *lx = T.cxyz.p + T.coff[L];
  const int32_t *np_ = T.near_ptr.p + T.near_ptr_off[L];
  const int32_t *ni_ = T.near_idx.p + T.near_off[L];
  for (int tr = 0; tr < 2; ++tr) {
    DBuf<int32_t> &ptr = tr ? T.nqT_ptr : T.nq_ptr;
    DBuf<int32_t> &idx = tr ? T.nqT_idx : T.nq_idx;
    DBuf<double> &coef = tr ? T.nqT_coef : T.nq_coef;
    DBuf<int32_t> cnt;
    cnt.alloc(N);
    ptr.alloc(N + 1);
    auto launch = [&](auto tpl_tr, auto tpl_fill) {
      constexpr int TR = decltype(tpl_tr)::value, FILL = decltype(tpl_fill)::value;
      k_nq_pairs<TR, FILL><<<nb, TB, 0, s>>>(N, cr.p, T.pleaf.p, lr, lx, np_, ni_, T.lo[0], T.lo[1], T.lo[2], sL, nu,
                                             reach, T.pperm.p, T.nrm.p, T.area.p, verts, tris, cnt.p, ptr.p, idx.p,
                                             coef.p);
      LAUNCH_OK();
    };
    if (tr) launch(std::integral_constant<int, 1>(), std::integral_constant<int, 0>());
    else launch(std::integral_constant<int, 0>(), std::integral_constant<int, 0>());
    DBuf<unsigned long long> tot;
    tot.alloc(1);
    tot.zero(s);
    k_sum_i32_to_u64<<<nb, TB, 0, s>>>(cnt.p, N, tot.p);
    LAUNCH_OK();
    unsigned long long h = 0;
    HIP_OK(hipMemcpyAsync(&h, tot.p, 8, hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    if (h >= (1ull << 31)) BF_THROW(BEMFMM_EINVAL, "near_quad: more than 2^31 close panel pairs; lower near_quad");
    exclusive_scan_i32(cnt.p, ptr.p, N, s, nullptr);
    const int32_t total = (int32_t)h;
    HIP_OK(hipMemcpyAsync(ptr.p + N, &total, sizeof(int32_t), hipMemcpyHostToDevice, s));
    idx.alloc(std::max<int64_t>(h, 1));
    coef.alloc(std::max<int64_t>(h, 1));
    if (tr) launch(std::integral_constant<int, 1>(), std::integral_constant<int, 1>());
    else launch(std::integral_constant<int, 0>(), std::integral_constant<int, 1>());
    if (tr) T.n_nqT = (int64_t)h;
    else T.n_nq = (int64_t)h;
  }
  HIP_OK(hipStreamSynchronize(s));
}

int64_t noalloc_max_charges() {
  // error word (256 B), then Q float4 and Q double4, each block 256-B aligned
  return (int64_t)((BEMFMM_NOALLOC_SCRATCH_BYTES - 2 * 256) / (sizeof(float4) + sizeof(double4)));
}

// set_charges without device allocation: the same kernels and checks, with
// the error word and the staged positions in `scratch` and the caller's
// positions read in place.  The tree is changed only after both checks pass.
void set_charges_noalloc(Tree &T, const double *qpos, hipStream_t s) {
  const int TB = 256;
  const int64_t nq = T.Q;
  if (nq == 0) return;
  if (nq > noalloc_max_charges())
    BF_THROW(BEMFMM_EINVAL, "set_charges_noalloc: " + std::to_string(nq) + " charges exceed the " +
                                std::to_string(noalloc_max_charges()) + " its fixed scratch holds; use bemfmm_set_charges");
  unsigned char *base = scratch_ptr();
  int *err = reinterpret_cast<int *>(base);
  float4 *q32 = reinterpret_cast<float4 *>(base + 256);
  const size_t off64 = (256 + (size_t)nq * sizeof(float4) + 255) / 256 * 256;
  double4 *q64 = reinterpret_cast<double4 *>(base + off64);
  if (off64 + (size_t)nq * sizeof(double4) > BEMFMM_NOALLOC_SCRATCH_BYTES)
    BF_THROW(BEMFMM_EDEVICE, "set_charges_noalloc: scratch layout overflow");
  k_zero_i32<<<1, 1, 0, s>>>(err);
  LAUNCH_OK();
  k_check_points<<<cdiv(nq, TB), TB, 0, s>>>(qpos, nq, err);
  LAUNCH_OK();
  if (read_err_ptr(err, s) & 4) BF_THROW(BEMFMM_EINVAL, "non-finite charge position");
  const double sL = T.side / double(1 << T.L);
  k_gather_charges<<<cdiv(nq, TB), TB, 0, s>>>(T.qperm.p, T.qleaf.p, nq, T.cxyz.p + T.coff[T.L], T.lo[0], T.lo[1],
                                               T.lo[2], sL, qpos, q32, q64, (0.5 + 1e-3) * sL, err);
  LAUNCH_OK();
  if (read_err_ptr(err, s) & 16)
    BF_THROW(BEMFMM_EINVAL, "set_charges: a charge left its leaf cell (by more than 1/1000 of its side); rebuild the tree");
  copy_d2d(T.qpos.p, qpos, 3 * nq, s);
  copy_d2d(T.q32pos.p, q32, nq, s);
  copy_d2d(T.q64pos.p, q64, nq, s);
  HIP_OK(hipStreamSynchronize(s));
}

void set_charges(Tree &T, const double *qpos, hipStream_t s) {
  const int TB = 256;
  const int64_t nq = T.Q;
  if (nq == 0) return;
  DBuf<int> err;
  err.alloc(1);
  err.zero(s);
  DBuf<double> tmp;
  tmp.alloc(3 * nq);
  HIP_OK(hipMemcpyAsync(tmp.p, qpos, 3 * nq * sizeof(double), hipMemcpyDeviceToDevice, s));
  k_check_points<<<cdiv(nq, TB), TB, 0, s>>>(tmp.p, nq, err.p);
  LAUNCH_OK();
  if (read_err(err, s) & 4) BF_THROW(BEMFMM_EINVAL, "non-finite charge position");
  const double sL = T.side / double(1 << T.L);
  DBuf<float4> q32;
  DBuf<double4> q64;
  q32.alloc(nq);
  q64.alloc(nq);
  // a charge may leave its leaf box by 1/1000 of the side at most: the near
  // and far lists were built for points inside the leaf boxes, and this
  // keeps the MAC's separation ratio within 0.2% of its design value
  k_gather_charges<<<cdiv(nq, TB), TB, 0, s>>>(T.qperm.p, T.qleaf.p, nq, T.cxyz.p + T.coff[T.L], T.lo[0], T.lo[1],
                                               T.lo[2], sL, tmp.p, q32.p, q64.p, (0.5 + 1e-3) * sL, err.p);
  LAUNCH_OK();
  if (read_err(err, s) & 16)
    BF_THROW(BEMFMM_EINVAL, "set_charges: a charge left its leaf cell (by more than 1/1000 of its side); rebuild the tree");
  copy_d2d(T.qpos.p, tmp.p, 3 * nq, s);
  copy_d2d(T.q32pos.p, q32.p, nq, s);
  copy_d2d(T.q64pos.p, q64.p, nq, s);
  HIP_OK(hipStreamSynchronize(s));
}

}  // namespace bemfmm
