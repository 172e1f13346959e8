// Device helpers shared by the step kernels (single problem and batched):
// smoothness indicators, order selection, limiter, per-class work lists.
#pragma once

#include <hip/hip_runtime.h>

#include "acat_internal.hpp"
#include "coeffs.hpp"

namespace acat {
namespace {

constexpr CoeffTables TB = make_tables();
constexpr int NXCD = 8;   // MI355X: 8 accelerator complex dies, each with its own L2

// ---------------------------------------------------------------- helpers
// Quotients below use div_rn (physics.hpp): the indicator's operands are sums
// of squares plus epsilon and the limiter's are state differences, inside the
// range where it equals IEEE division.
__device__ __forceinline__ double superbee(double r) { return fmax(0.0, fmax(fmin(2.0 * r, 1.0), fmin(r, 2.0))); }

// Modified p = 2 indicator of one component (Sec. 3.2): the lateral weights
// joined with the central sub-interval on either side, the larger ratio.
template <int G>
__device__ __forceinline__ double psi2_modified(const double (&v)[2 * G], double eps) {
  const double dl = v[G - 1] - v[G - 2], dc = v[G] - v[G - 1], dr = v[G + 1] - v[G];
  double I1L = dl * dl;
  I1L += eps;
  double I1R = dc * dc;
  I1R += dr * dr;
  I1R += eps;
  double I2L = dl * dl;
  I2L += dc * dc;
  I2L += eps;
  double I2R = dr * dr;
  I2R += eps;
  const double I1 = div_rn(I1L * I1R, I1L + I1R), I2 = div_rn(I2L * I2R, I2L + I2R);
  double s = 0.0;
#pragma unroll
  for (int j = -1; j <= 2; ++j) s += TB.TAU[2][j + 1] * v[j + G - 1];
  double tau = TB.FACT2PM1[2] * s;
  tau = tau * tau;
  return fmax(div_rn(I1, I1 + tau), div_rn(I2, I2 + tau));
}

// psi^p of one component; v holds offsets -G+1 .. G (index j + G - 1).
template <int G, int p>
__device__ __forceinline__ double psi_comp(const double (&v)[2 * G], double eps) {
  double IL = 0.0, IR = 0.0;
#pragma unroll
  for (int j = -p + 1; j <= -1; ++j) {
    const double d = v[j + G] - v[j + G - 1];
    IL += d * d;
  }
#pragma unroll
  for (int j = 1; j <= p - 1; ++j) {
    const double d = v[j + G] - v[j + G - 1];
    IR += d * d;
  }
  IL += eps;
  IR += eps;
  const double I = div_rn(IL * IR, IL + IR);
  double s = 0.0;
#pragma unroll
  for (int j = -p + 1; j <= p; ++j) s += TB.TAU[p][j + p - 1] * v[j + G - 1];
  double tau = TB.FACT2PM1[p] * s;
  tau = tau * tau;
  return div_rn(I, I + tau);
}

// p_s = max{p in 2..P : min_c psi^{c,p} >= theta}, else 1 (evaluated from P down)
template <int NV, int G, int p>
struct Select {
  __device__ static __forceinline__ int run(const double (&v)[NV][2 * G], double eps, double theta,
                                            bool mod2 = false) {
    double psi = 1.0;
#pragma unroll
    for (int c = 0; c < NV; ++c)
      psi = fmin(psi, (p == 2 && mod2) ? psi2_modified<G>(v[c], eps) : psi_comp<G, p>(v[c], eps));
    if (psi >= theta) return p;
    return Select<NV, G, p - 1>::run(v, eps, theta, mod2);
  }
};
template <int NV, int G>
struct Select<NV, G, 1> {
  __device__ static __forceinline__ int run(const double (&)[NV][2 * G], double, double, bool = false) { return 1; }
};

// Scalar law: psi^1 = phi(r) with the upwind ratio chosen by the sign of
// Roe's speed a = (f(u_{i+1}) - f(u_i)) / (u_{i+1} - u_i) (f'(u_i) if equal):
// r^- if a > 0, r^+ otherwise (Sec. 3.1).
template <int FLUX, int G>
__device__ __forceinline__ double limiter_roe(const Phys& ph, const double (&v)[1][2 * G], int d) {
  const double u0 = v[0][G - 1], u1 = v[0][G];
  const double dloc = u1 - u0;
  double f0, f1, fp;
  if constexpr (FLUX == BURG) {
    f0 = 0.5 * (u0 * u0);
    f1 = 0.5 * (u1 * u1);
    fp = u0;
  } else {
    const double a = d == 0 ? ph.ax : ph.ay;
    f0 = a * u0;
    f1 = a * u1;
    fp = a;
  }
  const double a = dloc != 0.0 ? div_rn(f1 - f0, dloc) : fp;
  const double dupw = a > 0.0 ? u0 - v[0][G - 2] : v[0][G + 1] - u1;
  if (dloc == 0.0) return dupw == 0.0 ? 1.0 : 0.0;
  return superbee(div_rn(dupw, dloc));
}

// psi^1 = min_c min(phi(r+), phi(r-)); a component with u_{i+1} = u_i gives 1
template <int NV, int G>
__device__ __forceinline__ double limiter(const double (&v)[NV][2 * G]) {
  double psi = 1e300;
#pragma unroll
  for (int c = 0; c < NV; ++c) {
    const double dl = v[c][G] - v[c][G - 1];
    const double dm = v[c][G - 1] - v[c][G - 2], dp = v[c][G + 1] - v[c][G];
    // ratio undefined when the central difference vanishes: a locally
    // constant component is smooth (1), a plateau next to a variation is an
    // extremum or a corner (0)
    double l = (dm == 0.0 && dp == 0.0) ? 1.0 : 0.0;
    if (dl != 0.0) l = fmin(superbee(div_rn(dp, dl)), superbee(div_rn(dm, dl)));
    psi = fmin(psi, l);
  }
  return psi;
}

// Balanced slice of one class list: the n items of class c (spatial order)
// are cut into gridDim.x contiguous slices, and the slices of the blocks on
// XCD x (blockIdx % 8) are adjacent, so neighbouring items share that XCD's L2.
struct Slice {
  const int32_t* items;
  int64_t lo, hi;
  __device__ Slice(const int32_t* counts, const int32_t* list, int c) {
    init(counts, list, c, blockIdx.x, gridDim.x);
  }
  // block `blk` of `nblk` blocks working on class c (nblk a multiple of the
  // XCD count, and blk on XCD blk % NXCD)
  __device__ Slice(const int32_t* counts, const int32_t* list, int c, int blk, int nblk) {
    init(counts, list, c, blk, nblk);
  }
  __device__ void init(const int32_t* counts, const int32_t* list, int c, int blk, int nblk) {
    int64_t base = 0;
    for (int k = 0; k < c; ++k) base += counts[k];
    const int64_t n = counts[c];
    const int nb = nblk / NXCD;
    const int r = (blk % NXCD) * nb + blk / NXCD;
    lo = n * r / nblk;
    hi = n * (r + 1) / nblk;
    items = list + base;
  }
};

// Per-block class histogram (LDS atomics), written without global atomics.
// Block maximum of (m0, m1) (non-negative values); the result is valid in thread 0.
__device__ __forceinline__ void block_max2(double& m0, double& m1) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    m0 = fmax(m0, __shfl_xor(m0, off));
    m1 = fmax(m1, __shfl_xor(m1, off));
  }
  __shared__ double red[2][BLOCK / 64];
  if (__lane_id() == 0) {
    red[0][threadIdx.x >> 6] = m0;
    red[1][threadIdx.x >> 6] = m1;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int w = 1; w < BLOCK / 64; ++w) {
      m0 = fmax(m0, red[0][w]);
      m1 = fmax(m1, red[1][w]);
    }
  }
}

__device__ __forceinline__ void block_hist(int* sh, bool valid, int cls, int32_t* out, int cls2 = -1) {
  if (threadIdx.x < MAX_CLASSES) sh[threadIdx.x] = 0;
  __syncthreads();
  if (valid) atomicAdd(&sh[cls], 1);
  if (valid && cls2 >= 0) atomicAdd(&sh[cls2], 1);
  __syncthreads();
  if (threadIdx.x < MAX_CLASSES) out[(int64_t)blockIdx.x * MAX_CLASSES + threadIdx.x] = sh[threadIdx.x];
}

// CFL rule: 1D cfl dx / s; 2D (Sec. 5.5) cfl/2 min(dx/s_x, dy/s_y); clipped at t_final
__device__ __forceinline__ void cfl_rule(int dim, double dx, double dy, double s0, double s1, double cfl,
                                         double t_final, double* t_dev, double* dt_dev) {
  double dt = dim == 1 ? cfl * dx / s0 : 0.5 * cfl * fmin(dx / s0, dy / s1);
  if (t_dev) {
    const double t = *t_dev;
    if (t >= t_final) dt = 0.0;
    else if (t + dt > t_final) dt = t_final - t;
    *t_dev = t + dt;
  }
  *dt_dev = dt;
}

// Optional time step from per-block partial wave-speed maxima [nparts][dim].
struct CflReduce {
  const double* part;   // null: none
  int nparts, dim;
  double dx, dy, cfl, t_final;
  double* t_dev;
  double* dt_out;
};

constexpr int SCAN_T = 1024;   // threads of the class-list prefix kernel

// offs[c][t] = items of class c in tiles < t, counts[c] = total: one block per
// class, each thread summing a contiguous chunk of tiles, then a block-wide
// exclusive scan of the chunk sums.  With cr.part, block ncls reduces the
// partial maxima and writes the CFL time step.
__global__ __launch_bounds__(SCAN_T) void k_scan_hist(const int32_t* hist, int ntiles, int32_t* offs,
                                                      int32_t* counts, int ncls, CflReduce cr) {
  __shared__ int wsum[SCAN_T / 64];
  __shared__ double wmax[2][SCAN_T / 64];
  const int c = blockIdx.x, tid = threadIdx.x, lane = __lane_id(), wid = tid >> 6;
  if (c == ncls) {   // time step
    double m0 = 0.0, m1 = 0.0;
    for (int i = tid; i < cr.nparts; i += SCAN_T) {
      m0 = fmax(m0, cr.part[cr.dim * i]);
      if (cr.dim == 2) m1 = fmax(m1, cr.part[2 * i + 1]);
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
      m0 = fmax(m0, __shfl_xor(m0, off));
      m1 = fmax(m1, __shfl_xor(m1, off));
    }
    if (lane == 0) {
      wmax[0][wid] = m0;
      wmax[1][wid] = m1;
    }
    __syncthreads();
    if (tid == 0) {
      for (int w = 1; w < SCAN_T / 64; ++w) {
        m0 = fmax(m0, wmax[0][w]);
        m1 = fmax(m1, wmax[1][w]);
      }
      cfl_rule(cr.dim, cr.dx, cr.dy, m0, m1, cr.cfl, cr.t_final, cr.t_dev, cr.dt_out);
    }
    return;
  }
  const int per = (ntiles + SCAN_T - 1) / SCAN_T;
  const int t0 = tid * per;
  const int t1 = min(t0 + per, ntiles);
  int acc = 0;
  for (int t = t0; t < t1; ++t) acc += hist[(int64_t)t * MAX_CLASSES + c];
  // block-wide exclusive scan of acc: wave inclusive scan, then the wave totals
  int inc = acc;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int v = __shfl_up(inc, off);
    if (lane >= off) inc += v;
  }
  if (lane == 63) wsum[wid] = inc;
  __syncthreads();
  if (tid == 0) {
    int run = 0;
    for (int w = 0; w < SCAN_T / 64; ++w) {
      const int v = wsum[w];
      wsum[w] = run;
      run += v;
    }
    counts[c] = run;
    offs[(int64_t)c * (ntiles + 1) + ntiles] = run;
  }
  __syncthreads();
  int run = wsum[wid] + inc - acc;
  for (int t = t0; t < t1; ++t) {
    offs[(int64_t)c * (ntiles + 1) + t] = run;
    run += hist[(int64_t)t * MAX_CLASSES + c];
  }
}

// list[base_c + offs[c][tile] + rank] = item, for the item of every thread
// (rank among the tile's items of the same class, in thread order).  One
// block per tile of the classification, with the same tiles: n1 consecutive
// items (1D, n2 = 1), or a 16 x 16 patch of the n2 x n1 corner grid (TILED).
// SQUARE (2D square-stencil variant, map = pair class of order square_P): a
// corner with q1 != q2 is listed in the square classes (q1, q1), tagged F
// only, and (q2, q2), tagged G only.  No atomics, deterministic.
template <int NCLS, bool TILED, bool SQUARE = false>
__global__ __launch_bounds__(BLOCK) void k_scatter(const int8_t* map, int map_bias, int64_t n1, int64_t n2,
                                                   int ntiles, const int32_t* offs, const int32_t* counts,
                                                   int32_t* list, int square_P = 0) {
  __shared__ int wc[NCLS][BLOCK / 64];
  int64_t e;
  bool inside;
  if constexpr (TILED) {
    const int64_t ntx = (n1 + TILE_X - 1) / TILE_X;
    const int64_t e1 = (blockIdx.x % ntx) * TILE_X + threadIdx.x % TILE_X;
    const int64_t e2 = (blockIdx.x / ntx) * TILE_Y + threadIdx.x / TILE_X;
    inside = e1 < n1 && e2 < n2;
    e = e2 * n1 + e1;
  } else {
    e = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    inside = e < n1;
  }
  int c1 = inside ? map[e] - map_bias : -1;
  int c2 = -1, t1 = 0, t2 = 0;
  if (SQUARE && c1 >= 0) {
    const int a = c1 / square_P, b = c1 % square_P;   // q1 - 1, q2 - 1
    if (a != b) {
      c1 = a * square_P + a;
      t1 = 1;
      c2 = b * square_P + b;
      t2 = 2;
    }
  }
  const int lane = __lane_id(), wid = threadIdx.x >> 6;
  unsigned long long m1 = 0ull, m2 = 0ull;
#pragma unroll
  for (int k = 0; k < NCLS; ++k) {
    const unsigned long long m = __ballot(c1 == k || c2 == k);
    if (c1 == k) m1 = m;
    if (c2 == k) m2 = m;
    if (lane == 0) wc[k][wid] = __popcll(m);
  }
  __syncthreads();
  const int cs[2] = {c1, c2}, ts[2] = {t1, t2};
  const unsigned long long ms[2] = {m1, m2};
#pragma unroll
  for (int s = 0; s < (SQUARE ? 2 : 1); ++s) {
    const int c = cs[s];
    if (c < 0 || c >= NCLS) continue;
    int64_t pos = 0;
    for (int k = 0; k < c; ++k) pos += counts[k];
    pos += offs[(int64_t)c * (ntiles + 1) + blockIdx.x];
    for (int w = 0; w < wid; ++w) pos += wc[c][w];
    pos += __popcll(ms[s] & ((1ull << lane) - 1ull));
    list[pos] = (int32_t)(e | ((int64_t)ts[s] << LIST_TAG_SHIFT));
  }
}


// p_s with a run-time largest half-width P <= p (batched problems): same
// decisions as Select with P fixed, on a window of half-width G >= P.
template <int NV, int G, int p>
struct SelectRT {
  __device__ static __forceinline__ int run(const double (&v)[NV][2 * G], int P, double eps, double theta) {
    if (p <= P) {
      double psi = 1.0;
#pragma unroll
      for (int c = 0; c < NV; ++c) psi = fmin(psi, psi_comp<G, p>(v[c], eps));
      if (psi >= theta) return p;
    }
    return SelectRT<NV, G, p - 1>::run(v, P, eps, theta);
  }
};
template <int NV, int G>
struct SelectRT<NV, G, 1> {
  __device__ static __forceinline__ int run(const double (&)[NV][2 * G], int, double, double) { return 1; }
};

// ------------------------------------------------------------ host side
int num_cus() {
  static int n = 0;
  if (!n) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        n <= 0)
      n = 256;
  }
  return n;
}

// Persistent grid of a tile-walking kernel of `bs` threads per block:
// enough blocks to fill every CU at the kernel's occupancy (or `per_cu`
// blocks per CU when that is > 0; cap > 0 overrides both), never more than
// the tiles, a multiple of the XCD count.
template <typename K>
int persistent_grid(K kernel, int64_t nitems, int cap, int bs = BLOCK, int per_cu = 0) {
  if (per_cu <= 0 &&
      (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, bs, 0) != hipSuccess || per_cu < 1))
    per_cu = 1;
  int64_t b = cap > 0 ? cap : (int64_t)per_cu * num_cus();
  const int64_t ntiles = (nitems + bs - 1) / bs;
  if (b > ntiles) b = ntiles;
  b = (b + NXCD - 1) / NXCD * NXCD;
  return (int)(b < NXCD ? NXCD : b);
}

}  // namespace

// Orders a wavefront's LDS stores before its later LDS loads.  The LDS
// operations of one wave are performed in issue order, so only the compiler
// has to be kept from moving loads above stores; no hardware barrier.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Assignment of a block's lanes to groups of L lanes (a 1D interface's or a
// 2D corner's stencil nodes).  When whole groups fill a 64-lane wavefront with
// at most 1/16 of its lanes idle, groups are packed per wave: no group spans
// two waves and its LDS exchange needs only wave_sync().  Otherwise groups
// are packed densely over the block and exchange across a workgroup barrier.
// Idle lanes get a spare group of their own (per wave, or one per block), so
// their stores never touch a live group's slots.
template <int L, int BS = BLOCK>
struct Groups {
  static constexpr int WAVE = 64;
  static constexpr int GPW = WAVE / L;
  static constexpr bool WAVE_LOCAL = L <= WAVE && (WAVE - GPW * L) * 16 <= WAVE;
  static constexpr int PER_BLOCK = WAVE_LOCAL ? (BS / WAVE) * GPW : BS / L;
  static constexpr int SPARE = WAVE_LOCAL ? (WAVE % L ? BS / WAVE : 0) : 1;
  static constexpr int TOTAL = PER_BLOCK + SPARE;     // groups with LDS slots, spares included
  int g;      // group of this lane
  int node;   // node within the group
  bool in;    // false for idle lanes
  __device__ __forceinline__ explicit Groups(int tid) {
    if constexpr (WAVE_LOCAL) {
      const int w = tid / WAVE, lw = tid % WAVE;
      in = lw / L < GPW;
      g = in ? w * GPW + lw / L : PER_BLOCK + w;
      node = lw % L;
    } else {
      g = tid / L;
      node = tid - g * L;
      in = g < PER_BLOCK;
    }
  }
  static __device__ __forceinline__ void sync() {
    if constexpr (WAVE_LOCAL) {
      wave_sync();
    } else {
      __syncthreads();
    }
  }
};

// Persistent grid of a lane-per-node kernel whose blocks take PER_BLOCK
// items (groups of L lanes) per round: at most one block per PER_BLOCK of
// the nitems items the kernel's lists can hold (a round's worth each), and
// otherwise as persistent_grid.
template <int L, class K>
int group_grid(K kernel, int64_t nitems, int cap) {
  constexpr int PB = Groups<L>::PER_BLOCK;
  return persistent_grid(kernel, (nitems + PB - 1) / PB * BLOCK, cap);
}

// LDS exchange of the time-derivative fluxes of a 2D corner: per node, the
// NV components of Fh and of Gh stored as double2 pairs in component-major
// planes (consecutive lanes write consecutive 16-byte words).
//   NV = 4: planes (F0,F1) (F2,F3) (G0,G1) (G2,G3);   NV = 1: plane (F0,G0)
template <int NV>
struct Xch {
  static constexpr int NP = NV == 1 ? 1 : NV;
  static __device__ __forceinline__ void put(double2* plane0, int stride, int slot, const double (&f)[NV],
                                             const double (&g)[NV]) {
    if constexpr (NV == 1) {
      plane0[slot] = make_double2(f[0], g[0]);
    } else {
#pragma unroll
      for (int c = 0; c < NV; c += 2) {
        plane0[(c / 2) * stride + slot] = make_double2(f[c], f[c + 1]);
        plane0[(NV / 2 + c / 2) * stride + slot] = make_double2(g[c], g[c + 1]);
      }
    }
  }
  // component c of Fh (G = false) or Gh (G = true) at a slot
  static __device__ __forceinline__ double get(const double* planes, int stride, int slot, int c, bool G) {
    if constexpr (NV == 1) {
      return planes[2 * slot + (G ? 1 : 0)];
    } else {
      const int pl = (G ? NV / 2 : 0) + c / 2;
      return planes[2 * (pl * stride + slot) + (c & 1)];
    }
  }
};

}  // namespace acat
