// Batched ACAT step: many independent 1D problems (own size N_b, largest
// half-width P_b, boundary, dx_b and time step dt_b; common flux) advanced
// together.  The interfaces of all problems are classified in one launch,
// grouped into per-order work lists shared by all problems, and each order
// class is one persistent launch over every problem, so the small problems
// of a batch fill the GPU together.  Per interface the arithmetic is that of
// the single-problem kernels (same rounding), so a batched step equals the
// per-problem steps bit for bit.
//
// Layout: states are SoA over the concatenated cells, u[var][coff_b + i];
// interface arrays are concatenated the same way with offsets ioff_b.
#include <hip/hip_runtime.h>

#include "acat_internal.hpp"
#include "coeffs.hpp"
#include "step_common.hpp"

namespace acat {

namespace {

constexpr int GW = BATCH_PMAX;   // indicator window half-width for every problem (offsets -3 .. 4)

template <int FLUX, int NV>
__global__ __launch_bounds__(BLOCK) void k_classify_b(KBatch bt, KBStep st) {
  const int64_t kg = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  const bool valid = kg < bt.nif;
  int ps = 1;
  if (valid) {
    const int b = bt.pif[kg];
    const int n = bt.N[b], bc = bt.bc[b];
    const int i = (int)(kg - bt.ioffs[b]) - (bc == PERIODIC ? 0 : 1);
    const double* ub = st.u + bt.coff[b];
    double v[NV][2 * GW];
#pragma unroll
    for (int a = 0; a < 2 * GW; ++a) {
      const int node = bc_index32(i - GW + 1 + a, n, bc);
#pragma unroll
      for (int c = 0; c < NV; ++c) v[c][a] = ub[c * bt.ncell + node];
    }
    ps = SelectRT<NV, GW, BATCH_PMAX>::run(v, bt.P[b], bt.eps, bt.theta);
    double psi1 = -1.0, al = -1.0;
    if (ps == 1) {
      psi1 = limiter<NV, GW>(v);
      double uL[NV], uR[NV];
#pragma unroll
      for (int c = 0; c < NV; ++c) {
        uL[c] = v[c][GW - 1];
        uR[c] = v[c][GW];
      }
      al = fmax(spectral_radius<FLUX, 1, NV>(bt.ph, uL, 0), spectral_radius<FLUX, 1, NV>(bt.ph, uR, 0));
    }
    st.ord[kg] = (int8_t)ps;
    st.psi[kg] = psi1;
    st.al[kg] = al;
  }
  __shared__ int sh[MAX_CLASSES];
  block_hist(sh, valid, ps - 1, st.hist);
}

// LDS doubles of the exchange buffers of order p at BS threads per block
template <int NV, int p, int BS>
constexpr int flux_b_lds() {
  return 2 * NV * Groups<2 * p, BS>::TOTAL * (2 * p + 1);
}

// Interfaces of order p of every problem (same arithmetic as k_flux1d), BS
// threads per block: BS / 2p interfaces per round; the block's share of the
// class list is `sl`; xsmem: the block's LDS exchange buffers
// (flux_b_lds<NV, p, BS>() doubles).
template <int FLUX, int NV, int p, int BS>
__device__ __forceinline__ void flux_b_body(const KBatch& bt, const KBStep& st, const Slice& sl, double* xsmem) {
  constexpr int L = 2 * p;
  using Grp = Groups<L, BS>;
  constexpr int GPB = Grp::PER_BLOCK;
  constexpr int SL = L + 1;
  constexpr int NS = Grp::TOTAL * SL;
  auto& xs = *reinterpret_cast<double (*)[2][NV][NS]>(xsmem);

  const Grp grp(threadIdx.x);
  const int g = grp.g;
  const int a = grp.node;
  const int slot = g * SL + a;
  const bool inblk = grp.in;

  double g1[L];
#pragma unroll
  for (int l = 0; l < L; ++l) g1[l] = TB.G1[p][a][l];

  int buf = 0;
  for (int64_t base = sl.lo; base < sl.hi; base += GPB) {
    const bool valid = inblk && base + g < sl.hi;
    const int64_t kg = valid ? sl.items[base + g] : 0;
    const int b = bt.pif[kg];
    const int n = bt.N[b], bc = bt.bc[b];
    const int i = (int)(kg - bt.ioffs[b]) - (bc == PERIODIC ? 0 : 1);
    const double* ub = st.u + bt.coff[b];
    const double lam = st.dt[b] / bt.dx[b];
    const int node = bc_index32(i + (a - p + 1), n, bc);
    double u[NV];
#pragma unroll
    for (int c = 0; c < NV; ++c) u[c] = valid ? ub[c * bt.ncell + node] : 1.0;

    double fh0[NV], cur[NV], S[NV];
    flux1d<FLUX, NV>(bt.ph, u, fh0);
#pragma unroll
    for (int c = 0; c < NV; ++c) {
      cur[c] = fh0[c];
      S[c] = fma(TB.INVFACT[1], fh0[c], 0.0);
    }
    double W[L][NV];   // Taylor predictions at the time nodes r != 0, one term per level
#pragma unroll
    for (int ri = 0; ri < L; ++ri)
#pragma unroll
      for (int c = 0; c < NV; ++c) W[ri][c] = u[c];
#pragma unroll
    for (int kk = 2; kk <= 2 * p; ++kk) {
#pragma unroll
      for (int c = 0; c < NV; ++c) xs[buf][c][slot] = cur[c];
      Grp::sync();
      double Uk[NV];
#pragma unroll
      for (int c = 0; c < NV; ++c) {
        double sacc = 0.0;
#pragma unroll
        for (int l = 0; l < L; ++l) sacc = fma(g1[l], xs[buf][c][g * SL + l], sacc);
        Uk[c] = -lam * sacc;
      }
      buf ^= 1;
#pragma unroll
      for (int ri = 0; ri < L; ++ri) {
        const int r = ri - p + 1;
        if (r == 0) continue;
#pragma unroll
        for (int c = 0; c < NV; ++c) W[ri][c] = fma(TB.TAYLOR[r + PMAX - 1][kk - 1], Uk[c], W[ri][c]);
      }
      double nxt[NV];
#pragma unroll
      for (int c = 0; c < NV; ++c) nxt[c] = 0.0;
#pragma unroll
      for (int ri = 0; ri < L; ++ri) {
        const int r = ri - p + 1;
        if (TB.GT[p][kk - 1][ri] == 0.0) continue;   // zero weight: nothing to add
        double ph[NV];
        if (r == 0) {
#pragma unroll
          for (int c = 0; c < NV; ++c) ph[c] = fh0[c];
        } else {
          flux1d<FLUX, NV>(bt.ph, W[ri], ph);
        }
#pragma unroll
        for (int c = 0; c < NV; ++c) nxt[c] = fma(TB.GT[p][kk - 1][ri], ph[c], nxt[c]);
      }
#pragma unroll
      for (int c = 0; c < NV; ++c) {
        cur[c] = nxt[c];
        S[c] = fma(TB.INVFACT[kk], nxt[c], S[c]);
      }
    }
#pragma unroll
    for (int c = 0; c < NV; ++c) xs[buf][c][slot] = S[c];
    Grp::sync();
    if (valid && a < NV) {
      for (int task = 0; task < 2; ++task) {
        const int c = a + task * L;
        if (c >= NV) break;
        double F = 0.0;
#pragma unroll
        for (int l = 0; l < L; ++l) F = fma(TB.ETA[p][l], xs[buf][c % NV][g * SL + l], F);
        if constexpr (p == 1) {
          const double psi = st.psi[kg], al = st.al[kg];
          const int nl = bc_index32(i, n, bc), nr = bc_index32(i + 1, n, bc);
          double uL[NV], uR[NV], fL[NV], fR[NV];
#pragma unroll
          for (int cc = 0; cc < NV; ++cc) {
            uL[cc] = ub[cc * bt.ncell + nl];
            uR[cc] = ub[cc * bt.ncell + nr];
          }
          flux1d<FLUX, NV>(bt.ph, uL, fL);
          flux1d<FLUX, NV>(bt.ph, uR, fR);
          double ul = 0.0, ur = 0.0, fl = 0.0, fr = 0.0;
#pragma unroll
          for (int cc = 0; cc < NV; ++cc)
            if (cc == c) {
              ul = uL[cc];
              ur = uR[cc];
              fl = fL[cc];
              fr = fR[cc];
            }
          const double flo = 0.5 * (fl + fr) - (0.5 * al) * (ur - ul);
          F = psi * F + (1.0 - psi) * flo;
        }
        st.F[c * bt.nif + kg] = F;
      }
    }
    buf ^= 1;
  }
}

template <int FLUX, int NV, int p, int BS>
__global__ __launch_bounds__(BS) void k_flux_b(KBatch bt, KBStep st) {
  __shared__ double xsmem[flux_b_lds<NV, p, BS>()];
  flux_b_body<FLUX, NV, p, BS>(bt, st, Slice(st.counts, st.list, p - 1), xsmem);
}

// Every order class in one persistent launch (256 threads per block): the
// grid is cut into runs of whole XCD groups of blocks, one run per class
// with interfaces, sized by the class's work (interfaces times the flops of
// one interface of that order); each block runs the kernel body of its
// class over its share of that class's list.  Same arithmetic per interface
// as the per-class launches.
template <int NV>
constexpr int flux_b_all_lds() {
  constexpr int a = flux_b_lds<NV, 1, BLOCK>(), b = flux_b_lds<NV, 2, BLOCK>();
  constexpr int c = flux_b_lds<NV, 3, BLOCK>(), d = flux_b_lds<NV, 4, BLOCK>();
  constexpr int ab = a > b ? a : b, cd = c > d ? c : d;
  return ab > cd ? ab : cd;
}

template <int FLUX, int NV>
__global__ __launch_bounds__(BLOCK) void k_flux_b_all(KBatch bt, KBStep st) {
  __shared__ double xsmem[flux_b_all_lds<NV>()];
  // relative cost of one interface of order p (1D Euler flops of the recursion)
  constexpr int64_t cost[BATCH_PMAX + 1] = {0, 172, 1212, 4482, 11192};
  const int units = (int)gridDim.x / NXCD;
  int64_t work[BATCH_PMAX + 1], total = 0;
  int nz = 0;
#pragma unroll
  for (int p = 1; p <= BATCH_PMAX; ++p) {
    work[p] = p <= bt.Pmax ? (int64_t)st.counts[p - 1] * cost[p] : 0;
    total += work[p];
    nz += work[p] > 0;
  }
  if (total == 0) return;
  // units per class: one each for classes with work, the rest in proportion to the work
  int u[BATCH_PMAX + 1], used = 0;
#pragma unroll
  for (int p = 1; p <= BATCH_PMAX; ++p) {
    u[p] = work[p] > 0 ? 1 + (int)((int64_t)(units - nz) * work[p] / total) : 0;
    used += u[p];
  }
  const int unit = (int)blockIdx.x / NXCD;
  if (unit >= used) return;
  int p = 1, first = 0;
  while (unit >= first + u[p]) {
    first += u[p];
    ++p;
  }
  const int blk = (int)blockIdx.x - first * NXCD, nblk = u[p] * NXCD;
  switch (p) {
    case 1: flux_b_body<FLUX, NV, 1, BLOCK>(bt, st, Slice(st.counts, st.list, 0, blk, nblk), xsmem); break;
    case 2: flux_b_body<FLUX, NV, 2, BLOCK>(bt, st, Slice(st.counts, st.list, 1, blk, nblk), xsmem); break;
    case 3: flux_b_body<FLUX, NV, 3, BLOCK>(bt, st, Slice(st.counts, st.list, 2, blk, nblk), xsmem); break;
    default: flux_b_body<FLUX, NV, 4, BLOCK>(bt, st, Slice(st.counts, st.list, 3, blk, nblk), xsmem); break;
  }
}

// A wave speed as a maximum candidate: NaN and -0 become +0, so that the bit
// pattern orders like the value under an unsigned integer maximum.
__device__ __forceinline__ double speed_floor(double m) { return m > 0.0 ? m : 0.0; }

template <int FLUX, int NV, bool CFL>
__global__ __launch_bounds__(BLOCK) void k_update_b(KBatch bt, KBStep st) {
  const int64_t e = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  const bool valid = e < bt.ncell;
  const int b = valid ? bt.pcell[e] : 0;
  double w[NV];
  if (valid) {
    const int n = bt.N[b], bc = bt.bc[b];
    const int i = (int)(e - bt.coff[b]);
    const double lam = st.dt[b] / bt.dx[b];
    const int64_t kr = bt.ioffs[b] + i + (bc == PERIODIC ? 0 : 1);
    const int64_t kl = bt.ioffs[b] + ((bc == PERIODIC) ? (i == 0 ? n - 1 : i - 1) : i);
    bool finite = true;
#pragma unroll
    for (int c = 0; c < NV; ++c) {
      w[c] = st.u[c * bt.ncell + e] + lam * (st.F[c * bt.nif + kl] - st.F[c * bt.nif + kr]);
      st.uout[c * bt.ncell + e] = w[c];
      finite = finite && isfinite(w[c]);
    }
    const uint32_t bad = (finite ? 0u : 1u) | (physical<FLUX, 1, NV>(bt.ph, w) ? 0u : 2u);
    if (bad) atomicOr(st.status, bad);
  }
  if constexpr (CFL) {
    // per-problem maximum of the new state's spectral radius (NaN and -0
    // count as +0, as in k_max_speed_b).  The lanes of a wave hold runs of
    // equal problem index: a segmented maximum over the runs, then the last
    // lane of each run stores it, with a plain store when the run is the
    // whole wave (most waves; folded per problem by k_dt_fold_b) and as an
    // atomic maximum on the bit patterns otherwise (only waves that straddle
    // problems; non-negative doubles order like their bit patterns, and max
    // is exact in any order).
    double m = valid ? speed_floor(spectral_radius<FLUX, 1, NV>(bt.ph, w, 0)) : 0.0;
    const int key = valid ? b : -1;
    const int lane = __lane_id();
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const double mo = __shfl_up(m, off);
      const int ko = __shfl_up(key, off);
      if (lane >= off && ko == key) m = fmax(m, mo);
    }
    const int key0 = __shfl(key, 0);
    const bool whole = __all(key == key0) && key0 >= 0;
    const int knext = __shfl_down(key, 1);
    if (valid && (lane == 63 || knext != key)) {
      if (whole) st.wmax[e >> 6] = m;
      else atomicMax(&st.smax[key], (unsigned long long)__double_as_longlong(m));
    }
  }
}

// smax[b] = max spectral radius over problem b: one 1024-thread block per
// problem (a few cells per thread even for the largest problems), no atomics.
constexpr int MSB_T = 1024;
template <int FLUX, int NV>
__global__ __launch_bounds__(MSB_T) void k_max_speed_b(KBatch bt, const double* __restrict__ u,
                                                      unsigned long long* smax) {
  const int b = blockIdx.x;
  const int64_t c0 = bt.coff[b], c1 = bt.coff[b + 1];
  double m = 0.0;
  for (int64_t e = c0 + threadIdx.x; e < c1; e += MSB_T) {
    double w[NV];
#pragma unroll
    for (int c = 0; c < NV; ++c) w[c] = u[c * bt.ncell + e];
    m = fmax(m, spectral_radius<FLUX, 1, NV>(bt.ph, w, 0));
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) m = fmax(m, __shfl_xor(m, off));
  __shared__ double red[MSB_T / 64];
  if (__lane_id() == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int w = 1; w < MSB_T / 64; ++w) m = fmax(m, red[w]);
    smax[b] = (unsigned long long)__double_as_longlong(speed_floor(m));
  }
}

// dt[b] = cfl dx[b] / smax[b]; smax is cleared for the next reduction
// One wave per problem: the maximum of the partial maxima of the waves whole
// inside problem b (cells coff[b] .. coff[b+1]-1) and of smax[b].
__global__ __launch_bounds__(64) void k_dt_fold_b(KBatch bt, unsigned long long* smax, const double* wmax,
                                                  double cfl, double* dt) {
  const int b = blockIdx.x;
  const int64_t w0 = (bt.coff[b] + 63) >> 6, w1 = bt.coff[b + 1] >> 6;
  double m = 0.0;
  for (int64_t v = w0 + threadIdx.x; v < w1; v += 64) m = fmax(m, wmax[v]);
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) m = fmax(m, __shfl_xor(m, off));
  if (threadIdx.x == 0) {
    m = fmax(m, __longlong_as_double((long long)smax[b]));
    dt[b] = cfl * bt.dx[b] / m;
    smax[b] = 0ull;
  }
}

__global__ void k_dt_b(KBatch bt, unsigned long long* smax, double cfl, double* dt) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < bt.nprob) {
    dt[b] = cfl * bt.dx[b] / __longlong_as_double((long long)smax[b]);
    smax[b] = 0ull;
  }
}

#define ACAT_CHECK_LAUNCH()                  \
  do {                                       \
    hipError_t e_ = hipGetLastError();       \
    if (e_ != hipSuccess) return e_;         \
  } while (0)

template <int FLUX, int NV, int p, int BS>
hipError_t launch_flux_b_bs(const KBatch& bt, const KBStep& st, hipStream_t s) {
  static const char* names[5] = {"", "flux_b_p1", "flux_b_p2", "flux_b_p3", "flux_b_p4"};
  auto kern = k_flux_b<FLUX, NV, p, BS>;
  const int grid = persistent_grid(kern, bt.nif, 0, BS, bt.per_cu[p]);
  {
    ProfScope ps(names[p], s);
    kern<<<grid, BS, 0, s>>>(bt, st);
  }
  ACAT_CHECK_LAUNCH();
  return hipSuccess;
}

// launch shape of class p from the batch's tuning table (waves per block)
template <int FLUX, int NV, int p>
hipError_t launch_flux_b(const KBatch& bt, const KBStep& st, hipStream_t s) {
  if (p > bt.Pmax) return hipSuccess;
  switch (bt.waves[p]) {
    case 1: return launch_flux_b_bs<FLUX, NV, p, 64>(bt, st, s);
    case 2: return launch_flux_b_bs<FLUX, NV, p, 128>(bt, st, s);
    default: return launch_flux_b_bs<FLUX, NV, p, 256>(bt, st, s);
  }
}

template <int FLUX, int NV>
hipError_t step_b_impl(const KBatch& bt, const KBStep& st, hipStream_t s) {
  const int cblocks = (int)((bt.nif + BLOCK - 1) / BLOCK);
  {
    ProfScope ps("classify_b", s);
    k_classify_b<FLUX, NV><<<cblocks, BLOCK, 0, s>>>(bt, st);
  }
  ACAT_CHECK_LAUNCH();
  k_scan_hist<<<bt.Pmax, SCAN_T, 0, s>>>(st.hist, cblocks, st.offs, st.counts, bt.Pmax, CflReduce{});
  ACAT_CHECK_LAUNCH();
  k_scatter<BATCH_PMAX, false><<<cblocks, BLOCK, 0, s>>>(st.ord, 1, bt.nif, 1, cblocks, st.offs, st.counts,
                                                         st.list);
  ACAT_CHECK_LAUNCH();
  hipError_t e;
  if (bt.fused_flux) {
    // one persistent launch for every order class
    auto kern = k_flux_b_all<FLUX, NV>;
    int grid = persistent_grid(kern, bt.nif, 0);
    if (grid < NXCD * BATCH_PMAX) grid = NXCD * BATCH_PMAX;   // at least one XCD group per class
    {
      ProfScope ps("flux_b_all", s);
      kern<<<grid, BLOCK, 0, s>>>(bt, st);
    }
    ACAT_CHECK_LAUNCH();
  } else {
    if ((e = launch_flux_b<FLUX, NV, 1>(bt, st, s)) != hipSuccess) return e;
    if ((e = launch_flux_b<FLUX, NV, 2>(bt, st, s)) != hipSuccess) return e;
    if ((e = launch_flux_b<FLUX, NV, 3>(bt, st, s)) != hipSuccess) return e;
    if ((e = launch_flux_b<FLUX, NV, 4>(bt, st, s)) != hipSuccess) return e;
  }
  {
    ProfScope ps("update_b", s);
    const unsigned grid = (unsigned)((bt.ncell + BLOCK - 1) / BLOCK);
    if (st.smax) k_update_b<FLUX, NV, true><<<grid, BLOCK, 0, s>>>(bt, st);
    else k_update_b<FLUX, NV, false><<<grid, BLOCK, 0, s>>>(bt, st);
  }
  ACAT_CHECK_LAUNCH();
  if (st.smax) {
    k_dt_fold_b<<<bt.nprob, 64, 0, s>>>(bt, st.smax, st.wmax, st.cfl, st.dt_next);
    ACAT_CHECK_LAUNCH();
  }
  return hipSuccess;
}

template <int FLUX, int NV>
hipError_t cfl_b_impl(const KBatch& bt, const double* u, double cfl, unsigned long long* smax, double* dt,
                      hipStream_t s) {
  {
    ProfScope ps("max_speed_b", s);
    k_max_speed_b<FLUX, NV><<<bt.nprob, MSB_T, 0, s>>>(bt, u, smax);
  }
  ACAT_CHECK_LAUNCH();
  k_dt_b<<<(bt.nprob + BLOCK - 1) / BLOCK, BLOCK, 0, s>>>(bt, smax, cfl, dt);
  ACAT_CHECK_LAUNCH();
  return hipSuccess;
}

}  // namespace

hipError_t launch_step_batched(const KBatch& bt, const KBStep& st, hipStream_t s) {
  if (bt.flux == EUL) return step_b_impl<EUL, 3>(bt, st, s);
  if (bt.flux == BURG) return step_b_impl<BURG, 1>(bt, st, s);
  return step_b_impl<ADV, 1>(bt, st, s);
}

hipError_t launch_cfl_batched(const KBatch& bt, const double* u, double cfl, unsigned long long* smax, double* dt,
                              hipStream_t s) {
  if (bt.flux == EUL) return cfl_b_impl<EUL, 3>(bt, u, cfl, smax, dt, s);
  if (bt.flux == BURG) return cfl_b_impl<BURG, 1>(bt, u, cfl, smax, dt, s);
  return cfl_b_impl<ADV, 1>(bt, u, cfl, smax, dt, s);
}

}  // namespace acat
