// ACAT forward step on gfx950: classification, per-order-class flux kernels,
// conservative update, CFL reduction.
//
// Data flow of one step (all on one stream, no host synchronisation):
//   k_classify*    one thread per 1D interface / 2D corner: smoothness
//                  indicators psi^p (Sec. 3.2, minimum over components,
//                  Sec. 3.4), order p_s (Sec. 3, admissible set), and where
//                  p_s = 1 the superbee weight psi^1 (Sec. 3.1) and the
//                  Rusanov speed; writes the order (1D) or the corner's
//                  order class (2D) as one byte, and a per-block histogram
//   k_scan_hist    per-class exclusive prefix of the tile histograms (and,
//                  in CFL mode, the time step from the classification's
//                  per-block maxima)
//   k_scatter      the item lists: every class's items in tile order
//                  (wave ballots, no global atomics)
//   k_flux*<class> persistent kernels, one per order class (2D: one per
//                  square class and one per mirror pair (q1,q2) + (q2,q1)).
//                  A block takes a contiguous slice of its class's list and
//                  processes it in rounds with one LANE PER STENCIL NODE: a
//                  1D interface of order p occupies 2p lanes, a 2D corner of
//                  orders (q1, q2) 2q1 x 2q2 lanes.  Each lane keeps its
//                  node's state and Taylor predictions in registers and
//                  evaluates the flux at its own predicted states; the
//                  spatial derivatives of the time-derivative fluxes go
//                  through LDS (Sec. 2.2 recursion, Sec. 4 corner recursion)
//   k_update*      conservative flux-difference update + status bits
#include <hip/hip_runtime.h>

#include <utility>

#include "acat_internal.hpp"
#include "coeffs.hpp"
#include "step_common.hpp"

namespace acat {
namespace {

__global__ void k_zero_u64(unsigned long long* p, int n) {
  const int t = threadIdx.x;
  if (t < n) p[t] = 0ull;
}

// ======================================================================= 1D
template <int FLUX, int NV, int P>
__global__ __launch_bounds__(BLOCK) void k_classify1d(KProb pb, KStep st) {
  constexpr int G = P > 2 ? P : 2;
  const int64_t k = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  const bool valid = k < pb.nIx;
  int ps = 1;
  double smax = 0.0;
  if (valid) {
    if (st.replay) {
      ps = st.ordx[k];
      if (ps < 1 || ps > P) {   // invalid recorded order: fall back to 1, flag it
        ps = 1;
        atomicOr(st.status, 4u);
      }
    } else {
      const int64_t i = k + pb.ioff;
      double v[NV][2 * G];
#pragma unroll
      for (int a = 0; a < 2 * G; ++a) {
        const int64_t node = bc_index(i - G + 1 + a, pb.nx, pb.bc);
#pragma unroll
        for (int c = 0; c < NV; ++c) v[c][a] = st.u[c * pb.nx + node];
      }
      if (st.cfl_mode) {   // the cell of node 0 (every cell is node 0 of one interface)
        double uc[NV];
#pragma unroll
        for (int c = 0; c < NV; ++c) uc[c] = v[c][G - 1];
        smax = spectral_radius<FLUX, 1, NV>(pb.ph, uc, 0);
      }
      ps = Select<NV, G, P>::run(v, pb.eps, pb.theta, (pb.flags & FLAG_PSI2_MODIFIED) != 0);
      double psi1 = -1.0, al = -1.0;
      if (ps == 1) {
        psi1 = limiter<NV, G>(v);
        if constexpr (NV == 1) {
          if (pb.flags & FLAG_PSI1_ROE) psi1 = limiter_roe<FLUX, G>(pb.ph, v, 0);
        }
        double uL[NV], uR[NV];
#pragma unroll
        for (int c = 0; c < NV; ++c) {
          uL[c] = v[c][G - 1];
          uR[c] = v[c][G];
        }
        al = fmax(spectral_radius<FLUX, 1, NV>(pb.ph, uL, 0), spectral_radius<FLUX, 1, NV>(pb.ph, uR, 0));
      }
      st.ordx[k] = (int8_t)ps;
      st.psix[k] = psi1;
      st.alx[k] = al;
    }
  }
  if (valid) st.cls[k] = (int8_t)(ps - 1);
  __shared__ int sh[MAX_CLASSES];
  block_hist(sh, valid, ps - 1, st.hist);
  if (st.cfl_mode) {
    double dummy = 0.0;
    block_max2(smax, dummy);
    if (threadIdx.x == 0) st.part[blockIdx.x] = smax;
  }
}

// CAT2p flux of the interfaces of order p (p = 1: FL-CAT2 blend).
// Rounding follows one fixed order: every weighted sum of the recursion is a
// chain of fused multiply-adds in index order, nothing else is contracted
// (the library is built with -ffp-contract=off).
template <int FLUX, int NV, int p>
__global__ __launch_bounds__(BLOCK) void k_flux1d(KProb pb, KStep st) {
  constexpr int L = 2 * p;            // lanes per interface = stencil nodes
  using Grp = Groups<L>;
  constexpr int GPB = Grp::PER_BLOCK; // interfaces per round
  constexpr int SL = L + 1;           // LDS slots per interface (one pad slot against bank conflicts)
  constexpr int NS = Grp::TOTAL * SL; // slots per component, idle lanes included
  __shared__ double xs[2][NV][NS];

  const Grp grp(threadIdx.x);
  const int g = grp.g;
  const int a = grp.node;             // node index, offset j = a - p + 1
  const int slot = g * SL + a;
  const bool inblk = grp.in;
  const double lam = step_dt(st) / pb.dx;
  const int64_t nx = pb.nx, nI = pb.nIx;

  double g1[L];
#pragma unroll
  for (int l = 0; l < L; ++l) g1[l] = TB.G1[p][a][l];

  int buf = 0;
  const Slice sl(st.counts, st.list, p - 1);
  for (int64_t base = sl.lo; base < sl.hi; base += GPB) {
    {
      const bool valid = inblk && base + g < sl.hi;
      const int32_t k = valid ? sl.items[base + g] : 0;
      const int i = k + (int)pb.ioff;
      const int node = bc_index32(i + (a - p + 1), (int)nx, pb.bc);
      double u[NV];
#pragma unroll
      for (int c = 0; c < NV; ++c) u[c] = valid ? st.u[c * nx + node] : 1.0;

      double fh0[NV], cur[NV], S[NV];
      flux1d<FLUX, NV>(pb.ph, u, fh0);
      // S = sum_k Fh^{k-1} / k! at this node (the CAT flux, Sec. 2.2, summed node by node)
#pragma unroll
      for (int c = 0; c < NV; ++c) {
        cur[c] = fh0[c];
        S[c] = fma(TB.INVFACT[1], fh0[c], 0.0);
      }
      // Taylor predictions W_r = u + sum_{l<kk} r^l/l! U^l, U^l = dt^l u~^(l), at the
      // time nodes r != 0, one term added per level (same fma chain as summing from u)
      double W[L][NV];
#pragma unroll
      for (int ri = 0; ri < L; ++ri)
#pragma unroll
        for (int c = 0; c < NV; ++c) W[ri][c] = u[c];
#pragma unroll
      for (int kk = 2; kk <= 2 * p; ++kk) {
        // share Fh^{kk-2} of every node of the stencil
#pragma unroll
        for (int c = 0; c < NV; ++c) xs[buf][c][slot] = cur[c];
        Grp::sync();
        // U^{kk-1} = -lambda * (spatial derivative of Fh^{kk-2} at this node)
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
        // flux at the Taylor-predicted states of the time nodes r, and its
        // (kk-1)-th time derivative at r = 0
        double nxt[NV];
#pragma unroll
        for (int c = 0; c < NV; ++c) nxt[c] = 0.0;
#pragma unroll
        for (int ri = 0; ri < L; ++ri) {
          const int r = ri - p + 1;
          // a time node whose weight is exactly zero adds nothing: its flux
          // is not evaluated (the same sum for finite values)
          if (TB.GT[p][kk - 1][ri] == 0.0) continue;
          double ph[NV];
          if (r == 0) {
#pragma unroll
            for (int c = 0; c < NV; ++c) ph[c] = fh0[c];
          } else {
            flux1d<FLUX, NV>(pb.ph, W[ri], ph);
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
      // F_c = sum_j eta_j S_j,c on lane a = c (and a + L when NV > L)
#pragma unroll
      for (int c = 0; c < NV; ++c) xs[buf][c][slot] = S[c];
      Grp::sync();
      double F0 = 0.0, F1 = 0.0;
      if (valid && a < NV) {
#pragma unroll
        for (int l = 0; l < L; ++l) F0 = fma(TB.ETA[p][l], xs[buf][a][g * SL + l], F0);
        if (NV > L && a + L < NV) {
#pragma unroll
          for (int l = 0; l < L; ++l) F1 = fma(TB.ETA[p][l], xs[buf][(a + L) % NV][g * SL + l], F1);
        }
      }
      buf ^= 1;   // the assembly above may still read this buffer
      if (valid && a < NV) {
        for (int task = 0; task < 2; ++task) {
          const int c = a + task * L;
          if (c >= NV) break;
          double F = task == 0 ? F0 : F1;
          if constexpr (p == 1) {
            // FL-CAT2 (Sec. 3.1): psi^1 CAT2 + (1 - psi^1) Rusanov
            const double psi = st.psix[k], al = st.alx[k];
            const int64_t nl = bc_index32(i, (int)nx, pb.bc), nr = bc_index32(i + 1, (int)nx, pb.bc);
            double uL[NV], uR[NV], fL[NV], fR[NV];
#pragma unroll
            for (int cc = 0; cc < NV; ++cc) {
              uL[cc] = st.u[cc * nx + nl];
              uR[cc] = st.u[cc * nx + nr];
            }
            flux1d<FLUX, NV>(pb.ph, uL, fL);
            flux1d<FLUX, NV>(pb.ph, uR, fR);
            double ul = 0.0, ur = 0.0, fl = 0.0, fr = 0.0;
#pragma unroll
            for (int cc = 0; cc < NV; ++cc)
              if (cc == c) { ul = uL[cc]; ur = uR[cc]; fl = fL[cc]; fr = fR[cc]; }
            const double alf = pb.dx / ((double)pb.dim * step_dt(st));
            const double flo = lo_flux<FLUX, 1, NV>(pb.ph, pb.flags, 0, uL, uR, fl, fr, ul, ur, al, alf);
            F = psi * F + (1.0 - psi) * flo;
          }
          st.Fx[c * nI + k] = F;
        }
      }
    }
  }
}

template <int FLUX, int NV>
__global__ __launch_bounds__(BLOCK) void k_update1d(KProb pb, KStep st) {
  const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (i >= pb.nx) return;
  const double lam = step_dt(st) / pb.dx;
  const int64_t kr = i - pb.ioff;
  const int64_t kl = (pb.bc == PERIODIC) ? (i == 0 ? pb.nx - 1 : i - 1) : i;
  double w[NV];
  bool finite = true;
#pragma unroll
  for (int c = 0; c < NV; ++c) {
    w[c] = st.u[c * pb.nx + i] + lam * (st.Fx[c * pb.nIx + kl] - st.Fx[c * pb.nIx + kr]);
    st.uout[c * pb.nx + i] = w[c];
    finite = finite && isfinite(w[c]);
  }
  uint32_t bad = (finite ? 0u : 1u) | (physical<FLUX, 1, NV>(pb.ph, w) ? 0u : 2u);
  if (bad) atomicOr(st.status, bad);
}

// ======================================================================= 2D
// One block per 16 x 16 tile of corners, one thread per corner.  The cells
// the tile's x- and y-stencils read (the tile and a halo of G - 1 below and
// G beyond it in each direction) are staged in LDS once per block.
template <int FLUX, int NV, int P>
__global__ __launch_bounds__(BLOCK) void k_classify2d(KProb pb, KStep st) {
  constexpr int G = P > 2 ? P : 2;
  constexpr int TW = TILE_X + 2 * G - 1, TH = TILE_Y + 2 * G - 1;
  static_assert(TILE_X * TILE_Y == BLOCK, "one thread per corner of the tile");
  __shared__ double tile[NV][TH][TW];
  const int64_t ntx = (pb.n1 + TILE_X - 1) / TILE_X;
  const int tx = threadIdx.x % TILE_X, ty = threadIdx.x / TILE_X;
  const int64_t e1 = (blockIdx.x % ntx) * TILE_X + tx;
  const int64_t e2 = (blockIdx.x / ntx) * TILE_Y + ty;
  const bool inside = e1 < pb.n1 && e2 < pb.n2;
  const int64_t e = e2 * pb.n1 + e1;
  const int64_t nx = pb.nx, ny = pb.ny;
  const int64_t i1 = inside ? e1 + pb.ioff : 0;
  const int64_t i2 = inside ? e2 + pb.ioff : 0;
  const bool needF = i2 >= 0, needG = i1 >= 0;
  const bool valid = inside && (needF || needG);
  if (!st.replay) {
    // tile cell (a, b) is cell (Y0 + a, X0 + b) before the boundary mapping;
    // cells beyond what the grid's last corner reads are not loaded (so the
    // periodic wrap stays within one period)
    const int64_t X0 = (blockIdx.x % ntx) * TILE_X + pb.ioff - G + 1;
    const int64_t Y0 = (blockIdx.x / ntx) * TILE_Y + pb.ioff - G + 1;
    const int64_t Xmax = pb.n1 - 1 + pb.ioff + G, Ymax = pb.n2 - 1 + pb.ioff + G;
    for (int t = threadIdx.x; t < TH * TW; t += BLOCK) {
      const int a = t / TW, b = t - a * TW;
      if (X0 + b <= Xmax && Y0 + a <= Ymax) {
        const int64_t x = bc_index(X0 + b, nx, pb.bc), y = bc_index(Y0 + a, ny, pb.bc);
#pragma unroll
        for (int c = 0; c < NV; ++c) tile[c][a][b] = st.u[(c * ny + y) * nx + x];
      }
    }
    __syncthreads();
  }
  int q1 = 1, q2 = 1;
  double sx = 0.0, sy = 0.0;
  if (valid) {
    const int64_t r2 = bc_index(i2, ny, pb.bc);   // ghost rows read the clamped row
    const int64_t r1 = bc_index(i1, nx, pb.bc);
    if (st.replay) {
      q1 = st.ordx[r2 * pb.nIx + (i1 - pb.ioff)];
      q2 = st.ordy[(i2 - pb.ioff) * nx + r1];
      if (q1 < 1 || q1 > P || q2 < 1 || q2 > P) {   // invalid recorded order: fall back to 1, flag it
        q1 = (q1 < 1 || q1 > P) ? 1 : q1;
        q2 = (q2 < 1 || q2 > P) ? 1 : q2;
        atomicOr(st.status, 4u);
      }
    } else {
      double v[NV][2 * G];
      // x-interface (i1 + 1/2, i2): cells (i2, i1 - G + 1 .. i1 + G)
#pragma unroll
      for (int a = 0; a < 2 * G; ++a)
#pragma unroll
        for (int c = 0; c < NV; ++c) v[c][a] = tile[c][ty + G - 1][tx + a];
      if (st.cfl_mode) {   // the corner's own cell (every cell is the cell of one corner)
        double uc[NV];
#pragma unroll
        for (int c = 0; c < NV; ++c) uc[c] = v[c][G - 1];
        sx = spectral_radius<FLUX, 2, NV>(pb.ph, uc, 0);
        sy = spectral_radius<FLUX, 2, NV>(pb.ph, uc, 1);
      }
      q1 = Select<NV, G, P>::run(v, pb.eps, pb.theta, (pb.flags & FLAG_PSI2_MODIFIED) != 0);
      if (needF) {
        double psi1 = -1.0, al = -1.0;
        if (q1 == 1) {
          psi1 = limiter<NV, G>(v);
          if constexpr (NV == 1) {
            if (pb.flags & FLAG_PSI1_ROE) psi1 = limiter_roe<FLUX, G>(pb.ph, v, 0);
          }
          double uL[NV], uR[NV];
#pragma unroll
          for (int c = 0; c < NV; ++c) {
            uL[c] = v[c][G - 1];
            uR[c] = v[c][G];
          }
          al = fmax(spectral_radius<FLUX, 2, NV>(pb.ph, uL, 0), spectral_radius<FLUX, 2, NV>(pb.ph, uR, 0));
        }
        const int64_t ex = i2 * pb.nIx + (i1 - pb.ioff);
        st.ordx[ex] = (int8_t)q1;
        st.psix[ex] = psi1;
        st.alx[ex] = al;
      }
      // y-interface (i1, i2 + 1/2): cells (i2 - G + 1 .. i2 + G, i1)
#pragma unroll
      for (int a = 0; a < 2 * G; ++a)
#pragma unroll
        for (int c = 0; c < NV; ++c) v[c][a] = tile[c][ty + a][tx + G - 1];
      q2 = Select<NV, G, P>::run(v, pb.eps, pb.theta, (pb.flags & FLAG_PSI2_MODIFIED) != 0);
      if (needG) {
        double psi1 = -1.0, al = -1.0;
        if (q2 == 1) {
          psi1 = limiter<NV, G>(v);
          if constexpr (NV == 1) {
            if (pb.flags & FLAG_PSI1_ROE) psi1 = limiter_roe<FLUX, G>(pb.ph, v, 1);
          }
          double uL[NV], uR[NV];
#pragma unroll
          for (int c = 0; c < NV; ++c) {
            uL[c] = v[c][G - 1];
            uR[c] = v[c][G];
          }
          al = fmax(spectral_radius<FLUX, 2, NV>(pb.ph, uL, 1), spectral_radius<FLUX, 2, NV>(pb.ph, uR, 1));
        }
        const int64_t ey = (i2 - pb.ioff) * nx + i1;
        st.ordy[ey] = (int8_t)q2;
        st.psiy[ey] = psi1;
        st.aly[ey] = al;
      }
    }
  }
  const int cls = (q1 - 1) * P + (q2 - 1);
  if (inside) st.cls[e] = valid ? (int8_t)cls : (int8_t)-1;
  // square-stencil variant: F in class (q1, q1), G in (q2, q2)
  const bool split = (pb.flags & FLAG_SQUARE_2D) && q1 != q2;
  __shared__ int sh[MAX_CLASSES];
  block_hist(sh, valid, split ? (q1 - 1) * P + (q1 - 1) : cls, st.hist, split ? (q2 - 1) * P + (q2 - 1) : -1);
  if (st.cfl_mode) {
    block_max2(sx, sy);
    if (threadIdx.x == 0) {
      st.part[2 * blockIdx.x] = sx;
      st.part[2 * blockIdx.x + 1] = sy;
    }
  }
}

// f(integral_constant<int, k>) for k = 2, 3, ... in order (the recursion
// levels, each compiled with its own constant k)
template <class F, int... K>
__device__ __forceinline__ void for_levels(F&& f, std::integer_sequence<int, K...>) {
  (f(std::integral_constant<int, K + 2>{}), ...);
}

// One recursion over the rectangle J_Q1 x J_Q2 with time nodes J_QT
// (Taylor order 2 QT).  Each lane is one node (a1, a2) and accumulates the
// series SF = sum_k Fh^{k-1} / k! (DOF) and SG = sum_k Gh^{k-1} / k! (DOG)
// of its node; the fluxes are the eta-weighted sums of SF over row j2 = 0
// and of SG over column j1 = 0.  Same fixed rounding as the 1D kernel.
// g1x, g1y: this node's derivative weights times -lamx and -lamy.
template <int FLUX, int NV, int Q1, int Q2, int QT, bool DOF, bool DOG>
__device__ __forceinline__ void corner_pass(const Phys& ph, const double (&u)[NV],
                                            const double (&f0)[NV], const double (&g0)[NV],
                                            const double* g1x, const double* g1y,
                                            double2* xsb0, double2* xsb1, int stride, int& buf, int slot,
                                            int gbase, int a1, int a2, double (&SF)[NV], double (&SG)[NV]) {
  constexpr int N1 = 2 * Q1;
  constexpr int N2 = 2 * Q2;
  double fc[NV], gc[NV];
#pragma unroll
  for (int c = 0; c < NV; ++c) {
    fc[c] = f0[c];
    gc[c] = g0[c];
    if (DOF) SF[c] = fma(TB.INVFACT[1], f0[c], 0.0);
    if (DOG) SG[c] = fma(TB.INVFACT[1], g0[c], 0.0);
  }
  // Taylor predictions W_r = u + sum_{l<kk} r^l/l! U^l at the time nodes r != 0,
  // extended by one term per level (the same chain of fused multiply-adds as
  // summing from u each level)
  // the row derivative weights of this node in registers for the pass; the
  // column weights too in the order-8 square class (two waves per SIMD with
  // or without them), elsewhere read from LDS at each use (held, they would
  // cost the order-6 square class its third wave per SIMD; the order-4 one
  // ran slower)
  constexpr bool WYR = Q1 == 4 && Q2 == 4;
  double wx[N1], wy[WYR ? N2 : 1];
#pragma unroll
  for (int l = 0; l < N1; ++l) wx[l] = g1x[l];
#pragma unroll
  for (int l = 0; l < (WYR ? N2 : 1); ++l) wy[l] = WYR ? g1y[l] : 0.0;
  double W[2 * QT][NV];
#pragma unroll
  for (int ri = 0; ri < 2 * QT; ++ri)
#pragma unroll
    for (int c = 0; c < NV; ++c) W[ri][c] = u[c];
  // one recursion level: exchange Fh^{kk-2}, Gh^{kk-2}; U^{kk-1}; predictions;
  // Fh^{kk-1}, Gh^{kk-1} and their series terms (each level compiled with
  // its own constant kk)
  auto level = [&](auto kkc) {
    constexpr int kk = decltype(kkc)::value;
    double2* xsw = buf ? xsb1 : xsb0;
    Xch<NV>::put(xsw, stride, slot, fc, gc);
    Groups<(2 * Q1) * (2 * Q2)>::sync();
    buf ^= 1;
    const double* xr = reinterpret_cast<const double*>(xsw);
    // U^{kk-1} = -lamx d_x Fh^{kk-2} - lamy d_y Gh^{kk-2} at this node: one
    // chain of fused multiply-adds over the row (x) and then the column (y)
    double Uk[NV];
#pragma unroll
    for (int c = 0; c < NV; ++c) {
      double s = 0.0;
#pragma unroll
      for (int l = 0; l < N1; ++l) s = fma(wx[l], Xch<NV>::get(xr, stride, gbase + a2 * N1 + l, c, false), s);
#pragma unroll
      for (int l = 0; l < N2; ++l)
        s = fma(WYR ? wy[WYR ? l : 0] : g1y[l], Xch<NV>::get(xr, stride, gbase + l * N1 + a1, c, true), s);
      Uk[c] = s;
    }
#pragma unroll
    for (int ri = 0; ri < 2 * QT; ++ri) {
      const int r = ri - QT + 1;
      if (r == 0) continue;
#pragma unroll
      for (int c = 0; c < NV; ++c) W[ri][c] = fma(TB.TAYLOR[r + PMAX - 1][kk - 1], Uk[c], W[ri][c]);
    }
    double nf[NV], ng[NV];
#pragma unroll
    for (int c = 0; c < NV; ++c) {
      nf[c] = 0.0;
      ng[c] = 0.0;
    }
    // Euler: the reciprocal densities of all predicted states first, their
    // Newton steps interleaved (time node r = 0 is the node state: its flux
    // is f0, g0)
    double rho[2 * QT - 1], ir[2 * QT - 1];
    if constexpr (FLUX == EUL) {
#pragma unroll
      for (int ri = 0; ri < 2 * QT; ++ri)
        if (ri != QT - 1) rho[ri < QT - 1 ? ri : ri - 1] = W[ri][0];
      recip_n(rho, ir);
    }
#pragma unroll
    for (int ri = 0; ri < 2 * QT; ++ri) {
      const int r = ri - QT + 1;
      // a time node whose weight is exactly zero adds nothing to Fh, Gh: its
      // fluxes (and reciprocal density) are not evaluated (the same sums
      // for finite values)
      if (TB.GT[QT][kk - 1][ri] == 0.0) continue;
      double pf[NV], pg[NV];
      if (r == 0) {
#pragma unroll
        for (int c = 0; c < NV; ++c) {
          pf[c] = f0[c];
          pg[c] = g0[c];
        }
      } else if constexpr (FLUX == EUL) {
        euler2d_ir(ph, W[ri], ir[ri < QT - 1 ? ri : ri - 1], pf, pg);
      } else {
        flux2d<FLUX, NV>(ph, W[ri], pf, pg);
      }
#pragma unroll
      for (int c = 0; c < NV; ++c) {
        nf[c] = fma(TB.GT[QT][kk - 1][ri], pf[c], nf[c]);
        ng[c] = fma(TB.GT[QT][kk - 1][ri], pg[c], ng[c]);
      }
    }
#pragma unroll
    for (int c = 0; c < NV; ++c) {
      fc[c] = nf[c];
      gc[c] = ng[c];
      if (DOF) SF[c] = fma(TB.INVFACT[kk], nf[c], SF[c]);
      if (DOG) SG[c] = fma(TB.INVFACT[kk], ng[c], SG[c]);
    }
  };
  for_levels(level, std::make_integer_sequence<int, 2 * QT - 1>{});
}

// Exchange slots of a group of L = (2 q1)(2 q2) corner nodes: node (a1, a2)
// of group g at g GS + a2 (2 q1) + a1.  Groups of 36 nodes (class (3, 3))
// start 38 slots apart: 36 apart, the first rows of two groups that share a
// 16-lane phase of a 128-bit LDS access fall on the same banks.
template <int L>
constexpr int corner_group_stride() {
  return L == 36 ? L + 2 : L;
}

// slots per exchange plane (spare groups of idle lanes included)
template <int L>
constexpr int corner_stride() {
  return Groups<L>::TOTAL * corner_group_stride<L>();
}

// Fluxes of the corners of order class (Q1, Q2) (Sec. 4; rectangle J_Q1 x J_Q2)
// in the block's share `sl` of the class list; every class but (1,1), which
// runs one lane per corner (k_flux2d_q11).  SQUARE: list entries carry
// the square-stencil variant's tags (square classes only).  xsm: the two
// exchange buffers (2 Xch<NV>::NP corner_stride<L>() double2), g1s: the
// derivative weights ((2 Q1)^2 + (2 Q2)^2 doubles), both in LDS.
template <int FLUX, int NV, int Q1, int Q2, bool SQUARE>
__device__ __forceinline__ void flux2d_body(const KProb& pb, const KStep& st, const Slice& sl, double2* xsm,
                                            double* g1s) {
  static_assert(Q1 > 1 || Q2 > 1, "class (1,1) runs in k_flux2d_q11");
  constexpr int N1 = 2 * Q1, N2 = 2 * Q2, L = N1 * N2;
  using Grp = Groups<L>;
  constexpr int CPB = Grp::PER_BLOCK;
  constexpr int NP = Xch<NV>::NP;
  constexpr int STRIDE = corner_stride<L>();
  constexpr int GS = corner_group_stride<L>();
  double2* const xs[2] = {xsm, xsm + NP * STRIDE};

  const int tid = threadIdx.x;
  const Grp grp(tid);
  const int g = grp.g;
  const int nd = grp.node;
  const int a1 = nd % N1, a2 = nd / N1;     // node (j1, j2) = (a1 - Q1 + 1, a2 - Q2 + 1)
  const bool inblk = grp.in;
  const double dt = step_dt(st);
  const double lamx = dt / pb.dx, lamy = dt / pb.dy;
  const int64_t nx = pb.nx, ny = pb.ny, plane = pb.nx * pb.ny;
  const int nx32 = (int)pb.nx, ny32 = (int)pb.ny, ioff = (int)pb.ioff;
  const uint32_t n1u = (uint32_t)pb.n1;

  // derivative weights times -lamx (rows) and -lamy (columns), in LDS (the
  // corner pass holds a node's row weights in registers and reads its column
  // weights at each use)
  for (int i = tid; i < N1 * N1 + N2 * N2; i += BLOCK)
    g1s[i] = i < N1 * N1 ? -lamx * TB.G1[Q1][i / N1][i % N1]
                         : -lamy * TB.G1[Q2][(i - N1 * N1) / N2][(i - N1 * N1) % N2];
  __syncthreads();
  const double* g1x = g1s + a1 * N1;
  const double* g1y = g1s + N1 * N1 + a2 * N2;

  int buf = 0;
  for (int64_t base = sl.lo; base < sl.hi; base += CPB) {
    {
      const bool valid = inblk && base + g < sl.hi;
      const int32_t raw = valid ? sl.items[base + g] : 0;
      // square-stencil variant: entries carry which flux to store (1 F, 2 G, 0 both)
      const int32_t e = SQUARE ? (raw & ((1 << LIST_TAG_SHIFT) - 1)) : raw;
      const int tag = SQUARE ? (raw >> LIST_TAG_SHIFT) : 0;
      const uint32_t eq = (uint32_t)e / n1u;
      const int i2 = (int)eq + ioff, i1 = (int)((uint32_t)e - eq * n1u) + ioff;
      const int x = bc_index32(i1 + (a1 - Q1 + 1), nx32, pb.bc);
      const int y = bc_index32(i2 + (a2 - Q2 + 1), ny32, pb.bc);
      const double* un = st.u + ((int64_t)y * nx + x);
      double u[NV];
#pragma unroll
      for (int c = 0; c < NV; ++c) u[c] = valid ? un[c * plane] : 1.0;
      double f0[NV], g0[NV];
      flux2d<FLUX, NV>(pb.ph, u, f0, g0);
      double SF[NV], SG[NV];
      const int slot = g * GS + nd;
      if constexpr (Q1 == Q2) {
        corner_pass<FLUX, NV, Q1, Q2, Q1, true, true>(pb.ph, u, f0, g0, g1x, g1y, xs[0], xs[1],
                                                      STRIDE, buf, slot, g * GS, a1, a2, SF, SG);
      } else {
        corner_pass<FLUX, NV, Q1, Q2, Q1, true, false>(pb.ph, u, f0, g0, g1x, g1y, xs[0], xs[1],
                                                       STRIDE, buf, slot, g * GS, a1, a2, SF, SG);
        corner_pass<FLUX, NV, Q1, Q2, Q2, false, true>(pb.ph, u, f0, g0, g1x, g1y, xs[0], xs[1],
                                                       STRIDE, buf, slot, g * GS, a1, a2, SF, SG);
      }
      // F_c = sum_l eta_l SF_(l,0),c and G_c = sum_l eta_l SG_(0,l),c on 2 NV lanes
      {
        double2* xsw = buf ? xs[1] : xs[0];
        Xch<NV>::put(xsw, STRIDE, slot, SF, SG);
        Grp::sync();
      }
      const double* xr = reinterpret_cast<const double*>(buf ? xs[1] : xs[0]);
      double acc[2] = {0.0, 0.0};
#pragma unroll
      for (int tk = 0; tk < 2; ++tk) {
        const int task = nd + tk * L;
        if (!valid || task >= 2 * NV) continue;
        const bool isG = task >= NV;
        const int c = isG ? task - NV : task;
        double t = 0.0;
        if (!isG) {
#pragma unroll
          for (int l = 0; l < N1; ++l) t = fma(TB.ETA[Q1][l], Xch<NV>::get(xr, STRIDE, g * GS + (Q2 - 1) * N1 + l, c, false), t);
        } else {
#pragma unroll
          for (int l = 0; l < N2; ++l) t = fma(TB.ETA[Q2][l], Xch<NV>::get(xr, STRIDE, g * GS + l * N1 + (Q1 - 1), c, true), t);
        }
        acc[tk] = t;
      }
      buf ^= 1;   // the assembly may still read this buffer
      // finish and store the assembled components
#pragma unroll
      for (int tk = 0; tk < 2; ++tk) {
        const int task = nd + tk * L;
        if (!valid || task >= 2 * NV) continue;
        const bool isG = task >= NV;
        const int c = isG ? task - NV : task;
        // transmissive ghost corners need one flux only; tagged entries one flux each
        const bool need = isG ? (i1 >= 0 && tag != 1) : (i2 >= 0 && tag != 2);
        if (!need) continue;
        double v = acc[tk];
        if ((!isG && Q1 == 1) || (isG && Q2 == 1)) {
          // 2D FL-CAT2 (Sec. 4): psi^1 CAT2 + (1 - psi^1) Rusanov in this direction
          const int64_t x0 = bc_index32(i1, nx32, pb.bc), y0 = bc_index32(i2, ny32, pb.bc);
          const int64_t xr = isG ? x0 : bc_index32(i1 + 1, nx32, pb.bc);
          const int64_t yr = isG ? bc_index32(i2 + 1, ny32, pb.bc) : y0;
          const int64_t ei = isG ? (int64_t)(i2 - ioff) * nx + i1 : (int64_t)i2 * pb.nIx + (i1 - ioff);
          const double psi = isG ? st.psiy[ei] : st.psix[ei];
          const double al = isG ? st.aly[ei] : st.alx[ei];
          double uL[NV], uR[NV], fL[NV], gL[NV], fR[NV], gR[NV];
#pragma unroll
          for (int cc = 0; cc < NV; ++cc) {
            uL[cc] = st.u[(cc * ny + y0) * nx + x0];
            uR[cc] = st.u[(cc * ny + yr) * nx + xr];
          }
          flux2d<FLUX, NV>(pb.ph, uL, fL, gL);
          flux2d<FLUX, NV>(pb.ph, uR, fR, gR);
          double ul = 0.0, ur = 0.0, hl = 0.0, hr = 0.0;
#pragma unroll
          for (int cc = 0; cc < NV; ++cc)
            if (cc == c) {
              ul = uL[cc];
              ur = uR[cc];
              hl = isG ? gL[cc] : fL[cc];
              hr = isG ? gR[cc] : fR[cc];
            }
          const double alf = (isG ? pb.dy : pb.dx) / ((double)pb.dim * dt);
          const double lo = lo_flux<FLUX, 2, NV>(pb.ph, pb.flags, isG ? 1 : 0, uL, uR, hl, hr, ul, ur, al, alf);
          v = psi * v + (1.0 - psi) * lo;
        }
        if (isG) st.Gy[((int64_t)c * pb.nIy + (i2 - ioff)) * nx + i1] = v;
        else st.Fx[((int64_t)c * ny + i2) * pb.nIx + (i1 - ioff)] = v;
      }
    }
  }
}


template <int FLUX, int NV, int Q1, int Q2, bool SQUARE = false>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(2))) void k_flux2d(KProb pb, KStep st) {
  constexpr int L = (2 * Q1) * (2 * Q2);
  __shared__ double2 xsm[2 * Xch<NV>::NP * corner_stride<L>()];
  __shared__ double g1s[(2 * Q1) * (2 * Q1) + (2 * Q2) * (2 * Q2)];
  flux2d_body<FLUX, NV, Q1, Q2, SQUARE>(pb, st, Slice(st.counts, st.list, (Q1 - 1) * pb.P + (Q2 - 1)), xsm, g1s);
}

// Order class (1,1) with ONE LANE PER CORNER.  The corner's four nodes
// (j1, j2) in {0,1}^2 (cells (i1 + j1, i2 + j2)) live in one lane, which
// computes, with the same operations in the same order as the node-per-lane
// kernel, just the quantities the corner's fluxes read (Sec. 4 with
// q1 = q2 = 1: one recursion level): the point fluxes at the four nodes, U^1
// at the three nodes of row j2 = 0 and column j1 = 0, the flux at their
// Taylor predictions, the series of F on the row and of G on the column,
// the eta-weighted sums and the FL-CAT2 blends.  No LDS exchange and no
// barrier; a wavefront holds 64 independent corners.
template <int FLUX, int NV, bool SQUARE = false>
__global__ __launch_bounds__(BLOCK) void k_flux2d_q11(KProb pb, KStep st) {
  const double dt = step_dt(st);
  const double lamx = dt / pb.dx, lamy = dt / pb.dy;
  // derivative weights times -lamx (x) and -lamy (y): gx[a][l], gy[a][l]
  double gx[2][2], gy[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int l = 0; l < 2; ++l) {
      gx[a][l] = -lamx * TB.G1[1][a][l];
      gy[a][l] = -lamy * TB.G1[1][a][l];
    }
  const double tay = TB.TAYLOR[PMAX][1];                      // r = 1, first term
  const double gt0 = TB.GT[1][1][0], gt1 = TB.GT[1][1][1];    // time derivative weights at r = 0, 1
  const int64_t nx = pb.nx, ny = pb.ny, plane = pb.nx * pb.ny;
  const int nx32 = (int)pb.nx, ny32 = (int)pb.ny, ioff = (int)pb.ioff;
  const uint32_t n1u = (uint32_t)pb.n1;
  const Slice sl(st.counts, st.list, 0);
  for (int64_t it = sl.lo + threadIdx.x; it < sl.hi; it += BLOCK) {
    const int32_t raw = sl.items[it];
    const int32_t e = SQUARE ? (raw & ((1 << LIST_TAG_SHIFT) - 1)) : raw;
    const int tag = SQUARE ? (raw >> LIST_TAG_SHIFT) : 0;
    const uint32_t eq = (uint32_t)e / n1u;
    const int i2 = (int)eq + ioff, i1 = (int)((uint32_t)e - eq * n1u) + ioff;
    int xs[2], ys[2];
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      xs[a] = bc_index32(i1 + a, nx32, pb.bc);
      ys[a] = bc_index32(i2 + a, ny32, pb.bc);
    }
    // node states and point fluxes, [j2][j1]
    double u[2][2][NV], f0[2][2][NV], g0[2][2][NV];
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int a = 0; a < 2; ++a) {
#pragma unroll
        for (int c = 0; c < NV; ++c) u[b][a][c] = st.u[c * plane + (int64_t)ys[b] * nx + xs[a]];
        flux2d<FLUX, NV>(pb.ph, u[b][a], f0[b][a], g0[b][a]);
      }
    // series of F on the row j2 = 0 (nodes (0,0), (1,0)) and of G on the
    // column j1 = 0 (nodes (0,0), (0,1)): S = Fh^0 / 1! + Fh^1 / 2!
    double SF[2][NV], SG[2][NV];
#pragma unroll
    for (int n = 0; n < 3; ++n) {
      const int a = n == 1 ? 1 : 0, b = n == 2 ? 1 : 0;   // nodes (0,0), (1,0), (0,1)
      double w[NV];
#pragma unroll
      for (int c = 0; c < NV; ++c) {
        // U^1 = -lamx d_x Fh^0 - lamy d_y Gh^0: one chain, row then column
        double s = 0.0;
        s = fma(gx[a][0], f0[b][0][c], s);
        s = fma(gx[a][1], f0[b][1][c], s);
        s = fma(gy[b][0], g0[0][a][c], s);
        s = fma(gy[b][1], g0[1][a][c], s);
        w[c] = fma(tay, s, u[b][a][c]);
      }
      double pf[NV], pg[NV];
      flux2d<FLUX, NV>(pb.ph, w, pf, pg);
#pragma unroll
      for (int c = 0; c < NV; ++c) {
        if (b == 0) {   // on the row: F's series
          const double nf = fma(gt1, pf[c], fma(gt0, f0[b][a][c], 0.0));
          SF[a][c] = fma(TB.INVFACT[2], nf, fma(TB.INVFACT[1], f0[b][a][c], 0.0));
        }
        if (a == 0) {   // on the column: G's series
          const double ng = fma(gt1, pg[c], fma(gt0, g0[b][a][c], 0.0));
          SG[b][c] = fma(TB.INVFACT[2], ng, fma(TB.INVFACT[1], g0[b][a][c], 0.0));
        }
      }
    }
    const bool needF = i2 >= 0 && tag != 2, needG = i1 >= 0 && tag != 1;
    if (needF) {
      // F: eta-weighted row sum, FL-CAT2 blend with the nodes (0,0), (1,0)
      const int64_t ei = (int64_t)i2 * pb.nIx + (i1 - ioff);
      const double psi = st.psix[ei], al = st.alx[ei];
      const double alf = pb.dx / ((double)pb.dim * dt);
#pragma unroll
      for (int c = 0; c < NV; ++c) {
        double v = fma(TB.ETA[1][1], SF[1][c], fma(TB.ETA[1][0], SF[0][c], 0.0));
        const double lo = lo_flux<FLUX, 2, NV>(pb.ph, pb.flags, 0, u[0][0], u[0][1], f0[0][0][c], f0[0][1][c],
                                               u[0][0][c], u[0][1][c], al, alf);
        v = psi * v + (1.0 - psi) * lo;
        st.Fx[((int64_t)c * ny + i2) * pb.nIx + (i1 - ioff)] = v;
      }
    }
    if (needG) {
      const int64_t ei = (int64_t)(i2 - ioff) * nx + i1;
      const double psi = st.psiy[ei], al = st.aly[ei];
      const double alf = pb.dy / ((double)pb.dim * dt);
#pragma unroll
      for (int c = 0; c < NV; ++c) {
        double v = fma(TB.ETA[1][1], SG[1][c], fma(TB.ETA[1][0], SG[0][c], 0.0));
        const double lo = lo_flux<FLUX, 2, NV>(pb.ph, pb.flags, 1, u[0][0], u[1][0], g0[0][0][c], g0[1][0][c],
                                               u[0][0][c], u[1][0][c], al, alf);
        v = psi * v + (1.0 - psi) * lo;
        st.Gy[((int64_t)c * pb.nIy + (i2 - ioff)) * nx + i1] = v;
      }
    }
  }
}

// The mirror classes (QA, QB) and (QB, QA), QA < QB, in one launch: the grid
// is cut into two runs of whole XCD groups of blocks, sized by the two
// classes' corner counts (at least one group for a class with corners),
// each block running its class's kernel body over its share of that class's
// list.  Both classes have the same corner size and the same work per
// corner; per corner the arithmetic is that of the one-class launch.
template <int FLUX, int NV, int QA, int QB>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(2))) void k_flux2d_pair(KProb pb, KStep st) {
  constexpr int L = (2 * QA) * (2 * QB);
  __shared__ double2 xsm[2 * Xch<NV>::NP * corner_stride<L>()];
  __shared__ double g1s[(2 * QA) * (2 * QA) + (2 * QB) * (2 * QB)];
  const int ca = (QA - 1) * pb.P + (QB - 1), cb = (QB - 1) * pb.P + (QA - 1);
  const int64_t na = st.counts[ca], nb = st.counts[cb];
  if (na + nb == 0) return;
  const int units = (int)gridDim.x / NXCD;
  const int ua = na == 0 ? 0 : (nb == 0 ? units : 1 + (int)((int64_t)(units - 2) * na / (na + nb)));
  const int unit = (int)blockIdx.x / NXCD;
  if (unit < ua) {
    flux2d_body<FLUX, NV, QA, QB, false>(pb, st, Slice(st.counts, st.list, ca, blockIdx.x, ua * NXCD), xsm, g1s);
  } else {
    const int ub = units - ua;
    flux2d_body<FLUX, NV, QB, QA, false>(pb, st, Slice(st.counts, st.list, cb, blockIdx.x - ua * NXCD, ub * NXCD),
                                         xsm, g1s);
  }
}

template <int FLUX, int NV>
__global__ __launch_bounds__(BLOCK) void k_update2d(KProb pb, KStep st) {
  const int64_t e = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  const int64_t nx = pb.nx, ny = pb.ny;
  if (e >= nx * ny) return;
  const int64_t i1 = e % nx, i2 = e / nx;
  const double dt = step_dt(st);
  const double lamx = dt / pb.dx, lamy = dt / pb.dy;
  const int64_t kxr = i1 - pb.ioff, kxl = (pb.bc == PERIODIC) ? (i1 == 0 ? nx - 1 : i1 - 1) : i1;
  const int64_t kyr = i2 - pb.ioff, kyl = (pb.bc == PERIODIC) ? (i2 == 0 ? ny - 1 : i2 - 1) : i2;
  double w[NV];
  bool finite = true;
#pragma unroll
  for (int c = 0; c < NV; ++c) {
    const double Fl = st.Fx[(c * ny + i2) * pb.nIx + kxl], Fr = st.Fx[(c * ny + i2) * pb.nIx + kxr];
    const double Gl = st.Gy[(c * pb.nIy + kyl) * nx + i1], Gr = st.Gy[(c * pb.nIy + kyr) * nx + i1];
    const int64_t idx = (c * ny + i2) * nx + i1;
    w[c] = st.u[idx] + lamx * (Fl - Fr) + lamy * (Gl - Gr);
    st.uout[idx] = w[c];
    finite = finite && isfinite(w[c]);
  }
  uint32_t bad = (finite ? 0u : 1u) | (physical<FLUX, 2, NV>(pb.ph, w) ? 0u : 2u);
  if (bad) atomicOr(st.status, bad);
}

// ====================================================================== CFL
template <int FLUX, int DIM, int NV>
__global__ __launch_bounds__(BLOCK) void k_max_speed(KProb pb, const double* __restrict__ u,
                                                     unsigned long long* smax) {
  const int64_t n = pb.nx * (DIM == 2 ? pb.ny : 1);
  double m0 = 0.0, m1 = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * BLOCK + threadIdx.x; e < n; e += (int64_t)gridDim.x * BLOCK) {
    double w[NV];
#pragma unroll
    for (int c = 0; c < NV; ++c) w[c] = u[c * n + e];
    m0 = fmax(m0, spectral_radius<FLUX, DIM, NV>(pb.ph, w, 0));
    if (DIM == 2) m1 = fmax(m1, spectral_radius<FLUX, DIM, NV>(pb.ph, w, 1));
  }
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
  // one atomic per block; the bit patterns of non-negative doubles order like the values
  if (threadIdx.x == 0) {
#pragma unroll
    for (int w = 1; w < BLOCK / 64; ++w) {
      m0 = fmax(m0, red[0][w]);
      m1 = fmax(m1, red[1][w]);
    }
    atomicMax(&smax[0], (unsigned long long)__double_as_longlong(m0));
    if (DIM == 2) atomicMax(&smax[1], (unsigned long long)__double_as_longlong(m1));
  }
}

__global__ void k_cfl_dt(int dim, double dx, double dy, const double* smax, double cfl, double t_final,
                         double* t_dev, double* dt_dev) {
  cfl_rule(dim, dx, dy, smax[0], dim == 2 ? smax[1] : 0.0, cfl, t_final, t_dev, dt_dev);
}


// ================================================================ launchers
CflReduce cfl_reduce(const KProb& pb, const KStep& st, int nparts) {
  CflReduce r{};
  if (st.cfl_mode) {
    r.part = st.part;
    r.nparts = nparts;
    r.dim = pb.dim;
    r.dx = pb.dx;
    r.dy = pb.dy;
    r.cfl = st.cfl;
    r.t_final = st.t_final;
    r.t_dev = st.t_dev;
    r.dt_out = st.dt_out;
  }
  return r;
}

#define ACAT_CHECK_LAUNCH()                  \
  do {                                       \
    hipError_t e_ = hipGetLastError();       \
    if (e_ != hipSuccess) return e_;         \
  } while (0)

template <int FLUX, int NV, int P, int p>
hipError_t launch_class1d(const KProb& pb, const KStep& st, int cap, hipStream_t s) {
  if constexpr (p <= P) {
    static const char* names[7] = {"", "flux1d_p1", "flux1d_p2", "flux1d_p3", "flux1d_p4", "flux1d_p5",
                                   "flux1d_p6"};
    auto kern = k_flux1d<FLUX, NV, p>;
    const int grid = group_grid<2 * p>(kern, pb.nIx, cap);
    {
      ProfScope ps(names[p], s);
      kern<<<grid, BLOCK, 0, s>>>(pb, st);
    }
    ACAT_CHECK_LAUNCH();
  }
  return hipSuccess;
}

// classification (or, in replay, the recorded orders) -> class map, then the
// per-class item lists
template <int FLUX, int NV, int P>
hipError_t lists1d_impl(const KProb& pb, const KStep& st, hipStream_t s) {
  const int64_t nI = pb.nIx;
  const int cblocks = (int)((nI + BLOCK - 1) / BLOCK);
  {
    ProfScope ps("classify1d", s);
    k_classify1d<FLUX, NV, P><<<cblocks, BLOCK, 0, s>>>(pb, st);
  }
  ACAT_CHECK_LAUNCH();
  {
    ProfScope ps("class_lists", s);
    k_scan_hist<<<P + (st.cfl_mode ? 1 : 0), SCAN_T, 0, s>>>(st.hist, cblocks, st.offs, st.counts, P,
                                                            cfl_reduce(pb, st, cblocks));
    k_scatter<P, false><<<cblocks, BLOCK, 0, s>>>(st.cls, 0, nI, 1, cblocks, st.offs, st.counts, st.list);
  }
  ACAT_CHECK_LAUNCH();
  return hipSuccess;
}

template <int FLUX, int NV, int P>
hipError_t step1d_impl(const KProb& pb, const KStep& st, int cap, hipStream_t s) {
  hipError_t e;
  if ((e = lists1d_impl<FLUX, NV, P>(pb, st, s)) != hipSuccess) return e;
  if ((e = launch_class1d<FLUX, NV, P, 1>(pb, st, cap, s)) != hipSuccess) return e;
  if ((e = launch_class1d<FLUX, NV, P, 2>(pb, st, cap, s)) != hipSuccess) return e;
  if ((e = launch_class1d<FLUX, NV, P, 3>(pb, st, cap, s)) != hipSuccess) return e;
  if ((e = launch_class1d<FLUX, NV, P, 4>(pb, st, cap, s)) != hipSuccess) return e;
  if ((e = launch_class1d<FLUX, NV, P, 5>(pb, st, cap, s)) != hipSuccess) return e;
  if ((e = launch_class1d<FLUX, NV, P, 6>(pb, st, cap, s)) != hipSuccess) return e;
  {
    ProfScope ps("update1d", s);
    k_update1d<FLUX, NV><<<(unsigned)((pb.nx + BLOCK - 1) / BLOCK), BLOCK, 0, s>>>(pb, st);
  }
  ACAT_CHECK_LAUNCH();
  return hipSuccess;
}

// A square class (Q, Q); the other classes run as mirror pairs (launch_pair2d).
template <int FLUX, int NV, int P, int Q>
hipError_t launch_class2d(const KProb& pb, const KStep& st, int cap, hipStream_t s) {
  if constexpr (Q <= P) {
    static const char* names[5] = {"", "flux2d_q11", "flux2d_q22", "flux2d_q33", "flux2d_q44"};
    // under the square-stencil variant only the square classes have items,
    // tagged with the flux they store
    // (1,1): one lane per corner (k_flux2d_q11); the others one lane per node
    const bool sq = (pb.flags & FLAG_SQUARE_2D) != 0;
    void (*kern)(KProb, KStep);
    int grid;
    if constexpr (Q == 1) {
      kern = sq ? k_flux2d_q11<FLUX, NV, true> : k_flux2d_q11<FLUX, NV>;
      grid = persistent_grid(kern, pb.n1 * pb.n2, cap);
    } else {
      kern = sq ? k_flux2d<FLUX, NV, Q, Q, true> : k_flux2d<FLUX, NV, Q, Q>;
      grid = group_grid<(2 * Q) * (2 * Q)>(kern, pb.n1 * pb.n2, cap);
    }
    {
      ProfScope ps(names[Q], s);
      kern<<<grid, BLOCK, 0, s>>>(pb, st);
    }
    ACAT_CHECK_LAUNCH();
  }
  return hipSuccess;
}

// The mirror classes (QA, QB) and (QB, QA), QA < QB, in one launch.
template <int FLUX, int NV, int P, int QA, int QB>
hipError_t launch_pair2d(const KProb& pb, const KStep& st, int cap, hipStream_t s) {
  static_assert(QA < QB, "pairs are named by their lower-left class");
  if constexpr (QB <= P) {
    static const char* names[5][5] = {{"", "", "", "", ""},
                                      {"", "", "flux2d_q12q21", "flux2d_q13q31", "flux2d_q14q41"},
                                      {"", "", "", "flux2d_q23q32", "flux2d_q24q42"},
                                      {"", "", "", "", "flux2d_q34q43"},
                                      {"", "", "", "", ""}};
    auto kern = k_flux2d_pair<FLUX, NV, QA, QB>;
    // two runs of XCD groups: at least one per class
    const int grid = std::max(group_grid<(2 * QA) * (2 * QB)>(kern, pb.n1 * pb.n2, cap), 2 * NXCD);
    {
      ProfScope ps(names[QA][QB], s);
      kern<<<grid, BLOCK, 0, s>>>(pb, st);
    }
    ACAT_CHECK_LAUNCH();
  }
  return hipSuccess;
}

template <int FLUX, int NV, int P>
hipError_t lists2d_impl(const KProb& pb, const KStep& st, hipStream_t s) {
  const int cblocks = (int)class_tiles(pb);
  {
    ProfScope ps("classify2d", s);
    k_classify2d<FLUX, NV, P><<<cblocks, BLOCK, 0, s>>>(pb, st);
  }
  ACAT_CHECK_LAUNCH();
  {
    ProfScope ps("class_lists", s);
    k_scan_hist<<<P * P + (st.cfl_mode ? 1 : 0), SCAN_T, 0, s>>>(st.hist, cblocks, st.offs, st.counts, P * P,
                                                                cfl_reduce(pb, st, cblocks));
    if (pb.flags & FLAG_SQUARE_2D)
      k_scatter<P * P, true, true><<<cblocks, BLOCK, 0, s>>>(st.cls, 0, pb.n1, pb.n2, cblocks, st.offs, st.counts,
                                                              st.list, P);
    else
      k_scatter<P * P, true><<<cblocks, BLOCK, 0, s>>>(st.cls, 0, pb.n1, pb.n2, cblocks, st.offs, st.counts,
                                                        st.list);
  }
  ACAT_CHECK_LAUNCH();
  return hipSuccess;
}

template <int FLUX, int NV, int P>
hipError_t step2d_impl(const KProb& pb, const KStep& st, int cap, hipStream_t s) {
  hipError_t e;
  if ((e = lists2d_impl<FLUX, NV, P>(pb, st, s)) != hipSuccess) return e;
  if ((e = launch_class2d<FLUX, NV, P, 1>(pb, st, cap, s)) != hipSuccess) return e;
  if ((e = launch_pair2d<FLUX, NV, P, 1, 2>(pb, st, cap, s)) != hipSuccess) return e;
  if ((e = launch_class2d<FLUX, NV, P, 2>(pb, st, cap, s)) != hipSuccess) return e;
  if ((e = launch_pair2d<FLUX, NV, P, 1, 3>(pb, st, cap, s)) != hipSuccess) return e;
  if ((e = launch_pair2d<FLUX, NV, P, 2, 3>(pb, st, cap, s)) != hipSuccess) return e;
  if ((e = launch_class2d<FLUX, NV, P, 3>(pb, st, cap, s)) != hipSuccess) return e;
  if ((e = launch_pair2d<FLUX, NV, P, 1, 4>(pb, st, cap, s)) != hipSuccess) return e;
  if ((e = launch_pair2d<FLUX, NV, P, 2, 4>(pb, st, cap, s)) != hipSuccess) return e;
  if ((e = launch_pair2d<FLUX, NV, P, 3, 4>(pb, st, cap, s)) != hipSuccess) return e;
  if ((e = launch_class2d<FLUX, NV, P, 4>(pb, st, cap, s)) != hipSuccess) return e;
  {
    ProfScope ps("update2d", s);
    k_update2d<FLUX, NV><<<(unsigned)((pb.nx * pb.ny + BLOCK - 1) / BLOCK), BLOCK, 0, s>>>(pb, st);
  }
  ACAT_CHECK_LAUNCH();
  return hipSuccess;
}

}  // namespace

hipError_t launch_step_1d(const KProb& pb, const KStep& st, int grid_blocks, hipStream_t s) {
  const int cap = grid_blocks;
  if (pb.flux == EUL) {
    switch (pb.P) {
      case 1: return step1d_impl<EUL, 3, 1>(pb, st, cap, s);
      case 2: return step1d_impl<EUL, 3, 2>(pb, st, cap, s);
      case 3: return step1d_impl<EUL, 3, 3>(pb, st, cap, s);
      case 4: return step1d_impl<EUL, 3, 4>(pb, st, cap, s);
      case 5: return step1d_impl<EUL, 3, 5>(pb, st, cap, s);
      case 6: return step1d_impl<EUL, 3, 6>(pb, st, cap, s);
    }
  } else if (pb.flux == BURG) {
    switch (pb.P) {
      case 1: return step1d_impl<BURG, 1, 1>(pb, st, cap, s);
      case 2: return step1d_impl<BURG, 1, 2>(pb, st, cap, s);
      case 3: return step1d_impl<BURG, 1, 3>(pb, st, cap, s);
      case 4: return step1d_impl<BURG, 1, 4>(pb, st, cap, s);
      case 5: return step1d_impl<BURG, 1, 5>(pb, st, cap, s);
      case 6: return step1d_impl<BURG, 1, 6>(pb, st, cap, s);
    }
  } else {
    switch (pb.P) {
      case 1: return step1d_impl<ADV, 1, 1>(pb, st, cap, s);
      case 2: return step1d_impl<ADV, 1, 2>(pb, st, cap, s);
      case 3: return step1d_impl<ADV, 1, 3>(pb, st, cap, s);
      case 4: return step1d_impl<ADV, 1, 4>(pb, st, cap, s);
      case 5: return step1d_impl<ADV, 1, 5>(pb, st, cap, s);
      case 6: return step1d_impl<ADV, 1, 6>(pb, st, cap, s);
    }
  }
  return hipErrorInvalidValue;
}

hipError_t launch_step_2d(const KProb& pb, const KStep& st, int grid_blocks, hipStream_t s) {
  const int cap = grid_blocks;
  if (pb.flux == EUL) {
    switch (pb.P) {
      case 1: return step2d_impl<EUL, 4, 1>(pb, st, cap, s);
      case 2: return step2d_impl<EUL, 4, 2>(pb, st, cap, s);
      case 3: return step2d_impl<EUL, 4, 3>(pb, st, cap, s);
      case 4: return step2d_impl<EUL, 4, 4>(pb, st, cap, s);
    }
  } else if (pb.flux == ADV) {
    switch (pb.P) {
      case 1: return step2d_impl<ADV, 1, 1>(pb, st, cap, s);
      case 2: return step2d_impl<ADV, 1, 2>(pb, st, cap, s);
      case 3: return step2d_impl<ADV, 1, 3>(pb, st, cap, s);
      case 4: return step2d_impl<ADV, 1, 4>(pb, st, cap, s);
    }
  }
  return hipErrorInvalidValue;
}

hipError_t launch_lists(const KProb& pb, const KStep& st, hipStream_t s) {
  if (pb.dim == 1) {
    if (pb.flux == EUL) {
      switch (pb.P) {
        case 1: return lists1d_impl<EUL, 3, 1>(pb, st, s);
        case 2: return lists1d_impl<EUL, 3, 2>(pb, st, s);
        case 3: return lists1d_impl<EUL, 3, 3>(pb, st, s);
        case 4: return lists1d_impl<EUL, 3, 4>(pb, st, s);
        case 5: return lists1d_impl<EUL, 3, 5>(pb, st, s);
        case 6: return lists1d_impl<EUL, 3, 6>(pb, st, s);
      }
    } else if (pb.flux == BURG) {
      switch (pb.P) {
        case 1: return lists1d_impl<BURG, 1, 1>(pb, st, s);
        case 2: return lists1d_impl<BURG, 1, 2>(pb, st, s);
        case 3: return lists1d_impl<BURG, 1, 3>(pb, st, s);
        case 4: return lists1d_impl<BURG, 1, 4>(pb, st, s);
        case 5: return lists1d_impl<BURG, 1, 5>(pb, st, s);
        case 6: return lists1d_impl<BURG, 1, 6>(pb, st, s);
      }
    } else {
      switch (pb.P) {
        case 1: return lists1d_impl<ADV, 1, 1>(pb, st, s);
        case 2: return lists1d_impl<ADV, 1, 2>(pb, st, s);
        case 3: return lists1d_impl<ADV, 1, 3>(pb, st, s);
        case 4: return lists1d_impl<ADV, 1, 4>(pb, st, s);
        case 5: return lists1d_impl<ADV, 1, 5>(pb, st, s);
        case 6: return lists1d_impl<ADV, 1, 6>(pb, st, s);
      }
    }
  } else if (pb.flux == EUL) {
    switch (pb.P) {
      case 1: return lists2d_impl<EUL, 4, 1>(pb, st, s);
      case 2: return lists2d_impl<EUL, 4, 2>(pb, st, s);
      case 3: return lists2d_impl<EUL, 4, 3>(pb, st, s);
      case 4: return lists2d_impl<EUL, 4, 4>(pb, st, s);
    }
  } else if (pb.flux == ADV) {
    switch (pb.P) {
      case 1: return lists2d_impl<ADV, 1, 1>(pb, st, s);
      case 2: return lists2d_impl<ADV, 1, 2>(pb, st, s);
      case 3: return lists2d_impl<ADV, 1, 3>(pb, st, s);
      case 4: return lists2d_impl<ADV, 1, 4>(pb, st, s);
    }
  }
  return hipErrorInvalidValue;
}

hipError_t launch_max_speed(const KProb& pb, const double* u, double* smax, hipStream_t s) {
  unsigned long long* sm = reinterpret_cast<unsigned long long*>(smax);
  ProfScope ps("max_speed", s);
  k_zero_u64<<<1, 64, 0, s>>>(sm, pb.dim);
  ACAT_CHECK_LAUNCH();
  const int64_t n = pb.nx * (pb.dim == 2 ? pb.ny : 1);
  int64_t blocks = (n + BLOCK - 1) / BLOCK;
  if (blocks > num_cus()) blocks = num_cus();   // one atomic per block: few blocks, many cells each
  const unsigned gb = (unsigned)blocks;
  if (pb.dim == 1) {
    if (pb.flux == EUL) k_max_speed<EUL, 1, 3><<<gb, BLOCK, 0, s>>>(pb, u, sm);
    else if (pb.flux == BURG) k_max_speed<BURG, 1, 1><<<gb, BLOCK, 0, s>>>(pb, u, sm);
    else k_max_speed<ADV, 1, 1><<<gb, BLOCK, 0, s>>>(pb, u, sm);
  } else {
    if (pb.flux == EUL) k_max_speed<EUL, 2, 4><<<gb, BLOCK, 0, s>>>(pb, u, sm);
    else k_max_speed<ADV, 2, 1><<<gb, BLOCK, 0, s>>>(pb, u, sm);
  }
  ACAT_CHECK_LAUNCH();
  return hipSuccess;
}

hipError_t launch_cfl_dt(const KProb& pb, const double* smax, double cfl, double t_final, double* t_dev,
                         double* dt_dev, hipStream_t s) {
  ProfScope ps("cfl_dt", s);
  k_cfl_dt<<<1, 1, 0, s>>>(pb.dim, pb.dx, pb.dy, smax, cfl, t_final, t_dev, dt_dev);
  ACAT_CHECK_LAUNCH();
  return hipSuccess;
}

// Coefficient tables as the kernels use them (host copy of the same constexpr data).
void copy_tables(int p, double* g1, double* gt, double* eta, double* tau) {
  const int n = 2 * p;
  for (int a = 0; a < n; ++a)
    for (int l = 0; l < n; ++l) {
      if (g1) g1[a * n + l] = TB.G1[p][a][l];
      if (gt) gt[a * n + l] = TB.GT[p][a][l];
    }
  for (int a = 0; a < n; ++a) {
    if (eta) eta[a] = TB.ETA[p][a];
    if (tau) tau[a] = TB.TAU[p][a];
  }
}

}  // namespace acat
