// Adjoint of one ACAT step with frozen decisions (orders, psi^1, Rusanov
// speed, time step): ubar_in = ubar_out + sum over interfaces of
// (dF/du)^T Fbar, with Fbar_k = lambda (ubar_{i+1} - ubar_i) for the
// interface between cells i and i+1 (in 2D likewise for G along y).
//
// Per interface (1D) or corner (2D) the kernels recompute the CAT recursion
// of the forward step (Sec. 2.2; Sec. 4 corner recursion) in registers, one
// lane per stencil node, keeping the Taylor history U^1..U^{2q-1} of the
// node, then run it backwards: flux Jacobian-transpose products at the
// predicted states, and for the spatial derivative of each level the
// transposed row/column sums through LDS.  Each lane writes the
// contribution to its node into a per-item buffer; a gather kernel adds, for
// every cell, the contributions of all items whose stencil covers it in a
// fixed order (deterministic, no atomics).
#include <hip/hip_runtime.h>

#include "acat_internal.hpp"
#include "coeffs.hpp"
#include "step_common.hpp"

namespace acat {
namespace {

// ======================================================================= 1D
// contribution buffer, slot-major: C[c][slot][k] with slot = j + P - 1 for the
// node at offset j in [-P+1, P] of interface k, so that a gather over one
// offset reads consecutive interfaces
template <int FLUX, int NV, int p>
__global__ __launch_bounds__(BLOCK) void k_adj1d(KProb pb, KStep st, const double* __restrict__ ubo,
                                                 double* __restrict__ C, int LMAX) {
  constexpr int L = 2 * p;
  using Grp = Groups<L>;
  constexpr int GPB = Grp::PER_BLOCK;
  constexpr int SL = L + 1;
  constexpr int NS = Grp::TOTAL * SL;
  __shared__ double xs[2][NV][NS];

  const Grp grp(threadIdx.x);
  const int g = grp.g;
  const int a = grp.node;
  const int slot = g * SL + a;
  const bool inblk = grp.in;
  const double lam = step_dt(st) / pb.dx;
  const int64_t nx = pb.nx, nI = pb.nIx;
  const int nx32 = (int)nx;
  const int64_t cstride = nI * LMAX;

  double g1[L], g1T[L];
#pragma unroll
  for (int l = 0; l < L; ++l) {
    g1[l] = TB.G1[p][a][l];
    g1T[l] = TB.G1[p][l][a];
  }
  const double eta = TB.ETA[p][a];

  int buf = 0;
  const Slice sl(st.counts, st.list, p - 1);
  for (int64_t base = sl.lo; base < sl.hi; base += GPB) {
    const bool valid = inblk && base + g < sl.hi;
    const int32_t k = valid ? sl.items[base + g] : 0;
    const int i = k + (int)pb.ioff;
    const int node = bc_index32(i + (a - p + 1), nx32, pb.bc);
    double u[NV], Fb[NV];
#pragma unroll
    for (int c = 0; c < NV; ++c) u[c] = valid ? st.u[c * nx + node] : 1.0;
    // Fbar = lambda (ubar_{i+1} - ubar_i); a transmissive boundary interface
    // updates only the cell inside the grid
    const bool hasR = valid && (pb.bc == PERIODIC || i + 1 < nx32);
    const bool hasL = valid && i >= 0;
    const int cr = bc_index32(i + 1, nx32, pb.bc), cl = bc_index32(i, nx32, pb.bc);
#pragma unroll
    for (int c = 0; c < NV; ++c) {
      const double ur = hasR ? ubo[c * nx + cr] : 0.0;
      const double ul = hasL ? ubo[c * nx + cl] : 0.0;
      Fb[c] = lam * (ur - ul);
    }
    double psi = 1.0, al = 0.0;
    if constexpr (p == 1) {
      if (valid) {
        psi = st.psix[k];
        al = st.alx[k];
      }
    }
    // ---- forward recomputation, keeping U^l at this node
    double fh0[NV], cur[NV];
    flux1d<FLUX, NV>(pb.ph, u, fh0);
#pragma unroll
    for (int c = 0; c < NV; ++c) cur[c] = fh0[c];
    double U[L][NV];
#pragma unroll
    for (int kk = 2; kk <= 2 * p - 1; ++kk) {   // Fh^{2p-1} is not needed backwards
#pragma unroll
      for (int c = 0; c < NV; ++c) xs[buf][c][slot] = cur[c];
      Grp::sync();
#pragma unroll
      for (int c = 0; c < NV; ++c) {
        double sacc = 0.0;
#pragma unroll
        for (int l = 0; l < L; ++l) sacc = fma(g1[l], xs[buf][c][g * SL + l], sacc);
        U[kk - 1][c] = -lam * sacc;
      }
      buf ^= 1;
      double nxt[NV];
#pragma unroll
      for (int c = 0; c < NV; ++c) nxt[c] = 0.0;
#pragma unroll
      for (int ri = 0; ri < L; ++ri) {
        const int r = ri - p + 1;
        double ph[NV];
        if (r == 0) {
#pragma unroll
          for (int c = 0; c < NV; ++c) ph[c] = fh0[c];
        } else {
          double w[NV];
#pragma unroll
          for (int c = 0; c < NV; ++c) {
            double sacc = u[c];
#pragma unroll
            for (int l = 1; l <= kk - 1; ++l) sacc = fma(TB.TAYLOR[r + PMAX - 1][l], U[l][c], sacc);
            w[c] = sacc;
          }
          flux1d<FLUX, NV>(pb.ph, w, ph);
        }
#pragma unroll
        for (int c = 0; c < NV; ++c) nxt[c] = fma(TB.GT[p][kk - 1][ri], ph[c], nxt[c]);
      }
#pragma unroll
      for (int c = 0; c < NV; ++c) cur[c] = nxt[c];
    }
    // U^{2p-1}
    if (2 * p >= 2) {
#pragma unroll
      for (int c = 0; c < NV; ++c) xs[buf][c][slot] = cur[c];
      Grp::sync();
#pragma unroll
      for (int c = 0; c < NV; ++c) {
        double sacc = 0.0;
#pragma unroll
        for (int l = 0; l < L; ++l) sacc = fma(g1[l], xs[buf][c][g * SL + l], sacc);
        U[2 * p - 1][c] = -lam * sacc;
      }
      buf ^= 1;
    }
    // ---- reverse sweep
    // F = sum_j eta_j S_j, S_j = sum_k Fh^{k-1}_j / k!  =>  Sbar_j = eta_j psi Fbar
    double sb[NV], ub[NV], f0b[NV], fhb[NV];
#pragma unroll
    for (int c = 0; c < NV; ++c) {
      sb[c] = eta * psi * Fb[c];
      ub[c] = 0.0;
      f0b[c] = 0.0;
      fhb[c] = TB.INVFACT[2 * p] * sb[c];   // Fhbar^{2p-1}
    }
    double Ub[L][NV];
#pragma unroll
    for (int l = 0; l < L; ++l)
#pragma unroll
      for (int c = 0; c < NV; ++c) Ub[l][c] = 0.0;
#pragma unroll
    for (int kk = 2 * p; kk >= 2; --kk) {
      // Fh^{kk-1} = sum_r GT_r phi_r
#pragma unroll
      for (int ri = 0; ri < L; ++ri) {
        const int r = ri - p + 1;
        double phb[NV];
#pragma unroll
        for (int c = 0; c < NV; ++c) phb[c] = TB.GT[p][kk - 1][ri] * fhb[c];
        if (r == 0) {
#pragma unroll
          for (int c = 0; c < NV; ++c) f0b[c] += phb[c];
        } else {
          double w[NV], wb[NV];
#pragma unroll
          for (int c = 0; c < NV; ++c) {
            double sacc = u[c];
#pragma unroll
            for (int l = 1; l <= kk - 1; ++l) sacc = fma(TB.TAYLOR[r + PMAX - 1][l], U[l][c], sacc);
            w[c] = sacc;
            wb[c] = 0.0;
          }
          flux1d_vjp<FLUX, NV>(pb.ph, w, phb, wb);
#pragma unroll
          for (int c = 0; c < NV; ++c) {
            ub[c] += wb[c];
#pragma unroll
            for (int l = 1; l <= kk - 1; ++l) Ub[l][c] += TB.TAYLOR[r + PMAX - 1][l] * wb[c];
          }
        }
      }
      // U^{kk-1}_a = -lam sum_l g1[a][l] Fh^{kk-2}_l  =>  Fhbar^{kk-2}_a += -lam sum_j g1[j][a] Ubar_j
#pragma unroll
      for (int c = 0; c < NV; ++c) xs[buf][c][slot] = Ub[kk - 1][c];
      Grp::sync();
#pragma unroll
      for (int c = 0; c < NV; ++c) {
        double sacc = 0.0;
#pragma unroll
        for (int j = 0; j < L; ++j) sacc += g1T[j] * xs[buf][c][g * SL + j];
        fhb[c] = TB.INVFACT[kk - 1] * sb[c] - lam * sacc;   // Fhbar^{kk-2}
      }
      buf ^= 1;
    }
    // Fh^0 = f(u) also enters every r = 0 term
#pragma unroll
    for (int c = 0; c < NV; ++c) f0b[c] += fhb[c];
    flux1d_vjp<FLUX, NV>(pb.ph, u, f0b, ub);
    if constexpr (p == 1) {
      // Rusanov part of the FL-CAT2 blend: (1 - psi) [(f_i + f_{i+1})/2 - alpha/2 (u_{i+1} - u_i)]
      double lb[NV], zero[NV];
#pragma unroll
      for (int c = 0; c < NV; ++c) {
        lb[c] = 0.5 * (1.0 - psi) * Fb[c];
        zero[c] = 0.0;
      }
      flux1d_vjp<FLUX, NV>(pb.ph, u, lb, zero);
      const double sp = (pb.flags & FLAG_FLO_LF) ? pb.dx / ((double)pb.dim * step_dt(st)) : al;
#pragma unroll
      for (int c = 0; c < NV; ++c) ub[c] += zero[c] + (a == 0 ? sp : -sp) * lb[c];
    }
    if (valid) {
#pragma unroll
      for (int c = 0; c < NV; ++c) C[c * cstride + (int64_t)(a - p + pb.P) * nI + k] = ub[c];
    }
  }
}

// ubar_in[m] = ubar_out[m] + the contributions of every interface with a
// stencil node at cell m (through the boundary map), interfaces in
// increasing order, nodes in increasing order.  Periodic: interfaces
// i = m - j, j in [-P+1, P] (node j of interface i is cell m exactly when
// i + j = m, as nx >= 2P).  Transmissive: the same window, extended to the
// first (last) interface for the P cells next to the left (right) edge,
// whose clamped nodes reach them.
template <int NV>
__global__ __launch_bounds__(BLOCK) void k_gather1d(KProb pb, KStep st, const double* __restrict__ ubo,
                                                    const double* __restrict__ C, int LMAX, double* ubi) {
  const int m = blockIdx.x * BLOCK + threadIdx.x;
  const int nx = (int)pb.nx, P = pb.P, ioff = (int)pb.ioff, nI = (int)pb.nIx;
  if (m >= nx) return;
  const int64_t cstride = (int64_t)nI * LMAX;
  const bool per = pb.bc == PERIODIC;
  double acc[NV];
#pragma unroll
  for (int c = 0; c < NV; ++c) acc[c] = ubo[c * pb.nx + m];
  const int ilo = (!per && m < P) ? ioff : m - P;
  const int ihi = (!per && m >= nx - P) ? nx - 1 : m + P - 1;
  for (int i0 = ilo; i0 <= ihi; ++i0) {
    const int i = per ? (i0 < 0 ? i0 + nx : (i0 >= nx ? i0 - nx : i0)) : i0;
    const int k = i - ioff;
    const int q = st.cls[k] + 1;
    for (int a = 0; a < 2 * q; ++a) {
      const int j = a - q + 1;
      const int node = per ? i0 + j : bc_index32(i0 + j, nx, pb.bc);
      if (node != m) continue;
#pragma unroll
      for (int c = 0; c < NV; ++c) acc[c] += C[c * cstride + (int64_t)(j + P - 1) * nI + k];
    }
  }
#pragma unroll
  for (int c = 0; c < NV; ++c) ubi[c * pb.nx + m] = acc[c];
}

// ======================================================================= 2D
// One corner recursion forward (keeping U), then backwards.  sfb/sgb: the
// adjoints of this node's series SF / SG; ub accumulates the adjoint of u,
// f0b/g0b those of f(u), g(u).
template <int FLUX, int NV, int Q1, int Q2, int QT>
__device__ __forceinline__ void corner_adjoint(const Phys& ph, const double (&u)[NV],
                                               const double (&f0)[NV], const double (&g0)[NV],
                                               const double* gx, const double* gy,
                                               double2* xsb0, double2* xsb1, int stride, int& buf, int slot,
                                               int gbase, int a1, int a2, const double (&sfb)[NV],
                                               const double (&sgb)[NV], double (&ub)[NV], double (&f0b)[NV],
                                               double (&g0b)[NV]) {
  constexpr int N1 = 2 * Q1, N2 = 2 * Q2, T = 2 * QT;
  double fc[NV], gc[NV];
#pragma unroll
  for (int c = 0; c < NV; ++c) {
    fc[c] = f0[c];
    gc[c] = g0[c];
  }
  double U[T][NV];
  // this node's derivative weights of the forward differences, in registers
  // for the pass (the transposed ones are read from LDS at each use)
  double wfx[N1], wfy[N2];
#pragma unroll
  for (int l = 0; l < N1; ++l) wfx[l] = gx[a1 * N1 + l];
#pragma unroll
  for (int l = 0; l < N2; ++l) wfy[l] = gy[a2 * N2 + l];
  // forward: U^1 .. U^{T-1}
#pragma unroll
  for (int kk = 2; kk <= T; ++kk) {
    double2* xsw = buf ? xsb1 : xsb0;
    Xch<NV>::put(xsw, stride, slot, fc, gc);
    Groups<(2 * Q1) * (2 * Q2)>::sync();
    const double* xr = reinterpret_cast<const double*>(xsw);
    // U^{kk-1} as the forward step forms it: one chain over the row, then
    // the column, with the weights -lamx gamma and -lamy gamma
#pragma unroll
    for (int c = 0; c < NV; ++c) {
      double s = 0.0;
#pragma unroll
      for (int l = 0; l < N1; ++l) s = fma(wfx[l], Xch<NV>::get(xr, stride, gbase + a2 * N1 + l, c, false), s);
#pragma unroll
      for (int l = 0; l < N2; ++l) s = fma(wfy[l], Xch<NV>::get(xr, stride, gbase + l * N1 + a1, c, true), s);
      U[kk - 1][c] = s;
    }
    buf ^= 1;
    if (kk == T) break;
    double nf[NV], ng[NV];
#pragma unroll
    for (int c = 0; c < NV; ++c) {
      nf[c] = 0.0;
      ng[c] = 0.0;
    }
#pragma unroll
    for (int ri = 0; ri < T; ++ri) {
      const int r = ri - QT + 1;
      double pf[NV], pg[NV];
      if (r == 0) {
#pragma unroll
        for (int c = 0; c < NV; ++c) {
          pf[c] = f0[c];
          pg[c] = g0[c];
        }
      } else {
        double w[NV];
#pragma unroll
        for (int c = 0; c < NV; ++c) {
          double sacc = u[c];
#pragma unroll
          for (int l = 1; l <= kk - 1; ++l) sacc = fma(TB.TAYLOR[r + PMAX - 1][l], U[l][c], sacc);
          w[c] = sacc;
        }
        flux2d<FLUX, NV>(ph, w, pf, pg);
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
    }
  }
  // backward
  double fhb[NV], ghb[NV];
#pragma unroll
  for (int c = 0; c < NV; ++c) {
    fhb[c] = TB.INVFACT[T] * sfb[c];
    ghb[c] = TB.INVFACT[T] * sgb[c];
  }
  double Ub[T][NV];
#pragma unroll
  for (int l = 0; l < T; ++l)
#pragma unroll
    for (int c = 0; c < NV; ++c) Ub[l][c] = 0.0;
#pragma unroll
  for (int kk = T; kk >= 2; --kk) {
#pragma unroll
    for (int ri = 0; ri < T; ++ri) {
      const int r = ri - QT + 1;
      double pfb[NV], pgb[NV];
#pragma unroll
      for (int c = 0; c < NV; ++c) {
        pfb[c] = TB.GT[QT][kk - 1][ri] * fhb[c];
        pgb[c] = TB.GT[QT][kk - 1][ri] * ghb[c];
      }
      if (r == 0) {
#pragma unroll
        for (int c = 0; c < NV; ++c) {
          f0b[c] += pfb[c];
          g0b[c] += pgb[c];
        }
      } else {
        double w[NV], wb[NV];
#pragma unroll
        for (int c = 0; c < NV; ++c) {
          double sacc = u[c];
#pragma unroll
          for (int l = 1; l <= kk - 1; ++l) sacc = fma(TB.TAYLOR[r + PMAX - 1][l], U[l][c], sacc);
          w[c] = sacc;
          wb[c] = 0.0;
        }
        flux2d_vjp<FLUX, NV>(ph, w, pfb, pgb, wb);
#pragma unroll
        for (int c = 0; c < NV; ++c) {
          ub[c] += wb[c];
#pragma unroll
          for (int l = 1; l <= kk - 1; ++l) Ub[l][c] += TB.TAYLOR[r + PMAX - 1][l] * wb[c];
        }
      }
    }
    // U^{kk-1} = sum_l wx[a1][l] Fh_(l,a2) + sum_l wy[a2][l] Gh_(a1,l)
    // (wx = -lamx gamma, wy = -lamy gamma)
    //  => Fhbar_(a1,a2) += sum_j wx[j][a1] Ubar_(j,a2); Ghbar likewise along the column
    double2* xsw = buf ? xsb1 : xsb0;
    Xch<NV>::put(xsw, stride, slot, Ub[kk - 1], Ub[kk - 1]);
    Groups<(2 * Q1) * (2 * Q2)>::sync();
    const double* xr = reinterpret_cast<const double*>(xsw);
#pragma unroll
    for (int c = 0; c < NV; ++c) {
      double sx = TB.INVFACT[kk - 1] * sfb[c], sy = TB.INVFACT[kk - 1] * sgb[c];
#pragma unroll
      for (int j = 0; j < N1; ++j) sx = fma(gx[j * N1 + a1], Xch<NV>::get(xr, stride, gbase + a2 * N1 + j, c, false), sx);
#pragma unroll
      for (int j = 0; j < N2; ++j) sy = fma(gy[j * N2 + a2], Xch<NV>::get(xr, stride, gbase + j * N1 + a1, c, true), sy);
      fhb[c] = sx;
      ghb[c] = sy;
    }
    buf ^= 1;
  }
#pragma unroll
  for (int c = 0; c < NV; ++c) {
    f0b[c] += fhb[c];
    g0b[c] += ghb[c];
  }
}

// contribution buffer, slot-major: C[c][slot][e], slot = (j2 + P - 1) 2P + (j1 + P - 1)
// for the node at offset (j1, j2) of corner e (a gather over one offset reads
// consecutive corners)
// PASSES (corners with q1 != q2): 1 = the F recursion only, 2 = the G recursion
// only, added to the contributions the first launch wrote, 3 = both.
// The body runs the block's share `sl` of the class list; xsm: the two LDS
// exchange buffers (2 Xch<NV>::NP adj_stride<L>() double2), g1s: LDS for the
// derivative weights ((2 Q1)^2 + (2 Q2)^2 doubles).
template <int L>
constexpr int adj_stride() {
  return Groups<L>::WAVE_LOCAL ? Groups<L>::TOTAL * L : BLOCK + L;
}

template <int FLUX, int NV, int Q1, int Q2, int PASSES>
__device__ __forceinline__ void adj2d_body(const KProb& pb, const KStep& st, const Slice& sl,
                                           const double* __restrict__ ubo, double* __restrict__ C, int LMAX,
                                           double2* xsm, double* g1s) {
  constexpr int N1 = 2 * Q1, N2 = 2 * Q2, L = N1 * N2;
  using Grp = Groups<L>;
  constexpr int CPB = Grp::PER_BLOCK;
  constexpr int NP = Xch<NV>::NP;
  constexpr int STRIDE = adj_stride<L>();
  double2* const xs[2] = {xsm, xsm + NP * STRIDE};

  const int tid = threadIdx.x;
  const Grp grp(tid);
  const int g = grp.g;
  const int nd = grp.node;
  const int a1 = nd % N1, a2 = nd / N1;
  const bool inblk = grp.in;
  const double dt = step_dt(st);
  const double lamx = dt / pb.dx, lamy = dt / pb.dy;
  const int64_t nx = pb.nx, plane = pb.nx * pb.ny;
  const int nx32 = (int)pb.nx, ny32 = (int)pb.ny, ioff = (int)pb.ioff;
  const uint32_t n1u = (uint32_t)pb.n1;
  const int64_t nitems = pb.n1 * pb.n2;
  const int64_t cstride = nitems * LMAX;

  // derivative weights times -lamx (x) and -lamy (y) in LDS, row-major: rows
  // for the recursion, columns for its transpose
  for (int i = tid; i < N1 * N1 + N2 * N2; i += BLOCK)
    g1s[i] = i < N1 * N1 ? -lamx * TB.G1[Q1][i / N1][i % N1]
                         : -lamy * TB.G1[Q2][(i - N1 * N1) / N2][(i - N1 * N1) % N2];
  __syncthreads();
  const double* gx = g1s;
  const double* gy = g1s + N1 * N1;
  const bool on_row = a2 == Q2 - 1, on_col = a1 == Q1 - 1;

  int buf = 0;
  for (int64_t base = sl.lo; base < sl.hi; base += CPB) {
    const bool valid = inblk && base + g < sl.hi;
    const int32_t e = valid ? sl.items[base + g] : 0;
    const uint32_t eq = (uint32_t)e / n1u;
    const int i2 = (int)eq + ioff, i1 = (int)((uint32_t)e - eq * n1u) + ioff;
    const int x = bc_index32(i1 + (a1 - Q1 + 1), nx32, pb.bc);
    const int y = bc_index32(i2 + (a2 - Q2 + 1), ny32, pb.bc);
    double u[NV];
#pragma unroll
    for (int c = 0; c < NV; ++c) u[c] = valid ? st.u[c * plane + (int64_t)y * nx + x] : 1.0;
    // Fbar = lamx (ubar_{i+e1} - ubar_i), Gbar = lamy (ubar_{i+e2} - ubar_i), the
    // terms of cells outside a transmissive grid dropped (an edge flux enters
    // one cell only); corners on the ghost row carry no x-flux, those on the
    // ghost column no y-flux
    const bool per = pb.bc == PERIODIC;
    const bool hasF = valid && i2 >= 0, hasG = valid && i1 >= 0;
    double Fb[NV], Gb[NV];
    {
      const bool in1 = per || i1 >= 0, inr1 = per || i1 + 1 < nx32;
      const bool in2 = per || i2 >= 0, inr2 = per || i2 + 1 < ny32;
      const int x0 = bc_index32(i1, nx32, pb.bc), y0 = bc_index32(i2, ny32, pb.bc);
      const int xr = bc_index32(i1 + 1, nx32, pb.bc), yr = bc_index32(i2 + 1, ny32, pb.bc);
#pragma unroll
      for (int c = 0; c < NV; ++c) {
        const double u0 = valid ? ubo[c * plane + (int64_t)y0 * nx + x0] : 0.0;
        const double ux = valid ? ubo[c * plane + (int64_t)y0 * nx + xr] : 0.0;
        const double uy = valid ? ubo[c * plane + (int64_t)yr * nx + x0] : 0.0;
        Fb[c] = hasF ? lamx * ((inr1 ? ux : 0.0) - (in1 ? u0 : 0.0)) : 0.0;
        Gb[c] = hasG ? lamy * ((inr2 ? uy : 0.0) - (in2 ? u0 : 0.0)) : 0.0;
      }
    }
    double psix = 1.0, alx = 0.0, psiy = 1.0, aly = 0.0;
    if (valid) {
      if (Q1 == 1 && hasF) {
        const int64_t ex = (int64_t)i2 * pb.nIx + (i1 - ioff);
        psix = st.psix[ex];
        alx = st.alx[ex];
      }
      if (Q2 == 1 && hasG) {
        const int64_t ey = (int64_t)(i2 - ioff) * nx + i1;
        psiy = st.psiy[ey];
        aly = st.aly[ey];
      }
    }
    double f0[NV], g0[NV];
    flux2d<FLUX, NV>(pb.ph, u, f0, g0);
    double sfb[NV], sgb[NV], zero[NV], ub[NV], f0b[NV], g0b[NV];
#pragma unroll
    for (int c = 0; c < NV; ++c) {
      sfb[c] = on_row ? TB.ETA[Q1][a1] * psix * Fb[c] : 0.0;
      sgb[c] = on_col ? TB.ETA[Q2][a2] * psiy * Gb[c] : 0.0;
      zero[c] = 0.0;
      ub[c] = 0.0;
      f0b[c] = 0.0;
      g0b[c] = 0.0;
    }
    const int slot = g * L + nd;
    if constexpr (Q1 == Q2) {
      corner_adjoint<FLUX, NV, Q1, Q2, Q1>(pb.ph, u, f0, g0, gx, gy, xs[0], xs[1], STRIDE, buf, slot,
                                           g * L, a1, a2, sfb, sgb, ub, f0b, g0b);
    } else {
      if constexpr ((PASSES & 1) != 0)
        corner_adjoint<FLUX, NV, Q1, Q2, Q1>(pb.ph, u, f0, g0, gx, gy, xs[0], xs[1], STRIDE, buf, slot,
                                             g * L, a1, a2, sfb, zero, ub, f0b, g0b);
      if constexpr ((PASSES & 2) != 0)
        corner_adjoint<FLUX, NV, Q1, Q2, Q2>(pb.ph, u, f0, g0, gx, gy, xs[0], xs[1], STRIDE, buf, slot,
                                             g * L, a1, a2, zero, sgb, ub, f0b, g0b);
    }
    // first-order parts (Rusanov or Lax-Friedrichs) of the FL-CAT2 blends, on
    // the two nodes each one reads
    if (pb.flags & FLAG_FLO_LF) {
      alx = pb.dx / ((double)pb.dim * dt);
      aly = pb.dy / ((double)pb.dim * dt);
    }
    if ((PASSES & 1) != 0 && Q1 == 1 && on_row && (a1 == Q1 - 1 || a1 == Q1)) {
#pragma unroll
      for (int c = 0; c < NV; ++c) {
        const double lb = 0.5 * (1.0 - psix) * Fb[c];
        f0b[c] += lb;
        ub[c] += (a1 == Q1 - 1 ? alx : -alx) * lb;
      }
    }
    if ((PASSES & 2) != 0 && Q2 == 1 && on_col && (a2 == Q2 - 1 || a2 == Q2)) {
#pragma unroll
      for (int c = 0; c < NV; ++c) {
        const double lb = 0.5 * (1.0 - psiy) * Gb[c];
        g0b[c] += lb;
        ub[c] += (a2 == Q2 - 1 ? aly : -aly) * lb;
      }
    }
    flux2d_vjp<FLUX, NV>(pb.ph, u, f0b, g0b, ub);
    const int cslot = (a2 - Q2 + pb.P) * (2 * pb.P) + (a1 - Q1 + pb.P);
    if (valid) {
#pragma unroll
      for (int c = 0; c < NV; ++c) {
        double* dst = C + c * cstride + (int64_t)cslot * nitems + e;
        *dst = PASSES == 2 ? *dst + ub[c] : ub[c];
      }
    }
  }
}

template <int FLUX, int NV, int Q1, int Q2, int PASSES = 3>
__global__ __launch_bounds__(BLOCK) void k_adj2d(KProb pb, KStep st, const double* __restrict__ ubo,
                                                 double* __restrict__ C, int LMAX) {
  constexpr int L = (2 * Q1) * (2 * Q2);
  __shared__ double2 xsm[2 * Xch<NV>::NP * adj_stride<L>()];
  __shared__ double g1s[(2 * Q1) * (2 * Q1) + (2 * Q2) * (2 * Q2)];
  adj2d_body<FLUX, NV, Q1, Q2, PASSES>(pb, st, Slice(st.counts, st.list, (Q1 - 1) * pb.P + (Q2 - 1)), ubo, C,
                                       LMAX, xsm, g1s);
}

// Order class (1,1) with ONE LANE PER CORNER: the adjoint of the one-lane
// forward kernel.  The lane holds the corner's four nodes (j1, j2) in
// {0,1}^2 and runs the same reverse sweep as the node-per-lane kernel
// (recursion level 2 backwards, the transposed centred differences, the
// blends' first-order parts, the Jacobian-transpose products), skipping
// the terms that are zero for this class: the predicted-state adjoint at
// node (1,1), which no flux reads.  Writes the four nodes' contributions.
template <int FLUX, int NV>
__global__ __launch_bounds__(BLOCK) void k_adj2d_q11(KProb pb, KStep st, const double* __restrict__ ubo,
                                                     double* __restrict__ C, int LMAX) {
  const double dt = step_dt(st);
  const double lamx = dt / pb.dx, lamy = dt / pb.dy;
  double gx[2][2], gy[2][2];   // -lamx G1[1][a][l], -lamy G1[1][a][l]
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int l = 0; l < 2; ++l) {
      gx[a][l] = -lamx * TB.G1[1][a][l];
      gy[a][l] = -lamy * TB.G1[1][a][l];
    }
  const double tay = TB.TAYLOR[PMAX][1];
  const double gt0 = TB.GT[1][1][0], gt1 = TB.GT[1][1][1];
  const int64_t nx = pb.nx, plane = pb.nx * pb.ny;
  const int nx32 = (int)pb.nx, ny32 = (int)pb.ny, ioff = (int)pb.ioff;
  const uint32_t n1u = (uint32_t)pb.n1;
  const int64_t nitems = pb.n1 * pb.n2;
  const int64_t cstride = nitems * LMAX;
  const bool per = pb.bc == PERIODIC;
  const Slice sl(st.counts, st.list, 0);
  for (int64_t it = sl.lo + threadIdx.x; it < sl.hi; it += BLOCK) {
    const int32_t e = sl.items[it];
    const uint32_t eq = (uint32_t)e / n1u;
    const int i2 = (int)eq + ioff, i1 = (int)((uint32_t)e - eq * n1u) + ioff;
    int xs[2], ys[2];
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      xs[a] = bc_index32(i1 + a, nx32, pb.bc);
      ys[a] = bc_index32(i2 + a, ny32, pb.bc);
    }
    // Fbar = lamx (ubar_{i+e1} - ubar_i), Gbar = lamy (ubar_{i+e2} - ubar_i);
    // ghost-row corners carry no x-flux, ghost-column corners no y-flux
    const bool hasF = i2 >= 0, hasG = i1 >= 0;
    double Fb[NV], Gb[NV];
    {
      const bool in1 = per || i1 >= 0, inr1 = per || i1 + 1 < nx32;
      const bool in2 = per || i2 >= 0, inr2 = per || i2 + 1 < ny32;
#pragma unroll
      for (int c = 0; c < NV; ++c) {
        const double u0 = ubo[c * plane + (int64_t)ys[0] * nx + xs[0]];
        const double ux = ubo[c * plane + (int64_t)ys[0] * nx + xs[1]];
        const double uy = ubo[c * plane + (int64_t)ys[1] * nx + xs[0]];
        Fb[c] = hasF ? lamx * ((inr1 ? ux : 0.0) - (in1 ? u0 : 0.0)) : 0.0;
        Gb[c] = hasG ? lamy * ((inr2 ? uy : 0.0) - (in2 ? u0 : 0.0)) : 0.0;
      }
    }
    double psix = 1.0, alx = 0.0, psiy = 1.0, aly = 0.0;
    if (hasF) {
      const int64_t ex = (int64_t)i2 * pb.nIx + (i1 - ioff);
      psix = st.psix[ex];
      alx = st.alx[ex];
    }
    if (hasG) {
      const int64_t ey = (int64_t)(i2 - ioff) * nx + i1;
      psiy = st.psiy[ey];
      aly = st.aly[ey];
    }
    if (pb.flags & FLAG_FLO_LF) {
      alx = pb.dx / ((double)pb.dim * dt);
      aly = pb.dy / ((double)pb.dim * dt);
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
    // adjoints: ub of the node states, f0b/g0b of the point fluxes, Ub1 of U^1
    double ub[2][2][NV], f0b[2][2][NV], g0b[2][2][NV], Ub1[2][2][NV];
    // series adjoints: sfb on the row j2 = 0, sgb on the column j1 = 0
    double sfb[2][NV], sgb[2][NV];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int c = 0; c < NV; ++c) {
        sfb[a][c] = TB.ETA[1][a] * psix * Fb[c];
        sgb[a][c] = TB.ETA[1][a] * psiy * Gb[c];
      }
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int c = 0; c < NV; ++c) {
          // level 2 backwards, time node r = 0: the point fluxes' share
          const double fhb = (b == 0) ? TB.INVFACT[2] * sfb[a][c] : 0.0;
          const double ghb = (a == 0) ? TB.INVFACT[2] * sgb[b][c] : 0.0;
          f0b[b][a][c] = gt0 * fhb;
          g0b[b][a][c] = gt0 * ghb;
          ub[b][a][c] = 0.0;
          Ub1[b][a][c] = 0.0;
        }
    // time node r = 1 at the row and column nodes: the prediction
    // w = u + tay U^1, the flux Jacobians' transpose at w
#pragma unroll
    for (int n = 0; n < 3; ++n) {
      const int a = n == 1 ? 1 : 0, b = n == 2 ? 1 : 0;
      double w[NV], pfb[NV], pgb[NV], wb[NV];
#pragma unroll
      for (int c = 0; c < NV; ++c) {
        double s = 0.0;
        s = fma(gx[a][0], f0[b][0][c], s);
        s = fma(gx[a][1], f0[b][1][c], s);
        s = fma(gy[b][0], g0[0][a][c], s);
        s = fma(gy[b][1], g0[1][a][c], s);
        w[c] = fma(tay, s, u[b][a][c]);
        pfb[c] = (b == 0) ? gt1 * (TB.INVFACT[2] * sfb[a][c]) : 0.0;
        pgb[c] = (a == 0) ? gt1 * (TB.INVFACT[2] * sgb[b][c]) : 0.0;
        wb[c] = 0.0;
      }
      flux2d_vjp<FLUX, NV>(pb.ph, w, pfb, pgb, wb);
#pragma unroll
      for (int c = 0; c < NV; ++c) {
        ub[b][a][c] += wb[c];
        Ub1[b][a][c] = tay * wb[c];
      }
    }
    // U^1 = sum_l gx[a1][l] Fh_(l,a2) + sum_l gy[a2][l] Gh_(a1,l) transposed:
    // Fh^0bar_(a1,a2) = Fh^0 series term + sum_j gx[j][a1] Ub1_(j,a2), and
    // Gh^0bar along the column
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int c = 0; c < NV; ++c) {
          double sx = (b == 0) ? TB.INVFACT[1] * sfb[a][c] : 0.0;
          double sy = (a == 0) ? TB.INVFACT[1] * sgb[b][c] : 0.0;
          sx = fma(gx[0][a], Ub1[b][0][c], sx);
          sx = fma(gx[1][a], Ub1[b][1][c], sx);
          sy = fma(gy[0][b], Ub1[0][a][c], sy);
          sy = fma(gy[1][b], Ub1[1][a][c], sy);
          f0b[b][a][c] += sx;
          g0b[b][a][c] += sy;
        }
    // first-order parts of the FL-CAT2 blends on the two nodes each reads:
    // x on (0,0), (1,0); y on (0,0), (0,1)
#pragma unroll
    for (int c = 0; c < NV; ++c) {
      const double lx = 0.5 * (1.0 - psix) * Fb[c];
      f0b[0][0][c] += lx;
      ub[0][0][c] += alx * lx;
      f0b[0][1][c] += lx;
      ub[0][1][c] += -alx * lx;
      const double ly = 0.5 * (1.0 - psiy) * Gb[c];
      g0b[0][0][c] += ly;
      ub[0][0][c] += aly * ly;
      g0b[1][0][c] += ly;
      ub[1][0][c] += -aly * ly;
    }
    // Jacobian-transpose products at the node states; contributions
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        flux2d_vjp<FLUX, NV>(pb.ph, u[b][a], f0b[b][a], g0b[b][a], ub[b][a]);
        const int cslot = (b - 1 + pb.P) * (2 * pb.P) + (a - 1 + pb.P);
#pragma unroll
        for (int c = 0; c < NV; ++c) C[c * cstride + (int64_t)cslot * nitems + e] = ub[b][a][c];
      }
  }
}

// The mirror classes (QA, QB) and (QB, QA), QA < QB, in one launch (both
// recursions in one pass): the grid is cut into two runs of whole XCD groups
// of blocks sized by the classes' corner counts, at least one per class with
// corners; each block runs its class's body over its share of the list.
// The (1,2) pair is held to two waves per SIMD: unbounded it takes 264
// registers (one wave); bounded, 9 spill to scratch, and it runs 6 % faster.
template <int FLUX, int NV, int QA, int QB>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu((QB <= 2) ? 2 : 1))) void k_adj2d_pair(
    KProb pb, KStep st, const double* __restrict__ ubo, double* __restrict__ C, int LMAX) {
  constexpr int L = (2 * QA) * (2 * QB);
  __shared__ double2 xsm[2 * Xch<NV>::NP * adj_stride<L>()];
  __shared__ double g1s[(2 * QA) * (2 * QA) + (2 * QB) * (2 * QB)];
  const int ca = (QA - 1) * pb.P + (QB - 1), cb = (QB - 1) * pb.P + (QA - 1);
  const int64_t na = st.counts[ca], nb = st.counts[cb];
  if (na + nb == 0) return;
  const int units = (int)gridDim.x / NXCD;
  const int ua = na == 0 ? 0 : (nb == 0 ? units : 1 + (int)((int64_t)(units - 2) * na / (na + nb)));
  const int unit = (int)blockIdx.x / NXCD;
  if (unit < ua)
    adj2d_body<FLUX, NV, QA, QB, 3>(pb, st, Slice(st.counts, st.list, ca, blockIdx.x, ua * NXCD), ubo, C, LMAX,
                                    xsm, g1s);
  else
    adj2d_body<FLUX, NV, QB, QA, 3>(pb, st,
                                    Slice(st.counts, st.list, cb, blockIdx.x - ua * NXCD, (units - ua) * NXCD),
                                    ubo, C, LMAX, xsm, g1s);
}

// Corners k whose node at offset j reads cell m along one direction of n
// cells: k = m - j (wrapped when periodic); with the transmissive clamp, an
// edge cell is also read by every corner whose node lies beyond it
// (k + j <= 0 for m = 0, k + j >= n - 1 for m = n - 1); corners run over
// [-1, n - 1] there.
__device__ __forceinline__ void corners_reading(int m, int j, int n, bool per, int& lo, int& hi) {
  lo = hi = m - j;
  if (per) return;
  if (m == 0) lo = -1;
  if (m == n - 1) hi = n - 1;
  lo = lo < -1 ? -1 : lo;
  hi = hi > n - 1 ? n - 1 : hi;
}

// 2D gather: cell m collects node (j1, j2) of every corner whose rectangle
// holds that node and whose node reads cell m (j2, corner row, j1, corner
// column: one fixed order).  P (the problem's largest half-width) is a
// template argument: with periodic boundaries every offset has exactly one
// corner, the loops unroll and the (2P)^2 class-map loads are issued
// together instead of one after another.
template <int NV, bool PER, int P>
__global__ __launch_bounds__(BLOCK) void k_gather2d(KProb pb, KStep st, const double* __restrict__ ubo,
                                                    const double* __restrict__ C, int LMAX, double* ubi) {
  const int64_t m = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  const int nx = (int)pb.nx, ny = (int)pb.ny, ioff = (int)pb.ioff;
  if (m >= (int64_t)nx * ny) return;
  constexpr bool per = PER;
  const int m1 = (int)(m % nx), m2 = (int)(m / nx);
  const int64_t plane = (int64_t)nx * ny;
  const int64_t nitems = pb.n1 * pb.n2;
  const int64_t cstride = nitems * LMAX;
  double acc[NV];
#pragma unroll
  for (int c = 0; c < NV; ++c) acc[c] = ubo[c * plane + m];
  if constexpr (PER) {
    int8_t cl[2 * P][2 * P];
    int64_t ek[2 * P][2 * P];
#pragma unroll
    for (int j2 = -P + 1; j2 <= P; ++j2)
#pragma unroll
      for (int j1 = -P + 1; j1 <= P; ++j1) {
        const int r2 = bc_index32(m2 - j2, ny, PERIODIC), r1 = bc_index32(m1 - j1, nx, PERIODIC);
        const int64_t e = (int64_t)r2 * pb.n1 + r1;
        ek[j2 + P - 1][j1 + P - 1] = e;
        cl[j2 + P - 1][j1 + P - 1] = st.cls[e];
      }
#pragma unroll
    for (int j2 = -P + 1; j2 <= P; ++j2)
#pragma unroll
      for (int j1 = -P + 1; j1 <= P; ++j1) {
        const int c0 = cl[j2 + P - 1][j1 + P - 1];
        if (c0 < 0) continue;
        const int q1 = c0 / P + 1, q2 = c0 % P + 1;
        if (j1 < -q1 + 1 || j1 > q1 || j2 < -q2 + 1 || j2 > q2) continue;
        const int64_t e = ek[j2 + P - 1][j1 + P - 1];
        const int64_t slot = (int64_t)(j2 + P - 1) * (2 * P) + (j1 + P - 1);
#pragma unroll
        for (int c = 0; c < NV; ++c) acc[c] += C[c * cstride + slot * nitems + e];
      }
#pragma unroll
    for (int c = 0; c < NV; ++c) ubi[c * plane + m] = acc[c];
    return;
  }
  for (int j2 = -P + 1; j2 <= P; ++j2) {
    int lo2, hi2;
    corners_reading(m2, j2, ny, per, lo2, hi2);
    for (int k2 = lo2; k2 <= hi2; ++k2) {
      const int r2 = per ? bc_index32(k2, ny, PERIODIC) : k2;
      for (int j1 = -P + 1; j1 <= P; ++j1) {
        int lo1, hi1;
        corners_reading(m1, j1, nx, per, lo1, hi1);
        for (int k1 = lo1; k1 <= hi1; ++k1) {
          const int r1 = per ? bc_index32(k1, nx, PERIODIC) : k1;
          const int64_t e = (int64_t)(r2 - ioff) * pb.n1 + (r1 - ioff);
          const int cl = st.cls[e];
          if (cl < 0) continue;
          const int q1 = cl / P + 1, q2 = cl % P + 1;
          if (j1 < -q1 + 1 || j1 > q1 || j2 < -q2 + 1 || j2 > q2) continue;
          const int64_t slot = (int64_t)(j2 + P - 1) * (2 * P) + (j1 + P - 1);
#pragma unroll
          for (int c = 0; c < NV; ++c) acc[c] += C[c * cstride + slot * nitems + e];
        }
      }
    }
  }
#pragma unroll
  for (int c = 0; c < NV; ++c) ubi[c * plane + m] = acc[c];
}

#define ACAT_CHECK_LAUNCH()                  \
  do {                                       \
    hipError_t e_ = hipGetLastError();       \
    if (e_ != hipSuccess) return e_;         \
  } while (0)

template <int FLUX, int NV, int P, int p>
hipError_t launch_adj1d(const KProb& pb, const KStep& st, const double* ubo, double* C, hipStream_t s) {
  if constexpr (p <= P) {
    static const char* names[7] = {"", "adjoint1d_p1", "adjoint1d_p2", "adjoint1d_p3", "adjoint1d_p4",
                                   "adjoint1d_p5", "adjoint1d_p6"};
    auto kern = k_adj1d<FLUX, NV, p>;
    const int grid = group_grid<2 * p>(kern, pb.nIx, 0);
    {
      ProfScope ps(names[p], s);
      kern<<<grid, BLOCK, 0, s>>>(pb, st, ubo, C, 2 * P);
    }
    ACAT_CHECK_LAUNCH();
  }
  return hipSuccess;
}

template <int FLUX, int NV, int P>
hipError_t adj1d_impl(const KProb& pb, const KStep& st, const double* ubo, double* ubi, double* C, hipStream_t s) {
  hipError_t e;
  if ((e = launch_adj1d<FLUX, NV, P, 1>(pb, st, ubo, C, s)) != hipSuccess) return e;
  if ((e = launch_adj1d<FLUX, NV, P, 2>(pb, st, ubo, C, s)) != hipSuccess) return e;
  if ((e = launch_adj1d<FLUX, NV, P, 3>(pb, st, ubo, C, s)) != hipSuccess) return e;
  if ((e = launch_adj1d<FLUX, NV, P, 4>(pb, st, ubo, C, s)) != hipSuccess) return e;
  if ((e = launch_adj1d<FLUX, NV, P, 5>(pb, st, ubo, C, s)) != hipSuccess) return e;
  if ((e = launch_adj1d<FLUX, NV, P, 6>(pb, st, ubo, C, s)) != hipSuccess) return e;
  {
    ProfScope ps("gather1d", s);
    k_gather1d<NV><<<(unsigned)((pb.nx + BLOCK - 1) / BLOCK), BLOCK, 0, s>>>(pb, st, ubo, C, 2 * P, ubi);
  }
  ACAT_CHECK_LAUNCH();
  return hipSuccess;
}

template <int FLUX, int NV, int P, int Q1, int Q2>
hipError_t launch_adj2d(const KProb& pb, const KStep& st, const double* ubo, double* C, hipStream_t s) {
  if constexpr (Q1 <= P && Q2 <= P) {
    static const char* names[5][5] = {{"", "", "", "", ""},
                                      {"", "adjoint2d_q11", "adjoint2d_q12", "adjoint2d_q13", "adjoint2d_q14"},
                                      {"", "adjoint2d_q21", "adjoint2d_q22", "adjoint2d_q23", "adjoint2d_q24"},
                                      {"", "adjoint2d_q31", "adjoint2d_q32", "adjoint2d_q33", "adjoint2d_q34"},
                                      {"", "adjoint2d_q41", "adjoint2d_q42", "adjoint2d_q43", "adjoint2d_q44"}};
    // the rectangles with two recursions of orders 4 and 8 or 6 and 8 run
    // them in two launches (one recursion each, in order on the stream):
    // together in one kernel they exceed the register file several times
    constexpr bool SPLIT = Q1 != Q2 && Q1 >= 2 && Q2 >= 2 && Q1 + Q2 >= 6;
    if constexpr (Q1 == 1 && Q2 == 1) {
      // one lane per corner
      auto kern = k_adj2d_q11<FLUX, NV>;
      const int grid = persistent_grid(kern, pb.n1 * pb.n2, 0);
      ProfScope ps(names[1][1], s);
      kern<<<grid, BLOCK, 0, s>>>(pb, st, ubo, C, 4 * P * P);
    } else if constexpr (SPLIT) {
      auto k1 = k_adj2d<FLUX, NV, Q1, Q2, 1>;
      auto k2 = k_adj2d<FLUX, NV, Q1, Q2, 2>;
      ProfScope ps(names[Q1][Q2], s);
      k1<<<group_grid<(2 * Q1) * (2 * Q2)>(k1, pb.n1 * pb.n2, 0), BLOCK, 0, s>>>(pb, st, ubo, C, 4 * P * P);
      k2<<<group_grid<(2 * Q1) * (2 * Q2)>(k2, pb.n1 * pb.n2, 0), BLOCK, 0, s>>>(pb, st, ubo, C, 4 * P * P);
    } else {
      auto kern = k_adj2d<FLUX, NV, Q1, Q2>;
      const int grid = group_grid<(2 * Q1) * (2 * Q2)>(kern, pb.n1 * pb.n2, 0);
      ProfScope ps(names[Q1][Q2], s);
      kern<<<grid, BLOCK, 0, s>>>(pb, st, ubo, C, 4 * P * P);
    }
    ACAT_CHECK_LAUNCH();
  }
  return hipSuccess;
}

// The mirror classes (QA, QB) and (QB, QA), QA < QB, in one launch; only for
// the rectangles of orders up to 3 (those of order 4 keep one launch per class,
// the (1, 4) pair included: its device build gave wrong values).
template <int FLUX, int NV, int P, int QA, int QB>
hipError_t launch_adjpair2d(const KProb& pb, const KStep& st, const double* ubo, double* C, hipStream_t s) {
  static_assert(QA < QB && QB <= 3, "pairs of rectangles of orders up to 3 only");
  if constexpr (QB <= P) {
    static const char* names[4][4] = {{"", "", "", ""},
                                      {"", "", "adjoint2d_q12q21", "adjoint2d_q13q31"},
                                      {"", "", "", "adjoint2d_q23q32"},
                                      {"", "", "", ""}};
    auto kern = k_adj2d_pair<FLUX, NV, QA, QB>;
    // two runs of XCD groups: at least one per class
    const int grid = std::max(group_grid<(2 * QA) * (2 * QB)>(kern, pb.n1 * pb.n2, 0), 2 * NXCD);
    ProfScope ps(names[QA][QB], s);
    kern<<<grid, BLOCK, 0, s>>>(pb, st, ubo, C, 4 * P * P);
    ACAT_CHECK_LAUNCH();
  }
  return hipSuccess;
}

template <int FLUX, int NV, int P>
hipError_t adj2d_impl(const KProb& pb, const KStep& st, const double* ubo, double* ubi, double* C, hipStream_t s) {
  hipError_t e;
  if ((e = launch_adj2d<FLUX, NV, P, 1, 1>(pb, st, ubo, C, s)) != hipSuccess) return e;
  if ((e = launch_adjpair2d<FLUX, NV, P, 1, 2>(pb, st, ubo, C, s)) != hipSuccess) return e;
  if ((e = launch_adj2d<FLUX, NV, P, 2, 2>(pb, st, ubo, C, s)) != hipSuccess) return e;
  if ((e = launch_adjpair2d<FLUX, NV, P, 1, 3>(pb, st, ubo, C, s)) != hipSuccess) return e;
  if ((e = launch_adjpair2d<FLUX, NV, P, 2, 3>(pb, st, ubo, C, s)) != hipSuccess) return e;
  if ((e = launch_adj2d<FLUX, NV, P, 3, 3>(pb, st, ubo, C, s)) != hipSuccess) return e;
  if ((e = launch_adj2d<FLUX, NV, P, 1, 4>(pb, st, ubo, C, s)) != hipSuccess) return e;
  if ((e = launch_adj2d<FLUX, NV, P, 4, 1>(pb, st, ubo, C, s)) != hipSuccess) return e;
  if ((e = launch_adj2d<FLUX, NV, P, 2, 4>(pb, st, ubo, C, s)) != hipSuccess) return e;
  if ((e = launch_adj2d<FLUX, NV, P, 4, 2>(pb, st, ubo, C, s)) != hipSuccess) return e;
  if ((e = launch_adj2d<FLUX, NV, P, 3, 4>(pb, st, ubo, C, s)) != hipSuccess) return e;
  if ((e = launch_adj2d<FLUX, NV, P, 4, 3>(pb, st, ubo, C, s)) != hipSuccess) return e;
  if ((e = launch_adj2d<FLUX, NV, P, 4, 4>(pb, st, ubo, C, s)) != hipSuccess) return e;
  {
    ProfScope ps("gather2d", s);
    const unsigned gb = (unsigned)((pb.nx * pb.ny + BLOCK - 1) / BLOCK);
    if (pb.bc == PERIODIC) k_gather2d<NV, true, P><<<gb, BLOCK, 0, s>>>(pb, st, ubo, C, 4 * P * P, ubi);
    else k_gather2d<NV, false, P><<<gb, BLOCK, 0, s>>>(pb, st, ubo, C, 4 * P * P, ubi);
  }
  ACAT_CHECK_LAUNCH();
  return hipSuccess;
}

}  // namespace

hipError_t launch_adjoint(const KProb& pb, const KStep& st, const double* ubo, double* ubi, double* C,
                          hipStream_t s) {
  if (pb.dim == 1) {
    if (pb.flux == EUL) {
      switch (pb.P) {
        case 1: return adj1d_impl<EUL, 3, 1>(pb, st, ubo, ubi, C, s);
        case 2: return adj1d_impl<EUL, 3, 2>(pb, st, ubo, ubi, C, s);
        case 3: return adj1d_impl<EUL, 3, 3>(pb, st, ubo, ubi, C, s);
        case 4: return adj1d_impl<EUL, 3, 4>(pb, st, ubo, ubi, C, s);
        case 5: return adj1d_impl<EUL, 3, 5>(pb, st, ubo, ubi, C, s);
        case 6: return adj1d_impl<EUL, 3, 6>(pb, st, ubo, ubi, C, s);
      }
    } else if (pb.flux == BURG) {
      switch (pb.P) {
        case 1: return adj1d_impl<BURG, 1, 1>(pb, st, ubo, ubi, C, s);
        case 2: return adj1d_impl<BURG, 1, 2>(pb, st, ubo, ubi, C, s);
        case 3: return adj1d_impl<BURG, 1, 3>(pb, st, ubo, ubi, C, s);
        case 4: return adj1d_impl<BURG, 1, 4>(pb, st, ubo, ubi, C, s);
        case 5: return adj1d_impl<BURG, 1, 5>(pb, st, ubo, ubi, C, s);
        case 6: return adj1d_impl<BURG, 1, 6>(pb, st, ubo, ubi, C, s);
      }
    } else {
      switch (pb.P) {
        case 1: return adj1d_impl<ADV, 1, 1>(pb, st, ubo, ubi, C, s);
        case 2: return adj1d_impl<ADV, 1, 2>(pb, st, ubo, ubi, C, s);
        case 3: return adj1d_impl<ADV, 1, 3>(pb, st, ubo, ubi, C, s);
        case 4: return adj1d_impl<ADV, 1, 4>(pb, st, ubo, ubi, C, s);
        case 5: return adj1d_impl<ADV, 1, 5>(pb, st, ubo, ubi, C, s);
        case 6: return adj1d_impl<ADV, 1, 6>(pb, st, ubo, ubi, C, s);
      }
    }
  } else {
    if (pb.flux == EUL) {
      switch (pb.P) {
        case 1: return adj2d_impl<EUL, 4, 1>(pb, st, ubo, ubi, C, s);
        case 2: return adj2d_impl<EUL, 4, 2>(pb, st, ubo, ubi, C, s);
        case 3: return adj2d_impl<EUL, 4, 3>(pb, st, ubo, ubi, C, s);
        case 4: return adj2d_impl<EUL, 4, 4>(pb, st, ubo, ubi, C, s);
      }
    } else {
      switch (pb.P) {
        case 1: return adj2d_impl<ADV, 1, 1>(pb, st, ubo, ubi, C, s);
        case 2: return adj2d_impl<ADV, 1, 2>(pb, st, ubo, ubi, C, s);
        case 3: return adj2d_impl<ADV, 1, 3>(pb, st, ubo, ubi, C, s);
        case 4: return adj2d_impl<ADV, 1, 4>(pb, st, ubo, ubi, C, s);
      }
    }
  }
  return hipErrorInvalidValue;
}

}  // namespace acat
