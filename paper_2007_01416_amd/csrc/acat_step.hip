// ACAT forward step on gfx950: classification, per-order-class flux kernels,
// conservative update, CFL reduction.
//
// Data flow of one step (all on one stream, no host synchronisation):
//   k_zero         clears the per-class counters
//   k_classify*    one thread per 1D interface / 2D corner: smoothness
//                  indicators psi^p (Sec. 3.2, minimum over components,
//                  Sec. 3.4), order p_s (Sec. 3, admissible set), and where
//                  p_s = 1 the superbee weight psi^1 (Sec. 3.1) and the
//                  Rusanov speed; appends the item to the work list of its
//                  order class (wave ballot + one atomic per wave and class)
//   k_flux*<class> persistent kernels, one per order class: one LANE PER
//                  STENCIL NODE, so a 1D interface of order p occupies 2p
//                  lanes and a 2D corner of orders (q1, q2) occupies
//                  2q1 x 2q2 lanes.  Each lane keeps its node's state and
//                  Taylor history in registers and evaluates the flux at its
//                  own predicted states; the only cross-lane step, the
//                  spatial derivative of the time-derivative fluxes, goes
//                  through LDS (Sec. 2.2 recursion, Sec. 4 corner recursion)
//   k_update*      conservative flux-difference update + status bits
#include <hip/hip_runtime.h>

#include "acat_internal.hpp"
#include "coeffs.hpp"

namespace acat {
namespace {

constexpr CoeffTables TB = make_tables();
constexpr int NXCD = 8;   // MI355X: 8 accelerator complex dies, each with its own L2

// ---------------------------------------------------------------- helpers
__device__ __forceinline__ double superbee(double r) { return fmax(0.0, fmax(fmin(2.0 * r, 1.0), fmin(r, 2.0))); }

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
  const double I = IL * IR / (IL + IR);
  double s = 0.0;
#pragma unroll
  for (int j = -p + 1; j <= p; ++j) s += TB.TAU[p][j + p - 1] * v[j + G - 1];
  double tau = TB.FACT2PM1[p] * s;
  tau = tau * tau;
  return I / (I + tau);
}

// p_s = max{p in 2..P : min_c psi^{c,p} >= theta}, else 1 (evaluated from P down)
template <int NV, int G, int p>
struct Select {
  __device__ static __forceinline__ int run(const double (&v)[NV][2 * G], double eps, double theta) {
    double psi = 1.0;
#pragma unroll
    for (int c = 0; c < NV; ++c) psi = fmin(psi, psi_comp<G, p>(v[c], eps));
    if (psi >= theta) return p;
    return Select<NV, G, p - 1>::run(v, eps, theta);
  }
};
template <int NV, int G>
struct Select<NV, G, 1> {
  __device__ static __forceinline__ int run(const double (&)[NV][2 * G], double, double) { return 1; }
};

// psi^1 = min_c min(phi(r+), phi(r-)); a component with u_{i+1} = u_i gives 1
template <int NV, int G>
__device__ __forceinline__ double limiter(const double (&v)[NV][2 * G]) {
  double psi = 1e300;
#pragma unroll
  for (int c = 0; c < NV; ++c) {
    const double dl = v[c][G] - v[c][G - 1];
    double l = 1.0;
    if (dl != 0.0) {
      const double rm = (v[c][G - 1] - v[c][G - 2]) / dl;
      const double rp = (v[c][G + 1] - v[c][G]) / dl;
      l = fmin(superbee(rp), superbee(rm));
    }
    psi = fmin(psi, l);
  }
  return psi;
}

// Append `id` to the list of class `cls` (all lanes of the wave call this).
__device__ __forceinline__ void append(int32_t* counts, int32_t* lists, int64_t stride, int ncls, bool valid,
                                       int cls, int32_t id) {
  const int lane = __lane_id();
  for (int c = 0; c < ncls; ++c) {
    const unsigned long long m = __ballot(valid && cls == c);
    if (m == 0ull) continue;
    const int leader = __ffsll((long long)m) - 1;
    int base = 0;
    if (lane == leader) base = atomicAdd(&counts[c], __popcll(m));
    base = __shfl(base, leader);
    if (valid && cls == c) {
      const unsigned long long below = m & ((1ull << lane) - 1ull);
      lists[(int64_t)c * stride + base + __popcll(below)] = id;
    }
  }
}

// Persistent-loop partition: blocks on XCD x (blockIdx % 8) walk a contiguous
// eighth of the work list, so neighbouring items share that XCD's L2.
struct Part {
  int64_t beg, end, first, step;
  __device__ Part(int32_t count, int per_block) {
    const int xcd = blockIdx.x % NXCD;
    const int nb = gridDim.x / NXCD;
    const int bx = blockIdx.x / NXCD;
    beg = (int64_t)count * xcd / NXCD;
    end = (int64_t)count * (xcd + 1) / NXCD;
    first = beg + (int64_t)bx * per_block;
    step = (int64_t)nb * per_block;
  }
};

__global__ void k_zero_i32(int32_t* p, int n) {
  const int t = threadIdx.x;
  if (t < n) p[t] = 0;
}

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
  if (valid) {
    if (st.replay) {
      ps = st.ordx[k];
    } else {
      const int64_t i = k + pb.ioff;
      double v[NV][2 * G];
#pragma unroll
      for (int a = 0; a < 2 * G; ++a) {
        const int64_t node = bc_index(i - G + 1 + a, pb.nx, pb.bc);
#pragma unroll
        for (int c = 0; c < NV; ++c) v[c][a] = st.u[c * pb.nx + node];
      }
      ps = Select<NV, G, P>::run(v, pb.eps, pb.theta);
      double psi1 = -1.0, al = -1.0;
      if (ps == 1) {
        psi1 = limiter<NV, G>(v);
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
  append(st.counts, st.lists, st.list_stride, P, valid, ps - 1, (int32_t)k);
}

// CAT2p flux of the interfaces of order class p (p = 1: FL-CAT2 blend).
// Rounding follows one fixed order: every weighted sum of the recursion is a
// chain of fused multiply-adds in index order, nothing else is contracted
// (the library is built with -ffp-contract=off).
template <int FLUX, int NV, int p>
__global__ __launch_bounds__(BLOCK) void k_flux1d(KProb pb, KStep st) {
  constexpr int L = 2 * p;            // lanes per interface = stencil nodes
  constexpr int GPB = BLOCK / L;      // interfaces per block
  __shared__ double xs[2][(BLOCK + L) * NV];

  const int tid = threadIdx.x;
  const int g = tid / L;
  const int a = tid - g * L;          // node index, offset j = a - p + 1
  const bool inblk = g < GPB;
  const int32_t count = st.counts[p - 1];
  const int32_t* list = st.lists + (int64_t)(p - 1) * st.list_stride;
  const double lam = step_dt(st) / pb.dx;
  const int64_t nx = pb.nx;

  double g1[L];
#pragma unroll
  for (int l = 0; l < L; ++l) g1[l] = TB.G1[p][a][l];

  int buf = 0;
  const Part part(count, GPB);
  for (int64_t base = part.first; base < part.end; base += part.step) {
    const int64_t item = base + g;
    const bool valid = inblk && item < part.end;
    const bool lead = valid && a == 0;   // lane that assembles the interface flux
    const int32_t k = valid ? list[item] : 0;
    const int64_t i = k + pb.ioff;
    const int64_t node = bc_index(i + (a - p + 1), nx, pb.bc);
    double u[NV];
#pragma unroll
    for (int c = 0; c < NV; ++c) u[c] = valid ? st.u[c * nx + node] : 1.0;

    double fh0[NV], cur[NV], F[NV];
    flux1d<FLUX, NV>(pb.ph, u, fh0);
#pragma unroll
    for (int c = 0; c < NV; ++c) {
      cur[c] = fh0[c];
      F[c] = 0.0;
    }
    double U[L][NV];   // U[l] = dt^l u~^(l) at this node, l = 1 .. 2p-1
#pragma unroll
    for (int kk = 2; kk <= 2 * p + 1; ++kk) {
      // share Fh^{kk-2} of every node of the stencil
#pragma unroll
      for (int c = 0; c < NV; ++c) xs[buf][tid * NV + c] = cur[c];
      __syncthreads();
      const double* row = &xs[buf][g * L * NV];
      if (lead) {
        // F += (1/(kk-1)!) sum_j eta_j Fh^{kk-2}_j  (the CAT flux, Sec. 2.2)
#pragma unroll
        for (int c = 0; c < NV; ++c) {
          double t = 0.0;
#pragma unroll
          for (int l = 0; l < L; ++l) t = fma(TB.ETA[p][l], row[l * NV + c], t);
          F[c] = fma(TB.INVFACT[kk - 1], t, F[c]);
        }
      }
      if (kk == 2 * p + 1) break;
      // U^{kk-1} = -lambda * (spatial derivative of Fh^{kk-2} at this node)
#pragma unroll
      for (int c = 0; c < NV; ++c) {
        double sacc = 0.0;
#pragma unroll
        for (int l = 0; l < L; ++l) sacc = fma(g1[l], row[l * NV + c], sacc);
        U[kk - 1][c] = -lam * sacc;
      }
      buf ^= 1;
      // flux at the Taylor-predicted states of the time nodes r, and its
      // (kk-1)-th time derivative at r = 0
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
    if (lead) {
      if constexpr (p == 1) {
        // FL-CAT2 (Sec. 3.1): psi^1 CAT2 + (1 - psi^1) Rusanov
        const double psi = st.psix[k], al = st.alx[k];
        const int64_t nr = bc_index(i + 1, nx, pb.bc);
        double uR[NV], fR[NV];
#pragma unroll
        for (int c = 0; c < NV; ++c) uR[c] = st.u[c * nx + nr];
        flux1d<FLUX, NV>(pb.ph, uR, fR);
#pragma unroll
        for (int c = 0; c < NV; ++c) {
          const double flo = 0.5 * (fh0[c] + fR[c]) - (0.5 * al) * (uR[c] - u[c]);
          F[c] = psi * F[c] + (1.0 - psi) * flo;
        }
      }
#pragma unroll
      for (int c = 0; c < NV; ++c) st.Fx[c * pb.nIx + k] = F[c];
    }
    buf ^= 1;
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
template <int FLUX, int NV, int P>
__global__ __launch_bounds__(BLOCK) void k_classify2d(KProb pb, KStep st) {
  constexpr int G = P > 2 ? P : 2;
  const int64_t e = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  const int64_t nx = pb.nx, ny = pb.ny;
  const int64_t i1 = (e < pb.n1 * pb.n2) ? e % pb.n1 + pb.ioff : 0;
  const int64_t i2 = (e < pb.n1 * pb.n2) ? e / pb.n1 + pb.ioff : 0;
  const bool needF = i2 >= 0, needG = i1 >= 0;
  const bool valid = e < pb.n1 * pb.n2 && (needF || needG);
  int q1 = 1, q2 = 1;
  if (valid) {
    const int64_t r2 = bc_index(i2, ny, pb.bc);   // ghost rows read the clamped row
    const int64_t r1 = bc_index(i1, nx, pb.bc);
    if (st.replay) {
      q1 = st.ordx[r2 * pb.nIx + (i1 - pb.ioff)];
      q2 = st.ordy[(i2 - pb.ioff) * nx + r1];
    } else {
      double v[NV][2 * G];
      // x-interface (i1 + 1/2, i2)
#pragma unroll
      for (int a = 0; a < 2 * G; ++a) {
        const int64_t x = bc_index(i1 - G + 1 + a, nx, pb.bc);
#pragma unroll
        for (int c = 0; c < NV; ++c) v[c][a] = st.u[(c * ny + r2) * nx + x];
      }
      q1 = Select<NV, G, P>::run(v, pb.eps, pb.theta);
      if (needF) {
        double psi1 = -1.0, al = -1.0;
        if (q1 == 1) {
          psi1 = limiter<NV, G>(v);
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
      // y-interface (i1, i2 + 1/2)
#pragma unroll
      for (int a = 0; a < 2 * G; ++a) {
        const int64_t y = bc_index(i2 - G + 1 + a, ny, pb.bc);
#pragma unroll
        for (int c = 0; c < NV; ++c) v[c][a] = st.u[(c * ny + y) * nx + r1];
      }
      q2 = Select<NV, G, P>::run(v, pb.eps, pb.theta);
      if (needG) {
        double psi1 = -1.0, al = -1.0;
        if (q2 == 1) {
          psi1 = limiter<NV, G>(v);
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
  append(st.counts, st.lists, st.list_stride, P * P, valid, (q1 - 1) * P + (q2 - 1), (int32_t)e);
}

// One recursion over the rectangle J_Q1 x J_Q2 with time nodes J_QT
// (Taylor order 2 QT).  Each lane is one node (a1, a2); the lead lane (node
// (0, 0)) assembles F from row j2 = 0 (DOF) and G from column j1 = 0 (DOG).
// Same fixed rounding as the 1D kernel.
template <int FLUX, int NV, int Q1, int Q2, int QT, bool DOF, bool DOG>
__device__ __forceinline__ void corner_pass(const Phys& ph, double lamx, double lamy, const double (&u)[NV],
                                            const double (&f0)[NV], const double (&g0)[NV],
                                            const double (&g1x)[2 * Q1], const double (&g1y)[2 * Q2],
                                            double (*xs)[(BLOCK + 4 * Q1 * Q2) * 2 * NV], int& buf, int tid,
                                            int gbase, int a1, int a2, bool lead, double (&F)[NV],
                                            double (&G)[NV]) {
  constexpr int N1 = 2 * Q1, N2 = 2 * Q2, S = 2 * NV;
  double fc[NV], gc[NV];
#pragma unroll
  for (int c = 0; c < NV; ++c) {
    fc[c] = f0[c];
    gc[c] = g0[c];
    if (DOF) F[c] = 0.0;
    if (DOG) G[c] = 0.0;
  }
  double U[2 * QT][NV];
#pragma unroll
  for (int kk = 2; kk <= 2 * QT + 1; ++kk) {
#pragma unroll
    for (int c = 0; c < NV; ++c) {
      xs[buf][tid * S + c] = fc[c];
      xs[buf][tid * S + NV + c] = gc[c];
    }
    __syncthreads();
    const double* rowp = &xs[buf][(gbase + a2 * N1) * S];   // this node's row  (l, j2)
    const double* colp = &xs[buf][(gbase + a1) * S + NV];   // this node's column (j1, l)
    if (lead) {
      // F += (1/(kk-1)!) sum_l eta_l Fh^{kk-2}_(l,0);  G likewise on column 0
#pragma unroll
      for (int c = 0; c < NV; ++c) {
        if (DOF) {
          double t = 0.0;
#pragma unroll
          for (int l = 0; l < N1; ++l) t = fma(TB.ETA[Q1][l], rowp[l * S + c], t);
          F[c] = fma(TB.INVFACT[kk - 1], t, F[c]);
        }
        if (DOG) {
          double t = 0.0;
#pragma unroll
          for (int l = 0; l < N2; ++l) t = fma(TB.ETA[Q2][l], colp[l * N1 * S + c], t);
          G[c] = fma(TB.INVFACT[kk - 1], t, G[c]);
        }
      }
    }
    if (kk == 2 * QT + 1) break;
    // U^{kk-1} = -lamx d_x Fh^{kk-2} - lamy d_y Gh^{kk-2} at this node
#pragma unroll
    for (int c = 0; c < NV; ++c) {
      double sx = 0.0, sy = 0.0;
#pragma unroll
      for (int l = 0; l < N1; ++l) sx = fma(g1x[l], rowp[l * S + c], sx);
#pragma unroll
      for (int l = 0; l < N2; ++l) sy = fma(g1y[l], colp[l * N1 * S + c], sy);
      U[kk - 1][c] = -lamx * sx - lamy * sy;
    }
    buf ^= 1;
    double nf[NV], ng[NV];
#pragma unroll
    for (int c = 0; c < NV; ++c) {
      nf[c] = 0.0;
      ng[c] = 0.0;
    }
#pragma unroll
    for (int ri = 0; ri < 2 * QT; ++ri) {
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
  // the lead lane may still read the buffer of the final exchange: the next
  // writer (a second pass or the next corner) must use the other one
  buf ^= 1;
}

// Fluxes of the corners of order class (Q1, Q2) (Sec. 4; rectangle J_Q1 x J_Q2).
template <int FLUX, int NV, int Q1, int Q2>
__global__ __launch_bounds__(BLOCK) void k_flux2d(KProb pb, KStep st) {
  constexpr int N1 = 2 * Q1, N2 = 2 * Q2, L = N1 * N2, CPB = BLOCK / L, S = 2 * NV;
  __shared__ double xs[2][(BLOCK + L) * S];

  const int tid = threadIdx.x;
  const int g = tid / L;
  const int nd = tid - g * L;
  const int a1 = nd % N1, a2 = nd / N1;     // node (j1, j2) = (a1 - Q1 + 1, a2 - Q2 + 1)
  const bool inblk = g < CPB;
  const int P = pb.P;
  const int cls = (Q1 - 1) * P + (Q2 - 1);
  const int32_t count = st.counts[cls];
  const int32_t* list = st.lists + (int64_t)cls * st.list_stride;
  const double dt = step_dt(st);
  const double lamx = dt / pb.dx, lamy = dt / pb.dy;
  const int64_t nx = pb.nx, ny = pb.ny;

  double g1x[N1], g1y[N2];
#pragma unroll
  for (int l = 0; l < N1; ++l) g1x[l] = TB.G1[Q1][a1][l];
#pragma unroll
  for (int l = 0; l < N2; ++l) g1y[l] = TB.G1[Q2][a2][l];

  int buf = 0;
  const Part part(count, CPB);
  for (int64_t base = part.first; base < part.end; base += part.step) {
    const int64_t item = base + g;
    const bool valid = inblk && item < part.end;
    const bool lead = valid && a1 == Q1 - 1 && a2 == Q2 - 1;
    const int32_t e = valid ? list[item] : 0;
    const int64_t i1 = e % pb.n1 + pb.ioff, i2 = e / pb.n1 + pb.ioff;
    const int64_t x = bc_index(i1 + (a1 - Q1 + 1), nx, pb.bc);
    const int64_t y = bc_index(i2 + (a2 - Q2 + 1), ny, pb.bc);
    double u[NV];
#pragma unroll
    for (int c = 0; c < NV; ++c) u[c] = valid ? st.u[(c * ny + y) * nx + x] : 1.0;
    double f0[NV], g0[NV], F[NV], Gv[NV];
    flux2d<FLUX, NV>(pb.ph, u, f0, g0);
    if constexpr (Q1 == Q2) {
      corner_pass<FLUX, NV, Q1, Q2, Q1, true, true>(pb.ph, lamx, lamy, u, f0, g0, g1x, g1y, xs, buf, tid, g * L,
                                                    a1, a2, lead, F, Gv);
    } else {
      corner_pass<FLUX, NV, Q1, Q2, Q1, true, false>(pb.ph, lamx, lamy, u, f0, g0, g1x, g1y, xs, buf, tid, g * L,
                                                     a1, a2, lead, F, Gv);
      corner_pass<FLUX, NV, Q1, Q2, Q2, false, true>(pb.ph, lamx, lamy, u, f0, g0, g1x, g1y, xs, buf, tid, g * L,
                                                     a1, a2, lead, F, Gv);
    }
    if (lead) {
      const bool needF = i2 >= 0, needG = i1 >= 0;
      if constexpr (Q1 == 1) {
        if (needF) {   // 2D FL-CAT2 in x (Sec. 4)
          const int64_t ex = i2 * pb.nIx + (i1 - pb.ioff);
          const double psi = st.psix[ex], al = st.alx[ex];
          const int64_t xr = bc_index(i1 + 1, nx, pb.bc);
          double uR[NV], fR[NV], gR[NV];
#pragma unroll
          for (int c = 0; c < NV; ++c) uR[c] = st.u[(c * ny + y) * nx + xr];
          flux2d<FLUX, NV>(pb.ph, uR, fR, gR);
#pragma unroll
          for (int c = 0; c < NV; ++c) {
            const double flo = 0.5 * (f0[c] + fR[c]) - (0.5 * al) * (uR[c] - u[c]);
            F[c] = psi * F[c] + (1.0 - psi) * flo;
          }
        }
      }
      if constexpr (Q2 == 1) {
        if (needG) {   // 2D FL-CAT2 in y
          const int64_t ey = (i2 - pb.ioff) * nx + i1;
          const double psi = st.psiy[ey], al = st.aly[ey];
          const int64_t yr = bc_index(i2 + 1, ny, pb.bc);
          double uR[NV], fR[NV], gR[NV];
#pragma unroll
          for (int c = 0; c < NV; ++c) uR[c] = st.u[(c * ny + yr) * nx + x];
          flux2d<FLUX, NV>(pb.ph, uR, fR, gR);
#pragma unroll
          for (int c = 0; c < NV; ++c) {
            const double glo = 0.5 * (g0[c] + gR[c]) - (0.5 * al) * (uR[c] - u[c]);
            Gv[c] = psi * Gv[c] + (1.0 - psi) * glo;
          }
        }
      }
      if (needF) {
#pragma unroll
        for (int c = 0; c < NV; ++c) st.Fx[(c * ny + i2) * pb.nIx + (i1 - pb.ioff)] = F[c];
      }
      if (needG) {
#pragma unroll
        for (int c = 0; c < NV; ++c) st.Gy[(c * pb.nIy + (i2 - pb.ioff)) * nx + i1] = Gv[c];
      }
    }
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
  // the bit patterns of non-negative doubles order like the values
  if (__lane_id() == 0) {
    atomicMax(&smax[0], (unsigned long long)__double_as_longlong(m0));
    if (DIM == 2) atomicMax(&smax[1], (unsigned long long)__double_as_longlong(m1));
  }
}

__global__ void k_cfl_dt(int dim, double dx, double dy, const double* smax, double cfl, double t_final,
                         double* t_dev, double* dt_dev) {
  double dt = dim == 1 ? cfl * dx / smax[0] : 0.5 * cfl * fmin(dx / smax[0], dy / smax[1]);
  if (t_dev) {
    const double t = *t_dev;
    if (t >= t_final) dt = 0.0;
    else if (t + dt > t_final) dt = t_final - t;
    *t_dev = t + dt;
  }
  *dt_dev = dt;
}

// ================================================================ launchers
int flux_grid(int64_t nitems, int per_block, int cap) {
  int64_t b = (nitems + per_block - 1) / per_block;
  if (b > cap) b = cap;
  if (b < 1) b = 1;
  b = (b + NXCD - 1) / NXCD * NXCD;   // whole XCD rounds
  return (int)b;
}

#define ACAT_CHECK_LAUNCH()                  \
  do {                                       \
    hipError_t e_ = hipGetLastError();       \
    if (e_ != hipSuccess) return e_;         \
  } while (0)

template <int FLUX, int NV, int P>
hipError_t step1d_impl(const KProb& pb, const KStep& st, int cap, hipStream_t s) {
  {
    ProfScope ps("zero", s);
    k_zero_i32<<<1, 64, 0, s>>>(st.counts, MAX_CLASSES);
  }
  ACAT_CHECK_LAUNCH();
  const int64_t nI = pb.nIx;
  {
    ProfScope ps("classify1d", s);
    k_classify1d<FLUX, NV, P><<<(unsigned)((nI + BLOCK - 1) / BLOCK), BLOCK, 0, s>>>(pb, st);
  }
  ACAT_CHECK_LAUNCH();
  {
    ProfScope ps("flux1d_p1", s);
    k_flux1d<FLUX, NV, 1><<<flux_grid(nI, BLOCK / 2, cap), BLOCK, 0, s>>>(pb, st);
  }
  ACAT_CHECK_LAUNCH();
  if constexpr (P >= 2) {
    ProfScope ps("flux1d_p2", s);
    k_flux1d<FLUX, NV, 2><<<flux_grid(nI, BLOCK / 4, cap), BLOCK, 0, s>>>(pb, st);
  }
  ACAT_CHECK_LAUNCH();
  if constexpr (P >= 3) {
    ProfScope ps("flux1d_p3", s);
    k_flux1d<FLUX, NV, 3><<<flux_grid(nI, BLOCK / 6, cap), BLOCK, 0, s>>>(pb, st);
  }
  ACAT_CHECK_LAUNCH();
  if constexpr (P >= 4) {
    ProfScope ps("flux1d_p4", s);
    k_flux1d<FLUX, NV, 4><<<flux_grid(nI, BLOCK / 8, cap), BLOCK, 0, s>>>(pb, st);
  }
  ACAT_CHECK_LAUNCH();
  {
    ProfScope ps("update1d", s);
    k_update1d<FLUX, NV><<<(unsigned)((pb.nx + BLOCK - 1) / BLOCK), BLOCK, 0, s>>>(pb, st);
  }
  ACAT_CHECK_LAUNCH();
  return hipSuccess;
}

template <int FLUX, int NV, int P, int Q1, int Q2>
hipError_t launch_class2d(const KProb& pb, const KStep& st, int64_t ncorner, int cap, hipStream_t s) {
  if constexpr (Q1 <= P && Q2 <= P) {
    constexpr int L = 4 * Q1 * Q2;
    static const char* names[4][4] = {{"", "", "", ""},
                                      {"", "flux2d_q11", "flux2d_q12", "flux2d_q13"},
                                      {"", "flux2d_q21", "flux2d_q22", "flux2d_q23"},
                                      {"", "flux2d_q31", "flux2d_q32", "flux2d_q33"}};
    {
      ProfScope ps(names[Q1][Q2], s);
      k_flux2d<FLUX, NV, Q1, Q2><<<flux_grid(ncorner, BLOCK / L, cap), BLOCK, 0, s>>>(pb, st);
    }
    ACAT_CHECK_LAUNCH();
  }
  return hipSuccess;
}

template <int FLUX, int NV, int P>
hipError_t step2d_impl(const KProb& pb, const KStep& st, int cap, hipStream_t s) {
  {
    ProfScope ps("zero", s);
    k_zero_i32<<<1, 64, 0, s>>>(st.counts, MAX_CLASSES);
  }
  ACAT_CHECK_LAUNCH();
  const int64_t nc = pb.n1 * pb.n2;
  {
    ProfScope ps("classify2d", s);
    k_classify2d<FLUX, NV, P><<<(unsigned)((nc + BLOCK - 1) / BLOCK), BLOCK, 0, s>>>(pb, st);
  }
  ACAT_CHECK_LAUNCH();
  hipError_t e;
  if ((e = launch_class2d<FLUX, NV, P, 1, 1>(pb, st, nc, cap, s)) != hipSuccess) return e;
  if ((e = launch_class2d<FLUX, NV, P, 1, 2>(pb, st, nc, cap, s)) != hipSuccess) return e;
  if ((e = launch_class2d<FLUX, NV, P, 2, 1>(pb, st, nc, cap, s)) != hipSuccess) return e;
  if ((e = launch_class2d<FLUX, NV, P, 2, 2>(pb, st, nc, cap, s)) != hipSuccess) return e;
  if ((e = launch_class2d<FLUX, NV, P, 1, 3>(pb, st, nc, cap, s)) != hipSuccess) return e;
  if ((e = launch_class2d<FLUX, NV, P, 3, 1>(pb, st, nc, cap, s)) != hipSuccess) return e;
  if ((e = launch_class2d<FLUX, NV, P, 2, 3>(pb, st, nc, cap, s)) != hipSuccess) return e;
  if ((e = launch_class2d<FLUX, NV, P, 3, 2>(pb, st, nc, cap, s)) != hipSuccess) return e;
  if ((e = launch_class2d<FLUX, NV, P, 3, 3>(pb, st, nc, cap, s)) != hipSuccess) return e;
  {
    ProfScope ps("update2d", s);
    k_update2d<FLUX, NV><<<(unsigned)((pb.nx * pb.ny + BLOCK - 1) / BLOCK), BLOCK, 0, s>>>(pb, st);
  }
  ACAT_CHECK_LAUNCH();
  return hipSuccess;
}

constexpr int kFluxBlockCap = 256 * 8;   // persistent grid: at most 8 blocks per CU

}  // namespace

hipError_t launch_step_1d(const KProb& pb, const KStep& st, int grid_blocks, hipStream_t s) {
  const int cap = grid_blocks > 0 ? grid_blocks : kFluxBlockCap;
  if (pb.flux == EUL) {
    switch (pb.P) {
      case 1: return step1d_impl<EUL, 3, 1>(pb, st, cap, s);
      case 2: return step1d_impl<EUL, 3, 2>(pb, st, cap, s);
      case 3: return step1d_impl<EUL, 3, 3>(pb, st, cap, s);
      case 4: return step1d_impl<EUL, 3, 4>(pb, st, cap, s);
    }
  } else if (pb.flux == BURG) {
    switch (pb.P) {
      case 1: return step1d_impl<BURG, 1, 1>(pb, st, cap, s);
      case 2: return step1d_impl<BURG, 1, 2>(pb, st, cap, s);
      case 3: return step1d_impl<BURG, 1, 3>(pb, st, cap, s);
      case 4: return step1d_impl<BURG, 1, 4>(pb, st, cap, s);
    }
  } else {
    switch (pb.P) {
      case 1: return step1d_impl<ADV, 1, 1>(pb, st, cap, s);
      case 2: return step1d_impl<ADV, 1, 2>(pb, st, cap, s);
      case 3: return step1d_impl<ADV, 1, 3>(pb, st, cap, s);
      case 4: return step1d_impl<ADV, 1, 4>(pb, st, cap, s);
    }
  }
  return hipErrorInvalidValue;
}

hipError_t launch_step_2d(const KProb& pb, const KStep& st, int grid_blocks, hipStream_t s) {
  const int cap = grid_blocks > 0 ? grid_blocks : kFluxBlockCap;
  if (pb.flux == EUL) {
    switch (pb.P) {
      case 1: return step2d_impl<EUL, 4, 1>(pb, st, cap, s);
      case 2: return step2d_impl<EUL, 4, 2>(pb, st, cap, s);
      case 3: return step2d_impl<EUL, 4, 3>(pb, st, cap, s);
    }
  } else if (pb.flux == ADV) {
    switch (pb.P) {
      case 1: return step2d_impl<ADV, 1, 1>(pb, st, cap, s);
      case 2: return step2d_impl<ADV, 1, 2>(pb, st, cap, s);
      case 3: return step2d_impl<ADV, 1, 3>(pb, st, cap, s);
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
  if (blocks > 2048) blocks = 2048;
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
