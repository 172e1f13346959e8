// Fluxes and spectral radii of the supported conservation laws (device code).
//   advection  f = ax u, g = ay u                  (Sec. 5.1 / 5.4)
//   Burgers    f = u^2 / 2                          (Sec. 5.2)
//   Euler 1D   u = (rho, rho v, E), ideal gas      (Sec. 5.3)
//   Euler 2D   u = (rho, rho v, rho w, E)          (Sec. 5.5)
#pragma once

#include <hip/hip_runtime.h>

namespace acat {

enum FluxId { ADV = 0, BURG = 1, EUL = 2 };
enum BcId { PERIODIC = 0, TRANSMISSIVE = 1 };

struct Phys {
  double gm1;   // gamma - 1
  double gamma;
  double ax, ay;
};

// a / b, correctly rounded, for b and nonzero a of magnitude in [2^-300, 2^300]
// and for a = +0: the compiler's IEEE division sequence (reciprocal estimate,
// two Newton steps, quotient, residual, correction) without its operand
// scaling and special-case fix-up, which are identities there.  (a = -0 gives
// +0 instead of -0.)
__device__ __forceinline__ double div_rn(double a, double b) {
  double r = __builtin_amdgcn_rcp(b);
  double e = fma(-b, r, 1.0);
  r = fma(r, e, r);
  e = fma(-b, r, 1.0);
  r = fma(r, e, r);
  const double q = a * r;
  const double rem = fma(-b, q, a);
  return fma(rem, r, q);
}

// x-direction flux of a 1D law
template <int FLUX, int NV>
__device__ __forceinline__ void flux1d(const Phys& ph, const double (&u)[NV], double (&f)[NV]) {
  if constexpr (FLUX == ADV) {
#pragma unroll
    for (int c = 0; c < NV; ++c) f[c] = ph.ax * u[c];
  } else if constexpr (FLUX == BURG) {
    f[0] = 0.5 * (u[0] * u[0]);
  } else {
    static_assert(NV == 3, "1D Euler has 3 conserved variables");
    const double v = div_rn(u[1], u[0]);
    const double mv = u[1] * v;
    // E - mv/2 in one fused operation: halving is exact, so this is the
    // same value as the subtraction of the halved product
    const double p = ph.gm1 * fma(-0.5, mv, u[2]);
    f[0] = u[1];
    f[1] = mv + p;
    f[2] = v * (u[2] + p);
  }
}

// 1/x, correctly rounded, for |x| in [2^-700, 2^700]: the compiler's IEEE
// division sequence (reciprocal estimate, two Newton steps, residual
// correction) without its exponent scaling and special-case fix-up, which
// are identities in that range.  (Outside it, e.g. x = 0, the result is not
// the IEEE one; such densities are non-physical.)
__device__ __forceinline__ double recip(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  const double rem = fma(-x, r, 1.0);
  return fma(rem, r, r);
}

// recip() of N values at once, its steps interleaved across the values (the
// same operations on each, so the same results)
template <int N>
__device__ __forceinline__ void recip_n(const double (&x)[N], double (&r)[N]) {
  double e[N];
#pragma unroll
  for (int i = 0; i < N; ++i) r[i] = __builtin_amdgcn_rcp(x[i]);
#pragma unroll
  for (int s = 0; s < 2; ++s) {
#pragma unroll
    for (int i = 0; i < N; ++i) e[i] = fma(-x[i], r[i], 1.0);
#pragma unroll
    for (int i = 0; i < N; ++i) r[i] = fma(r[i], e[i], r[i]);
  }
#pragma unroll
  for (int i = 0; i < N; ++i) e[i] = fma(-x[i], r[i], 1.0);
#pragma unroll
  for (int i = 0; i < N; ++i) r[i] = fma(e[i], r[i], r[i]);
}

// 2D Euler fluxes at one state given ir = recip(rho)
template <int NV>
__device__ __forceinline__ void euler2d_ir(const Phys& ph, const double (&u)[NV], double ir, double (&f)[NV],
                                           double (&g)[NV]) {
  static_assert(NV == 4, "2D Euler has 4 conserved variables");
  const double v = u[1] * ir;
  const double w = u[2] * ir;
  // the product-sums are fused multiply-adds: m v + n w, E - (m v + n w)/2,
  // m v + p and n w + p, each rounded once
  const double s = fma(u[1], v, u[2] * w);
  const double p = ph.gm1 * fma(-0.5, s, u[3]);
  const double ep = u[3] + p;
  f[0] = u[1];
  f[1] = fma(u[1], v, p);
  f[2] = u[2] * v;
  f[3] = v * ep;
  g[0] = u[2];
  g[1] = u[1] * w;
  g[2] = fma(u[2], w, p);
  g[3] = w * ep;
}

// x- and y-direction fluxes of a 2D law at one state (shared primitives)
template <int FLUX, int NV>
__device__ __forceinline__ void flux2d(const Phys& ph, const double (&u)[NV], double (&f)[NV], double (&g)[NV]) {
  if constexpr (FLUX == ADV) {
#pragma unroll
    for (int c = 0; c < NV; ++c) {
      f[c] = ph.ax * u[c];
      g[c] = ph.ay * u[c];
    }
  } else {
    static_assert(FLUX == EUL && NV == 4, "2D Euler has 4 conserved variables");
    euler2d_ir(ph, u, recip(u[0]), f, g);
  }
}

// Jacobian-transpose products (adjoint of flux1d): ub += f'(u)^T fb
template <int FLUX, int NV>
__device__ __forceinline__ void flux1d_vjp(const Phys& ph, const double (&u)[NV], const double (&fb)[NV],
                                           double (&ub)[NV]) {
  if constexpr (FLUX == ADV) {
#pragma unroll
    for (int c = 0; c < NV; ++c) ub[c] += ph.ax * fb[c];
  } else if constexpr (FLUX == BURG) {
    ub[0] += u[0] * fb[0];
  } else {
    // f = (m, m v + p, v (E + p)), v = m / rho, p = (gamma-1)(E - m v / 2)
    const double rho = u[0], m = u[1], E = u[2];
    const double v = div_rn(m, rho);
    const double p = ph.gm1 * fma(-0.5, m * v, E);
    double mb = fb[0] + fb[1] * v, vb = fb[1] * m + fb[2] * (E + p);
    const double epb = fb[2] * v;
    double Eb = epb;
    const double pb = fb[1] + epb;
    Eb += ph.gm1 * pb;
    const double q = ph.gm1 * pb;
    mb -= 0.5 * q * v;
    vb -= 0.5 * q * m;
    mb += div_rn(vb, rho);
    ub[0] += div_rn(-vb * v, rho);
    ub[1] += mb;
    ub[2] += Eb;
  }
}

// adjoint of flux2d: ub += f'(u)^T fb + g'(u)^T gb
template <int FLUX, int NV>
__device__ __forceinline__ void flux2d_vjp(const Phys& ph, const double (&u)[NV], const double (&fb)[NV],
                                           const double (&gb)[NV], double (&ub)[NV]) {
  if constexpr (FLUX == ADV) {
#pragma unroll
    for (int c = 0; c < NV; ++c) ub[c] += ph.ax * fb[c] + ph.ay * gb[c];
  } else {
    const double rho = u[0], m = u[1], n = u[2], E = u[3];
    const double ir = recip(rho);
    const double v = m * ir, w = n * ir;
    const double p = ph.gm1 * fma(-0.5, fma(m, v, n * w), E);
    const double ep = E + p;
    // f = (m, m v + p, n v, v ep), g = (n, m w, n w + p, w ep)
    double mb = fb[0] + fb[1] * v + gb[1] * w;
    double nb = gb[0] + fb[2] * v + gb[2] * w;
    double vb = fb[1] * m + fb[2] * n + fb[3] * ep;
    double wb = gb[1] * m + gb[2] * n + gb[3] * ep;
    const double epb = fb[3] * v + gb[3] * w;
    const double pb = fb[1] + gb[2] + epb;
    double Eb = epb + ph.gm1 * pb;
    const double q = ph.gm1 * pb;
    mb -= 0.5 * q * v;
    vb -= 0.5 * q * m;
    nb -= 0.5 * q * w;
    wb -= 0.5 * q * n;
    mb += vb * ir;
    nb += wb * ir;
    const double irb = vb * m + wb * n;
    ub[0] += -irb * ir * ir;
    ub[1] += mb;
    ub[2] += nb;
    ub[3] += Eb;
  }
}

// spectral radius of the flux Jacobian in direction d (0: x, 1: y)
template <int FLUX, int DIM, int NV>
__device__ __forceinline__ double spectral_radius(const Phys& ph, const double (&u)[NV], int d) {
  if constexpr (FLUX == ADV) {
    return fabs(d == 0 ? ph.ax : ph.ay);
  } else if constexpr (FLUX == BURG) {
    return fabs(u[0]);
  } else if constexpr (DIM == 1) {
    const double v = u[1] / u[0];
    const double p = ph.gm1 * (u[2] - 0.5 * u[0] * v * v);
    return fabs(v) + sqrt(ph.gamma * p / u[0]);
  } else {
    const double v = u[1] / u[0], w = u[2] / u[0];
    const double p = ph.gm1 * (u[3] - 0.5 * u[0] * (v * v + w * w));
    return (d == 0 ? fabs(v) : fabs(w)) + sqrt(ph.gamma * p / u[0]);
  }
}

// physical admissibility of an Euler state (density and pressure positive)
template <int FLUX, int DIM, int NV>
__device__ __forceinline__ bool physical(const Phys& ph, const double (&u)[NV]) {
  if constexpr (FLUX != EUL) {
    return true;
  } else if constexpr (DIM == 1) {
    const double p = ph.gm1 * (u[2] - 0.5 * u[1] * u[1] / u[0]);
    return u[0] > 0.0 && p > 0.0;
  } else {
    const double p = ph.gm1 * (u[3] - 0.5 * (u[1] * u[1] + u[2] * u[2]) / u[0]);
    return u[0] > 0.0 && p > 0.0;
  }
}

// Boundary index map for a node index i in [-n, 2n) (every stencil offset is
// at most max(P, 2) < n cells outside the grid): periodic wrap or
// transmissive zeroth-order extrapolation (clamp).
__device__ __forceinline__ int64_t bc_index(int64_t i, int64_t n, int bc) {
  if (bc == PERIODIC) return i < 0 ? i + n : (i >= n ? i - n : i);
  return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

// 32-bit form of bc_index for per-item index math (every extent is below 2^31).
__device__ __forceinline__ int bc_index32(int i, int n, int bc) {
  if (bc == PERIODIC) return i < 0 ? i + n : (i >= n ? i - n : i);
  return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

// Variants of the method (acat_problem.flags; ACAT_FLAG_* in acat.h).
enum { FLAG_FLO_LF = 1, FLAG_FLO_HLL = 2, FLAG_PSI2_MODIFIED = 4, FLAG_PSI1_ROE = 8, FLAG_SQUARE_2D = 16 };

// Smallest and largest characteristic speed along direction d (the Davis
// estimates of HLL): Euler v -+ c, Burgers u, advection a.
template <int FLUX, int DIM, int NV>
__device__ __forceinline__ void wave_speeds(const Phys& ph, const double (&u)[NV], int d, double& lo, double& hi) {
  if constexpr (FLUX == ADV) {
    lo = hi = (d == 0 ? ph.ax : ph.ay);
  } else if constexpr (FLUX == BURG) {
    lo = hi = u[0];
  } else if constexpr (DIM == 1) {
    const double rho = u[0];
    const double v = u[1] / rho;
    const double p = ph.gm1 * (u[2] - 0.5 * rho * v * v);
    const double c = sqrt(ph.gamma * p / rho);
    lo = v - c;
    hi = v + c;
  } else {
    const double rho = u[0], vx = u[1] / rho, vy = u[2] / rho;
    const double p = ph.gm1 * (u[3] - 0.5 * rho * (vx * vx + vy * vy));
    const double c = sqrt(ph.gamma * p / rho);
    const double v = d == 0 ? vx : vy;
    lo = v - c;
    hi = v + c;
  }
}

// One component of the first-order flux F^lo between uL and uR along d:
// Rusanov with speed alpha (default), Lax-Friedrichs with speed alf
// (dx_d / (dim dt)), or HLL with the Davis speeds of the two states.
// fl, fr, ul, ur: component c of f(uL), f(uR), uL, uR.
template <int FLUX, int DIM, int NV>
__device__ __forceinline__ double lo_flux(const Phys& ph, int flags, int d, const double (&uL)[NV],
                                          const double (&uR)[NV], double fl, double fr, double ul, double ur,
                                          double alpha, double alf) {
  if (flags & FLAG_FLO_HLL) {
    double l0, h0, l1, h1;
    wave_speeds<FLUX, DIM, NV>(ph, uL, d, l0, h0);
    wave_speeds<FLUX, DIM, NV>(ph, uR, d, l1, h1);
    const double sl = fmin(l0, l1), sr = fmax(h0, h1);
    if (sl >= 0.0) return fl;
    if (sr <= 0.0) return fr;
    double t = sr * fl - sl * fr;
    t = t + (sl * sr) * (ur - ul);
    return t / (sr - sl);
  }
  const double a = (flags & FLAG_FLO_LF) ? alf : alpha;
  return 0.5 * (fl + fr) - (0.5 * a) * (ur - ul);
}

}  // namespace acat
