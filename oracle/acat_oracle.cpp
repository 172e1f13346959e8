// ACAT oracle: a plain, slow, obviously-written CPU implementation of one
// time step of the Adaptive Compact Approximate Taylor method (Carrillo,
// Macca, Pares, Russo, Zorio, "An order-adaptive compact approximation Taylor
// method for systems of conservation laws", arXiv:2007.01416).
//
// TEST INFRASTRUCTURE ONLY.  This file is the correctness reference for the
// HIP library.  It shares no code, header, table or generator with the
// library; only tests, the package smoke check and the CPU-baseline leg of
// the benchmark load it.  The product path never calls it.
//
// Conventions (each one is a reading of the paper):
//   * point values on a uniform grid, nodes at cell centres (Sec. 2, Taylor
//     update of point values);
//   * scaled recursion variables U^l = dt^l u~^(l), Fh^l = dt^l f~^(l): an
//     exact rewriting of the CAT recursion of Sec. 2.2 that leaves only
//     lambda = dt/dx;
//   * the interface weights eta used in the final CAT flux are the ones
//     defined by the telescoping relation between centred and interpolatory
//     formulas (Sec. 2.1, relation between D^k and A^{k-1,1/2}, taken with
//     k = 1); every other coefficient is a Lagrange derivative on the 2p
//     stencil nodes;
//   * indicators read the conserved variables, componentwise, and the
//     system takes the minimum over components (Sec. 3.4);
//   * the admissibility test "psi^p ~ 1" is psi^p >= theta (default 0.5);
//   * epsilon (Sec. 3.2) is an absolute constant, default 1e-12;
//   * tau_p keeps the (2p-1)! factor exactly as printed (Sec. 3.2);
//   * the robust first-order flux F^lo is Rusanov (local Lax-Friedrichs)
//     with alpha = max of the two cells' spectral radii;
//   * psi^1 is the speed-free min form of the superbee limiter (Sec. 3.1),
//     applied per conserved component; where u_{i+1} = u_i the ratios are
//     undefined: the component contributes 1 if it is constant on the four
//     points, 0 otherwise (a plateau beside a variation is an extremum or a
//     corner; for a scalar law F^1 = F^lo there and the value is immaterial);
//   * 2D: corner i uses the rectangle J_{q1} x J_{q2}, q1 the order of the
//     x-interface i+e1/2 and q2 the order of the y-interface i+e2/2 (Sec. 4,
//     rectangular stencils); F is computed with Taylor order 2 q1 and time
//     nodes J_{q1}, G with 2 q2 and J_{q2}; one recursion when q1 = q2.
//     Variant FLAG_SQUARE_2D: F on the square J_{q1} x J_{q1}, G on
//     J_{q2} x J_{q2} (the square algorithm of Sec. 4 per direction);
//   * boundaries: periodic wrap or transmissive zeroth-order extrapolation.
//   * rounding: the paper fixes none.  Two frozen modes (see mad below):
//     "fixed" (default) writes the weighted sums of the recursion, the 2D U^k
//     (one chain with the weights -lamx gamma and -lamy gamma) and the 2D
//     Euler flux's product-sums as fused multiply-adds in index order;
//     "plain" rounds every operation on its own in the order the paper writes
//     the formulas.  Nothing is contracted implicitly (-ffp-contract=off).
//     An implementation that follows the fixed mode reproduces its results
//     bit for bit, which matters because the limiter and the admissibility
//     test are discontinuous in the data; the plain mode checks an
//     implementation at a tolerance against a rounding it did not choose.
//
// Pins (tests/test_oracle_*.py, tests/golden/): exact-rational coefficient
// identities and tables, closed forms (CAT2 in 1D and 2D, the order-2p
// Lax-Wendroff stencil and the q1 != q2 rectangles for linear flux), exact
// shift at unit Courant number, convergence orders, conservation, symmetries,
// reductions (every forced corner class, nonlinear Euler data constant along
// one direction, against the 1D fluxes of that direction's order), and exact
// Riemann solutions of the paper's shock tubes.  Parity unpinned: the values
// of nonlinear shocked states, and the coupling of the two directions in the
// nonlinear flux evaluations on q1 != q2 rectangles (pinned for linear flux by
// the closed form), for which no closed form or printed value exists.
//
// Build: g++ -O2 -ffp-contract=off -fopenmp -shared -fPIC (no fast-math).
#include <cmath>
#include <cstdint>
#include <cstring>
#include <cstdlib>
#include <algorithm>
#include <vector>
#include <omp.h>

namespace {

// ---------------------------------------------------------------------------
// Exact rationals, used only to build the coefficient tables.
// ---------------------------------------------------------------------------
typedef __int128 i128;

i128 gcd128(i128 a, i128 b) {
  if (a < 0) a = -a;
  if (b < 0) b = -b;
  while (b) { i128 t = a % b; a = b; b = t; }
  return a;
}

struct Rat {
  i128 n, d;
  Rat(i128 n_ = 0, i128 d_ = 1) : n(n_), d(d_) { norm(); }
  void norm() {
    if (d < 0) { n = -n; d = -d; }
    i128 g = gcd128(n, d);
    if (g > 1) { n /= g; d /= g; }
    if (n == 0) d = 1;
  }
  Rat operator+(const Rat& o) const { return Rat(n * o.d + o.n * d, d * o.d); }
  Rat operator-(const Rat& o) const { return Rat(n * o.d - o.n * d, d * o.d); }
  Rat operator*(const Rat& o) const { return Rat(n * o.n, d * o.d); }
  Rat operator/(const Rat& o) const { return Rat(n * o.d, d * o.n); }
  // Rounded once: numerator and denominator are exact doubles (< 2^53 for
  // every table used here), so one IEEE division rounds the exact value.
  double to_double() const { return (double)(long long)n / (double)(long long)d; }
};

// d^k/dx^k of the Lagrange interpolant through integer nodes x[0..nn-1],
// evaluated at the rational point q: weights w[j] with sum_j w[j] f(x_j).
// Built from the expanded Lagrange basis polynomials (a plain definition,
// Sec. 2.1: interpolatory differentiation formulas A^{k,q}).
void lagrange_weights(int nn, const int* x, Rat q, int k, Rat* w) {
  for (int j = 0; j < nn; ++j) {
    // basis polynomial l_j(t) = prod_{m != j} (t - x_m) / (x_j - x_m), in monomials
    std::vector<Rat> c(nn, Rat(0));
    c[0] = Rat(1);
    int deg = 0;
    for (int m = 0; m < nn; ++m) {
      if (m == j) continue;
      Rat den(x[j] - x[m]);
      std::vector<Rat> nc(nn, Rat(0));
      for (int e = 0; e <= deg; ++e) {
        nc[e + 1] = nc[e + 1] + c[e] / den;
        nc[e] = nc[e] - c[e] * Rat(x[m]) / den;
      }
      c = nc;
      ++deg;
    }
    // k-th derivative evaluated at q
    Rat s(0);
    for (int e = k; e <= deg; ++e) {
      Rat term = c[e];
      for (int t = 0; t < k; ++t) term = term * Rat(e - t);
      for (int t = 0; t < e - k; ++t) term = term * q;
      s = s + term;
    }
    w[j] = s;
  }
}

const int PMAX = 6;   // largest stencil half-width supported (1D; 4 in 2D)
const int NMAX = 12;  // 2 * PMAX nodes
const int VMAX = 4;   // largest number of conserved variables

struct Tables {
  // g1[p][j][l]: gamma^{1,j}_{p,l}, first derivative at node j from the 2p
  //              nodes J_p = {-p+1..p}; j, l stored with offset p-1.
  double g1[PMAX + 1][NMAX][NMAX];
  // gt[p][k][r]: gamma^{k,0}_{p,r}, k-th derivative at 0 from nodes J_p.
  double gt[PMAX + 1][NMAX][NMAX];
  // eta[p][l]: interface weights of the final CAT flux (telescoping
  //            relation with the centred first-derivative formula).
  double eta[PMAX + 1][NMAX];
  // tau[p][l]: gamma^{2p-1,1/2}_{p,l}, the (2p-1)-th derivative weights.
  double tau[PMAX + 1][NMAX];
  // d1[p][m]: centred (2p+1)-point first derivative delta^1_{p,m}, m = -p..p.
  double d1[PMAX + 1][2 * PMAX + 1];
  // taylor[r+PMAX-1][l] = r^l / l! for the local time nodes r.
  double taylor[NMAX][NMAX];
  // inverse factorials 1/k! and factorials k! (exact in binary64 for k <= 12)
  double invfact[NMAX + 1];
  double fact[NMAX + 1];
  // (2p-1)!
  double fact2pm1[PMAX + 1];
};

Tables build_tables() {
  Tables T;
  std::memset(&T, 0, sizeof(T));
  for (int p = 1; p <= PMAX; ++p) {
    int nn = 2 * p;
    int x[NMAX];
    for (int a = 0; a < nn; ++a) x[a] = a - p + 1;
    Rat w[NMAX];
    for (int j = 0; j < nn; ++j) {
      lagrange_weights(nn, x, Rat(x[j]), 1, w);
      for (int l = 0; l < nn; ++l) T.g1[p][j][l] = w[l].to_double();
    }
    for (int k = 0; k < nn; ++k) {
      lagrange_weights(nn, x, Rat(0), k, w);
      for (int r = 0; r < nn; ++r) T.gt[p][k][r] = w[r].to_double();
    }
    lagrange_weights(nn, x, Rat(1, 2), nn - 1, w);
    for (int l = 0; l < nn; ++l) T.tau[p][l] = w[l].to_double();
    // centred first derivative on -p..p
    int xc[2 * PMAX + 1];
    for (int a = 0; a < 2 * p + 1; ++a) xc[a] = a - p;
    Rat dc[2 * PMAX + 1];
    lagrange_weights(2 * p + 1, xc, Rat(0), 1, dc);
    for (int a = 0; a < 2 * p + 1; ++a) T.d1[p][a] = dc[a].to_double();
    // eta_m - eta_{m+1} = delta_m, eta_{-p} = 0  =>  eta_{m+1} = eta_m - delta_m
    Rat e(0);
    for (int a = 0; a < nn; ++a) {   // a = m + p, m = -p .. p-1  -> eta_{m+1}
      e = e - dc[a];
      T.eta[p][a] = e.to_double();    // eta at node m+1 = a - p + 1, offset p-1 -> index a
    }
    i128 f = 1;
    for (int t = 2; t <= 2 * p - 1; ++t) f *= t;
    T.fact2pm1[p] = (double)(long long)f;
  }
  for (int ri = 0; ri < NMAX; ++ri) {
    int r = ri - (PMAX - 1);
    Rat v(1);
    for (int l = 0; l < NMAX; ++l) {
      T.taylor[ri][l] = v.to_double();
      v = v * Rat(r) / Rat(l + 1);
    }
  }
  i128 f = 1;
  for (int k = 0; k <= NMAX; ++k) {
    if (k > 0) f *= k;
    T.invfact[k] = Rat(1, f).to_double();
    T.fact[k] = Rat(f).to_double();
  }
  return T;
}

const Tables& tables() {
  static Tables T = build_tables();
  return T;
}

// ---------------------------------------------------------------------------
// Dual numbers (value + K tangents) for the forward-mode JVP oracle: each
// tangent follows the derivative rules of the operations on the value.
template <int K>
struct DualN {
  double v, d[K];
  DualN(double v_ = 0) : v(v_) {
    for (int k = 0; k < K; ++k) d[k] = 0.0;
  }
};
template <int K>
inline DualN<K> operator+(const DualN<K>& a, const DualN<K>& b) {
  DualN<K> r(a.v + b.v);
  for (int k = 0; k < K; ++k) r.d[k] = a.d[k] + b.d[k];
  return r;
}
template <int K>
inline DualN<K> operator-(const DualN<K>& a, const DualN<K>& b) {
  DualN<K> r(a.v - b.v);
  for (int k = 0; k < K; ++k) r.d[k] = a.d[k] - b.d[k];
  return r;
}
template <int K>
inline DualN<K> operator-(const DualN<K>& a) {
  DualN<K> r(-a.v);
  for (int k = 0; k < K; ++k) r.d[k] = -a.d[k];
  return r;
}
template <int K>
inline DualN<K> operator*(const DualN<K>& a, const DualN<K>& b) {
  DualN<K> r(a.v * b.v);
  for (int k = 0; k < K; ++k) r.d[k] = a.d[k] * b.v + a.v * b.d[k];
  return r;
}
template <int K>
inline DualN<K> operator/(const DualN<K>& a, const DualN<K>& b) {
  const double q = a.v / b.v;
  DualN<K> r(q);
  for (int k = 0; k < K; ++k) r.d[k] = (a.d[k] - q * b.d[k]) / b.v;
  return r;
}
template <int K>
inline DualN<K> operator*(double s, const DualN<K>& b) {
  DualN<K> r(s * b.v);
  for (int k = 0; k < K; ++k) r.d[k] = s * b.d[k];
  return r;
}
template <int K>
inline DualN<K> operator/(double s, const DualN<K>& b) { return DualN<K>(s) / b; }
template <int K>
inline DualN<K> operator/(const DualN<K>& a, double s) { return a / DualN<K>(s); }
template <int K>
inline DualN<K> operator*(const DualN<K>& b, double s) {
  DualN<K> r(b.v * s);
  for (int k = 0; k < K; ++k) r.d[k] = b.d[k] * s;
  return r;
}
template <int K>
inline DualN<K> operator+(const DualN<K>& a, double s) {
  DualN<K> r(a);
  r.v = a.v + s;
  return r;
}
template <int K>
inline DualN<K> operator-(double s, const DualN<K>& a) {
  DualN<K> r(s - a.v);
  for (int k = 0; k < K; ++k) r.d[k] = -a.d[k];
  return r;
}
typedef DualN<1> Dual;
typedef DualN<2> Dual2;
inline double val(double x) { return x; }
template <int K>
inline double val(const DualN<K>& x) { return x.v; }

// a*b + c.  Two rounding modes, chosen per problem (FLAG_PLAIN_ROUNDING):
//   fixed (default): one rounding, a fused multiply-add.  Every weighted sum
//     of the recursion (the differentiation formulas in space and time, the
//     Taylor predictions and the final flux sum) accumulates in index order
//     with it, and so do the 2D Euler flux's product-sums (m v + n w,
//     E - (m v + n w)/2, m v + p, n w + p); the 2D U^k is one such chain over
//     the row and then the column, with the weights -lamx gamma and
//     -lamy gamma; the final flux is summed node by node.
//   plain: the product and the sum each rounded (no fused operation
//     anywhere), the sums in the order the paper writes them: U^k as
//     -lamx (sum) - lamy (sum), the final flux k-outer with 1/k! as a
//     division, velocities as m / rho.
// All other arithmetic is plain IEEE operations in both modes.  Both modes
// are frozen: each is a fixed reading of the paper's formulas, and neither
// is changed to follow an implementation.
inline double fmad(double a, double b, double c) { return std::fma(a, b, c); }
template <int K>
inline DualN<K> fmad(double a, const DualN<K>& b, const DualN<K>& c) {
  DualN<K> r(std::fma(a, b.v, c.v));
  for (int k = 0; k < K; ++k) r.d[k] = std::fma(a, b.d[k], c.d[k]);
  return r;
}
template <int K>
inline DualN<K> fmad(const DualN<K>& a, const DualN<K>& b, const DualN<K>& c) {
  DualN<K> r(std::fma(a.v, b.v, c.v));
  for (int k = 0; k < K; ++k) r.d[k] = a.d[k] * b.v + a.v * b.d[k] + c.d[k];
  return r;
}
template <class A, class B, class C>
inline auto mad(bool plain, const A& a, const B& b, const C& c) -> decltype(fmad(a, b, c)) {
  if (plain) return a * b + c;
  return fmad(a, b, c);
}

// ---------------------------------------------------------------------------
// Physics: fluxes and spectral radii.
// ---------------------------------------------------------------------------
enum { FLUX_ADVECTION = 0, FLUX_BURGERS = 1, FLUX_EULER = 2 };
enum { BC_PERIODIC = 0, BC_TRANSMISSIVE = 1 };
// Variants the paper describes beside the default method (bits of flags):
// the first-order flux F^lo of the blend is Lax-Friedrichs or HLL instead of
// Rusanov (Sec. 5 lists LF and HLL as the first-order schemes), the p = 2
// indicator is the modified one of Sec. 3.2, for scalar laws psi^1 may use
// the upwind ratio chosen by the sign of Roe's speed (Sec. 3.1), and 2D
// corners may use square stencils per direction.  FLAG_PLAIN_ROUNDING
// selects the plain rounding mode (see mad).
enum { FLAG_FLO_LF = 1, FLAG_FLO_HLL = 2, FLAG_PSI2_MODIFIED = 4, FLAG_PSI1_ROE = 8, FLAG_SQUARE_2D = 16,
       FLAG_PLAIN_ROUNDING = 256 };

}  // namespace

extern "C" {
// Problem description shared with the Python side of the oracle (ctypes).
typedef struct {
  int32_t dim, nvar;
  int64_t nx, ny;
  int32_t flux, P, bc, flags;
  double gamma, ax, ay, dx, dy, eps, theta;
} oracle_problem;
}

namespace {

inline bool plain(const oracle_problem& pb) { return (pb.flags & FLAG_PLAIN_ROUNDING) != 0; }

// 2D velocities v = m / rho, w = n / rho: fixed rounding through one
// reciprocal, plain rounding by division
template <class T>
void velocities(bool pl, const T& rho, const T& mx, const T& my, T& v, T& w) {
  if (pl) {
    v = mx / rho;
    w = my / rho;
  } else {
    T ir = 1.0 / rho;
    v = mx * ir;
    w = my * ir;
  }
}

// x-direction flux f(u) (1D flux, or the x-flux in 2D)
template <class T>
void flux_f(const oracle_problem& pb, const T* u, T* f) {
  if (pb.flux == FLUX_ADVECTION) {
    for (int c = 0; c < pb.nvar; ++c) f[c] = pb.ax * u[c];
  } else if (pb.flux == FLUX_BURGERS) {
    f[0] = 0.5 * (u[0] * u[0]);
  } else if (pb.dim == 1) {
    // 1D Euler (Sec. 5.3): u = (rho, rho v, E), p = (gamma-1)(E - rho v^2/2)
    T rho = u[0], m = u[1], E = u[2];
    T v = m / rho;
    T p = (pb.gamma - 1.0) * (E - 0.5 * (m * v));
    f[0] = m;
    f[1] = m * v + p;
    f[2] = v * (E + p);
  } else {
    // 2D Euler (Sec. 5.5): u = (rho, rho v, rho w, E); fixed rounding: both
    // velocity components use one reciprocal of the density
    const bool pl = plain(pb);
    T rho = u[0], mx = u[1], my = u[2], E = u[3];
    T v, w;
    velocities(pl, rho, mx, my, v, w);
    T p = (pb.gamma - 1.0) * mad(pl, -0.5, mad(pl, mx, v, my * w), E);
    f[0] = mx;
    f[1] = mad(pl, mx, v, p);
    f[2] = my * v;
    f[3] = v * (E + p);
  }
}

// y-direction flux g(u) (2D only)
template <class T>
void flux_g(const oracle_problem& pb, const T* u, T* g) {
  if (pb.flux == FLUX_ADVECTION) {
    for (int c = 0; c < pb.nvar; ++c) g[c] = pb.ay * u[c];
  } else {
    const bool pl = plain(pb);
    T rho = u[0], mx = u[1], my = u[2], E = u[3];
    T v, w;
    velocities(pl, rho, mx, my, v, w);
    T p = (pb.gamma - 1.0) * mad(pl, -0.5, mad(pl, mx, v, my * w), E);
    g[0] = my;
    g[1] = mx * w;
    g[2] = mad(pl, my, w, p);
    g[3] = w * (E + p);
  }
}

// spectral radius of the flux Jacobian in direction d (0 = x, 1 = y)
double spectral_radius(const oracle_problem& pb, const double* u, int d) {
  if (pb.flux == FLUX_ADVECTION) return std::fabs(d == 0 ? pb.ax : pb.ay);
  if (pb.flux == FLUX_BURGERS) return std::fabs(u[0]);
  if (pb.dim == 1) {
    double rho = u[0], v = u[1] / rho;
    double p = (pb.gamma - 1.0) * (u[2] - 0.5 * rho * v * v);
    return std::fabs(v) + std::sqrt(pb.gamma * p / rho);
  }
  double rho = u[0], v = u[1] / rho, w = u[2] / rho;
  double p = (pb.gamma - 1.0) * (u[3] - 0.5 * rho * (v * v + w * w));
  double c = std::sqrt(pb.gamma * p / rho);
  return (d == 0 ? std::fabs(v) : std::fabs(w)) + c;
}

// ---------------------------------------------------------------------------
// Boundary extension (periodic wrap or transmissive clamp).
// ---------------------------------------------------------------------------
int64_t bc_index(int64_t i, int64_t n, int bc) {
  if (bc == BC_PERIODIC) {
    int64_t r = i % n;
    return r < 0 ? r + n : r;
  }
  return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

// ---------------------------------------------------------------------------
// Smoothness indicators and the limiter (Sec. 3.1, 3.2, 3.4).
// v[a] holds one conserved component at the nodes i-P+1 .. i+P
// (a = j + P - 1 for stencil offset j).
// ---------------------------------------------------------------------------


// Modified p = 2 indicator (Sec. 3.2): two pairs of lateral weights, each
// joining the central sub-interval to one side; the larger ratio.
double indicator_psi2_modified(const double* v, int P, double eps) {
  const Tables& T = tables();
  auto at = [&](int j) { return v[j + P - 1]; };
  const double dl = at(0) - at(-1), dc = at(1) - at(0), dr = at(2) - at(1);
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
  const double I1 = I1L * I1R / (I1L + I1R), I2 = I2L * I2R / (I2L + I2R);
  double s = 0.0;
  for (int j = -1; j <= 2; ++j) s += T.tau[2][j + 1] * at(j);
  double tau = T.fact2pm1[2] * s;
  tau = tau * tau;
  return std::max(I1 / (I1 + tau), I2 / (I2 + tau));
}

double indicator_psi(const double* v, int P, int p, double eps) {
  const Tables& T = tables();
  auto at = [&](int j) { return v[j + P - 1]; };
  double IL = 0.0, IR = 0.0;
  for (int j = -p + 1; j <= -1; ++j) { double d = at(j + 1) - at(j); IL += d * d; }
  for (int j = 1; j <= p - 1; ++j) { double d = at(j + 1) - at(j); IR += d * d; }
  IL += eps;
  IR += eps;
  double I = IL * IR / (IL + IR);
  double s = 0.0;
  for (int j = -p + 1; j <= p; ++j) s += T.tau[p][j + p - 1] * at(j);
  double tau = T.fact2pm1[p] * s;
  tau = tau * tau;
  return I / (I + tau);
}

double superbee(double r) {
  return std::max(0.0, std::max(std::min(2.0 * r, 1.0), std::min(r, 2.0)));
}

// psi^1 for one component: min(phi(r+), phi(r-)) (Sec. 3.1, min form).
double limiter_psi1(const double* v, int P) {
  auto at = [&](int j) { return v[j + P - 1]; };
  double dloc = at(1) - at(0);
  if (dloc == 0.0) return (at(0) - at(-1) == 0.0 && at(2) - at(1) == 0.0) ? 1.0 : 0.0;
  double rm = (at(0) - at(-1)) / dloc;
  double rp = (at(2) - at(1)) / dloc;
  return std::min(superbee(rp), superbee(rm));
}

// psi^1 of a scalar law with the upwind ratio chosen by the sign of Roe's
// speed a = (f(u_{i+1}) - f(u_i)) / (u_{i+1} - u_i) (f'(u_i) if equal):
// r^- if a > 0, r^+ otherwise (Sec. 3.1).
double limiter_psi1_roe(const oracle_problem& pb, const double* v, int P, int d) {
  auto at = [&](int j) { return v[j + P - 1]; };
  const double u0 = at(0), u1 = at(1);
  const double dloc = u1 - u0;
  double f0, f1, fp;
  if (pb.flux == FLUX_BURGERS) { f0 = 0.5 * (u0 * u0); f1 = 0.5 * (u1 * u1); fp = u0; }
  else { const double a = d == 0 ? pb.ax : pb.ay; f0 = a * u0; f1 = a * u1; fp = a; }
  const double a = dloc != 0.0 ? (f1 - f0) / dloc : fp;
  const double dupw = a > 0.0 ? u0 - at(-1) : at(2) - u1;
  if (dloc == 0.0) return dupw == 0.0 ? 1.0 : 0.0;
  return superbee(dupw / dloc);
}

// Order selection at one interface: p_s = max{p in 2..P : psi^p >= theta},
// 1 if the admissible set is empty (Sec. 3, admissible set; Sec. 3.4 min over
// components).  comp[c] holds component c at offsets -P+1..P (P >= 2 needs
// offsets -1..2 as well, which the caller guarantees by using max(P,2)).
int select_order(const oracle_problem& pb, const double* const* comp, int G, double* psi1_out, int d = 0) {
  int ps = 1;
  for (int p = pb.P; p >= 2; --p) {
    double psi = 1.0;
    for (int c = 0; c < pb.nvar; ++c)
      psi = std::min(psi, (p == 2 && (pb.flags & FLAG_PSI2_MODIFIED))
                              ? indicator_psi2_modified(comp[c] + (G - pb.P) + (pb.P - 2), 2, pb.eps)
                              : indicator_psi(comp[c] + (G - pb.P), pb.P, p, pb.eps));
    if (psi >= pb.theta) { ps = p; break; }
  }
  if (ps == 1) {
    double psi1 = 1e300;
    for (int c = 0; c < pb.nvar; ++c)
      psi1 = std::min(psi1, (pb.flags & FLAG_PSI1_ROE) ? limiter_psi1_roe(pb, comp[c] + (G - 2), 2, d)
                                                       : limiter_psi1(comp[c] + (G - 2), 2));
    *psi1_out = psi1;
  } else {
    *psi1_out = -1.0;
  }
  return ps;
}

// The CAT flux F = sum_{k=1}^{m} 1/k! sum_l eta_l Fh^{k-1}_l (Sec. 2.2, the
// interpolation A^{0,1/2} with the weights eta) from Fh^{k-1}_l = fh(k-1, l),
// l = 0 .. nn-1, m = nn.  Fixed rounding: summed node by node,
// sum_l eta_l (sum_k Fh^{k-1}_l / k!), fused; plain rounding: k-outer as
// written, each term's interpolation divided by k!.
template <class T, class FH>
T final_flux(bool pl, int p, int nn, FH fh) {
  const Tables& Tb = tables();
  T s = 0.0;
  if (pl) {
    for (int k = 1; k <= nn; ++k) {
      T a = 0.0;
      for (int l = 0; l < nn; ++l) a = a + Tb.eta[p][l] * fh(k - 1, l);
      s = s + a / Tb.fact[k];
    }
    return s;
  }
  for (int l = 0; l < nn; ++l) {
    T t = 0.0;
    for (int k = 1; k <= nn; ++k) t = fmad(Tb.invfact[k], fh(k - 1, l), t);
    s = fmad(Tb.eta[p][l], t, s);
  }
  return s;
}

// ---------------------------------------------------------------------------
// 1D CAT2p flux at one interface (Sec. 2.2 algorithm, scaled variables).
// u[a][c]: state at node j = a - p + 1, a = 0 .. 2p-1.
// ---------------------------------------------------------------------------
template <class T>
void cat_flux_1d(const oracle_problem& pb, int p, const T (*u)[VMAX], double lam, T* F) {
  const Tables& Tb = tables();
  const bool pl = plain(pb);
  const int nn = 2 * p, nv = pb.nvar;
  T Fh[NMAX][NMAX][VMAX];   // Fh[k][a][c] = dt^k f~^(k) at node a
  T U[NMAX][NMAX][VMAX];    // U[l][a][c]  = dt^l u~^(l) at node a
  for (int a = 0; a < nn; ++a) flux_f(pb, u[a], Fh[0][a]);
  for (int k = 2; k <= 2 * p; ++k) {
    // (a) U^{k-1}_j = -lam * sum_l gamma^{1,j}_{p,l} Fh^{k-2}_l
    for (int a = 0; a < nn; ++a)
      for (int c = 0; c < nv; ++c) {
        T s = 0.0;
        for (int l = 0; l < nn; ++l) s = mad(pl, Tb.g1[p][a][l], Fh[k - 2][l][c], s);
        U[k - 1][a][c] = -lam * s;
      }
    // (b) flux at the Taylor-predicted states at the time nodes r, and
    // (c) its (k-1)-th time derivative at r = 0.
    for (int a = 0; a < nn; ++a) {
      for (int c = 0; c < nv; ++c) Fh[k - 1][a][c] = 0.0;
      for (int ri = 0; ri < nn; ++ri) {
        int r = ri - p + 1;
        T phi[VMAX];
        if (r == 0) {
          for (int c = 0; c < nv; ++c) phi[c] = Fh[0][a][c];
        } else {
          T w[VMAX];
          for (int c = 0; c < nv; ++c) {
            T s = u[a][c];
            for (int l = 1; l <= k - 1; ++l) s = mad(pl, Tb.taylor[r + PMAX - 1][l], U[l][a][c], s);
            w[c] = s;
          }
          flux_f(pb, w, phi);
        }
        for (int c = 0; c < nv; ++c) Fh[k - 1][a][c] = mad(pl, Tb.gt[p][k - 1][ri], phi[c], Fh[k - 1][a][c]);
      }
    }
  }
  // F = sum_{k=1}^{2p} 1/k! sum_l eta_l Fh^{k-1}_l
  for (int c = 0; c < nv; ++c) F[c] = final_flux<T>(pl, p, nn, [&](int k, int a) { return Fh[k][a][c]; });
}

// Smallest and largest characteristic speed along direction d (Davis
// estimates for HLL): Euler v -+ c, Burgers u, advection a.
void wave_speeds(const oracle_problem& pb, const double* u, int d, double* lo, double* hi) {
  if (pb.flux == FLUX_ADVECTION) { *lo = *hi = d == 0 ? pb.ax : pb.ay; return; }
  if (pb.flux == FLUX_BURGERS) { *lo = *hi = u[0]; return; }
  double v, c;
  if (pb.dim == 1) {
    const double rho = u[0];
    v = u[1] / rho;
    const double p = (pb.gamma - 1.0) * (u[2] - 0.5 * rho * v * v);
    c = std::sqrt(pb.gamma * p / rho);
  } else {
    const double rho = u[0], vx = u[1] / rho, vy = u[2] / rho;
    const double p = (pb.gamma - 1.0) * (u[3] - 0.5 * rho * (vx * vx + vy * vy));
    c = std::sqrt(pb.gamma * p / rho);
    v = d == 0 ? vx : vy;
  }
  *lo = v - c;
  *hi = v + c;
}

// First-order flux F^lo along direction d between states uL, uR: Rusanov
// with speed alpha (default), Lax-Friedrichs with dx_d / (dim dt) (so that
// the unsplit 2D sum is the classical 2D scheme), or HLL with the Davis
// speeds of the two states (taken at their values: frozen in a tangent).
template <class T>
void lo_flux(const oracle_problem& pb, int d, const T* uL, const T* uR, double alpha, double dt, T* F) {
  T fL[VMAX], fR[VMAX];
  if (d == 0) { flux_f(pb, uL, fL); flux_f(pb, uR, fR); }
  else { flux_g(pb, uL, fL); flux_g(pb, uR, fR); }
  if (pb.flags & FLAG_FLO_HLL) {
    double uLd[VMAX], uRd[VMAX], l0, h0, l1, h1;
    for (int c = 0; c < pb.nvar; ++c) { uLd[c] = val(uL[c]); uRd[c] = val(uR[c]); }
    wave_speeds(pb, uLd, d, &l0, &h0);
    wave_speeds(pb, uRd, d, &l1, &h1);
    const double sl = std::min(l0, l1), sr = std::max(h0, h1);
    for (int c = 0; c < pb.nvar; ++c) {
      if (sl >= 0.0) { F[c] = fL[c]; continue; }
      if (sr <= 0.0) { F[c] = fR[c]; continue; }
      T t = sr * fL[c] - sl * fR[c];
      t = t + (sl * sr) * (uR[c] - uL[c]);
      F[c] = t / (sr - sl);
    }
    return;
  }
  double a = alpha;
  if (pb.flags & FLAG_FLO_LF) a = (d == 0 ? pb.dx : pb.dy) / (pb.dim * dt);
  for (int c = 0; c < pb.nvar; ++c) F[c] = 0.5 * (fL[c] + fR[c]) - (0.5 * a) * (uR[c] - uL[c]);
}

// ---------------------------------------------------------------------------
// 1D step.
// ---------------------------------------------------------------------------
template <class T>
struct Step1D {
  const oracle_problem& pb;
  const T* u;         // [nvar][nx]
  int64_t nx, nI, ioff;
  int G;
  double dt = 0.0;     // time step (the Lax-Friedrichs flux uses it)
  Step1D(const oracle_problem& p, const T* u_) : pb(p), u(u_) {
    nx = pb.nx;
    nI = (pb.bc == BC_PERIODIC) ? nx : nx + 1;
    ioff = (pb.bc == BC_PERIODIC) ? 0 : -1;   // interface k <-> i = k + ioff
    G = std::max(pb.P, 2);
  }
  T at(int c, int64_t i) const { return u[(int64_t)c * nx + bc_index(i, nx, pb.bc)]; }

  // Numerical flux at interface k.  decide = true: choose the order, psi^1
  // and alpha here and return them; decide = false: use the given ones
  // (frozen replay).
  void flux(int64_t k, double lam, bool decide, int& ps, double& ps1, double& al, T* F) const {
    int64_t i = k + ioff;
    if (decide) {
      double vals[VMAX][2 * NMAX];
      const double* comp[VMAX];
      for (int c = 0; c < pb.nvar; ++c) {
        for (int j = -G + 1; j <= G; ++j) vals[c][j + G - 1] = val(at(c, i + j));
        comp[c] = vals[c];
      }
      ps = select_order(pb, comp, G, &ps1);
      al = -1.0;
    }
    T us[NMAX][VMAX];
    for (int j = -ps + 1; j <= ps; ++j)
      for (int c = 0; c < pb.nvar; ++c) us[j + ps - 1][c] = at(c, i + j);
    cat_flux_1d(pb, ps, us, lam, F);
    if (ps == 1) {
      T uL[VMAX], uR[VMAX];
      double uLd[VMAX], uRd[VMAX];
      for (int c = 0; c < pb.nvar; ++c) {
        uL[c] = at(c, i); uR[c] = at(c, i + 1);
        uLd[c] = val(uL[c]); uRd[c] = val(uR[c]);
      }
      if (decide) al = std::max(spectral_radius(pb, uLd, 0), spectral_radius(pb, uRd, 0));
      T Flo[VMAX];
      lo_flux(pb, 0, uL, uR, al, dt, Flo);
      // FL-CAT2 blend (Sec. 3.1)
      for (int c = 0; c < pb.nvar; ++c) F[c] = ps1 * F[c] + (1.0 - ps1) * Flo[c];
    }
  }
};

template <class T>
int step1d(const oracle_problem& pb, const T* u, T* uout, double dt, int mode, int8_t* ord,
           double* psi1, double* alpha, T* flux_out, int nthreads) {
  Step1D<T> S(pb, u);
  S.dt = dt;
  const int64_t nx = pb.nx, nI = S.nI;
  const int nv = pb.nvar;
  const double lam = dt / pb.dx;
  std::vector<T> F((size_t)nI * nv);
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t k = 0; k < nI; ++k) {
    T f[VMAX];
    int ps = 0;
    double ps1 = -1.0, al = -1.0;
    if (mode == 1) { ps = ord[k]; ps1 = psi1[k]; al = alpha[k]; }
    S.flux(k, lam, mode == 0, ps, ps1, al, f);
    if (mode == 0) {
      if (ord) ord[k] = (int8_t)ps;
      if (psi1) psi1[k] = ps1;
      if (alpha) alpha[k] = al;
    }
    for (int c = 0; c < nv; ++c) F[(size_t)c * nI + k] = f[c];
  }
  // conservative update (Sec. 2.1 conservative form; Sec. 3.3 ACAT2P update)
  for (int c = 0; c < nv; ++c)
    for (int64_t i = 0; i < nx; ++i) {
      int64_t kr = i - S.ioff;                       // interface i+1/2
      int64_t kl = (pb.bc == BC_PERIODIC) ? (i == 0 ? nx - 1 : i - 1) : i;  // interface i-1/2
      uout[(size_t)c * nx + i] = u[(size_t)c * nx + i] + lam * (F[(size_t)c * nI + kl] - F[(size_t)c * nI + kr]);
    }
  if (flux_out)
    for (size_t a = 0; a < F.size(); ++a) flux_out[a] = F[a];
  return 0;
}

// ---------------------------------------------------------------------------
// 2D corner recursion on the rectangle J_{q1} x J_{q2} (Sec. 4).
// u[a1][a2][c]: state at node (j1, j2) = (a1 - q1 + 1, a2 - q2 + 1).
// qt is the half-width of the time stencil (q1 for F, q2 for G); the Taylor
// order is 2 qt.  Outputs F (row j2 = 0) and/or G (column j1 = 0).
// ---------------------------------------------------------------------------
template <class T>
void cat_corner_2d(const oracle_problem& pb, int q1, int q2, int qt, const T (*u)[NMAX][VMAX],
                   double lamx, double lamy, T* F, T* G) {
  const Tables& Tb = tables();
  const bool pl = plain(pb);
  const int n1 = 2 * q1, n2 = 2 * q2, nt = 2 * qt, nv = pb.nvar;
  static thread_local T Fh[NMAX][NMAX][NMAX][VMAX];
  static thread_local T Gh[NMAX][NMAX][NMAX][VMAX];
  static thread_local T U[NMAX][NMAX][NMAX][VMAX];
  for (int a1 = 0; a1 < n1; ++a1)
    for (int a2 = 0; a2 < n2; ++a2) {
      flux_f(pb, u[a1][a2], Fh[0][a1][a2]);
      flux_g(pb, u[a1][a2], Gh[0][a1][a2]);
    }
  for (int k = 2; k <= nt; ++k) {
    // (a) U^{k-1}_j = -lamx sum_l gamma^{1,j1}_{q1,l} Fh^{k-2}_{(l,j2)}
    //                 -lamy sum_l gamma^{1,j2}_{q2,l} Gh^{k-2}_{(j1,l)}
    //     fixed rounding: one fused chain, row terms then column terms, with
    //     the weights -lamx gamma and -lamy gamma; plain: the two sums, then
    //     -lamx sx - lamy sy
    for (int a1 = 0; a1 < n1; ++a1)
      for (int a2 = 0; a2 < n2; ++a2)
        for (int c = 0; c < nv; ++c) {
          if (pl) {
            T sx = 0.0, sy = 0.0;
            for (int l = 0; l < n1; ++l) sx = sx + Tb.g1[q1][a1][l] * Fh[k - 2][l][a2][c];
            for (int l = 0; l < n2; ++l) sy = sy + Tb.g1[q2][a2][l] * Gh[k - 2][a1][l][c];
            U[k - 1][a1][a2][c] = -lamx * sx - lamy * sy;
            continue;
          }
          T s = 0.0;
          for (int l = 0; l < n1; ++l) s = fmad(-lamx * Tb.g1[q1][a1][l], Fh[k - 2][l][a2][c], s);
          for (int l = 0; l < n2; ++l) s = fmad(-lamy * Tb.g1[q2][a2][l], Gh[k - 2][a1][l][c], s);
          U[k - 1][a1][a2][c] = s;
        }
    // (b), (c): f and g at the predicted states, time derivative at r = 0
    for (int a1 = 0; a1 < n1; ++a1)
      for (int a2 = 0; a2 < n2; ++a2) {
        for (int c = 0; c < nv; ++c) { Fh[k - 1][a1][a2][c] = 0.0; Gh[k - 1][a1][a2][c] = 0.0; }
        for (int ri = 0; ri < nt; ++ri) {
          int r = ri - qt + 1;
          T pf[VMAX], pg[VMAX];
          if (r == 0) {
            for (int c = 0; c < nv; ++c) { pf[c] = Fh[0][a1][a2][c]; pg[c] = Gh[0][a1][a2][c]; }
          } else {
            T w[VMAX];
            for (int c = 0; c < nv; ++c) {
              T s = u[a1][a2][c];
              for (int l = 1; l <= k - 1; ++l) s = mad(pl, Tb.taylor[r + PMAX - 1][l], U[l][a1][a2][c], s);
              w[c] = s;
            }
            flux_f(pb, w, pf);
            flux_g(pb, w, pg);
          }
          for (int c = 0; c < nv; ++c) {
            Fh[k - 1][a1][a2][c] = mad(pl, Tb.gt[qt][k - 1][ri], pf[c], Fh[k - 1][a1][a2][c]);
            Gh[k - 1][a1][a2][c] = mad(pl, Tb.gt[qt][k - 1][ri], pg[c], Gh[k - 1][a1][a2][c]);
          }
        }
      }
  }
  // F = sum_k 1/k! sum_l eta_l Fh^{k-1}_(l,0) on row j2 = 0 (Taylor order
  // nt = 2 q1 for F: qt = q1 whenever F is asked for)
  if (F) {
    const int a2 = q2 - 1;
    for (int c = 0; c < nv; ++c)
      F[c] = final_flux<T>(pl, q1, n1, [&](int k, int a) { return Fh[k][a][a2][c]; });
  }
  // G likewise on column j1 = 0 (nt = 2 q2)
  if (G) {
    const int a1 = q1 - 1;
    for (int c = 0; c < nv; ++c)
      G[c] = final_flux<T>(pl, q2, n2, [&](int k, int a) { return Gh[k][a1][a][c]; });
  }
}

// ---------------------------------------------------------------------------
// 2D step.  x-interfaces: array [ny][nIx], entry kx <-> i1 = kx + ioff;
// y-interfaces: array [nIy][nx], entry ky <-> i2 = ky + ioff.
// ---------------------------------------------------------------------------
template <class T>
struct Step2D {
  const oracle_problem& pb;
  const T* u;   // [nvar][ny][nx]
  int64_t nx, ny, nIx, nIy, ioff;
  int G;
  double dt = 0.0;     // time step (the Lax-Friedrichs flux uses it)
  Step2D(const oracle_problem& p, const T* u_) : pb(p), u(u_) {
    nx = pb.nx; ny = pb.ny;
    bool per = pb.bc == BC_PERIODIC;
    nIx = per ? nx : nx + 1;
    nIy = per ? ny : ny + 1;
    ioff = per ? 0 : -1;
    G = std::max(pb.P, 2);
  }
  T at(int c, int64_t i1, int64_t i2) const {
    return u[((int64_t)c * ny + bc_index(i2, ny, pb.bc)) * nx + bc_index(i1, nx, pb.bc)];
  }
  // Decide the order of the interface i + e_d/2 (d = 0: x, 1: y).
  int decide(int d, int64_t i1, int64_t i2, double* psi1, double* alpha) const {
    double vals[VMAX][2 * NMAX];
    const double* comp[VMAX];
    for (int c = 0; c < pb.nvar; ++c) {
      for (int j = -G + 1; j <= G; ++j)
        vals[c][j + G - 1] = val(d == 0 ? at(c, i1 + j, i2) : at(c, i1, i2 + j));
      comp[c] = vals[c];
    }
    int ps = select_order(pb, comp, G, psi1, d);
    *alpha = -1.0;
    if (ps == 1) {
      double uL[VMAX], uR[VMAX];
      for (int c = 0; c < pb.nvar; ++c) {
        uL[c] = val(at(c, i1, i2));
        uR[c] = val(d == 0 ? at(c, i1 + 1, i2) : at(c, i1, i2 + 1));
      }
      *alpha = std::max(spectral_radius(pb, uL, d), spectral_radius(pb, uR, d));
    }
    return ps;
  }
  // States of the stencil J_{s1} x J_{s2} around corner (i1, i2).
  void gather(int64_t i1, int64_t i2, int s1, int s2, T (*us)[NMAX][VMAX]) const {
    for (int j1 = -s1 + 1; j1 <= s1; ++j1)
      for (int j2 = -s2 + 1; j2 <= s2; ++j2)
        for (int c = 0; c < pb.nvar; ++c) us[j1 + s1 - 1][j2 + s2 - 1][c] = at(c, i1 + j1, i2 + j2);
  }
  // Fluxes of corner (i1, i2).  q/psi/alpha for both directions are given.
  // Default: both fluxes on the rectangle J_{q1} x J_{q2}.  FLAG_SQUARE_2D
  // (q1 != q2): F on the square J_{q1} x J_{q1} and G on J_{q2} x J_{q2},
  // each the square algorithm of Sec. 4 with its own half-width.
  void corner(int64_t i1, int64_t i2, int q1, int q2, double ps1x, double ps1y, double alx, double aly,
              double lamx, double lamy, T* F, T* G_) const {
    T us[NMAX][NMAX][VMAX];
    if (q1 == q2) {
      gather(i1, i2, q1, q2, us);
      cat_corner_2d(pb, q1, q2, q1, us, lamx, lamy, F, G_);
    } else if (pb.flags & FLAG_SQUARE_2D) {
      if (F) {
        gather(i1, i2, q1, q1, us);
        cat_corner_2d<T>(pb, q1, q1, q1, us, lamx, lamy, F, nullptr);
      }
      if (G_) {
        gather(i1, i2, q2, q2, us);
        cat_corner_2d<T>(pb, q2, q2, q2, us, lamx, lamy, nullptr, G_);
      }
    } else {
      gather(i1, i2, q1, q2, us);
      if (F) cat_corner_2d<T>(pb, q1, q2, q1, us, lamx, lamy, F, nullptr);
      if (G_) cat_corner_2d<T>(pb, q1, q2, q2, us, lamx, lamy, nullptr, G_);
    }
    T u0[VMAX], ux[VMAX], uy[VMAX];
    for (int c = 0; c < pb.nvar; ++c) { u0[c] = at(c, i1, i2); ux[c] = at(c, i1 + 1, i2); uy[c] = at(c, i1, i2 + 1); }
    // 2D FL-CAT2 blends (Sec. 4), one per direction with order 1
    if (F && q1 == 1) {
      T Flo[VMAX];
      lo_flux(pb, 0, u0, ux, alx, dt, Flo);
      for (int c = 0; c < pb.nvar; ++c) F[c] = ps1x * F[c] + (1.0 - ps1x) * Flo[c];
    }
    if (G_ && q2 == 1) {
      T Glo[VMAX];
      lo_flux(pb, 1, u0, uy, aly, dt, Glo);
      for (int c = 0; c < pb.nvar; ++c) G_[c] = ps1y * G_[c] + (1.0 - ps1y) * Glo[c];
    }
  }
};

template <class T>
int step2d(const oracle_problem& pb, const T* u, T* uout, double dt, int mode, int8_t* ordx, int8_t* ordy,
           double* psix, double* psiy, double* alx, double* aly, T* Fout, T* Gout, int nthreads) {
  Step2D<T> S(pb, u);
  S.dt = dt;
  const int64_t nx = S.nx, ny = S.ny, nIx = S.nIx, nIy = S.nIy, off = S.ioff;
  const int nv = pb.nvar;
  const double lamx = dt / pb.dx, lamy = dt / pb.dy;
  if (nthreads > 0) omp_set_num_threads(nthreads);
  // orders of every x- and y-interface (decided or given)
  std::vector<int8_t> ox((size_t)ny * nIx), oy((size_t)nIy * nx);
  std::vector<double> px((size_t)ny * nIx), py((size_t)nIy * nx), ax((size_t)ny * nIx), ay((size_t)nIy * nx);
  if (mode == 0) {
#pragma omp parallel for schedule(static)
    for (int64_t i2 = 0; i2 < ny; ++i2)
      for (int64_t kx = 0; kx < nIx; ++kx) {
        size_t e = (size_t)i2 * nIx + kx;
        ox[e] = (int8_t)S.decide(0, kx + off, i2, &px[e], &ax[e]);
      }
#pragma omp parallel for schedule(static)
    for (int64_t ky = 0; ky < nIy; ++ky)
      for (int64_t i1 = 0; i1 < nx; ++i1) {
        size_t e = (size_t)ky * nx + i1;
        oy[e] = (int8_t)S.decide(1, i1, ky + off, &py[e], &ay[e]);
      }
  } else {
    for (size_t e = 0; e < ox.size(); ++e) { ox[e] = ordx[e]; px[e] = psix[e]; ax[e] = alx[e]; }
    for (size_t e = 0; e < oy.size(); ++e) { oy[e] = ordy[e]; py[e] = psiy[e]; ay[e] = aly[e]; }
  }
  // order of x-interface (i1+1/2, i2) for any i2 (ghost rows take the clamped
  // or wrapped row: the extended data there is a copy of a real row).
  auto qx = [&](int64_t i1, int64_t i2) { return (int)ox[(size_t)bc_index(i2, ny, pb.bc) * nIx + (i1 - off)]; };
  auto qy = [&](int64_t i1, int64_t i2) { return (int)oy[(size_t)(i2 - off) * nx + bc_index(i1, nx, pb.bc)]; };
  std::vector<T> F((size_t)nv * ny * nIx), Gf((size_t)nv * nIy * nx);
  // corners (i1, i2) with i1 in [off, nx), i2 in [off, ny)
  const int64_t n1 = nx - off, n2 = ny - off;
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t e = 0; e < n1 * n2; ++e) {
    int64_t i1 = e % n1 + off, i2 = e / n1 + off;
    bool needF = i2 >= 0;   // x-interface (i1+1/2, i2) is a real one
    bool needG = i1 >= 0;   // y-interface (i1, i2+1/2) is a real one
    if (!needF && !needG) continue;
    int q1 = qx(i1, i2), q2 = qy(i1, i2);
    double p1 = -1, p2 = -1, a1 = -1, a2 = -1;
    if (needF) { size_t ex = (size_t)i2 * nIx + (i1 - off); p1 = px[ex]; a1 = ax[ex]; }
    if (needG) { size_t ey = (size_t)(i2 - off) * nx + i1; p2 = py[ey]; a2 = ay[ey]; }
    T f[VMAX], g[VMAX];
    S.corner(i1, i2, q1, q2, p1, p2, a1, a2, lamx, lamy, needF ? f : nullptr, needG ? g : nullptr);
    if (needF)
      for (int c = 0; c < nv; ++c) F[((size_t)c * ny + i2) * nIx + (i1 - off)] = f[c];
    if (needG)
      for (int c = 0; c < nv; ++c) Gf[((size_t)c * nIy + (i2 - off)) * nx + i1] = g[c];
  }
  // unsplit conservative update (Sec. 4, ACAT2P scheme in 2D)
  for (int c = 0; c < nv; ++c)
    for (int64_t i2 = 0; i2 < ny; ++i2)
      for (int64_t i1 = 0; i1 < nx; ++i1) {
        int64_t kxr = i1 - off, kxl = (pb.bc == BC_PERIODIC) ? (i1 == 0 ? nx - 1 : i1 - 1) : i1;
        int64_t kyr = i2 - off, kyl = (pb.bc == BC_PERIODIC) ? (i2 == 0 ? ny - 1 : i2 - 1) : i2;
        T Fl = F[((size_t)c * ny + i2) * nIx + kxl], Fr = F[((size_t)c * ny + i2) * nIx + kxr];
        T Gl = Gf[((size_t)c * nIy + kyl) * nx + i1], Gr = Gf[((size_t)c * nIy + kyr) * nx + i1];
        size_t e = ((size_t)c * ny + i2) * nx + i1;
        uout[e] = u[e] + lamx * (Fl - Fr) + lamy * (Gl - Gr);
      }
  if (mode == 0) {
    if (ordx) for (size_t e = 0; e < ox.size(); ++e) ordx[e] = ox[e];
    if (ordy) for (size_t e = 0; e < oy.size(); ++e) ordy[e] = oy[e];
    if (psix) for (size_t e = 0; e < px.size(); ++e) psix[e] = px[e];
    if (psiy) for (size_t e = 0; e < py.size(); ++e) psiy[e] = py[e];
    if (alx) for (size_t e = 0; e < ax.size(); ++e) alx[e] = ax[e];
    if (aly) for (size_t e = 0; e < ay.size(); ++e) aly[e] = ay[e];
  }
  if (Fout) for (size_t a = 0; a < F.size(); ++a) Fout[a] = F[a];
  if (Gout) for (size_t a = 0; a < Gf.size(); ++a) Gout[a] = Gf[a];
  return 0;
}

int check_problem(const oracle_problem* pb) {
  if (!pb) return -1;
  if (pb->dim != 1 && pb->dim != 2) return -2;
  if (pb->P < 1 || pb->P > PMAX || (pb->dim == 2 && pb->P > 4)) return -2;
  if (pb->nvar < 1 || pb->nvar > VMAX) return -2;
  if (pb->flux == FLUX_BURGERS && (pb->nvar != 1 || pb->dim != 1)) return -2;
  if (pb->flux == FLUX_EULER && pb->nvar != (pb->dim == 1 ? 3 : 4)) return -2;
  if (pb->nx < 2 * std::max(pb->P, 2) || (pb->dim == 2 && pb->ny < 2 * std::max(pb->P, 2))) return -2;
  if (pb->flags & ~(FLAG_FLO_LF | FLAG_FLO_HLL | FLAG_PSI2_MODIFIED | FLAG_PSI1_ROE | FLAG_SQUARE_2D |
                    FLAG_PLAIN_ROUNDING))
    return -2;
  if ((pb->flags & FLAG_SQUARE_2D) && pb->dim != 2) return -2;
  if ((pb->flags & FLAG_FLO_LF) && (pb->flags & FLAG_FLO_HLL)) return -2;
  if ((pb->flags & FLAG_PSI1_ROE) && pb->flux == FLUX_EULER) return -2;   // scalar laws only
  return 0;
}

}  // namespace

extern "C" {

// Coefficient tables for half-width p (each array has the documented shape).
int oracle_coeffs(int p, double* g1, double* gt, double* eta, double* tau, double* d1) {
  if (p < 1 || p > PMAX) return -2;
  const Tables& T = tables();
  int nn = 2 * p;
  for (int a = 0; a < nn; ++a)
    for (int l = 0; l < nn; ++l) {
      if (g1) g1[a * nn + l] = T.g1[p][a][l];
      if (gt) gt[a * nn + l] = T.gt[p][a][l];
    }
  for (int a = 0; a < nn; ++a) {
    if (eta) eta[a] = T.eta[p][a];
    if (tau) tau[a] = T.tau[p][a];
  }
  if (d1) for (int a = 0; a < 2 * p + 1; ++a) d1[a] = T.d1[p][a];
  return 0;
}

// psi^p of one component on 2p values (offsets -p+1..p), for pins.
double oracle_indicator(const double* v, int p, double eps) { return indicator_psi(v, p, p, eps); }
// psi^1 of one component on 4 values (offsets -1..2).
double oracle_limiter(const double* v) { return limiter_psi1(v, 2); }
// Modified p = 2 indicator on 4 values (offsets -1..2), for pins.
double oracle_indicator2_modified(const double* v, double eps) { return indicator_psi2_modified(v, 2, eps); }

// One ACAT step.  mode 0: adaptive (decisions written to ord/psi1/alpha when
// non-null); mode 1: frozen replay of the given decisions.
int oracle_step1d(const oracle_problem* pb, const double* u, double* uout, double dt, int mode, int8_t* ord,
                  double* psi1, double* alpha, double* flux_out, int nthreads) {
  int e = check_problem(pb);
  if (e) return e;
  if (mode == 1 && (!ord || !psi1 || !alpha)) return -1;
  return step1d<double>(*pb, u, uout, dt, mode, ord, psi1, alpha, flux_out, nthreads);
}

// Forward-mode tangent of the frozen replay step: du_out = J du.
int oracle_step1d_jvp(const oracle_problem* pb, const double* u, const double* du, double* uout, double* duout,
                      double dt, int8_t* ord, double* psi1, double* alpha, int nthreads) {
  int e = check_problem(pb);
  if (e) return e;
  size_t n = (size_t)pb->nvar * pb->nx;
  std::vector<Dual> x(n), y(n);
  for (size_t a = 0; a < n; ++a) { x[a] = Dual(u[a]); x[a].d[0] = du[a]; }
  step1d<Dual>(*pb, x.data(), y.data(), dt, 1, ord, psi1, alpha, nullptr, nthreads);
  for (size_t a = 0; a < n; ++a) { uout[a] = y[a].v; duout[a] = y[a].d[0]; }
  return 0;
}

int oracle_step2d(const oracle_problem* pb, const double* u, double* uout, double dt, int mode, int8_t* ordx,
                  int8_t* ordy, double* psix, double* psiy, double* alx, double* aly, double* Fout, double* Gout,
                  int nthreads) {
  int e = check_problem(pb);
  if (e) return e;
  if (pb->dim != 2) return -2;
  if (mode == 1 && (!ordx || !ordy || !psix || !psiy || !alx || !aly)) return -1;
  return step2d<double>(*pb, u, uout, dt, mode, ordx, ordy, psix, psiy, alx, aly, Fout, Gout, nthreads);
}

int oracle_step2d_jvp(const oracle_problem* pb, const double* u, const double* du, double* uout, double* duout,
                      double dt, int8_t* ordx, int8_t* ordy, double* psix, double* psiy, double* alx, double* aly,
                      int nthreads) {
  int e = check_problem(pb);
  if (e) return e;
  size_t n = (size_t)pb->nvar * pb->nx * pb->ny;
  std::vector<Dual> x(n), y(n);
  for (size_t a = 0; a < n; ++a) { x[a] = Dual(u[a]); x[a].d[0] = du[a]; }
  step2d<Dual>(*pb, x.data(), y.data(), dt, 1, ordx, ordy, psix, psiy, alx, aly, nullptr, nullptr, nthreads);
  for (size_t a = 0; a < n; ++a) { uout[a] = y[a].v; duout[a] = y[a].d[0]; }
  return 0;
}

// The same tangent along two directions at once: du and duout are [2][state].
// decide = 0: the given decisions (frozen replay); decide = 1: the step
// decides from the values of u (the decisions are written to the arrays),
// which is the tangent of the replay map of the step's own decisions.
int oracle_step2d_jvp2(const oracle_problem* pb, const double* u, const double* du, double* uout, double* duout,
                       double dt, int8_t* ordx, int8_t* ordy, double* psix, double* psiy, double* alx, double* aly,
                       int nthreads, int decide) {
  int e = check_problem(pb);
  if (e) return e;
  if (!ordx || !ordy || !psix || !psiy || !alx || !aly) return -1;
  size_t n = (size_t)pb->nvar * pb->nx * pb->ny;
  std::vector<Dual2> x(n), y(n);
  for (size_t a = 0; a < n; ++a) {
    x[a] = Dual2(u[a]);
    x[a].d[0] = du[a];
    x[a].d[1] = du[n + a];
  }
  step2d<Dual2>(*pb, x.data(), y.data(), dt, decide ? 0 : 1, ordx, ordy, psix, psiy, alx, aly, nullptr, nullptr,
                nthreads);
  for (size_t a = 0; a < n; ++a) {
    uout[a] = y[a].v;
    duout[a] = y[a].d[0];
    duout[n + a] = y[a].d[1];
  }
  return 0;
}

// Updated state at selected cells only (adaptive decisions), for sampled
// checks on grids too large for a full oracle step.  cells: (i1, i2) pairs
// (i2 = 0 in 1D); out: [ncell][nvar]; ord_out: [ncell][4] orders of the
// x-left, x-right, y-left, y-right interfaces of each cell (1D: two).
int oracle_update_cells(const oracle_problem* pb, const double* u, double dt, int64_t ncell, const int64_t* cells,
                        double* out, int8_t* ord_out, int nthreads) {
  int e = check_problem(pb);
  if (e) return e;
  const int nv = pb->nvar;
  if (nthreads > 0) omp_set_num_threads(nthreads);
  if (pb->dim == 1) {
    Step1D<double> S(*pb, u);
    S.dt = dt;
    const double lam = dt / pb->dx;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t s = 0; s < ncell; ++s) {
      int64_t i = cells[2 * s];
      double Fl[VMAX], Fr[VMAX];
      int ol = 0, orr = 0;
      double d1, d2;
      S.flux(i - 1 - S.ioff, lam, true, ol, d1, d2, Fl);
      S.flux(i - S.ioff, lam, true, orr, d1, d2, Fr);
      for (int c = 0; c < nv; ++c) out[s * nv + c] = S.at(c, i) + lam * (Fl[c] - Fr[c]);
      if (ord_out) { ord_out[4 * s] = (int8_t)ol; ord_out[4 * s + 1] = (int8_t)orr; ord_out[4 * s + 2] = 0; ord_out[4 * s + 3] = 0; }
    }
    return 0;
  }
  Step2D<double> S(*pb, u);
  S.dt = dt;
  const double lamx = dt / pb->dx, lamy = dt / pb->dy;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t s = 0; s < ncell; ++s) {
    int64_t i1 = cells[2 * s], i2 = cells[2 * s + 1];
    // corners (i1-1, i2) [F left], (i1, i2) [F right, G right], (i1, i2-1) [G left]
    double fl[VMAX], fr[VMAX], gl[VMAX], gr[VMAX];
    double p, a, px, ax;
    int qxl = S.decide(0, i1 - 1, i2, &px, &ax);
    int qyl_c = S.decide(1, i1 - 1, i2, &p, &a);    // y-order at corner (i1-1, i2)
    S.corner(i1 - 1, i2, qxl, qyl_c, px, -1, ax, -1, lamx, lamy, fl, nullptr);
    double pxr, axr, pyr, ayr;
    int qxr = S.decide(0, i1, i2, &pxr, &axr);
    int qyr = S.decide(1, i1, i2, &pyr, &ayr);
    S.corner(i1, i2, qxr, qyr, pxr, pyr, axr, ayr, lamx, lamy, fr, gr);
    double pyl, ayl;
    int qxl2 = S.decide(0, i1, i2 - 1, &p, &a);      // x-order at corner (i1, i2-1)
    int qyl = S.decide(1, i1, i2 - 1, &pyl, &ayl);
    S.corner(i1, i2 - 1, qxl2, qyl, -1, pyl, -1, ayl, lamx, lamy, nullptr, gl);
    for (int c = 0; c < nv; ++c)
      out[s * nv + c] = S.at(c, i1, i2) + lamx * (fl[c] - fr[c]) + lamy * (gl[c] - gr[c]);
    if (ord_out) {
      ord_out[4 * s] = (int8_t)qxl; ord_out[4 * s + 1] = (int8_t)qxr;
      ord_out[4 * s + 2] = (int8_t)qyl; ord_out[4 * s + 3] = (int8_t)qyr;
    }
  }
  return 0;
}

// Largest spectral radius per direction over the grid (CFL rule input).
int oracle_max_speed(const oracle_problem* pb, const double* u, double* smax) {
  int e = check_problem(pb);
  if (e) return e;
  const int nv = pb->nvar;
  const int64_t n = pb->nx * (pb->dim == 2 ? pb->ny : 1);
  for (int d = 0; d < pb->dim; ++d) {
    double m = 0.0;
    for (int64_t a = 0; a < n; ++a) {
      double w[VMAX];
      for (int c = 0; c < nv; ++c) w[c] = u[(size_t)c * n + a];
      m = std::max(m, spectral_radius(*pb, w, d));
    }
    smax[d] = m;
  }
  return 0;
}

}  // extern "C"
