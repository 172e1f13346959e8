// Differentiation coefficients of the ACAT recursion, generated at compile
// time in exact rational arithmetic and rounded once to binary64.
//
// Sec. 2.1 defines the interpolatory formulas A^{k,q}_{p} on the 2p nodes
// J_p = {-p+1, .., p}; their weights gamma^{k,q}_{p,j} are obtained here
// with Fornberg's recursion for finite-difference weights (the algorithm the
// paper names for these coefficients), carried out on exact fractions.
//   G1[p][j][l]  gamma^{1,j}_{p,l}: first derivative at node j (space, Sec. 2.2 step a)
//   GT[p][k][r]  gamma^{k,0}_{p,r}: k-th derivative at 0 (time, Sec. 2.2 step c)
//   TAU[p][l]    gamma^{2p-1,1/2}_{p,l}: the undivided difference of tau_p (Sec. 3.2)
//   ETA[p][l]    weights of the interface value in the CAT flux: fixed by the
//                relation D^1_{p,i} = (A_{p,i} - A_{p,i-1}) / dx between the
//                centred (2p+1)-point first derivative and the interface
//                formula (Sec. 2.1, relation with k = 1), i.e.
//                eta_{m+1} = eta_m - delta^1_{p,m}, eta_{-p} = 0.
//   TAYLOR[r][l] r^l / l! (Taylor weights of the local time nodes)
//   INVFACT[k]   1 / k!
// Indices j, l, r of a p-stencil are stored with offset p-1.
#pragma once

#include <cstdint>

namespace acat {

constexpr int PMAX = 6;     // largest stencil half-width (1D; 2D stops at 4)
constexpr int PMAX_2D = 4;
constexpr int NMAX = 2 * PMAX;

namespace detail {

struct Frac {
  __int128 n, d;
};

constexpr __int128 iabs(__int128 a) { return a < 0 ? -a : a; }

constexpr __int128 igcd(__int128 a, __int128 b) {
  a = iabs(a);
  b = iabs(b);
  while (b != 0) {
    __int128 t = a % b;
    a = b;
    b = t;
  }
  return a;
}

constexpr Frac mk(__int128 n, __int128 d = 1) {
  if (d < 0) { n = -n; d = -d; }
  __int128 g = igcd(n, d);
  if (g > 1) { n /= g; d /= g; }
  if (n == 0) d = 1;
  return Frac{n, d};
}
constexpr Frac add(Frac a, Frac b) { return mk(a.n * b.d + b.n * a.d, a.d * b.d); }
constexpr Frac sub(Frac a, Frac b) { return mk(a.n * b.d - b.n * a.d, a.d * b.d); }
constexpr Frac mul(Frac a, Frac b) { return mk(a.n * b.n, a.d * b.d); }
constexpr Frac dvd(Frac a, Frac b) { return mk(a.n * b.d, a.d * b.n); }
// numerator and denominator stay below 2^53 for every table here (checked:
// a larger one stops the constant evaluation), so one IEEE division rounds
// the exact value correctly
constexpr __int128 TWO53 = (__int128)1 << 53;
constexpr double exact_or_fail(double v, bool ok) { return ok ? v : throw "table entry not exact"; }
constexpr double to_f64(Frac a) {
  return exact_or_fail((double)(int64_t)a.n / (double)(int64_t)a.d, iabs(a.n) < TWO53 && a.d < TWO53);
}

// Fornberg's recursion: weights w[k][j] of the k-th derivative (k <= m) at
// z from the values at nodes x[0..n-1].
struct FWeights {
  Frac w[NMAX + 1][2 * PMAX + 1];
};

constexpr FWeights fornberg(int n, const int* x, Frac z, int m) {
  FWeights C{};
  for (int k = 0; k <= NMAX; ++k)
    for (int j = 0; j < 2 * PMAX + 1; ++j) C.w[k][j] = mk(0);
  Frac c1 = mk(1);
  Frac c4 = sub(mk(x[0]), z);
  C.w[0][0] = mk(1);
  for (int i = 1; i < n; ++i) {
    int mn = i < m ? i : m;
    Frac c2 = mk(1);
    Frac c5 = c4;
    c4 = sub(mk(x[i]), z);
    for (int j = 0; j < i; ++j) {
      Frac c3 = mk(x[i] - x[j]);
      c2 = mul(c2, c3);
      if (j == i - 1) {
        for (int k = mn; k >= 1; --k)
          C.w[k][i] = dvd(mul(c1, sub(mul(mk(k), C.w[k - 1][i - 1]), mul(c5, C.w[k][i - 1]))), c2);
        C.w[0][i] = dvd(mul(mk(-1), mul(c1, mul(c5, C.w[0][i - 1]))), c2);
      }
      for (int k = mn; k >= 1; --k) C.w[k][j] = dvd(sub(mul(c4, C.w[k][j]), mul(mk(k), C.w[k - 1][j])), c3);
      C.w[0][j] = dvd(mul(c4, C.w[0][j]), c3);
    }
    c1 = c2;
  }
  return C;
}

}  // namespace detail

struct CoeffTables {
  double G1[PMAX + 1][NMAX][NMAX];
  double GT[PMAX + 1][NMAX][NMAX];
  double TAU[PMAX + 1][NMAX];
  double ETA[PMAX + 1][NMAX];
  double FACT2PM1[PMAX + 1];
  double TAYLOR[NMAX][NMAX];   // [r + PMAX - 1][l]
  double INVFACT[NMAX + 1];
};

constexpr CoeffTables make_tables() {
  using namespace detail;
  CoeffTables T{};
  for (int p = 1; p <= PMAX; ++p) {
    const int n = 2 * p;
    int x[NMAX] = {};
    for (int a = 0; a < n; ++a) x[a] = a - p + 1;
    for (int a = 0; a < n; ++a) {
      FWeights W = fornberg(n, x, mk(x[a]), 1);
      for (int l = 0; l < n; ++l) T.G1[p][a][l] = to_f64(W.w[1][l]);
    }
    {
      FWeights W = fornberg(n, x, mk(0), n - 1);
      for (int k = 0; k < n; ++k)
        for (int r = 0; r < n; ++r) T.GT[p][k][r] = to_f64(W.w[k][r]);
    }
    {
      FWeights W = fornberg(n, x, mk(1, 2), n - 1);
      for (int l = 0; l < n; ++l) T.TAU[p][l] = to_f64(W.w[n - 1][l]);
    }
    {
      int xc[2 * PMAX + 1] = {};
      for (int a = 0; a <= n; ++a) xc[a] = a - p;
      FWeights W = fornberg(n + 1, xc, mk(0), 1);
      Frac e = mk(0);
      for (int a = 0; a < n; ++a) {   // node m = a - p; eta_{m+1} = eta_m - delta_m
        e = sub(e, W.w[1][a]);
        T.ETA[p][a] = to_f64(e);
      }
    }
    int64_t f = 1;
    for (int t = 2; t <= 2 * p - 1; ++t) f *= t;
    T.FACT2PM1[p] = (double)f;
  }
  for (int ri = 0; ri < NMAX; ++ri) {
    const int r = ri - (PMAX - 1);
    Frac v = mk(1);
    for (int l = 0; l < NMAX; ++l) {
      T.TAYLOR[ri][l] = to_f64(v);
      v = dvd(mul(v, mk(r)), mk(l + 1));
    }
  }
  int64_t f = 1;
  for (int k = 0; k <= NMAX; ++k) {
    if (k > 0) f *= k;
    T.INVFACT[k] = to_f64(mk(1, f));
  }
  return T;
}

}  // namespace acat
