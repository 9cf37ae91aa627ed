// Host plan construction in binary128 arithmetic (see planner.h).
//
// The boundary construction follows Sec. 3.2: boundary scaling functions and
// wavelets with staggered supports [0, nu+m] (left) and [-m-nu, 0] (right),
// finite combinations of interior functions, orthonormal and preserving the
// nu vanishing moments.  The paper states supports and staggering; the
// construction below is the Cohen-Daubechies-Vial one written from the
// mathematics:
//   * left edge space = { sum_{k=-nu+1}^{nu-1} p(k) phi(. - k) on [0,inf) :
//     deg p < nu }, interior translates k >= nu;
//   * phi^left_m spans the tails supported in [0, nu+m] (p(m+1..nu-1) = 0)
//     orthogonally to those supported in [0, nu+m-1]; positive coefficient on
//     the translate k = m;
//   * psi^left_m spans { f in V_1 supported in [0, nu+m], orthogonal to V_0
//     and to the interior wavelets } orthogonally to the same space for
//     m-1; its coefficient on the level-1 translate nu+2m has the sign of g_nu;
//   * the right edge is the mirror statement on (-inf, 0] (translates
//     [-nu, nu-2], positive coefficient on k = -m-1; wavelet sign of g_{-nu+1}).
// Inner products use the exact half-line Gram matrix, obtained here from the
// cell Gram matrix K[a][b] = int_0^1 phi(x+a) phi(x+b) dx, the eigenvalue-1
// solution of its two-scale relation, summed over the cells of the half-line.
#include "planner.h"

#include <quadmath.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>

namespace wh2wav {
namespace {

using R = __float128;

R rabs(R x) { return x < 0 ? -x : x; }
R rsqrt(R x) { return sqrtq(x); }

struct Cx {
  R re, im;
};
Cx operator+(Cx a, Cx b) { return {a.re + b.re, a.im + b.im}; }
Cx operator-(Cx a, Cx b) { return {a.re - b.re, a.im - b.im}; }
Cx operator*(Cx a, Cx b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
Cx operator/(Cx a, Cx b) {
  R d = b.re * b.re + b.im * b.im;
  return {(a.re * b.re + a.im * b.im) / d, (a.im * b.re - a.re * b.im) / d};
}
R cabs2(Cx a) { return a.re * a.re + a.im * a.im; }
R cabs(Cx a) { return rsqrt(cabs2(a)); }
Cx csqrt(Cx a) {
  R r = cabs(a);
  R re = rsqrt((r + a.re) / 2);
  R im = rsqrt(rabs((r - a.re) / 2));
  if (a.im < 0) im = -im;
  return {re, im};
}

// ---------------------------------------------------------------- filters
// Spectral factorisation (Sec. 3.2: compactly supported orthonormal wavelets
// with nu vanishing moments).  The roots of P(y) = sum_{k<nu} C(nu-1+k, k) y^k
// are found with the Aberth-Ehrlich iteration; each root gives the pair z, 1/z
// with (2 - z - 1/z)/4 = y, and a filter is the coefficient list of
// (1+z)^nu prod (z - z_i) over one member of each pair, from the highest power
// down, scaled to sum sqrt(2).
bool y_roots(int nu, std::vector<Cx>* out, std::string* err) {
  const int d = nu - 1;
  std::vector<R> p(nu);  // p[k] = coefficient of y^k
  for (int k = 0; k < nu; ++k) {
    R b = 1;  // binom(nu-1+k, k)
    for (int i = 1; i <= k; ++i) b = b * (nu - 1 + i) / i;
    p[k] = b;
  }
  auto eval = [&](Cx y, Cx* dp) {
    Cx v{p[d], 0}, dv{0, 0};
    for (int k = d - 1; k >= 0; --k) {
      dv = dv * y + v;
      v = v * y + Cx{p[k], 0};
    }
    *dp = dv;
    return v;
  };
  R bound = 0;
  for (int k = 0; k < d; ++k) bound = std::max(bound, rabs(p[k] / p[d]));
  const R rad = (bound + 1) / 2;
  std::vector<Cx> z(d);
  for (int i = 0; i < d; ++i) {
    R a = 2 * M_PIq * (i + 0.25Q) / d + 0.4Q;
    z[i] = {rad * cosq(a), rad * sinq(a)};
  }
  bool converged = false;
  for (int it = 0; it < 1000 && !converged; ++it) {
    R worst = 0;
    for (int i = 0; i < d; ++i) {
      Cx dp;
      Cx v = eval(z[i], &dp);
      if (cabs2(dp) == 0) continue;
      Cx w = v / dp;
      Cx s{0, 0};
      for (int k = 0; k < d; ++k)
        if (k != i) s = s + Cx{1, 0} / (z[i] - z[k]);
      Cx step = w / (Cx{1, 0} - w * s);
      z[i] = z[i] - step;
      worst = std::max(worst, cabs(step) / std::max(R(1), cabs(z[i])));
    }
    converged = worst < 1e-32Q;
  }
  for (int pol = 0; pol < 3; ++pol)
    for (int i = 0; i < d; ++i) {
      Cx dp;
      Cx v = eval(z[i], &dp);
      if (cabs2(dp) > 0) z[i] = z[i] - v / dp;
    }
  if (!converged) {
    *err = "filter root finding did not converge";
    return false;
  }
  *out = z;
  return true;
}

// The member z, |z| < 1, of the pair belonging to the root y.
Cx inside_root(Cx y) {
  Cx b = Cx{2, 0} - Cx{4, 0} * y;
  Cx disc = csqrt(b * b - Cx{4, 0});
  Cx z1 = (b + disc) / Cx{2, 0}, z2 = (b - disc) / Cx{2, 0};
  return cabs2(z1) < 1 ? z1 : z2;
}

std::vector<R> taps_from_roots(int nu, const std::vector<Cx>& zs) {
  std::vector<Cx> poly{{1, 0}};
  auto mul = [&](Cx a0, Cx a1) {  // poly *= (a0 z + a1)
    std::vector<Cx> o(poly.size() + 1, Cx{0, 0});
    for (size_t i = 0; i < poly.size(); ++i) {
      o[i] = o[i] + poly[i] * a0;
      o[i + 1] = o[i + 1] + poly[i] * a1;
    }
    poly.swap(o);
  };
  for (int i = 0; i < nu; ++i) mul({1, 0}, {1, 0});
  for (const Cx& zi : zs) mul({1, 0}, Cx{0, 0} - zi);
  R total = 0;
  for (auto& c : poly) total += c.re;
  std::vector<R> out(poly.size());
  for (size_t i = 0; i < poly.size(); ++i) out[i] = poly[i].re * rsqrt(2) / total;
  return out;
}

// Daubechies filter: the minimum-phase choice (every z inside the unit circle).
bool daubechies(int nu, std::vector<R>* out, std::string* err) {
  out->clear();
  if (nu == 1) {
    R s = rsqrt(2) / 2;
    *out = {s, s};
    return true;
  }
  std::vector<Cx> ys;
  if (!y_roots(nu, &ys, err)) return false;
  std::vector<Cx> zs;
  for (const Cx& y : ys) zs.push_back(inside_root(y));
  *out = taps_from_roots(nu, zs);
  return true;
}

// Deviation from linear phase of the filter with factor roots zs.  Read from
// (1+z)^nu prod (z - z_i), highest power first, the filter's response is
// e^{-i(2nu-1)w} c (1 + e^{iw})^nu prod (e^{iw} - z_i): its phase is linear in
// w plus phi(w) = sum_i arg(e^{iw} - z_i), taken here from the roots on
// w_k = pi k / 256 (k = 0 .. 256) and unwrapped along k.  Returns the largest
// distance of phi from its least-squares straight line.  (From the taps, the
// phase near w = pi, a zero of order nu, would carry no accurate digits.)
R phase_deviation(const std::vector<Cx>& zs) {
  constexpr int K = 256;
  std::vector<R> w(K + 1), th(K + 1);
  for (int k = 0; k <= K; ++k) {
    w[k] = M_PIq * k / K;
    const Cx u{cosq(w[k]), sinq(w[k])};
    R a = 0;
    for (const Cx& z : zs) {
      const Cx d = u - z;
      a += atan2q(d.im, d.re);
    }
    if (k > 0) {
      while (a - th[k - 1] > M_PIq) a -= 2 * M_PIq;
      while (a - th[k - 1] <= -M_PIq) a += 2 * M_PIq;
    }
    th[k] = a;
  }
  R sw = 0, st = 0, sww = 0, swt = 0;
  for (int k = 0; k <= K; ++k) sw += w[k], st += th[k], sww += w[k] * w[k], swt += w[k] * th[k];
  const R n = K + 1;
  const R c = (n * swt - sw * st) / (n * sww - sw * sw);
  const R a0 = (st - c * sw) / n;
  R dev = 0;
  for (int k = 0; k <= K; ++k) dev = std::max(dev, rabs(th[k] - a0 - c * w[k]));
  return dev;
}

// Least-asymmetric filter (symlet).  Each root group of P(y) -- a real root,
// or a conjugate pair taken together so the taps stay real -- takes the pair
// member inside or outside the unit circle; groups are ordered by the real,
// then the imaginary part of their member with Im y >= 0, and bit g of the
// choice mask selects the outside member for group g.  The filter of least
// phase_deviation wins; a mask and its complement give the same filter
// reversed (equal deviation) and the smaller mask is kept.
bool symlet(int nu, std::vector<R>* out, std::string* err) {
  if (nu <= 1) return daubechies(nu, out, err);
  std::vector<Cx> ys;
  if (!y_roots(nu, &ys, err)) return false;
  const R tol = 1e-20Q;
  std::vector<Cx> reps;
  for (const Cx& y : ys)
    if (y.im >= -tol) reps.push_back(y);
  std::sort(reps.begin(), reps.end(), [](const Cx& a, const Cx& b) {
    return a.re != b.re ? a.re < b.re : a.im < b.im;
  });
  std::vector<std::vector<Cx>> groups;
  for (const Cx& y : reps) {
    const Cx zin = inside_root(y);
    if (rabs(y.im) <= tol)
      groups.push_back({zin});
    else
      groups.push_back({zin, Cx{zin.re, -zin.im}});
  }
  if (groups.size() > 16) {
    *err = "too many root groups for the symlet search";
    return false;
  }
  R best_dev = -1;
  std::vector<Cx> best;
  for (uint32_t mask = 0; mask < (1u << groups.size()); ++mask) {
    std::vector<Cx> zs;
    for (size_t g = 0; g < groups.size(); ++g)
      for (const Cx& z : groups[g]) zs.push_back(((mask >> g) & 1u) ? Cx{1, 0} / z : z);
    const R dev = phase_deviation(zs);
    if (best_dev < 0 || dev < best_dev - 1e-20Q) {
      best_dev = dev;
      best = zs;
    }
  }
  *out = taps_from_roots(nu, best);
  return true;
}

// -------------------------------------------------------- linear algebra
using Mat = std::vector<std::vector<R>>;

// Null vector of a square matrix of rank n-1, by Gaussian elimination with
// complete pivoting.  Fails if the rank is not exactly n-1.
bool null_vector(Mat A, std::vector<R>* x, std::string* err) {
  const int n = (int)A.size();
  std::vector<int> col(n);
  for (int i = 0; i < n; ++i) col[i] = i;
  R scale = 1;  // callers pass (operator - identity): rank is judged against O(1) entries
  for (auto& r : A)
    for (R v : r) scale = std::max(scale, rabs(v));
  std::vector<R> piv(n);
  for (int k = 0; k < n; ++k) {
    int bi = k, bj = k;
    R best = -1;
    for (int i = k; i < n; ++i)
      for (int jj = k; jj < n; ++jj)
        if (rabs(A[i][jj]) > best) best = rabs(A[i][jj]), bi = i, bj = jj;
    std::swap(A[k], A[bi]);
    if (bj != k) {
      for (int i = 0; i < n; ++i) std::swap(A[i][k], A[i][bj]);
      std::swap(col[k], col[bj]);
    }
    piv[k] = A[k][k];
    if (k == n - 1) break;
    if (rabs(piv[k]) <= scale * 1e-28Q) {
      *err = "eigenvalue-1 space is not one-dimensional";
      return false;
    }
    for (int i = k + 1; i < n; ++i) {
      R f = A[i][k] / A[k][k];
      if (f == 0) continue;
      for (int jj = k; jj < n; ++jj) A[i][jj] -= f * A[k][jj];
    }
  }
  if (rabs(piv[n - 1]) > scale * 1e-26Q) {
    *err = "matrix is not singular: no eigenvalue 1";
    return false;
  }
  std::vector<R> y(n, 0);
  y[n - 1] = 1;
  for (int k = n - 2; k >= 0; --k) {
    R s = 0;
    for (int jj = k + 1; jj < n; ++jj) s += A[k][jj] * y[jj];
    y[k] = -s / A[k][k];
  }
  x->assign(n, 0);
  for (int k = 0; k < n; ++k) (*x)[col[k]] = y[k];
  return true;
}

// One-sided Jacobi SVD (Hestenes): returns the right singular vectors whose
// singular value is below tol * (largest singular value).
bool null_space(Mat A, R tol, Mat* basis) {
  const int rows = (int)A.size(), n = rows ? (int)A[0].size() : 0;
  Mat V(n, std::vector<R>(n, 0));
  for (int i = 0; i < n; ++i) V[i][i] = 1;
  for (int sweep = 0; sweep < 80; ++sweep) {
    bool changed = false;
    for (int p = 0; p < n; ++p)
      for (int qq = p + 1; qq < n; ++qq) {
        R a = 0, b = 0, c = 0;
        for (int i = 0; i < rows; ++i) {
          a += A[i][p] * A[i][p];
          b += A[i][qq] * A[i][qq];
          c += A[i][p] * A[i][qq];
        }
        if (c == 0 || rabs(c) <= 1e-33Q * rsqrt(a * b)) continue;
        changed = true;
        R zeta = (b - a) / (2 * c);
        R t = (zeta >= 0 ? 1 : -1) / (rabs(zeta) + rsqrt(1 + zeta * zeta));
        R cs = 1 / rsqrt(1 + t * t), sn = cs * t;
        for (int i = 0; i < rows; ++i) {
          R x = A[i][p], y = A[i][qq];
          A[i][p] = cs * x - sn * y;
          A[i][qq] = sn * x + cs * y;
        }
        for (int i = 0; i < n; ++i) {
          R x = V[i][p], y = V[i][qq];
          V[i][p] = cs * x - sn * y;
          V[i][qq] = sn * x + cs * y;
        }
      }
    if (!changed) break;
  }
  std::vector<R> sv(n, 0);
  R smax = 0;
  for (int jcol = 0; jcol < n; ++jcol) {
    R s = 0;
    for (int i = 0; i < rows; ++i) s += A[i][jcol] * A[i][jcol];
    sv[jcol] = rsqrt(s);
    smax = std::max(smax, sv[jcol]);
  }
  basis->clear();
  for (int jcol = 0; jcol < n; ++jcol)
    if (sv[jcol] <= tol * smax) {
      std::vector<R> v(n);
      for (int i = 0; i < n; ++i) v[i] = V[i][jcol];
      basis->push_back(v);
    }
  return true;
}

// ------------------------------------------------------------- cascade
// Cell integrals of phi at resolution 2^-r: Phi_r[s], s in [(-nu+1) 2^r, nu 2^r).
struct Cells {
  int64_t lo = 0;
  std::vector<R> v;
  R at(int64_t s) const {
    int64_t i = s - lo;
    return (i >= 0 && i < (int64_t)v.size()) ? v[i] : R(0);
  }
};

bool phi_cells(const std::vector<R>& h, int nu, int r, Cells* out, std::string* err) {
  const int n = 2 * nu - 1;
  Mat A(n, std::vector<R>(n, 0));
  const R inv_sqrt2 = 1 / rsqrt(2);
  for (int a = 0; a < n; ++a) {
    int s = a - nu + 1;
    for (int c = -nu + 1; c <= nu; ++c)
      for (int t : {2 * s - c, 2 * s - c + 1})
        if (t >= -nu + 1 && t <= nu - 1) A[a][t + nu - 1] += h[c + nu - 1] * inv_sqrt2;
    A[a][a] -= 1;
  }
  std::vector<R> v;
  if (!null_vector(A, &v, err)) return false;
  R sum = 0;
  for (R x : v) sum += x;
  Cells cur;
  cur.lo = -nu + 1;
  cur.v.resize(n);
  for (int i = 0; i < n; ++i) cur.v[i] = v[i] / sum;
  for (int level = 1; level <= r; ++level) {
    Cells nxt;
    nxt.lo = (int64_t)(-nu + 1) << level;
    nxt.v.assign((size_t)(2 * nu - 1) << level, 0);
    const int64_t half = (int64_t)1 << (level - 1);
    for (size_t i = 0; i < nxt.v.size(); ++i) {
      int64_t s = nxt.lo + (int64_t)i;
      R acc = 0;
      for (int c = -nu + 1; c <= nu; ++c) acc += h[c + nu - 1] * cur.at(s - c * half);
      nxt.v[i] = acc * inv_sqrt2;
    }
    cur = nxt;
  }
  *out = cur;
  return true;
}

// ------------------------------------------------------ half-line Gram
struct Gram {
  int nu = 0;
  std::vector<R> K;  // cell Gram (2nu-1)^2
  R cell(int a, int b) const {
    if (a < -nu + 1 || a > nu - 1 || b < -nu + 1 || b > nu - 1) return 0;
    return K[(a + nu - 1) * (2 * nu - 1) + (b + nu - 1)];
  }
  // int over [0, inf) of phi(x-k) phi(x-kp)
  R left(int k, int kp) const {
    R s = 0;
    int lo = std::max(0, std::max(k, kp) - nu + 1), hi = std::min(k, kp) + nu - 1;
    for (int i = lo; i <= hi; ++i) s += cell(i - k, i - kp);
    return s;
  }
  // int over (-inf, 0] of phi(x-k) phi(x-kp)
  R right(int k, int kp) const {
    R s = 0;
    int lo = std::max(k, kp) - nu + 1, hi = std::min(-1, std::min(k, kp) + nu - 1);
    for (int i = lo; i <= hi; ++i) s += cell(i - k, i - kp);
    return s;
  }
  R side(bool left_side, int k, int kp) const { return left_side ? left(k, kp) : right(k, kp); }
};

bool cell_gram(const std::vector<R>& h, int nu, Gram* G, std::string* err) {
  const int n = 2 * nu - 1, n2 = n * n;
  Mat A(n2, std::vector<R>(n2, 0));
  auto id = [&](int a, int b) { return (a + nu - 1) * n + (b + nu - 1); };
  auto inside = [&](int a) { return a >= -nu + 1 && a <= nu - 1; };
  for (int a = -nu + 1; a <= nu - 1; ++a)
    for (int b = -nu + 1; b <= nu - 1; ++b) {
      int row = id(a, b);
      for (int c = -nu + 1; c <= nu; ++c)
        for (int d = -nu + 1; d <= nu; ++d) {
          R w = h[c + nu - 1] * h[d + nu - 1];
          int a1 = 2 * a - c, b1 = 2 * b - d;
          if (inside(a1) && inside(b1)) A[row][id(a1, b1)] += w;
          if (inside(a1 + 1) && inside(b1 + 1)) A[row][id(a1 + 1, b1 + 1)] += w;
        }
      A[row][row] -= 1;
    }
  std::vector<R> v;
  if (!null_vector(A, &v, err)) return false;
  R tr = 0;
  for (int a = -nu + 1; a <= nu - 1; ++a) tr += v[id(a, a)];
  G->nu = nu;
  G->K.resize(n2);
  for (int i = 0; i < n2; ++i) G->K[i] = v[i] / tr;
  // whole-line orthonormality of the integer translates
  for (int k = -2 * nu; k <= 2 * nu; ++k)
    for (int kp = -2 * nu; kp <= 2 * nu; ++kp) {
      R s = 0;
      for (int i = -4 * nu; i <= 4 * nu; ++i) s += G->cell(i - k, i - kp);
      if (rabs(s - (k == kp ? 1 : 0)) > 1e-26Q) {
        *err = "cell Gram matrix fails the orthonormality self-check";
        return false;
      }
    }
  return true;
}

// ------------------------------------------------------------ vectors
// Sparse-in-spirit dense vectors over an index window [lo, lo + size).
struct Vec {
  int lo = 0;
  std::vector<R> v;
  Vec() = default;
  Vec(int lo_, int size) : lo(lo_), v(size, 0) {}
  R& operator[](int k) { return v[k - lo]; }
  R at(int k) const {
    int i = k - lo;
    return (i >= 0 && i < (int)v.size()) ? v[i] : R(0);
  }
  int hi() const { return lo + (int)v.size(); }
};

R dot(const Vec& a, const Vec& b, const Gram& G, bool left_side) {
  R s = 0;
  for (int x = a.lo; x < a.hi(); ++x) {
    R ax = a.at(x);
    if (ax == 0) continue;
    int lo = std::max(b.lo, x - 2 * G.nu + 2), hi = std::min(b.hi(), x + 2 * G.nu - 1);
    for (int y = lo; y < hi; ++y) {
      R by = b.at(y);
      if (by != 0) s += ax * by * G.side(left_side, x, y);
    }
  }
  return s;
}

void axpy(R alpha, const Vec& x, Vec* y) {
  for (int k = x.lo; k < x.hi(); ++k) (*y)[k] += alpha * x.at(k);
}

// Window of level-1 indices used for every half-line computation.
struct Window {
  int lo, size;
};
Window level1_window(int nu, bool left_side) {
  return left_side ? Window{-nu + 1, 10 * nu + 4} : Window{-9 * nu - 5, 10 * nu + 4};
}

Vec level0_to_level1(const Vec& f0, const std::vector<R>& taps, int nu, bool left_side) {
  Window w = level1_window(nu, left_side);
  Vec out(w.lo, w.size);
  for (int k = f0.lo; k < f0.hi(); ++k) {
    R a = f0.at(k);
    if (a == 0) continue;
    for (int c = -nu + 1; c <= nu; ++c) {
      int n = 2 * k + c;
      if (left_side && n + nu <= 0) continue;       // vanishes on [0, inf)
      if (!left_side && n - nu + 1 >= 0) continue;  // vanishes on (-inf, 0]
      out[n] += a * taps[c + nu - 1];
    }
  }
  return out;
}

Vec lift(const Vec& f0, int nu, bool left_side) {  // same coefficients, level-1 window
  Window w = level1_window(nu, left_side);
  Vec out(w.lo, w.size);
  for (int k = f0.lo; k < f0.hi(); ++k) out[k] = f0.at(k);
  return out;
}

bool edge_scaling(int nu, bool left_side, const Gram& G, std::vector<Vec>* out, std::string* err) {
  out->clear();
  for (int m = 0; m < nu; ++m) {
    Vec u = left_side ? Vec(-nu + 1, 2 * nu - 1) : Vec(-nu, 2 * nu - 1);
    int lead = left_side ? m : -m - 1;
    for (int k = u.lo; k < u.hi(); ++k) {
      R val = 1;
      if (left_side)
        for (int i = m + 1; i <= nu - 1; ++i) val *= (k - i);
      else
        for (int i = -nu; i <= -m - 2; ++i) val *= (k - i);
      u[k] = val;
    }
    for (int pass = 0; pass < 2; ++pass)
      for (auto& e : *out) axpy(-dot(e, u, G, left_side), e, &u);
    R nrm = dot(u, u, G, left_side);
    if (!(nrm > 0)) {
      *err = "boundary scaling construction: degenerate tail space";
      return false;
    }
    R inv = 1 / rsqrt(nrm);
    for (auto& x : u.v) x *= inv;
    if (u.at(lead) < 0)
      for (auto& x : u.v) x = -x;
    out->push_back(u);
  }
  return true;
}

bool edge_wavelets(int nu, bool left_side, const Gram& G, const std::vector<R>& h,
                   const std::vector<R>& g, const std::vector<Vec>& scal, std::vector<Vec>* out,
                   std::string* err) {
  out->clear();
  Window w = level1_window(nu, left_side);
  std::vector<Vec> e1, cons;
  for (auto& f : scal) e1.push_back(lift(f, nu, left_side));
  for (auto& f : scal) cons.push_back(level0_to_level1(f, h, nu, left_side));
  for (int i = 0; i <= 2 * nu; ++i) {
    int k = left_side ? nu + i : -nu - 1 - i;
    Vec unit(k, 1);
    unit[k] = 1;
    cons.push_back(level0_to_level1(unit, h, nu, left_side));
    cons.push_back(level0_to_level1(unit, g, nu, left_side));
  }
  const R ref_sign = left_side ? g[2 * nu - 1] : g[0];
  for (int m = 0; m < nu; ++m) {
    std::vector<Vec> cands = e1;
    int newest = left_side ? nu + 2 * m : -nu - 2 * m - 1;
    for (int i = 0; i <= 2 * m; ++i) {
      int n = left_side ? nu + i : -nu - 2 * m - 1 + i;
      Vec unit(w.lo, w.size);
      unit[n] = 1;
      cands.push_back(unit);
    }
    Mat K(cons.size(), std::vector<R>(cands.size(), 0));
    for (size_t i = 0; i < cons.size(); ++i)
      for (size_t jc = 0; jc < cands.size(); ++jc) K[i][jc] = dot(cons[i], cands[jc], G, left_side);
    Mat ns;
    null_space(K, 1e-24Q, &ns);
    if ((int)ns.size() != m + 1) {
      *err = "boundary wavelet space has unexpected dimension";
      return false;
    }
    Vec best;
    R best_n = -1;
    for (auto& z : ns) {
      Vec f(w.lo, w.size);
      for (size_t jc = 0; jc < cands.size(); ++jc) axpy(z[jc], cands[jc], &f);
      for (int pass = 0; pass < 2; ++pass)
        for (auto& e : *out) axpy(-dot(e, f, G, left_side), e, &f);
      R nrm = rsqrt(dot(f, f, G, left_side));
      if (nrm > best_n) best_n = nrm, best = f;
    }
    for (auto& x : best.v) x /= best_n;
    R lead = best.at(newest);
    if (rabs(lead) < 1e-20Q) {
      *err = "boundary wavelet has no weight on its newest translate";
      return false;
    }
    if ((lead < 0) != (ref_sign < 0))
      for (auto& x : best.v) x = -x;
    out->push_back(best);
  }
  return true;
}

// Walsh function of Def. 3.1 at x = k / 2^J.
int walsh_sign(int64_t n, int64_t k, int J) {
  int e = 0;
  for (int i = 1; i <= J; ++i) {
    int xi = (int)((k >> (J - i)) & 1);
    int ni = (int)((n >> (i - 1)) & 1), ni1 = (int)((n >> i) & 1);
    e += (ni + ni1) * xi;
  }
  return (e & 1) ? -1 : 1;
}

}  // namespace

int build_tables(int family, int nu, int q, int j, HostPlan* P, std::string* err) {
  std::vector<R> h;
  if (!(family == WH2WAV_SYM ? symlet(nu, &h, err) : daubechies(nu, &h, err))) return WH2WAV_EINTERNAL;
  std::vector<R> g(2 * nu);
  for (int c = -nu + 1; c <= nu; ++c) {
    R v = h[(1 - c) + nu - 1];
    g[c + nu - 1] = (c & 1) ? -v : v;
  }
  Gram G;
  if (!cell_gram(h, nu, &G, err)) return WH2WAV_EINTERNAL;
  std::vector<Vec> sL, sR, wL, wR;
  if (!edge_scaling(nu, true, G, &sL, err) || !edge_scaling(nu, false, G, &sR, err))
    return WH2WAV_EINTERNAL;
  if (!edge_wavelets(nu, true, G, h, g, sL, &wL, err) ||
      !edge_wavelets(nu, false, G, h, g, sR, &wR, err))
    return WH2WAV_EINTERNAL;
  Cells phi;
  if (!phi_cells(h, nu, q, &phi, err)) return WH2WAV_EINTERNAL;

  const int Q = 1 << q;
  P->Q = Q;
  P->h.assign(2 * nu, 0);
  P->g.assign(2 * nu, 0);
  for (int i = 0; i < 2 * nu; ++i) P->h[i] = (double)h[i], P->g[i] = (double)g[i];

  const R scale = powq(2, -R(j) / 2);
  auto walsh_of = [&](auto cell_value, int s) {  // sum_r w_s(r 2^-q) cell_value(r)
    R acc = 0;
    for (int r = 0; r < Q; ++r) acc += walsh_sign(s, r, q) * cell_value(r);
    return acc;
  };
  // interior table (operator D_l of Sec. 4.1; Lemma 3.3 with h = phi)
  P->tabT.assign((size_t)(2 * nu - 1) * Q, 0);
  for (int l = -nu + 1; l <= nu - 1; ++l)
    for (int s = 0; s < Q; ++s)
      P->tabT[(l + nu - 1) * Q + s] =
          (double)(scale * walsh_of([&](int r) { return phi.at((int64_t)l * Q + r); }, s));
  // boundary bands (Prop. 4.2, bd)
  const int band = 2 * nu - 1;
  P->tabBL.assign((size_t)band * nu * Q, 0);
  P->tabBR.assign((size_t)band * nu * Q, 0);
  for (int p = 0; p < band; ++p)
    for (int m = 0; m < nu; ++m)
      for (int s = 0; s < Q; ++s) {
        if (p <= nu + m - 1) {
          auto cellL = [&](int r) {
            R acc = 0;
            for (int t = sL[m].lo; t < sL[m].hi(); ++t)
              acc += sL[m].at(t) * phi.at((int64_t)(p - t) * Q + r);
            return acc;
          };
          P->tabBL[((size_t)p * nu + m) * Q + s] = (double)(scale * walsh_of(cellL, s));
        }
        int prel = p - band;  // cell index relative to the right end, in [-2nu+1, -1]
        if (prel >= -nu - m) {
          auto cellR = [&](int r) {
            R acc = 0;
            for (int t = sR[m].lo; t < sR[m].hi(); ++t)
              acc += sR[m].at(t) * phi.at((int64_t)(prel - t) * Q + r);
            return acc;
          };
          P->tabBR[((size_t)p * nu + m) * Q + s] = (double)(scale * walsh_of(cellR, s));
        }
      }
  // one-level synthesis boundary blocks
  const int rowsB = 3 * nu - 1, colsB = 2 * nu;
  P->synL.assign((size_t)rowsB * colsB, 0);
  P->synR.assign((size_t)rowsB * colsB, 0);
  for (int side = 0; side < 2; ++side) {
    bool left_side = side == 0;
    Window w = level1_window(nu, left_side);
    const auto& sc = left_side ? sL : sR;
    const auto& wv = left_side ? wL : wR;
    std::vector<Vec> colv;
    for (int c = 0; c < nu; ++c) colv.push_back(level0_to_level1(sc[c], h, nu, left_side));
    for (int c = 0; c < nu; ++c) colv.push_back(wv[c]);
    for (int i = 0; i < rowsB; ++i) {
      Vec rowv(w.lo, w.size);
      if (left_side) {
        if (i < nu) rowv = lift(sc[i], nu, true);
        else rowv[i] = 1;
      } else {
        int nrel = i - rowsB;  // [-3nu+1, -1]
        if (nrel >= -nu) rowv = lift(sc[-1 - nrel], nu, false);
        else rowv[nrel] = 1;
      }
      auto& dst = left_side ? P->synL : P->synR;
      for (int c = 0; c < colsB; ++c) dst[(size_t)i * colsB + c] = (double)dot(rowv, colv[c], G, left_side);
    }
  }
  // self-check: the one-level synthesis matrix at 2^k = 2 nu (smallest level)
  // built from these pieces must be orthogonal.
  {
    const int half = std::max(2 * nu, 1), size = 2 * half;
    std::vector<double> S((size_t)size * size, 0);  // S[row * size + col]
    for (int mcol = 0; mcol < half; ++mcol) {
      bool interior = mcol >= nu && mcol < half - nu;
      for (int kind = 0; kind < 2; ++kind) {
        int col = kind * half + mcol;
        if (interior) {
          const auto& taps = kind == 0 ? P->h : P->g;
          for (int c = -nu + 1; c <= nu; ++c) S[(size_t)(2 * mcol + c) * size + col] += taps[c + nu - 1];
        } else if (mcol < nu) {
          for (int i = 0; i < rowsB; ++i) S[(size_t)i * size + col] += P->synL[(size_t)i * colsB + kind * nu + mcol];
        } else {
          int mp = half - 1 - mcol;
          for (int i = 0; i < rowsB; ++i)
            S[(size_t)(size - rowsB + i) * size + col] += P->synR[(size_t)i * colsB + kind * nu + mp];
        }
      }
    }
    double worst = 0;
    for (int a = 0; a < size; ++a)
      for (int b = 0; b < size; ++b) {
        double s = 0;
        for (int r = 0; r < size; ++r) s += S[(size_t)r * size + a] * S[(size_t)r * size + b];
        worst = std::max(worst, std::fabs(s - (a == b ? 1.0 : 0.0)));
      }
    if (nu >= 2 && worst > 1e-12) {
      *err = "one-level synthesis matrix fails the orthogonality self-check";
      return WH2WAV_EINTERNAL;
    }
  }
  return WH2WAV_OK;
}

int build_host_plan(const wh2wav_desc* d, HostPlan* P, std::string* err) {
  if (!d) {
    *err = "descriptor is NULL";
    return WH2WAV_EINVAL;
  }
  if (d->dim < 1 || d->dim > 3) return *err = "dim must be 1, 2 or 3", WH2WAV_EINVAL;
  if (d->nu < 1 || d->nu > 10) return *err = "nu must be in [1, 10]", WH2WAV_EINVAL;
  if (d->q < 1) return *err = "q must be >= 1", WH2WAV_EINVAL;
  if (d->j0 < 0 || d->j < d->j0) return *err = "need 0 <= j0 <= j", WH2WAV_EINVAL;
  if (d->nu >= 2 && ((int64_t)1 << d->j0) < 2 * d->nu)
    return *err = "coarsest level too small: need 2^j0 >= 2 nu", WH2WAV_EINVAL;
  if (d->family != WH2WAV_DB && d->family != WH2WAV_SYM)
    return *err = "family must be WH2WAV_DB or WH2WAV_SYM", WH2WAV_EINVAL;
  if (d->boundary != WH2WAV_BD && d->boundary != WH2WAV_PER)
    return *err = "boundary must be WH2WAV_BD or WH2WAV_PER", WH2WAV_EINVAL;
  if (d->dtype != WH2WAV_F32 && d->dtype != WH2WAV_F64) return *err = "dtype must be F32 or F64", WH2WAV_EINVAL;
  if (d->basis2d != WH2WAV_ISOTROPIC && d->basis2d != WH2WAV_TENSOR)
    return *err = "basis2d must be WH2WAV_ISOTROPIC or WH2WAV_TENSOR", WH2WAV_EINVAL;
  // per-axis sizes: j_axes[a] for a < dim (0 takes j), zero beyond dim
  bool unequal = false;
  for (int a = 0; a < 3; ++a) {
    const int v = d->j_axes[a];
    if (a >= d->dim || d->dim == 1) {
      if (v != 0 && !(d->dim == 1 && a == 0 && v == d->j))
        return *err = "j_axes entries beyond dim (and all of them in 1D) must be 0", WH2WAV_EINVAL;
      continue;
    }
    if (v < 0) return *err = "j_axes entries must be >= 0", WH2WAV_EINVAL;
    const int ja = v ? v : d->j;
    if (ja < d->j0) return *err = "need j0 <= j_axes[a] on every axis", WH2WAV_EINVAL;
    P->ja[a] = ja;
    unequal = unequal || ja != d->j;
  }
  if (unequal && d->basis2d != WH2WAV_TENSOR)
    return *err = "unequal sides need the tensor basis (WH2WAV_TENSOR)", WH2WAV_EINVAL;
  const int J = d->j + d->q;
  if ((d->dim == 1 && J > 28) || (d->dim == 2 && J > 15))
    return *err = "size exceeds the supported range", WH2WAV_EUNSUPPORTED;
  int64_t total = 1;
  if (d->dim >= 2) {
    int jsum = 0;
    for (int a = 0; a < d->dim; ++a) {
      if (P->ja[a] + d->q > 15) return *err = "size exceeds the supported range", WH2WAV_EUNSUPPORTED;
      jsum += P->ja[a] + d->q;
    }
    if (jsum > 32) return *err = "size exceeds the supported range (N_1 ... N_dim > 2^32)", WH2WAV_EUNSUPPORTED;
  }
  P->dim = d->dim, P->j = d->j, P->q = d->q, P->j0 = d->j0, P->nu = d->nu, P->dtype = d->dtype;
  P->M = (int64_t)1 << d->j;
  P->N = (int64_t)1 << J;
  P->family = d->family;
  P->per = d->boundary == WH2WAV_PER;
  P->tensor = d->dim >= 2 && d->basis2d == WH2WAV_TENSOR;
  P->nd = d->dim == 3 || unequal;
  int rc = build_tables(d->family, d->nu, d->q, d->j, P, err);
  if (rc != WH2WAV_OK) return rc;
  if (P->nd) {
    for (int a = 0; a < d->dim; ++a) {
      P->Ma[a] = (int64_t)1 << P->ja[a];
      P->Na[a] = (int64_t)1 << (P->ja[a] + d->q);
      if (P->ja[a] == d->j) {
        P->tabT_ax[a] = P->tabT, P->tabBL_ax[a] = P->tabBL, P->tabBR_ax[a] = P->tabBR;
      } else {
        HostPlan axis;
        rc = build_tables(d->family, d->nu, d->q, P->ja[a], &axis, err);
        if (rc != WH2WAV_OK) return rc;
        P->tabT_ax[a] = std::move(axis.tabT);
        P->tabBL_ax[a] = std::move(axis.tabBL);
        P->tabBR_ax[a] = std::move(axis.tabBR);
      }
      if (P->per) {
        std::fill(P->tabBL_ax[a].begin(), P->tabBL_ax[a].end(), 0.0);
        std::fill(P->tabBR_ax[a].begin(), P->tabBR_ax[a].end(), 0.0);
      }
    }
  }
  if (P->per) {
    // periodic extension: every function is an interior one, periodised
    std::fill(P->tabBL.begin(), P->tabBL.end(), 0.0);
    std::fill(P->tabBR.begin(), P->tabBR.end(), 0.0);
    std::fill(P->synL.begin(), P->synL.end(), 0.0);
    std::fill(P->synR.begin(), P->synR.end(), 0.0);
  }

  if (P->nd) {
    for (int a = 0; a < d->dim; ++a) total *= P->Na[a];
    P->row_len = P->Na[d->dim - 1];
  } else {
    total = d->dim == 1 ? P->N : P->N * P->N;
    P->row_len = P->N;
  }
  if (d->m < 0 || d->m > total) return *err = "m out of range", WH2WAV_EINVAL;
  P->m = d->m;
  P->rows = d->dim == 1 ? 1 : total / P->row_len;
  P->words_per_row = (P->row_len + 31) / 32;
  if (!d->omega) {
    if (d->m != total) return *err = "omega is NULL but m != N_1 ... N_dim", WH2WAV_EINVAL;
    P->full_omega = true;
  } else {
    bool full = d->m == total;
    for (int64_t i = 0; i < d->m; ++i) {
      int64_t v = d->omega[i];
      if (v < 0 || v >= total) return *err = "omega index out of range", WH2WAV_EINVAL;
      if (i > 0 && v <= d->omega[i - 1]) return *err = "omega must be strictly increasing", WH2WAV_EINVAL;
      full = full && v == i;
    }
    P->full_omega = full;
  }
  P->mask.clear();
  P->row_ptr.assign(P->rows + 1, 0);
  if (!P->full_omega) {
    P->mask.assign((size_t)(P->rows * P->words_per_row), 0u);
    for (int64_t i = 0; i < d->m; ++i) {
      int64_t v = d->omega[i];
      int64_t r = d->dim == 1 ? 0 : v / P->row_len, c = d->dim == 1 ? v : v % P->row_len;
      P->mask[(size_t)(r * P->words_per_row + c / 32)] |= 1u << (c % 32);
      P->row_ptr[r + 1]++;
    }
  } else {
    for (int64_t r = 0; r < P->rows; ++r) P->row_ptr[r + 1] = P->row_len;
  }
  for (int64_t r = 0; r < P->rows; ++r) P->row_ptr[r + 1] += P->row_ptr[r];
  P->pos16.clear();
  P->seg_ptr.clear();
  // 2D, and 1D lines of at most 2048 values (one wave per phase line): the
  // sample list per (row, phase); 1D has the single row n1 = 0
  if (!P->nd && (d->dim == 2 || d->j <= 11) && !P->full_omega && P->M <= 65536) {
    const int64_t Q = P->Q, M = P->M, nrows = d->dim == 2 ? P->N : 1;
    P->seg_ptr.assign((size_t)(nrows * Q + 1), 0);
    P->pos16.resize((size_t)d->m);
    for (int64_t i = 0; i < d->m; ++i) {
      const int64_t v = d->omega[i];
      const int64_t n1 = d->dim == 2 ? v / P->N : 0, n2 = d->dim == 2 ? v % P->N : v;
      const int64_t s = n2 / M, b = n2 % M;
      P->seg_ptr[(size_t)(n1 * Q + s + 1)]++;
      const uint64_t g = (uint64_t)(b ^ (b >> 1));
      uint64_t k = 0;
      for (int bit = 0; bit < d->j; ++bit) k |= ((g >> bit) & 1u) << (d->j - 1 - bit);
      P->pos16[(size_t)i] = (uint16_t)(k ^ (uint64_t)(s & 1));
    }
    for (size_t e = 1; e < P->seg_ptr.size(); ++e) P->seg_ptr[e] += P->seg_ptr[e - 1];
  }
  P->pos32.clear();
  if (d->dim == 1 && !P->full_omega && P->N <= ((int64_t)1 << 30)) {
    const int64_t M = P->M;
    P->pos32.resize((size_t)d->m);
    for (int64_t i = 0; i < d->m; ++i) {
      const int64_t v = d->omega[i], s = v / M, b = v % M;
      const uint64_t g = (uint64_t)(b ^ (b >> 1));
      uint64_t k = 0;
      for (int bit = 0; bit < d->j; ++bit) k |= ((g >> bit) & 1u) << (d->j - 1 - bit);
      P->pos32[(size_t)i] = (int32_t)(s * M + (int64_t)(k ^ (uint64_t)(s & 1)));
    }
  }
  return WH2WAV_OK;
}

}  // namespace wh2wav
