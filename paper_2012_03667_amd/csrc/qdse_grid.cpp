// qdse_grid.cpp -- host-side discretisation for the gfx950 gap-equation
// solver: Gauss-Legendre rules, the interleaved external/loop radial grids and
// the interpolation stencils with brackets known in advance.
//
// Radial variable u = ln p^2 on [ln s_min, ln s_max]. External nodes are the
// N-point Gauss-Legendre nodes in u, loop nodes the (N+1)-point ones on the
// same interval. Zeros of consecutive Legendre polynomials interlace strictly,
// so t_0 < s_0 < t_1 < ... < s_{N-1} < t_N: every loop momentum differs from
// every external one and the bracket of t_j is (s_{j-1}, s_j) without any
// search. This is the ordering of Sec. III A, eq. pqrelationship, which the
// paper's modified interpolation (eq. chazhiresult) relies on.
#include "qdse_internal.h"

#include <algorithm>
#include <cmath>

// The grid is defined by correctly rounded values: with x, w the correctly
// rounded Gauss-Legendre rule and a = ln s_min, b = ln s_max (exact),
//   u = RN(a + (b - a)(x + 1)/2),  s = RN(exp(u)),  W = RN((b - a)/2 w t^2),
// each evaluated in double-double arithmetic and rounded once (the same for
// the finite-mu grids). No fused multiply-add contraction in the helpers.
#pragma clang fp contract(off)

namespace qdse {

// Double-double arithmetic (value = hi + lo, |lo| <= ulp(hi)/2), used to
// polish the Gauss-Legendre rule to correct FP64 rounding.
struct dd {
  double hi, lo;
};
static inline dd two_sum(double a, double b) {
  const double s = a + b, bb = s - a;
  return {s, (a - (s - bb)) + (b - bb)};
}
static inline dd quick_two_sum(double a, double b) {
  const double s = a + b;
  return {s, b - (s - a)};
}
static inline dd dd_add(dd a, dd b) {
  dd s = two_sum(a.hi, b.hi);
  dd t = two_sum(a.lo, b.lo);
  s.lo += t.hi;
  s = quick_two_sum(s.hi, s.lo);
  s.lo += t.lo;
  return quick_two_sum(s.hi, s.lo);
}
static inline dd dd_neg(dd a) { return {-a.hi, -a.lo}; }
static inline dd dd_mul(dd a, dd b) {
  const double p = a.hi * b.hi;
  const double e = std::fma(a.hi, b.hi, -p) + (a.hi * b.lo + a.lo * b.hi);
  return quick_two_sum(p, e);
}
static inline dd dd_mul_d(dd a, double b) { return dd_mul(a, dd{b, 0.0}); }
static inline dd dd_div(dd a, dd b) {
  const double q1 = a.hi / b.hi;
  dd r = dd_add(a, dd_neg(dd_mul_d(b, q1)));
  const double q2 = r.hi / b.hi;
  r = dd_add(r, dd_neg(dd_mul_d(b, q2)));
  const double q3 = r.hi / b.hi;
  return dd_add(quick_two_sum(q1, q2), dd{q3, 0.0});
}
static inline dd dd_from(double a) { return dd{a, 0.0}; }
static inline dd dd_sub(dd a, dd b) { return dd_add(a, dd_neg(b)); }
static inline double dd_round(dd a) { return a.hi + a.lo; }
static inline dd dd_ldexp(dd a, int e) { return dd{std::ldexp(a.hi, e), std::ldexp(a.lo, e)}; }

static const dd kDdLn2{0.6931471805599453094, 2.319046813846299558e-17};
static const dd kDdPi{3.141592653589793116, 1.224646799147353207e-16};

// exp in double-double: x = k ln 2 + r, exp(r / 2^10) by its Taylor series
// (|r / 2^10| < 3.4e-4, 12 terms), squared ten times, scaled by 2^k.
static dd dd_exp(dd x) {
  const double kf = std::nearbyint(x.hi / kDdLn2.hi);
  const dd r = dd_ldexp(dd_sub(x, dd_mul_d(kDdLn2, kf)), -10);
  dd term = dd_from(1.0), sum = dd_from(1.0);
  for (int i = 1; i <= 12; ++i) {
    term = dd_div(dd_mul(term, r), dd_from((double)i));
    sum = dd_add(sum, term);
  }
  for (int i = 0; i < 10; ++i) sum = dd_mul(sum, sum);
  return dd_ldexp(sum, (int)kf);
}

// ln x (x > 0) in double-double: Newton steps y += x exp(-y) - 1 from the
// FP64 logarithm (each step squares the relative error).
static dd dd_log(dd x) {
  dd y = dd_from(std::log(x.hi));
  for (int it = 0; it < 2; ++it)
    y = dd_add(y, dd_sub(dd_mul(x, dd_exp(dd_neg(y))), dd_from(1.0)));
  return y;
}

static dd dd_sqrt(dd a) {
  const double y = std::sqrt(a.hi);
  const dd y2 = dd_mul(dd_from(y), dd_from(y));
  return dd_add(dd_from(y), dd_div(dd_sub(a, y2), dd_from(2.0 * y)));
}

static dd dd_sinh(dd v) { return dd_ldexp(dd_sub(dd_exp(v), dd_exp(dd_neg(v))), -1); }
static dd dd_cosh(dd v) { return dd_ldexp(dd_add(dd_exp(v), dd_exp(dd_neg(v))), -1); }
static dd dd_asinh(dd x) { return dd_log(dd_add(x, dd_sqrt(dd_add(dd_mul(x, x), dd_from(1.0))))); }

// RN(a + h (x + 1)) for a Gauss-Legendre node x of [-1, 1] mapped to an
// interval of left end a and half length h (both double-double).
static inline double map_node(dd a, dd h, double x) {
  return dd_round(dd_add(a, dd_mul(h, two_sum(x, 1.0))));
}

static inline dd two_prod(double a, double b) {
  const double p = a * b;
  return {p, std::fma(a, b, -p)};
}

// The node u = RN(ln lo + (ln hi - ln lo)(x + 1)/2) of the grid in ln p on
// [lo, hi]. The middle node of an odd rule (x = 0) is (ln lo + ln hi)/2 =
// ln(lo hi)/2, which can be far smaller than ln lo (a range symmetric about
// 1 up to the rounding of lo): it is taken from ln(1 + d), d = lo hi - 1
// exact, by its series when |d| is small, so that it too is correctly
// rounded.
static double log_node(double lo, double hi, dd a, dd h, double x) {
  if (x != 0.0) return map_node(a, h, x);
  const dd d = dd_sub(two_prod(lo, hi), dd_from(1.0));
  if (std::fabs(d.hi) > 1e-3) return map_node(a, h, x);
  dd sum = dd_from(0.0), pw = d;
  for (int k = 1; k <= 16; ++k) {  // ln(1 + d) = sum (-1)^(k+1) d^k / k
    const dd term = dd_div(pw, dd_from((double)k));
    sum = (k & 1) ? dd_add(sum, term) : dd_sub(sum, term);
    pw = dd_mul(pw, d);
  }
  return dd_round(dd_ldexp(sum, -1));
}

// P_n(r) and P_n'(r) by the three-term recurrence in double-double.
static void legendre_dd(int n, dd r, dd* p, dd* dp) {
  dd p0{1.0, 0.0}, p1 = r;
  for (int l = 2; l <= n; ++l) {
    const dd a = dd_mul_d(dd_mul(r, p1), 2.0 * l - 1.0);
    const dd b = dd_mul_d(p0, l - 1.0);
    const dd p2 = dd_div(dd_add(a, dd_neg(b)), dd{(double)l, 0.0});
    p0 = p1;
    p1 = p2;
  }
  *p = p1;
  // P_n' = n (r P_n - P_{n-1}) / (r^2 - 1)
  const dd num = dd_mul_d(dd_add(dd_mul(r, p1), dd_neg(p0)), (double)n);
  *dp = dd_div(num, dd_add(dd_mul(r, r), dd{-1.0, 0.0}));
}

// Nodes x[k] (ascending) and weights w[k] of the n-point Gauss-Legendre rule
// on [-1, 1], correctly rounded to FP64: Newton's method on P_n in FP64 from
// the asymptotic (Tricomi) estimate of each zero, then two Newton steps and
// the weight 2 / ((1 - x^2) P_n'(x)^2) in double-double arithmetic. Correct
// rounding matters: at large p^2 the quadrature sums react to single-ulp moves
// of the angular nodes through exp(-k^2/omega^2), k^2 ~ 2|p||q|(1 - z).
void gauss_legendre(int n, double* x, double* w) {
  const double pi = 3.14159265358979323846;
  if (n == 1) {
    x[0] = 0.0;
    w[0] = 2.0;
    return;
  }
  for (int k = 0; k < (n + 1) / 2; ++k) {
    const double th = pi * (k + 0.75) / (n + 0.5);
    double r = std::cos(th) * (1.0 - (n - 1.0) / (8.0 * n * n * n));
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = r;
      for (int l = 2; l <= n; ++l) {
        const double p2 = ((2.0 * l - 1.0) * r * p1 - (l - 1.0) * p0) / l;
        p0 = p1;
        p1 = p2;
      }
      const double dr = p1 / (n * (r * p1 - p0) / (r * r - 1.0));
      r -= dr;
      if (std::fabs(dr) < 1e-15) break;
    }
    dd rr{r, 0.0}, p, dp;
    for (int it = 0; it < 2; ++it) {
      legendre_dd(n, rr, &p, &dp);
      rr = dd_add(rr, dd_neg(dd_div(p, dp)));
    }
    legendre_dd(n, rr, &p, &dp);
    const dd one_m_r2 = dd_add(dd{1.0, 0.0}, dd_neg(dd_mul(rr, rr)));
    const dd wk = dd_div(dd{2.0, 0.0}, dd_mul(one_m_r2, dd_mul(dp, dp)));
    const double root = rr.hi + rr.lo;  // round to FP64
    const double wt = wk.hi + wk.lo;
    x[n - 1 - k] = root;  // largest roots first in k
    x[k] = -root;
    w[k] = w[n - 1 - k] = wt;
  }
  if (n % 2 == 1) x[n / 2] = 0.0;
}

void gl_mapped(int n, double a, double b, double* x, double* w) {
  gauss_legendre(n, x, w);
  const dd da = dd_from(a), half = dd_ldexp(two_sum(b, -a), -1);
  for (int i = 0; i < n; ++i) {
    // the middle node of an odd rule is (a + b)/2, exact in double-double
    x[i] = x[i] == 0.0 ? dd_round(dd_ldexp(two_sum(a, b), -1)) : map_node(da, half, x[i]);
    w[i] = dd_round(dd_mul_d(half, w[i]));
  }
}

// 4-point stencil (base index, weights) of Lagrange interpolation in u for
// every loop node, using the bracket (s_{j-1}, s_j) known from the
// interleaving. order 3: nodes j-2..j+1 shifted to stay inside the grid.
// order 1: nodes j-1, j (eq. chazhiresult), the end value beyond either end.
void build_stencils(int n, int order, const double* u, const double* uq, int* lo, double* sw) {
  const int nq = n + 1;
  for (int j = 0; j < nq; ++j) {
    double* w = sw + 4 * j;
    w[0] = w[1] = w[2] = w[3] = 0.0;
    int base = j - 2;
    if (base < 0) base = 0;
    if (base > n - 4) base = n - 4;
    lo[j] = base;
    if (order == 1) {
      if (j == 0) {
        w[0 - base] = 1.0;
      } else if (j == n) {
        w[n - 1 - base] = 1.0;
      } else {
        const int a = j - 1, b = j;
        const double h = u[b] - u[a];
        w[a - base] = (u[b] - uq[j]) / h;
        w[b - base] = (uq[j] - u[a]) / h;
      }
    } else {
      for (int l = 0; l < 4; ++l) {
        double c = 1.0;
        for (int k = 0; k < 4; ++k)
          if (k != l) c *= (uq[j] - u[base + k]) / (u[base + l] - u[base + k]);
        w[l] = c;
      }
    }
  }
}

int build_grid(const qdse_grid& g, HostGrid* hg) {
  const int n = g.n_radial, nq = n + 1, na = g.n_angle;
  hg->n = n;
  hg->nq = nq;
  hg->na = na;
  hg->ldk = (nq + 7) & ~7;
  const dd a = dd_log(dd_from(g.s_min)), b = dd_log(dd_from(g.s_max));
  const dd half = dd_ldexp(dd_sub(b, a), -1);

  std::vector<double> x(nq), w(nq);
  hg->u.resize(n);
  hg->s.resize(n);
  gauss_legendre(n, x.data(), w.data());
  for (int i = 0; i < n; ++i) {
    hg->u[i] = log_node(g.s_min, g.s_max, a, half, x[i]);
    hg->s[i] = dd_round(dd_exp(dd_from(hg->u[i])));
  }
  hg->uq.resize(nq);
  hg->t.resize(nq);
  hg->W.resize(nq);
  gauss_legendre(nq, x.data(), w.data());
  for (int j = 0; j < nq; ++j) {
    hg->uq[j] = log_node(g.s_min, g.s_max, a, half, x[j]);
    hg->t[j] = dd_round(dd_exp(dd_from(hg->uq[j])));
    const dd t = dd_from(hg->t[j]);
    hg->W[j] = dd_round(dd_mul(dd_mul_d(half, w[j]), dd_mul(t, t)));  // t dt = t^2 du
  }
  std::vector<double> za(na), wa(na);
  gauss_legendre(na, za.data(), wa.data());
  hg->z = za;
  hg->wz.resize(na);
  for (int k = 0; k < na; ++k) hg->wz[k] = wa[k] * std::sqrt((1.0 - za[k]) * (1.0 + za[k]));

  for (int i = 0; i < n; ++i) {  // interleaving must hold strictly
    if (!(hg->t[i] < hg->s[i] && hg->s[i] < hg->t[i + 1])) return -1;
  }
  hg->lo.resize(nq);
  hg->sw.resize(4 * nq);
  build_stencils(n, g.interp_order, hg->u.data(), hg->uq.data(), hg->lo.data(), hg->sw.data());
  return 0;
}

int build_mu_grid(const qdse_mu_grid& g, HostMuGrid* h) {
  const int ns = g.n_space, n4 = g.n_time, na = g.n_angle;
  h->ns = ns;
  h->n4 = n4;
  h->nqs = ns + 1;
  h->nq4 = n4 + 1;
  h->na = na;
  const dd a = dd_log(dd_from(g.r_min)), b = dd_log(dd_from(g.r_max));
  const dd half = dd_ldexp(dd_sub(b, a), -1);
  std::vector<double> x(ns + 2), w(ns + 2);
  // |p_vec|: Gauss-Legendre in ln|p|; loop |q|: one more node, weight |q|^3 dln|q|
  h->us.resize(ns);
  h->ps.resize(ns);
  gauss_legendre(ns, x.data(), w.data());
  for (int i = 0; i < ns; ++i) {
    h->us[i] = log_node(g.r_min, g.r_max, a, half, x[i]);
    h->ps[i] = dd_round(dd_exp(dd_from(h->us[i])));
  }
  h->uqs.resize(ns + 1);
  h->qs.resize(ns + 1);
  h->wqs.resize(ns + 1);
  gauss_legendre(ns + 1, x.data(), w.data());
  for (int j = 0; j <= ns; ++j) {
    h->uqs[j] = log_node(g.r_min, g.r_max, a, half, x[j]);
    h->qs[j] = dd_round(dd_exp(dd_from(h->uqs[j])));
    const dd q = dd_from(h->qs[j]);
    h->wqs[j] = dd_round(dd_mul(dd_mul_d(half, w[j]), dd_mul(q, dd_mul(q, q))));
  }
  if (g.T > 0.0) {
    // Matsubara frequencies w_n = (2n+1) pi T; the loop runs over the same
    // frequencies (both signs in the sweep), weight 2 pi T each; the time
    // stencil is the identity (lo at n, clamped so that lo + 3 < n4)
    h->nq4 = n4;
    const dd piT = dd_mul_d(kDdPi, g.T);
    h->v4.resize(n4);
    h->p4.resize(n4);
    h->vq4.resize(n4);
    h->q4.resize(n4);
    h->wq4.resize(n4);
    for (int i = 0; i < n4; ++i) {
      h->p4[i] = dd_round(dd_mul_d(piT, 2.0 * i + 1.0));
      h->v4[i] = h->p4[i];
      h->q4[i] = h->p4[i];
      h->vq4[i] = h->p4[i];
      h->wq4[i] = dd_round(dd_mul_d(piT, 2.0));
    }
    h->lo_4.resize(n4);
    h->sw_4.assign(4 * (size_t)n4, 0.0);
    for (int i = 0; i < n4; ++i) {
      const int lo = i < n4 - 4 ? i : n4 - 4;
      h->lo_4[i] = lo;
      h->sw_4[4 * (size_t)i + (i - lo)] = 1.0;
    }
  } else {
  // p4 = lam4 sinh(v), v Gauss-Legendre on [0, asinh(p4_max/lam4)]; dq4 = lam4 cosh(v) dv
  const dd hv = dd_ldexp(dd_asinh(dd_div(dd_from(g.p4_max), dd_from(g.lam4))), -1);
  std::vector<double> y(n4 + 2), wy(n4 + 2);
  h->v4.resize(n4);
  h->p4.resize(n4);
  gauss_legendre(n4, y.data(), wy.data());
  for (int i = 0; i < n4; ++i) {
    h->v4[i] = map_node(dd_from(0.0), hv, y[i]);
    h->p4[i] = dd_round(dd_mul_d(dd_sinh(dd_from(h->v4[i])), g.lam4));
  }
  h->vq4.resize(n4 + 1);
  h->q4.resize(n4 + 1);
  h->wq4.resize(n4 + 1);
  gauss_legendre(n4 + 1, y.data(), wy.data());
  for (int j = 0; j <= n4; ++j) {
    h->vq4[j] = map_node(dd_from(0.0), hv, y[j]);
    h->q4[j] = dd_round(dd_mul_d(dd_sinh(dd_from(h->vq4[j])), g.lam4));
    h->wq4[j] = dd_round(dd_mul(dd_mul_d(dd_mul_d(hv, wy[j]), g.lam4), dd_cosh(dd_from(h->vq4[j]))));
  }
  for (int i = 0; i < n4; ++i)
    if (!(h->q4[i] < h->p4[i] && h->p4[i] < h->q4[i + 1])) return -1;
  h->lo_4.resize(n4 + 1);
  h->sw_4.resize(4 * (n4 + 1));
  build_stencils(n4, g.interp_order, h->v4.data(), h->vq4.data(), h->lo_4.data(), h->sw_4.data());
  }
  h->z.resize(na);
  h->wz.resize(na);
  gauss_legendre(na, h->z.data(), h->wz.data());
  for (int i = 0; i < ns; ++i)
    if (!(h->qs[i] < h->ps[i] && h->ps[i] < h->qs[i + 1])) return -1;
  h->lo_s.resize(ns + 1);
  h->sw_s.resize(4 * (ns + 1));
  build_stencils(ns, g.interp_order, h->us.data(), h->uqs.data(), h->lo_s.data(), h->sw_s.data());
  return 0;
}

// Interpolation stencil at an arbitrary p^2 = s inside the grid, with the
// rule of the loop-node stencils: bracket u_b < ln s <= u_{b+1} by search;
// order 1: the two bracketing nodes (the end value beyond the grid), order 3:
// the four nodes b-1..b+2 shifted to stay inside the grid, Lagrange in u.
QcPoint qc_point(const HostGrid& g, int order, double s) {
  const int n = g.n;
  const double x = std::log(s);
  int b = -1;
  for (int i = 0; i < n; ++i)
    if (g.u[i] < x) b = i;
  QcPoint p{};
  p.s = s;
  if (order == 1) {
    if (b < 0) {
      p.base = 0;
      p.w[0] = 1.0;
    } else if (b >= n - 1) {
      p.base = n - 4;
      p.w[3] = 1.0;
    } else {
      p.base = std::min(b, n - 4);
      const double h = g.u[b + 1] - g.u[b];
      p.w[b - p.base] = (g.u[b + 1] - x) / h;
      p.w[b + 1 - p.base] = (x - g.u[b]) / h;
    }
    return p;
  }
  p.base = std::min(std::max(b - 1, 0), n - 4);
  for (int l = 0; l < 4; ++l) {
    double c = 1.0;
    for (int k = 0; k < 4; ++k)
      if (k != l) c *= (x - g.u[p.base + k]) / (g.u[p.base + l] - g.u[p.base + k]);
    p.w[l] = c;
  }
  return p;
}

}  // namespace qdse
