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

// The grid must round exactly as written (no fused multiply-add contraction):
// u = a + half (x + 1), W = half w t^2.
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
  const double a = std::log(g.s_min), b = std::log(g.s_max);
  const double half = 0.5 * (b - a);

  std::vector<double> x(nq), w(nq);
  hg->u.resize(n);
  hg->s.resize(n);
  gauss_legendre(n, x.data(), w.data());
  for (int i = 0; i < n; ++i) {
    hg->u[i] = a + half * (x[i] + 1.0);
    hg->s[i] = std::exp(hg->u[i]);
  }
  hg->uq.resize(nq);
  hg->t.resize(nq);
  hg->W.resize(nq);
  gauss_legendre(nq, x.data(), w.data());
  for (int j = 0; j < nq; ++j) {
    hg->uq[j] = a + half * (x[j] + 1.0);
    hg->t[j] = std::exp(hg->uq[j]);
    hg->W[j] = half * w[j] * hg->t[j] * hg->t[j];  // t dt = t^2 du
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
  const double a = std::log(g.r_min), b = std::log(g.r_max);
  const double half = 0.5 * (b - a);
  const double vmax = std::asinh(g.p4_max / g.lam4);
  const double hv = 0.5 * (vmax - 0.0);
  std::vector<double> x(ns + 2), w(ns + 2);
  // |p_vec|: Gauss-Legendre in ln|p|; loop |q|: one more node, weight |q|^3 dln|q|
  h->us.resize(ns);
  h->ps.resize(ns);
  gauss_legendre(ns, x.data(), w.data());
  for (int i = 0; i < ns; ++i) {
    h->us[i] = a + half * (x[i] + 1.0);
    h->ps[i] = std::exp(h->us[i]);
  }
  h->uqs.resize(ns + 1);
  h->qs.resize(ns + 1);
  h->wqs.resize(ns + 1);
  gauss_legendre(ns + 1, x.data(), w.data());
  for (int j = 0; j <= ns; ++j) {
    h->uqs[j] = a + half * (x[j] + 1.0);
    h->qs[j] = std::exp(h->uqs[j]);
    h->wqs[j] = half * w[j] * h->qs[j] * h->qs[j] * h->qs[j];
  }
  if (g.T > 0.0) {
    // Matsubara frequencies w_n = (2n+1) pi T; the loop runs over the same
    // frequencies (both signs in the sweep), weight 2 pi T each; the time
    // stencil is the identity (lo at n, clamped so that lo + 3 < n4)
    h->nq4 = n4;
    const double pi = 3.14159265358979323846;
    h->v4.resize(n4);
    h->p4.resize(n4);
    h->vq4.resize(n4);
    h->q4.resize(n4);
    h->wq4.resize(n4);
    for (int i = 0; i < n4; ++i) {
      h->p4[i] = (2.0 * i + 1.0) * pi * g.T;
      h->v4[i] = h->p4[i];
      h->q4[i] = h->p4[i];
      h->vq4[i] = h->p4[i];
      h->wq4[i] = 2.0 * pi * g.T;
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
  std::vector<double> y(n4 + 2), wy(n4 + 2);
  h->v4.resize(n4);
  h->p4.resize(n4);
  gauss_legendre(n4, y.data(), wy.data());
  for (int i = 0; i < n4; ++i) {
    h->v4[i] = 0.0 + hv * (y[i] + 1.0);
    h->p4[i] = g.lam4 * std::sinh(h->v4[i]);
  }
  h->vq4.resize(n4 + 1);
  h->q4.resize(n4 + 1);
  h->wq4.resize(n4 + 1);
  gauss_legendre(n4 + 1, y.data(), wy.data());
  for (int j = 0; j <= n4; ++j) {
    h->vq4[j] = 0.0 + hv * (y[j] + 1.0);
    h->q4[j] = g.lam4 * std::sinh(h->vq4[j]);
    h->wq4[j] = hv * wy[j] * (g.lam4 * std::cosh(h->vq4[j]));
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
