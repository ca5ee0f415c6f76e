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

#include <cmath>

namespace qdse {

// Nodes x[k] (ascending) and weights w[k] of the n-point Gauss-Legendre rule
// on [-1, 1]: Newton's method on P_n, evaluated by the three-term recurrence,
// started from the asymptotic (Tricomi) estimate of the k-th zero.
void gauss_legendre(int n, double* x, double* w) {
  const double pi = 3.14159265358979323846;
  for (int k = 0; k < (n + 1) / 2; ++k) {
    const double th = pi * (k + 0.75) / (n + 0.5);
    double r = std::cos(th) * (1.0 - (n - 1.0) / (8.0 * n * n * n));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = r;
      for (int l = 2; l <= n; ++l) {
        const double p2 = ((2.0 * l - 1.0) * r * p1 - (l - 1.0) * p0) / l;
        p0 = p1;
        p1 = p2;
      }
      if (n == 1) {
        p1 = r;
        p0 = 1.0;
      }
      dp = n * (r * p1 - p0) / (r * r - 1.0);  // P_n'(r)
      const double dr = p1 / dp;
      r -= dr;
      if (std::fabs(dr) < 1e-16) {
        // one more recurrence for the derivative at the converged root
        double q0 = 1.0, q1 = r;
        for (int l = 2; l <= n; ++l) {
          const double q2 = ((2.0 * l - 1.0) * r * q1 - (l - 1.0) * q0) / l;
          q0 = q1;
          q1 = q2;
        }
        dp = (n == 1) ? 1.0 : n * (r * q1 - q0) / (r * r - 1.0);
        break;
      }
    }
    const double wk = 2.0 / ((1.0 - r * r) * dp * dp);
    x[n - 1 - k] = r;   // largest roots first in k
    x[k] = -r;
    w[k] = w[n - 1 - k] = wk;
  }
  if (n % 2 == 1) x[n / 2] = 0.0;
}

// 4-point stencil (base index, weights) of Lagrange interpolation in u for
// every loop node, using the bracket (s_{j-1}, s_j) known from the
// interleaving. order 3: nodes j-2..j+1 shifted to stay inside the grid.
// order 1: nodes j-1, j (eq. chazhiresult), the end value beyond either end.
static void build_stencils(int n, int order, const double* u, const double* uq,
                           int* lo, double* sw) {
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

}  // namespace qdse
