// qdse_oracle.cpp -- plain FP64 CPU oracle for the vacuum quark gap equation
// with the Ball-Chiu vertex (Huang, Duan, Hu, Chen, arXiv:2012.03667).
//
// TEST INFRASTRUCTURE ONLY. Nothing in the product path links, loads or calls
// this file; only the tests, the smoke check and the CPU-baseline leg of the
// benchmark do. It shares no code, header, table or constant with the HIP
// library.
//
// What it computes (Sec. II, eqs. gendse, KernelAnsatz, bcvtxmu, eq. (2),
// IRGsQC, dsesys, dsesys2): one sweep of the successive-approximation map
// (Sec. I, eq. jifen12)
//     A'(p^2) = 1 + C_F/(8 pi^3) sum_q sum_angle  W g(k^2) I_A / Delta_q
//     B'(p^2) = m + C_F/(8 pi^3) sum_q sum_angle  W g(k^2) I_B / Delta_q
// evaluated for every external momentum by a direct double sum over the loop
// radial nodes and the angular nodes, one projection at a time (Sec. III), with
// an OpenMP parallel-for over external momenta for the parallel programs that
// Table 1 times. No angular kernel is precomputed.
//
// Readings of the paper taken here (each is also listed in the design notes):
//  * g(k^2) = G(k^2)/k^2 = (8 pi^2/omega^4) D exp(-k^2/omega^2): the Gaussian
//    of eq. IRGsQC multiplies the transverse projector directly; the literal
//    extra 1/k^2 is dimensionally inconsistent.
//  * The colour factor C_F = 4/3 of the lambda^a/2 pair in eq. gendse is kept.
//  * The denominator of eq. dsesys is the loop one, Delta_q = q^2 A(q^2)^2 +
//    B(q^2)^2 (it comes from S(q)); there is one overall 1/p^2 in the A
//    equation, the one written inside I_A1..I_A3.
//  * lambda_1 = (A(p^2)+A(q^2))/2 (eq. (2) misses a parenthesis); z_1 = 1.
//  * Measure: d^4q/(2pi)^4 = (1/(8 pi^3)) int dt t int_{-1}^{1} dz sqrt(1-z^2)
//    with t = q^2, z = cos(theta); the radial variable is u = ln t, so the
//    radial weight is w_u t^2.
//  * Off-grid A(q^2), B(q^2) come from Lagrange interpolation in u = ln p^2,
//    either 2-point (eq. chazhiresult, flat beyond the grid ends) or 4-point.
//    The bracket is found by searching the external grid, the "finding step"
//    of Sec. III A.
//  * A homotopy parameter lam scales the Ball-Chiu-specific parts of the
//    vertex (the two difference quotients and sigma_A - 1); lam = 1 is the
//    Ball-Chiu vertex of eq. bcvtxmu, lam = 0 the bare (rainbow) vertex.
//
// Beyond the paper (its Sec. II drops the ultraviolet part of the Qin-Chang
// interaction and sets the renormalisation constants to 1), an optional mode
// keeps both:
//  * g(k^2) gains g_UV(k^2) = 8 pi^2 gamma_m F(k^2) / ln[tau + (1 + k^2/L^2)^2],
//    F(k^2) = (1 - exp(-k^2/(4 m_t^2)))/k^2, gamma_m = 12/(33 - 2 N_f) with
//    N_f = 4, L = 0.234 GeV, tau = e^2 - 1, m_t = 0.5 GeV (the Qin-Chang form:
//    4 pi times the one-loop running coupling at large k^2);
//  * S^-1 = Z_2 (i gamma.p + Z_m m) + Z_1 Sigma with Z_1 = Z_2 (the
//    Ward-Takahashi identity the Ball-Chiu vertex satisfies), so
//    A = Z_2 (1 + Sigma_A), B = Z_4 m + Z_2 Sigma_B, Z_4 = Z_2 Z_m, with the
//    conditions A(zeta^2) = 1 and B(zeta^2) = m fixing Z_2 and Z_4 every sweep
//    from the sums at p^2 = zeta^2 (A, B interpolated there); at m = 0 the mass
//    term is absent. The top of the radial grid is the regulator.
//
// Scalar type: every routine is a template, instantiated for double and for
// std::complex<double>; the complex form gives Jacobian-vector products by the
// complex-step method (exact to rounding).

#include <cmath>
#include <complex>
#include <vector>
#include <omp.h>

typedef std::complex<double> cplx;

extern "C" {

// Vacuum discretisation. All arrays are host arrays owned by the caller.
struct qo_vac_grid {
  int n;            // external radial nodes p^2 = s[i]
  int nq;           // loop radial nodes q^2 = t[j]
  int na;           // angular nodes z = cos(theta)
  int order;        // interpolation order: 1 = 2-point, 3 = 4-point Lagrange
  const double* s;  // [n]  external p^2, ascending
  const double* u;  // [n]  ln s
  const double* t;  // [nq] loop q^2, ascending
  const double* uq; // [nq] ln t
  const double* W;  // [nq] radial weights: Gauss-Legendre weight in u = ln t
                    //      times t^2 (t dt = t^2 du), correctly rounded
  const double* z;  // [na] angular nodes on [-1, 1]
  const double* wz; // [na] angular weights (without sqrt(1-z^2))
};

struct qo_vac_par {
  double D;      // interaction strength, GeV^2
  double omega;  // interaction range, GeV
  double m;      // current-quark mass, GeV (renormalised at zeta when zeta > 0)
  double lam;    // vertex homotopy: 1 = Ball-Chiu, 0 = bare vertex
  int uv;        // 1: add the ultraviolet term of the Qin-Chang interaction
  double zeta;   // > 0: renormalise at p^2 = zeta^2 (GeV); 0: Z_1 = Z_2 = Z_4 = 1
};

}  // extern "C"

namespace {

const double PI = 3.14159265358979323846;

// Index b of the external node with u[b] < x <= u[b+1]; -1 below the grid,
// n-1 above it. This is the bracket search of Sec. III A.
int find_bracket(int n, const double* u, double x) {
  int b = -1;
  for (int i = 0; i < n; ++i)
    if (u[i] < x) b = i;
  return b;
}

// Lagrange interpolation in u of f given at nodes u[0..n-1], evaluated at x.
// order 1: the two nodes around x, constant beyond the ends (eq. chazhiresult).
// order 3: the four nodes b-1..b+2, shifted to stay inside the grid.
template <class T>
T interp_at(int n, const double* u, const T* f, double x, int order, int b) {
  int lo, cnt;
  if (order == 1) {
    if (b < 0) return f[0];
    if (b >= n - 1) return f[n - 1];
    lo = b;
    cnt = 2;
  } else {
    lo = b - 1;
    if (lo < 0) lo = 0;
    if (lo > n - 4) lo = n - 4;
    cnt = 4;
  }
  T acc = 0.0;
  for (int l = lo; l < lo + cnt; ++l) {
    double w = 1.0;
    for (int k = lo; k < lo + cnt; ++k)
      if (k != l) w *= (x - u[k]) / (u[l] - u[k]);
    acc += w * f[l];
  }
  return acc;
}

// The same with the bracket found by the search above (the paper's
// "traditional" interpolation).
template <class T>
T interp_one(int n, const double* u, const T* f, double x, int order) {
  return interp_at(n, u, f, x, order, find_bracket(n, u, x));
}

double dot4(const double* a, const double* b) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2] + a[3] * b[3];
}

// The bracketed integrands of eq. dsesys, i.e. I_A1+I_A2+I_A3 (with its one
// 1/p^2) and I_B1+I_B2+I_B3 of eq. dsesys2, at external p^2 = s, loop q^2 = t
// and z = cos(angle between p and q). Euclidean four-vectors: p along axis 4,
// q in the (3,4)-plane. k = p - q is the gluon momentum and P = p + q (the
// paper's "t" vector).
template <class T>
void integrand(double s, double t, double z, T Ap, T Bp, T Aq, T Bq, double lam,
               T* IA, T* IB, double* k2_out = nullptr) {
  const double p[4] = {0.0, 0.0, 0.0, std::sqrt(s)};
  const double sn = std::sqrt(1.0 - z * z);
  const double q[4] = {0.0, 0.0, std::sqrt(t) * sn, std::sqrt(t) * z};
  double k[4], P[4];
  for (int c = 0; c < 4; ++c) {
    k[c] = p[c] - q[c];
    P[c] = p[c] + q[c];
  }
  const double k2 = dot4(k, k), pq = dot4(p, q);
  if (k2_out) *k2_out = k2;
  const double pP = dot4(p, P), qP = dot4(q, P), PP = dot4(P, P);
  const double kp = dot4(k, p), kq = dot4(k, q), kP = dot4(k, P);

  // Ball-Chiu dressing functions, eq. (2): lambda_1 = sigA,
  // lambda_2 = -i dB, lambda_3 = dA / 2.
  T sigA = (Ap + Aq) / 2.0;
  T dA = (Aq - Ap) / (t - s);
  T dB = (Bq - Bp) / (t - s);
  sigA = 1.0 + lam * (sigA - 1.0);
  dA = lam * dA;
  dB = lam * dB;

  const T IA1 = -Bq * ((k2 * pP - kp * kP) / k2) * dB;
  const T IA2 = -Aq / 2.0 * ((s * qP * k2 + t * pP * k2 - t * kp * kP - s * kq * kP) / k2) * dA;
  const T IA3 = Aq * ((k2 * pq + 2.0 * kq * kp) / k2) * sigA;
  *IA = (IA1 + IA2 + IA3) / s;

  const T IB1 = -Aq * ((qP * k2 - kq * kP) / k2) * dB;
  const T IB2 = 3.0 * Bq * sigA;
  const T IB3 = Bq * ((k2 * PP - kP * kP) / (2.0 * k2)) * dA;
  *IB = IB1 + IB2 + IB3;
}

// Ultraviolet term of the Qin-Chang interaction (see the header).
double g_uv(double k2) {
  const double gamma_m = 12.0 / (33.0 - 2.0 * 4.0);
  const double lam2 = 0.234 * 0.234, mt2 = 0.5 * 0.5;
  const double tau = std::exp(2.0) - 1.0;
  const double f = -std::expm1(-k2 / (4.0 * mt2)) / k2;
  const double r = 1.0 + k2 / lam2;
  return 8.0 * PI * PI * gamma_m * f / std::log(tau + r * r);
}

// One external row i of the map: returns the two radial x angular sums.
template <class T>
void row_sums(const qo_vac_grid* g, const qo_vac_par* par, T Ai, T Bi,
              const T* Aq, const T* Bq, double s, T* sumA, T* sumB) {
  const double gnorm = 8.0 * PI * PI * par->D / std::pow(par->omega, 4);
  const double om2 = par->omega * par->omega;
  T accA = 0.0, accB = 0.0;
  for (int j = 0; j < g->nq; ++j) {
    const double t = g->t[j];
    const T Dq = t * Aq[j] * Aq[j] + Bq[j] * Bq[j];
    const double Wj = g->W[j];
    for (int a = 0; a < g->na; ++a) {
      const double z = g->z[a];
      T IA, IB;
      double k2;  // squared gluon momentum k = p - q, from the four-vectors
      integrand(s, t, z, Ai, Bi, Aq[j], Bq[j], par->lam, &IA, &IB, &k2);
      const double gk = gnorm * std::exp(-k2 / om2) + (par->uv ? g_uv(k2) : 0.0);
      const double w = Wj * g->wz[a] * std::sqrt(1.0 - z * z) * gk;
      accA += w * IA / Dq;
      accB += w * IB / Dq;
    }
  }
  *sumA = accA;
  *sumB = accB;
}

// The full map x' = F(x), x = [A(0..n-1) | B(0..n-1)], for the listed rows
// (rows == nullptr: all rows, written to x_out[i], x_out[n+i]; otherwise row
// rows[r] is written to x_out[r], x_out[nrows+r]).
template <class T>
void vac_map(const qo_vac_grid* g, const qo_vac_par* par, const T* x, T* out,
             const int* rows, int nrows, int nthreads) {
  const int n = g->n;
  std::vector<T> Aq(g->nq), Bq(g->nq);
  for (int j = 0; j < g->nq; ++j) {
    Aq[j] = interp_one(n, g->u, x, g->uq[j], g->order);
    Bq[j] = interp_one(n, g->u, x + n, g->uq[j], g->order);
  }
  const double c = (4.0 / 3.0) / (8.0 * PI * PI * PI);
  const int cnt = rows ? nrows : n;
  // renormalisation constants (1 without a renormalisation point)
  T Z2 = 1.0, Z4m = par->m;
  if (par->zeta > 0.0) {
    const double sz = par->zeta * par->zeta, uz = std::log(sz);
    const T Az = interp_one(n, g->u, x, uz, g->order);
    const T Bz = interp_one(n, g->u, x + n, uz, g->order);
    T sA, sB;
    row_sums(g, par, Az, Bz, Aq.data(), Bq.data(), sz, &sA, &sB);
    Z2 = 1.0 / (1.0 + c * sA);                              // A(zeta^2) = 1
    Z4m = par->m == 0.0 ? T(0.0) : par->m - Z2 * (c * sB);  // B(zeta^2) = m
  }
#pragma omp parallel for schedule(static) num_threads(nthreads)
  for (int r = 0; r < cnt; ++r) {
    const int i = rows ? rows[r] : r;
    T sA, sB;
    row_sums(g, par, x[i], x[n + i], Aq.data(), Bq.data(), g->s[i], &sA, &sB);
    if (par->zeta > 0.0) {
      out[r] = Z2 * (1.0 + c * sA);
      out[cnt + r] = Z4m + Z2 * (c * sB);
    } else {
      out[r] = 1.0 + c * sA;
      out[cnt + r] = par->m + c * sB;
    }
  }
}

// The map as the paper organises it (Sec. III, Table 1's programs): for
// every external momentum, functionA and functionB each run the whole radial x
// angular sum, and A(q^2), B(q^2) are interpolated where the integrand needs
// them, inside the angular loop. Traditional interpolation (Sec. III A) finds
// the bracket by searching the external grid at every call; the modified one
// takes it from the interleaving of eq. pqrelationship (loop node j lies
// between external nodes j-1 and j). Same arithmetic, in the same order, as
// vac_map: the results are identical; only the work differs.
double paper_function(const qo_vac_grid* g, const qo_vac_par* par, const double* x, int i,
                      int which, int modified) {
  const int n = g->n;
  const double gnorm = 8.0 * PI * PI * par->D / std::pow(par->omega, 4);
  const double om2 = par->omega * par->omega;
  double acc = 0.0;
  for (int j = 0; j < g->nq; ++j) {
    const double t = g->t[j];
    const double Wj = g->W[j];
    for (int a = 0; a < g->na; ++a) {
      double Aq, Bq;
      if (modified) {
        Aq = interp_at(n, g->u, x, g->uq[j], g->order, j - 1);
        Bq = interp_at(n, g->u, x + n, g->uq[j], g->order, j - 1);
      } else {
        Aq = interp_one(n, g->u, x, g->uq[j], g->order);
        Bq = interp_one(n, g->u, x + n, g->uq[j], g->order);
      }
      const double Dq = t * Aq * Aq + Bq * Bq;
      const double z = g->z[a];
      double IA, IB, k2;
      integrand(g->s[i], t, z, x[i], x[n + i], Aq, Bq, par->lam, &IA, &IB, &k2);
      const double gk = gnorm * std::exp(-k2 / om2);
      const double w = Wj * g->wz[a] * std::sqrt(1.0 - z * z) * gk;
      acc += w * (which == 0 ? IA : IB) / Dq;
    }
  }
  return acc;
}

int check_grid(const qo_vac_grid* g) {
  if (!g || g->n < 2 || g->nq < 1 || g->na < 1) return -1;
  if (g->order != 1 && g->order != 3) return -1;
  if (g->order == 3 && g->n < 4) return -1;
  return 0;
}

}  // namespace

extern "C" {

// x_out = F(x_in) for all rows; returns 0 or -1 on a bad grid.
int qo_vac_map(const qo_vac_grid* g, const qo_vac_par* par, const double* x_in,
               double* x_out, int nthreads) {
  if (check_grid(g)) return -1;
  vac_map<double>(g, par, x_in, x_out, nullptr, 0, nthreads);
  return 0;
}

// Rows rows[0..nrows-1] of F(x_in): out[r] = A'(rows[r]), out[nrows+r] = B'.
// One sweep in the paper's organisation (see paper_function): modified = 0
// traditional interpolation, 1 modified; nthreads = 1 sequential, more: OpenMP
// over external momenta (Table 1's algorithms 1-2 and 3-4).
int qo_vac_map_paper(const qo_vac_grid* g, const qo_vac_par* par, const double* x_in,
                     double* x_out, int modified, int nthreads) {
  if (check_grid(g) || !par || !x_in || !x_out || nthreads < 1) return -1;
  const double c = (4.0 / 3.0) / (8.0 * PI * PI * PI);
  const int n = g->n;
  const double f0[2] = {1.0, par->m};  // inhomogeneous terms of A and B
  // the two projections of every external momentum are separate integrals,
  // each with its own interpolation inside the loops; OpenMP over the rows
#pragma omp parallel for schedule(static) num_threads(nthreads)
  for (int i = 0; i < n; ++i)
    for (int which = 0; which < 2; ++which)
      x_out[which * n + i] = f0[which] + c * paper_function(g, par, x_in, i, which, modified);
  return 0;
}

int qo_vac_map_rows(const qo_vac_grid* g, const qo_vac_par* par, const double* x_in,
                    const int* rows, int nrows, double* out, int nthreads) {
  if (check_grid(g)) return -1;
  for (int r = 0; r < nrows; ++r)
    if (rows[r] < 0 || rows[r] >= g->n) return -1;
  vac_map<double>(g, par, x_in, out, rows, nrows, nthreads);
  return 0;
}

// Jacobian-vector product jv = (dF/dx) v at x by the complex step
// F(x + i h v) with h = 1e-30: Im / h is exact to rounding.
int qo_vac_jvp(const qo_vac_grid* g, const qo_vac_par* par, const double* x,
               const double* v, double* jv, int nthreads) {
  if (check_grid(g)) return -1;
  const int n2 = 2 * g->n;
  const double h = 1e-30;
  std::vector<cplx> xc(n2), oc(n2);
  for (int k = 0; k < n2; ++k) xc[k] = cplx(x[k], h * v[k]);
  vac_map<cplx>(g, par, xc.data(), oc.data(), nullptr, 0, nthreads);
  for (int k = 0; k < n2; ++k) jv[k] = oc[k].imag() / h;
  return 0;
}

// The complex-valued map itself (complex-step derivatives with respect to the
// parameters are taken by the caller through the inputs it perturbs).
int qo_vac_map_c(const qo_vac_grid* g, const qo_vac_par* par, const double* x_re,
                 const double* x_im, double* out_re, double* out_im, int nthreads) {
  if (check_grid(g)) return -1;
  const int n2 = 2 * g->n;
  std::vector<cplx> xc(n2), oc(n2);
  for (int k = 0; k < n2; ++k) xc[k] = cplx(x_re[k], x_im[k]);
  vac_map<cplx>(g, par, xc.data(), oc.data(), nullptr, 0, nthreads);
  for (int k = 0; k < n2; ++k) {
    out_re[k] = oc[k].real();
    out_im[k] = oc[k].imag();
  }
  return 0;
}

// Interpolated values f(x_j) at nq points, and the bracket found for each.
int qo_interp(int n, const double* u, const double* f, int nq, const double* x,
              int order, double* fx, int* bracket) {
  if (n < 2 || (order != 1 && order != 3) || (order == 3 && n < 4)) return -1;
  for (int j = 0; j < nq; ++j) {
    fx[j] = interp_one<double>(n, u, f, x[j], order);
    if (bracket) bracket[j] = find_bracket(n, u, x[j]);
  }
  return 0;
}

// The bracketed integrands I_A (with its 1/p^2) and I_B at one point.
void qo_integrand(double s, double t, double z, double Ap, double Bp, double Aq,
                  double Bq, double lam, double* IA, double* IB) {
  integrand<double>(s, t, z, Ap, Bp, Aq, Bq, lam, IA, IB);
}

int qo_max_threads(void) { return omp_get_max_threads(); }

double qo_g_uv(double k2) { return g_uv(k2); }

}  // extern "C"
