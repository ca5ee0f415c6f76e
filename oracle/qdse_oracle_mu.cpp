// qdse_oracle_mu.cpp -- plain FP64 CPU oracle for the quark gap equation at
// finite chemical potential mu (T = 0) with the Ball-Chiu vertex.
//
// TEST INFRASTRUCTURE ONLY. Nothing in the product path links, loads or calls
// this file; only the tests and the benchmark's CPU-baseline leg do. It shares
// no code, header, table or constant with the HIP library.
//
// The paper solves the vacuum equation and names the finite-mu problem as its
// extension (Sec. II: the propagator and vertex carry mu; Sec. V: one more
// integration dimension and two-dimensional interpolation). The equations are
// the vacuum ones (eqs. gendse, KernelAnsatz, bcvtxmu, eq. (2), IRGsQC) with
// the Euclidean quark momentum shifted, p~ = (p_vec, p4 + i mu):
//   S^-1(p~) = i gamma_vec.p_vec A(p~) + i gamma_4 p~_4 C(p~) + B(p~),
//   Sigma(p~) = C_F int d^4q/(2pi)^4 g(k^2) T_mu_nu(k) gamma_mu S(q~) Gamma_nu(q~, p~),
// k = p - q real (the shift cancels in the gluon momentum), and the Ball-Chiu
// vertex in its finite-mu form
//   Gamma_nu = Sigma_A gamma_nu (nu = 1..3) + Sigma_C gamma_4 (nu = 4)
//              + P~_nu [ Delta_A gamma_vec.P~_vec / 2 + Delta_C gamma_4 P~_4 / 2 - i Delta_B ],
// Sigma_F = (F(q~) + F(p~))/2, Delta_F = (F(q~) - F(p~))/(q~^2 - p~^2), P~ = p~ + q~,
// which satisfies i (q~ - p~).Gamma = S^-1(q~) - S^-1(p~). The projections are
//   A = 1 + tr[-i gamma_vec.p_vec Sigma]/(4 |p_vec|^2),
//   C = 1 + tr[-i gamma_4 p~_4 Sigma]/(4 p~_4^2),   B = m + tr[Sigma]/4.
// Here every trace is taken numerically from explicit complex 4x4 Euclidean
// Dirac matrices and a numerically inverted propagator: no scalar trace formula
// is used.
//
// Discretisation (readings): external |p_vec| on a Gauss-Legendre rule in
// ln|p_vec|, external p4 > 0 on a Gauss-Legendre rule in v with
// p4 = lambda sinh(v) (uniform near p4 = 0, logarithmic at large p4); loop
// |q_vec| and |q4| on the rules with one more node on the same intervals
// (interleaved); q4 runs over both signs with
// F(|q|, -q4) = F(|q|, q4)^* ; the angle between p_vec and q_vec on a
// Gauss-Legendre rule in z = cos(theta) with flat weight (d^3q = 2 pi |q|^2
// d|q| dz). A, B, C at loop points: tensor-product Lagrange interpolation in
// (ln|p_vec|, v), 2- or 4-point per direction, brackets found by searching.
#include <cmath>
#include <complex>
#include <vector>

typedef std::complex<double> cplx;

extern "C" {

struct qo_mu_grid {
  int ns, n4;       // external |p_vec| nodes, p4 nodes (p4 > 0)
  int nqs, nq4;     // loop |q_vec| nodes, |q4| nodes
  int na;           // angular nodes
  int order;        // 1 or 3
  const double* ps; const double* us;    // [ns]  |p_vec|, ln|p_vec|
  const double* p4; const double* v4;    // [n4]  p4, its grid variable v
  const double* qs; const double* uqs; const double* wqs;  // [nqs] |q|, ln|q|, |q|^2 d|q| weight
  const double* q4; const double* vq4; const double* wq4;  // [nq4] |q4|, its grid variable, dq4 weight
  const double* z;  const double* wz;    // [na] flat-weight rule in cos(theta)
};

struct qo_mu_par {
  double D, omega, m, mu;
};

}  // extern "C"

namespace {

const double PI = 3.14159265358979323846;
typedef cplx Mat[4][4];

struct Dirac {
  Mat g[4];
  Mat one;
  Dirac() {
    // Hermitian Euclidean matrices, chiral representation:
    // gamma_k = [[0, -i s_k], [i s_k, 0]], gamma_4 = [[0, 1], [1, 0]].
    const cplx I(0.0, 1.0);
    const cplx s[3][2][2] = {{{0.0, 1.0}, {1.0, 0.0}},
                             {{0.0, -I}, {I, 0.0}},
                             {{1.0, 0.0}, {0.0, -1.0}}};
    for (int m = 0; m < 4; ++m)
      for (int r = 0; r < 4; ++r)
        for (int c = 0; c < 4; ++c) g[m][r][c] = 0.0;
    for (int k = 0; k < 3; ++k)
      for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 2; ++c) {
          g[k][r][2 + c] = -I * s[k][r][c];
          g[k][2 + r][c] = I * s[k][r][c];
        }
    for (int r = 0; r < 2; ++r) {
      g[3][r][2 + r] = 1.0;
      g[3][2 + r][r] = 1.0;
    }
    for (int r = 0; r < 4; ++r)
      for (int c = 0; c < 4; ++c) one[r][c] = (r == c) ? 1.0 : 0.0;
  }
};

const Dirac& dirac() {
  static const Dirac d;
  return d;
}

void mat_zero(Mat a) {
  for (int r = 0; r < 4; ++r)
    for (int c = 0; c < 4; ++c) a[r][c] = 0.0;
}
void mat_axpy(Mat y, cplx a, const Mat x) {
  for (int r = 0; r < 4; ++r)
    for (int c = 0; c < 4; ++c) y[r][c] += a * x[r][c];
}
void mat_mul(Mat out, const Mat a, const Mat b) {
  for (int r = 0; r < 4; ++r)
    for (int c = 0; c < 4; ++c) {
      cplx acc = 0.0;
      for (int k = 0; k < 4; ++k) acc += a[r][k] * b[k][c];
      out[r][c] = acc;
    }
}
cplx trace(const Mat a) { return a[0][0] + a[1][1] + a[2][2] + a[3][3]; }

// Gauss-Jordan inverse with partial pivoting.
bool mat_inv(Mat out, const Mat a) {
  cplx w[4][8];
  for (int r = 0; r < 4; ++r)
    for (int c = 0; c < 4; ++c) {
      w[r][c] = a[r][c];
      w[r][4 + c] = (r == c) ? 1.0 : 0.0;
    }
  for (int col = 0; col < 4; ++col) {
    int piv = col;
    for (int r = col + 1; r < 4; ++r)
      if (std::abs(w[r][col]) > std::abs(w[piv][col])) piv = r;
    if (std::abs(w[piv][col]) == 0.0) return false;
    if (piv != col)
      for (int c = 0; c < 8; ++c) std::swap(w[piv][c], w[col][c]);
    const cplx d = w[col][col];
    for (int c = 0; c < 8; ++c) w[col][c] /= d;
    for (int r = 0; r < 4; ++r) {
      if (r == col) continue;
      const cplx f = w[r][col];
      if (f == 0.0) continue;
      for (int c = 0; c < 8; ++c) w[r][c] -= f * w[col][c];
    }
  }
  for (int r = 0; r < 4; ++r)
    for (int c = 0; c < 4; ++c) out[r][c] = w[r][4 + c];
  return true;
}

// slash(v) = sum_mu v_mu gamma_mu for a complex four-vector.
void slash(Mat out, const cplx v[4]) {
  mat_zero(out);
  for (int m = 0; m < 4; ++m) mat_axpy(out, v[m], dirac().g[m]);
}

// Inverse propagator i gamma_vec.x_vec A + i gamma_4 x4 C + B.
void sinv(Mat out, const cplx x[4], cplx A, cplx B, cplx C) {
  const cplx I(0.0, 1.0);
  mat_zero(out);
  for (int m = 0; m < 3; ++m) mat_axpy(out, I * x[m] * A, dirac().g[m]);
  mat_axpy(out, I * x[3] * C, dirac().g[3]);
  mat_axpy(out, B, dirac().one);
}

// The three projections of T_mu_nu(k) gamma_mu S(q~) Gamma_nu(q~, p~), without
// the interaction g(k^2): outA = tr[-i gamma_vec.p_vec M]/(4|p_vec|^2),
// outC = tr[-i gamma_4 p~_4 M]/(4 p~_4^2), outB = tr[M]/4.
void projections(const cplx p[4], const cplx q[4], const double k[4], cplx Ap, cplx Bp, cplx Cp,
                 cplx Aq, cplx Bq, cplx Cq, cplx* outA, cplx* outB, cplx* outC) {
  const Dirac& G = dirac();
  const cplx I(0.0, 1.0);
  Mat Si, S;
  sinv(Si, q, Aq, Bq, Cq);
  mat_inv(S, Si);
  cplx P[4];
  for (int m = 0; m < 4; ++m) P[m] = p[m] + q[m];
  const cplx p2 = p[0] * p[0] + p[1] * p[1] + p[2] * p[2] + p[3] * p[3];
  const cplx q2 = q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3];
  const cplx sA = (Aq + Ap) / 2.0, sC = (Cq + Cp) / 2.0;
  const cplx dA = (Aq - Ap) / (q2 - p2), dB = (Bq - Bp) / (q2 - p2), dC = (Cq - Cp) / (q2 - p2);
  // Gamma_nu
  Mat Gam[4], vecP;
  cplx Pvec[4] = {P[0], P[1], P[2], 0.0};
  slash(vecP, Pvec);
  for (int nu = 0; nu < 4; ++nu) {
    mat_zero(Gam[nu]);
    mat_axpy(Gam[nu], nu < 3 ? sA : sC, G.g[nu]);
    mat_axpy(Gam[nu], P[nu] * dA / 2.0, vecP);
    mat_axpy(Gam[nu], P[nu] * P[3] * dC / 2.0, G.g[3]);
    mat_axpy(Gam[nu], -I * P[nu] * dB, G.one);
  }
  const double k2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2] + k[3] * k[3];
  Mat M, T1, T2, Gm;
  mat_zero(M);
  for (int mu = 0; mu < 4; ++mu) {
    mat_zero(Gm);
    for (int nu = 0; nu < 4; ++nu) {
      const double Tmn = (mu == nu ? 1.0 : 0.0) - k[mu] * k[nu] / k2;
      mat_axpy(Gm, Tmn, Gam[nu]);
    }
    mat_mul(T1, S, Gm);
    mat_mul(T2, G.g[mu], T1);
    mat_axpy(M, 1.0, T2);
  }
  Mat pv, X;
  cplx pvec[4] = {p[0], p[1], p[2], 0.0};
  slash(pv, pvec);
  const double pv2 = (p[0] * p[0] + p[1] * p[1] + p[2] * p[2]).real();
  mat_mul(X, pv, M);
  *outA = -I * trace(X) / (4.0 * pv2);
  mat_mul(X, G.g[3], M);
  *outC = -I * p[3] * trace(X) / (4.0 * p[3] * p[3]);
  *outB = trace(M) / 4.0;
}

int find_bracket(int n, const double* u, double x) {
  int b = -1;
  for (int i = 0; i < n; ++i)
    if (u[i] < x) b = i;
  return b;
}

// 1-D Lagrange weights of node indices lo..lo+cnt-1 at x (order as in the
// vacuum oracle: 2-point flat beyond the ends, 4-point shifted stencil).
void weights_1d(int n, const double* u, double x, int order, int* lo, int* cnt, double w[4]) {
  const int b = find_bracket(n, u, x);
  if (order == 1) {
    if (b < 0) {
      *lo = 0; *cnt = 1; w[0] = 1.0; return;
    }
    if (b >= n - 1) {
      *lo = n - 1; *cnt = 1; w[0] = 1.0; return;
    }
    *lo = b; *cnt = 2;
  } else {
    int l = b - 1;
    if (l < 0) l = 0;
    if (l > n - 4) l = n - 4;
    *lo = l; *cnt = 4;
  }
  for (int a = 0; a < *cnt; ++a) {
    double c = 1.0;
    for (int k = 0; k < *cnt; ++k)
      if (k != a) c *= (x - u[*lo + k]) / (u[*lo + a] - u[*lo + k]);
    w[a] = c;
  }
}

}  // namespace

extern "C" {

// One sweep of the finite-mu map. x_re/x_im: [3][ns][n4] (A, B, C), out the
// same. rows: external points (a * n4 + b) to evaluate, or nullptr for all;
// out is then [3][nrows]. Returns 0, or -1 on a bad grid.
int qo_mu_map(const qo_mu_grid* g, const qo_mu_par* par, const double* x_re, const double* x_im,
              const int* rows, int nrows, double* out_re, double* out_im, int nthreads) {
  if (!g || g->ns < 2 || g->n4 < 2 || g->nqs < 1 || g->nq4 < 1 || g->na < 1) return -1;
  if (g->order != 1 && g->order != 3) return -1;
  if (g->order == 3 && (g->ns < 4 || g->n4 < 4)) return -1;
  const int ne = g->ns * g->n4;
  std::vector<cplx> X(3 * ne);
  for (int k = 0; k < 3 * ne; ++k) X[k] = cplx(x_re[k], x_im[k]);
  // A, B, C at the loop points (|q|, |q4|) by 2-D interpolation
  const int nl = g->nqs * g->nq4;
  std::vector<cplx> Lq(3 * nl);
  for (int c = 0; c < g->nqs; ++c) {
    int lo1, n1;
    double w1[4];
    weights_1d(g->ns, g->us, g->uqs[c], g->order, &lo1, &n1, w1);
    for (int d = 0; d < g->nq4; ++d) {
      int lo2, n2;
      double w2[4];
      weights_1d(g->n4, g->v4, g->vq4[d], g->order, &lo2, &n2, w2);
      for (int f = 0; f < 3; ++f) {
        cplx acc = 0.0;
        for (int a = 0; a < n1; ++a)
          for (int b = 0; b < n2; ++b)
            acc += w1[a] * w2[b] * X[(size_t)f * ne + (size_t)(lo1 + a) * g->n4 + lo2 + b];
        Lq[(size_t)f * nl + (size_t)c * g->nq4 + d] = acc;
      }
    }
  }
  const double gnorm = 8.0 * PI * PI * par->D / std::pow(par->omega, 4);
  const double om2 = par->omega * par->omega;
  const double cf = 4.0 / 3.0;
  const double meas = 1.0 / (8.0 * PI * PI * PI);  // d^4q/(2pi)^4 = dq4 2pi|q|^2 d|q| dz/(2pi)^4
  const int cnt = rows ? nrows : ne;
#pragma omp parallel for schedule(dynamic) num_threads(nthreads)
  for (int r = 0; r < cnt; ++r) {
    const int e = rows ? rows[r] : r;
    const int ia = e / g->n4, ib = e % g->n4;
    const double pabs = g->ps[ia], p4r = g->p4[ib];
    const cplx p[4] = {0.0, 0.0, pabs, cplx(p4r, par->mu)};
    const cplx Ap = X[e], Bp = X[ne + e], Cp = X[2 * ne + e];
    cplx sa = 0.0, sb = 0.0, sc = 0.0;
    for (int c = 0; c < g->nqs; ++c) {
      const double qa = g->qs[c];
      const double wr = g->wqs[c];  // |q|^2 d|q|
      for (int d = 0; d < g->nq4; ++d) {
        const double wq = g->wq4[d];  // dq4
        for (int sgn = -1; sgn <= 1; sgn += 2) {
          const double q4r = sgn * g->q4[d];
          cplx Aq = Lq[(size_t)c * g->nq4 + d], Bq = Lq[nl + (size_t)c * g->nq4 + d],
               Cq = Lq[2 * (size_t)nl + (size_t)c * g->nq4 + d];
          if (sgn < 0) {  // F(|q|, -q4) = F(|q|, q4)^*
            Aq = std::conj(Aq);
            Bq = std::conj(Bq);
            Cq = std::conj(Cq);
          }
          for (int a = 0; a < g->na; ++a) {
            const double z = g->z[a], sn = std::sqrt(1.0 - z * z);
            const cplx q[4] = {qa * sn, 0.0, qa * z, cplx(q4r, par->mu)};
            const double k[4] = {-qa * sn, 0.0, pabs - qa * z, p4r - q4r};
            const double k2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2] + k[3] * k[3];
            const double gk = gnorm * std::exp(-k2 / om2);
            cplx oA, oB, oC;
            projections(p, q, k, Ap, Bp, Cp, Aq, Bq, Cq, &oA, &oB, &oC);
            const double w = cf * meas * wr * wq * g->wz[a] * gk;
            sa += w * oA;
            sb += w * oB;
            sc += w * oC;
          }
        }
      }
    }
    const cplx An = 1.0 + sa, Bn = par->m + sb, Cn = 1.0 + sc;
    out_re[r] = An.real();
    out_im[r] = An.imag();
    out_re[cnt + r] = Bn.real();
    out_im[cnt + r] = Bn.imag();
    out_re[2 * cnt + r] = Cn.real();
    out_im[2 * cnt + r] = Cn.imag();
  }
  return 0;
}

// The three projections at one point (for tests): p = (0,0,|p|,p4+i mu),
// q = (|q| sin, 0, |q| cos, q4 + i mu).
void qo_mu_projections(double pabs, double p4, double qabs, double q4, double z, double mu,
                       const double* fp /*A,B,C re/im [6]*/, const double* fq /*[6]*/,
                       double* out /*[6]*/) {
  const double sn = std::sqrt(1.0 - z * z);
  const cplx p[4] = {0.0, 0.0, pabs, cplx(p4, mu)};
  const cplx q[4] = {qabs * sn, 0.0, qabs * z, cplx(q4, mu)};
  const double k[4] = {-qabs * sn, 0.0, pabs - qabs * z, p4 - q4};
  cplx oA, oB, oC;
  projections(p, q, k, cplx(fp[0], fp[1]), cplx(fp[2], fp[3]), cplx(fp[4], fp[5]),
              cplx(fq[0], fq[1]), cplx(fq[2], fq[3]), cplx(fq[4], fq[5]), &oA, &oB, &oC);
  out[0] = oA.real(); out[1] = oA.imag();
  out[2] = oB.real(); out[3] = oB.imag();
  out[4] = oC.real(); out[5] = oC.imag();
}

}  // extern "C"
