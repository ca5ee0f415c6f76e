// qdse_mu.hip -- the gap-equation sweep at finite chemical potential mu
// (T = 0) with the Ball-Chiu vertex, evaluated directly on gfx950.
//
// The paper names this extension (Sec. II carries mu in the propagator and
// vertex; Sec. V: one more integration dimension and two-dimensional
// interpolation). With p~ = (p_vec, p4 + i mu), real gluon momentum k = p - q,
//   S^-1(p~) = i gamma_vec.p_vec A + i gamma_4 p~_4 C + B,
//   Gamma_nu = Sigma'_nu gamma_nu + P~_nu [gamma.U / 2 - i Delta_B],
//   Sigma' = (Sigma_A, Sigma_A, Sigma_A, Sigma_C),
//   U = (Delta_A P~_vec, Delta_C P~_4),
// Sigma_F = (F(q~) + F(p~))/2, Delta_F = (F(q~) - F(p~))/(q~^2 - p~^2). With the
// dressed loop momentum Qh = (A(q~) q_vec, C(q~) q~_4), Delta = Qh.Qh + B(q~)^2,
// S(q~) = (-i gamma.Qh + B(q~))/Delta, T(a, b) = a.b - (a.k)(b.k)/k^2 (bilinear,
// no conjugation) and the Euclidean trace identities, the three projections of
// T_mu_nu gamma_mu S(q~) Gamma_nu reduce to four-vector algebra:
//   tr/4        = [ -Delta_B T(Qh, P~) + B(q~) TrW ] / Delta,
//   tr[-i gamma.X .]/4 = [ -T(X, Qh o Sigma') - (Qh.U) T(X, P~)/2 + (X.Qh) TrW
//                          - T(Qh, X o Sigma') - (X.U) T(Qh, P~)/2
//                          - B(q~) Delta_B T(X, P~) ] / Delta,
//   TrW = sum_nu Sigma'_nu + U.P~/2 - [ sum_nu k_nu^2 Sigma'_nu + (k.U)(k.P~)/2 ]/k^2,
// with X = (p_vec, 0) for A (divided by |p_vec|^2) and X = (0, p~_4) for C
// (divided by p~_4^2); (a o b)_nu = a_nu b_nu.
//
// Quadrature: external |p_vec| x p4 (> 0) grid, loop |q_vec| x |q4| grid (one
// more node per direction on the same intervals, interleaved), q4 of both signs
// with F(|q|, -q4) = F(|q|, q4)^*, angle z = cos(p_vec, q_vec) with flat weight;
// measure d^4q/(2pi)^4 = dq4 |q|^2 d|q| dz / (8 pi^3), weights precomputed.
// A, B, C at loop points by a tensor-product 4x4 stencil with brackets known
// from the interleaving. No angular kernel is precomputed: one wavefront per
// external point, lanes over loop points, angles in registers (FP64 VALU).
#include "qdse_internal.h"

namespace qdse {

namespace {

struct cd {
  double r, i;
};
__device__ inline cd mk(double r, double i = 0.0) { return {r, i}; }
__device__ inline cd operator+(cd a, cd b) { return {a.r + b.r, a.i + b.i}; }
__device__ inline cd operator-(cd a, cd b) { return {a.r - b.r, a.i - b.i}; }
__device__ inline cd operator-(cd a) { return {-a.r, -a.i}; }
__device__ inline cd operator*(cd a, cd b) { return {a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r}; }
__device__ inline cd operator*(double a, cd b) { return {a * b.r, a * b.i}; }
__device__ inline cd operator*(cd b, double a) { return {a * b.r, a * b.i}; }
__device__ inline cd inv(cd a) {
  const double d = a.r * a.r + a.i * a.i;
  return {a.r / d, -a.i / d};
}
__device__ inline cd conj(cd a) { return {a.r, -a.i}; }

// Four-vectors with a vanishing y component: (x, z, t).
struct v3 {
  cd x, z, t;
};
__device__ inline cd dot(v3 a, v3 b) { return a.x * b.x + a.z * b.z + a.t * b.t; }

constexpr int MU_WAVE = 64;

__device__ inline double wsum_mu(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// A, B, C at every loop point (|q| index c, |q4| index d), per instance.
__global__ void k_mu_interp(int ns, int n4, int nqs, int nq4, const int* __restrict__ lo_s,
                            const double* __restrict__ sw_s, const int* __restrict__ lo_4,
                            const double* __restrict__ sw_4, const double2* __restrict__ x,
                            double2* __restrict__ L) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  const int inst = blockIdx.y;
  const int nl = nqs * nq4, ne = ns * n4;
  if (l >= nl) return;
  const int c = l / nq4, d = l % nq4;
  const double2* xi = x + (size_t)inst * 3 * ne;
  double2* Li = L + (size_t)inst * 3 * nl;
  const int bs = lo_s[c], b4 = lo_4[d];
  for (int f = 0; f < 3; ++f) {
    double re = 0.0, im = 0.0;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const double wa = sw_s[4 * c + a];
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const double w = wa * sw_4[4 * d + b];
        const double2 v = xi[(size_t)f * ne + (size_t)(bs + a) * n4 + b4 + b];
        re = fma(w, v.x, re);
        im = fma(w, v.y, im);
      }
    }
    Li[(size_t)f * nl + l] = make_double2(re, im);
  }
}

struct MuArgs {
  int n_inst, ns, n4, nqs, nq4, na;
  double mu, gnorm, inv_om2, m, cw;  // cw = C_F / (8 pi^3)
  const double* ps;
  const double* p4;
  const double* qs;
  const double* q4;
  const double* wqs;
  const double* wq4;
  const double* z;
  const double* wz;
  const double2* x;  // [inst][3][ne]
  const double2* L;  // [inst][3][nl]
  double2* out;      // [inst][3][ne]
};

__global__ void __launch_bounds__(256) k_mu_sweep(MuArgs a) {
  __shared__ double zs[256], sns[256], wzs[256];
  const int lane = threadIdx.x & (MU_WAVE - 1);
  for (int t = threadIdx.x; t < a.na && t < 256; t += blockDim.x) {
    zs[t] = a.z[t];
    sns[t] = sqrt((1.0 - a.z[t]) * (1.0 + a.z[t]));
    wzs[t] = a.wz[t];
  }
  __syncthreads();
  const int ne = a.ns * a.n4, nl = a.nqs * a.nq4;
  const long row = (long)blockIdx.x * (blockDim.x / MU_WAVE) + threadIdx.x / MU_WAVE;
  if (row >= (long)a.n_inst * ne) return;
  const int inst = (int)(row / ne), e = (int)(row % ne);
  const int ia = e / a.n4, ib = e % a.n4;
  const double pabs = a.ps[ia], p4r = a.p4[ib];
  const double2* xi = a.x + (size_t)inst * 3 * ne;
  const double2* Li = a.L + (size_t)inst * 3 * nl;
  const cd Ap = mk(xi[e].x, xi[e].y), Bp = mk(xi[ne + e].x, xi[ne + e].y),
           Cp = mk(xi[2 * ne + e].x, xi[2 * ne + e].y);
  const cd pt4 = mk(p4r, a.mu);
  const cd p2 = mk(pabs * pabs) + pt4 * pt4;
  double sAr = 0, sAi = 0, sBr = 0, sBi = 0, sCr = 0, sCi = 0;
  for (int l = lane; l < nl; l += MU_WAVE) {
    const int c = l / a.nq4, d = l % a.nq4;
    const double qa = a.qs[c];
    const double wl = a.cw * a.wqs[c] * a.wq4[d];
    const cd A0 = mk(Li[l].x, Li[l].y), B0 = mk(Li[nl + l].x, Li[nl + l].y),
             C0 = mk(Li[2 * nl + l].x, Li[2 * nl + l].y);
    for (int sgn = -1; sgn <= 1; sgn += 2) {
      const double q4r = sgn * a.q4[d];
      const cd Aq = sgn < 0 ? conj(A0) : A0, Bq = sgn < 0 ? conj(B0) : B0,
               Cq = sgn < 0 ? conj(C0) : C0;
      const cd qt4 = mk(q4r, a.mu);
      const cd q2 = mk(qa * qa) + qt4 * qt4;
      const cd idq = inv(q2 - p2);
      const cd sA = 0.5 * (Aq + Ap), sC = 0.5 * (Cq + Cp);
      const cd dA = (Aq - Ap) * idq, dB = (Bq - Bp) * idq, dC = (Cq - Cp) * idq;
      const cd Dl = Aq * Aq * (qa * qa) + Cq * Cq * (qt4 * qt4) + Bq * Bq;
      const cd iD = inv(Dl);
      const cd P4 = pt4 + qt4;
      const double k4 = p4r - q4r;
      for (int t = 0; t < a.na; ++t) {
        const double z = zs[t], sn = sns[t];
        const double qx = qa * sn, qz = qa * z;
        const double kx = -qx, kz = pabs - qz;
        const double k2 = kx * kx + kz * kz + k4 * k4;
        const double ik2 = 1.0 / k2;
        const double gw = wl * wzs[t] * a.gnorm * exp(-k2 * a.inv_om2);
        const v3 P{mk(qx), mk(pabs + qz), P4};
        const v3 Qh{Aq * qx, Aq * qz, Cq * qt4};
        const v3 U{dA * P.x, dA * P.z, dC * P.t};
        const v3 K{mk(kx), mk(kz), mk(k4)};
        const cd kP = dot(K, P), kQ = dot(K, Qh), kU = dot(K, U);
        const cd QP = dot(Qh, P), QU = dot(Qh, U), UP = dot(U, P);
        const cd TQP = QP - kQ * kP * ik2;
        const cd TrW = 3.0 * sA + sC + 0.5 * UP -
                       (sA * (kx * kx + kz * kz) + sC * (k4 * k4) + 0.5 * kU * kP) * ik2;
        const cd Bproj = (Bq * TrW - dB * TQP) * iD;
        // X = (0, |p|, 0): A projection
        const v3 QS{sA * Qh.x, sA * Qh.z, sC * Qh.t};  // Qh o Sigma'
        const cd kQS = dot(K, QS);
        const double Xz = pabs;
        const cd TXQS = Xz * QS.z - (Xz * kz) * kQS * ik2;      // T(X, Qh o Sigma')
        const cd TXP = Xz * P.z - (Xz * kz) * kP * ik2;         // T(X, P)
        const cd XSz = sA * Xz;                                 // X o Sigma' = (0, sA |p|, 0)
        const cd TQXS = Qh.z * XSz - kQ * (kz * XSz) * ik2;     // T(Qh, X o Sigma')
        const cd XQ = Xz * Qh.z, XU = Xz * U.z;
        const cd numA = -TXQS - 0.5 * QU * TXP + XQ * TrW - TQXS - 0.5 * XU * TQP -
                        Bq * dB * TXP;
        const cd Aproj = numA * iD * (1.0 / (pabs * pabs));
        // X = (0, 0, p~4): C projection
        const cd TXQS4 = pt4 * QS.t - (k4 * pt4) * kQS * ik2;
        const cd TXP4 = pt4 * P.t - (k4 * pt4) * kP * ik2;
        const cd XS4 = sC * pt4;
        const cd TQXS4 = Qh.t * XS4 - kQ * (k4 * XS4) * ik2;
        const cd XQ4 = pt4 * Qh.t, XU4 = pt4 * U.t;
        const cd numC = -TXQS4 - 0.5 * QU * TXP4 + XQ4 * TrW - TQXS4 - 0.5 * XU4 * TQP -
                        Bq * dB * TXP4;
        const cd Cproj = numC * iD * inv(pt4 * pt4);
        sAr = fma(gw, Aproj.r, sAr);
        sAi = fma(gw, Aproj.i, sAi);
        sBr = fma(gw, Bproj.r, sBr);
        sBi = fma(gw, Bproj.i, sBi);
        sCr = fma(gw, Cproj.r, sCr);
        sCi = fma(gw, Cproj.i, sCi);
      }
    }
  }
  sAr = wsum_mu(sAr);
  sAi = wsum_mu(sAi);
  sBr = wsum_mu(sBr);
  sBi = wsum_mu(sBi);
  sCr = wsum_mu(sCr);
  sCi = wsum_mu(sCi);
  if (lane == 0) {
    double2* o = a.out + (size_t)inst * 3 * ne;
    o[e] = make_double2(1.0 + sAr, sAi);
    o[ne + e] = make_double2(a.m + sBr, sBi);
    o[2 * ne + e] = make_double2(1.0 + sCr, sCi);
  }
}

// Per-instance max over external points of |A'-A|, |B'-B|, |C'-C|, as bits of
// a non-negative double (atomic max).
__global__ void k_mu_stat(int n_inst, int ne, const double2* __restrict__ xo,
                          const double2* __restrict__ xn, unsigned long long* __restrict__ stat) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const int inst = blockIdx.y;
  if (t >= 3l * ne) return;
  const size_t o = (size_t)inst * 3 * ne + t;
  const double dr = xn[o].x - xo[o].x, di = xn[o].y - xo[o].y;
  double r = sqrt(dr * dr + di * di);
  unsigned long long bits =
      isnan(r) ? 0x7ff8000000000000ull : (unsigned long long)__double_as_longlong(r);
  atomicMax(&stat[inst], bits);
}

}  // namespace

hipError_t launch_mu_sweep(hipStream_t st, int n_inst, int ns, int n4, int nqs, int nq4, int na,
                           const double* ps, const double* p4, const double* qs, const double* q4,
                           const double* wqs, const double* wq4, const double* z, const double* wz,
                           const int* lo_s, const double* sw_s, const int* lo_4,
                           const double* sw_4, double mu, double D, double omega, double m,
                           const double* x_in, double* x_out, double* L) {
  if (na > 256) return hipErrorInvalidValue;
  const int nl = nqs * nq4, ne = ns * n4;
  hipLaunchKernelGGL(k_mu_interp, dim3((nl + 255) / 256, n_inst), dim3(256), 0, st, ns, n4, nqs,
                     nq4, lo_s, sw_s, lo_4, sw_4, (const double2*)x_in, (double2*)L);
  const double pi = 3.14159265358979323846;
  MuArgs a{n_inst, ns, n4, nqs, nq4, na, mu, 8.0 * pi * pi * D / (omega * omega * omega * omega),
           1.0 / (omega * omega), m, (4.0 / 3.0) / (8.0 * pi * pi * pi), ps, p4, qs, q4, wqs, wq4,
           z, wz, (const double2*)x_in, (const double2*)L, (double2*)x_out};
  const long rows = (long)n_inst * ne;
  hipLaunchKernelGGL(k_mu_sweep, dim3((unsigned)((rows + 3) / 4)), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_mu_stat(hipStream_t st, int n_inst, int ne, const double* x_old,
                          const double* x_new, unsigned long long* stat) {
  hipLaunchKernelGGL(k_mu_stat, dim3((unsigned)((3l * ne + 255) / 256), n_inst), dim3(256), 0, st,
                     n_inst, ne, (const double2*)x_old, (const double2*)x_new, stat);
  return hipGetLastError();
}

}  // namespace qdse
