// Near-diagonal band of the sweep Jacobian J = dF/dx at a point x, and a
// banded preconditioner for the adjoint system (I - J)^T lambda = g built
// from it.
//
// The sweep (Sec. II eqs. dsesys, dsesys2 in the direct-difference form) maps
// x = [A | B] to F(x); row i depends on A_i, B_i directly and on the node
// functions of every loop node j (A, B interpolated at t_j, sigma_V =
// A/Delta, sigma_S = B/Delta, Delta = t A^2 + B^2), which depend on the four
// external nodes of j's stencil. Hence
//   J[(a,i),(b,l)] = delta_il D^{ab}_i + sum_{j : l in stencil(j)} w_{j,l} G^{ab}_{ij},
// with D_i the derivatives through A_i, B_i (a full row sum over j) and G_ij
// the derivatives through A(t_j), B(t_j) (local to the pair (i, j)). The
// loop-node weights 1/(t_j - s_i) inside the kernel matrices make the entries
// with t_j next to s_i large and the spectrum of J spread with the grid size;
// the band |i - l| <= bw holds that part, and a banded solve with
// I - band(J)^T removes it from the Krylov iteration.
#include "qdse_internal.h"

namespace qdse {

namespace {

constexpr int WAVE = 64;

__device__ inline double shfl_sum(double v) {
#pragma unroll
  for (int o = WAVE / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
  return v;
}

// D_i per instance: d(F^A, F^B)/d(A_i, B_i) through dA, dB and A + A_i, one
// wavefront per row: D[inst][i][4] = {AA, AB, BA, BB}.
__global__ void __launch_bounds__(256) k_jdiag(int n_inst, int n, int nq, int ldk,
                                               const InstDev* __restrict__ inst_,
                                               const double* __restrict__ K, size_t kstride,
                                               const double* __restrict__ s_,
                                               const double* __restrict__ t_,
                                               const double* __restrict__ nodes,
                                               double* __restrict__ D) {
  const int lane = threadIdx.x & (WAVE - 1);
  const long row = (long)blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE;
  if (row >= (long)n_inst * n) return;
  const int inst = (int)(row / n), i = (int)(row % n);
  const InstDev P = inst_[inst];
  const size_t mat = (size_t)n * ldk;
  const double* Ki = K + (size_t)P.kblock * kstride + (size_t)i * ldk;
  const double* nd = nodes + (size_t)inst * 5 * ldk;
  const double s = s_[i];
  double aa = 0.0, ab = 0.0, ba = 0.0, bb = 0.0;
  for (int j = lane; j < nq; j += WAVE) {
    const double kT = Ki[j], k3 = Ki[mat + j], k0 = Ki[2 * mat + j];
    const double sV = nd[2 * ldk + j], sS = nd[3 * ldk + j], t = t_[j];
    aa += (k3 + kT * (s + t)) * sV;
    ab += 2.0 * kT * sS;
    ba += (k0 - 2.0 * s * kT) * sS;
    bb += 2.0 * s * kT * sV;
  }
  aa = shfl_sum(aa);
  ab = shfl_sum(ab);
  ba = shfl_sum(ba);
  bb = shfl_sum(bb);
  if (lane == 0) {
    double* o = D + ((size_t)inst * n + i) * 4;
    o[0] = P.pref * aa;
    o[1] = P.pref * ab;
    o[2] = P.pref * ba;
    o[3] = P.pref * bb;
  }
}

// Band entries: one thread per (instance, row i, offset o), l = i - bw + o.
// Output block order {AA, AB, BA, BB} (first letter: component of F, second:
// of x). Layout instance-major [inst][i][o][4], or instance-minor
// [i][o][4][inst] when minor != 0 (for the per-instance factorisation).
__global__ void k_jband(int n_inst, int n, int nq, int ldk, int bw, const InstDev* __restrict__ inst_,
                        const double* __restrict__ K, size_t kstride, const int* __restrict__ lo,
                        const double* __restrict__ sw, const double* __restrict__ s_,
                        const double* __restrict__ t_, const double* __restrict__ nodes,
                        const double* __restrict__ x, const double* __restrict__ D,
                        double* __restrict__ out, int minor) {
  const int wb = 2 * bw + 1;
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)n_inst * n * wb) return;
  const int inst = (int)(e / ((long)n * wb));
  const int rem = (int)(e % ((long)n * wb));
  const int i = rem / wb, o = rem % wb, l = i - bw + o;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  if (l >= 0 && l < n) {
    const InstDev P = inst_[inst];
    const size_t mat = (size_t)n * ldk;
    const double* Ki = K + (size_t)P.kblock * kstride + (size_t)i * ldk;
    const double* nd = nodes + (size_t)inst * 5 * ldk;
    const double* xi = x + (size_t)inst * 2 * n;
    const double s = s_[i], Ai = xi[i], Bi = xi[n + i];
    if (l == i) {
      const double* Di = D + ((size_t)inst * n + i) * 4;
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[q] = Di[q];
    }
    // stencil bases clamp(j - 2, 0, N - 4): node l is in the stencils of
    // loop nodes l - 3 .. l + 4 at most (l + 4 for the last loop node)
    const int j0 = l - 3 < 0 ? 0 : l - 3, j1 = l + 4 > nq - 1 ? nq - 1 : l + 4;
    for (int j = j0; j <= j1; ++j) {
      const int b = lo[j];
      if (l < b || l >= b + 4) continue;
      const double wl = sw[4 * j + (l - b)];
      const double kT = Ki[j], k3 = Ki[mat + j], k0 = Ki[2 * mat + j];
      const double Aq = nd[j], Bq = nd[ldk + j], sV = nd[2 * ldk + j], sS = nd[3 * ldk + j];
      const double t = t_[j];
      const double dA = Aq - Ai, dB = Bq - Bi, sA = Aq + Ai;
      // derivatives of sigma_V, sigma_S with respect to A(t_j), B(t_j)
      const double Dl = t * Aq * Aq + Bq * Bq, iD2 = 1.0 / (Dl * Dl);
      const double vA = (Bq * Bq - t * Aq * Aq) * iD2, vB = -2.0 * Aq * Bq * iD2;
      const double sAq = -2.0 * t * Aq * Bq * iD2, sBq = (t * Aq * Aq - Bq * Bq) * iD2;
      // F^A = 1 + pref (sum k3 sV sA - sum kT [2 sS dB + (s + t) sV dA])
      const double fA_sV = k3 * sA - kT * (s + t) * dA, fA_sS = -2.0 * kT * dB;
      const double fA_A = k3 * sV - kT * (s + t) * sV, fA_B = -2.0 * kT * sS;
      // F^B = m + pref (2 s sum kT (sS dA - sV dB) + sum k0 sS sA)
      const double fB_sV = -2.0 * s * kT * dB, fB_sS = 2.0 * s * kT * dA + k0 * sA;
      const double fB_A = 2.0 * s * kT * sS + k0 * sS, fB_B = -2.0 * s * kT * sV;
      const double c = P.pref * wl;
      acc[0] += c * (fA_A + fA_sV * vA + fA_sS * sAq);
      acc[1] += c * (fA_B + fA_sV * vB + fA_sS * sBq);
      acc[2] += c * (fB_A + fB_sV * vA + fB_sS * sAq);
      acc[3] += c * (fB_B + fB_sV * vB + fB_sS * sBq);
    }
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const size_t idx = minor ? (((size_t)i * wb + o) * 4 + q) * n_inst + inst
                             : (((size_t)inst * n + i) * wb + o) * 4 + q;
    out[idx] = acc[q];
  }
}

// M = I - band(J)^T with the unknowns interleaved, r = 2 l + b (b = 0: A, 1: B):
// M[2l+b][2i+a] = delta - J[(a,i),(b,l)], |i - l| <= BW, so |r - c| <= HB =
// 2 BW + 1. LU without pivoting, one wavefront per instance: the HB + 1
// active rows of the band sit in registers (the same values in every lane),
// the rows entering the window over the next 64 steps are assembled from the
// band by the 64 lanes (one row each) into LDS while the current 64 steps
// run, and lane u keeps factor row k0 + u to write it. Factor rows
// [inst][r][2 HB + 1]: unit lower multipliers left of the diagonal, the
// reciprocal of U's diagonal at offset HB, U's other entries right of it.
// ok[inst] = 0 when a pivot is not safely away from zero (the solve then
// leaves that instance unpreconditioned).
template <int BW>
__global__ void __launch_bounds__(64) k_band_lu(int n_inst, int n, const double* __restrict__ Jb,
                                                double* __restrict__ F, int* __restrict__ ok) {
  constexpr int HB = 2 * BW + 1, W = 2 * HB + 1, WB = 2 * BW + 1;
  __shared__ double rows[WAVE][W];
  const int inst = blockIdx.x;
  const int lane = threadIdx.x;
  const int N = 2 * n;
  // row r of M, entries at offsets d = c - r + HB (rows past the end: identity)
  auto load_row = [&](int r, double* R) {
#pragma unroll
    for (int d = 0; d < W; ++d) R[d] = 0.0;
    if (r >= N) {
      R[HB] = 1.0;
      return;
    }
#pragma unroll
    for (int d = 0; d < W; ++d) {
      const int c = r + d - HB;
      if (c < 0 || c >= N) continue;
      // (a, i): component and node of F (the column); (b, l): of x (the row)
      const int i = c >> 1, a = c & 1, l = r >> 1, b = r & 1;
      const int o = l - i + BW;
      if (o < 0 || o >= WB) continue;
      const double jv = Jb[(((size_t)i * WB + o) * 4 + (a * 2 + b)) * n_inst + inst];
      R[d] = (c == r ? 1.0 : 0.0) - jv;
    }
  };
  double R[HB + 1][W];
#pragma unroll
  for (int q = 0; q <= HB; ++q) load_row(q, R[q]);
  double nxt[W], keep[W];
  load_row(HB + 1 + lane, nxt);  // rows entering at steps 0 .. 63
  int good = 1;
  double* Fi = F + (size_t)inst * N * W;
  for (int k0 = 0; k0 < N; k0 += WAVE) {
#pragma unroll
    for (int d = 0; d < W; ++d) rows[lane][d] = nxt[d];
    __syncthreads();
    load_row(k0 + WAVE + HB + 1 + lane, nxt);  // overlaps this chunk's steps
    const int cnt = min(WAVE, N - k0);
    for (int u = 0; u < cnt; ++u) {
      const double piv = R[0][HB];
      double scale = 0.0;
#pragma unroll
      for (int d = HB; d < W; ++d) scale = fmax(scale, fabs(R[0][d]));
      if (!(fabs(piv) > 1e-8 * scale)) good = 0;
      const double ip = good ? 1.0 / piv : 0.0;
#pragma unroll
      for (int q = 1; q <= HB; ++q) {
        const double f = R[q][HB - q] * ip;
        R[q][HB - q] = f;
#pragma unroll
        for (int cc = 1; cc <= HB; ++cc)
          R[q][HB - q + cc] = fma(-f, R[0][HB + cc], R[q][HB - q + cc]);
      }
#pragma unroll
      for (int d = 0; d < W; ++d) keep[d] = lane == u ? (d == HB ? ip : R[0][d]) : keep[d];
#pragma unroll
      for (int q = 0; q < HB; ++q)
#pragma unroll
        for (int d = 0; d < W; ++d) R[q][d] = R[q + 1][d];
#pragma unroll
      for (int d = 0; d < W; ++d) R[HB][d] = rows[u][d];
    }
    if (lane < cnt) {
#pragma unroll
      for (int d = 0; d < W; ++d) Fi[(size_t)(k0 + lane) * W + d] = keep[d];
    }
    __syncthreads();
  }
  if (lane == 0) ok[inst] = good;
}

// out = M^{-1} in for every active instance (act may be null), one wavefront
// per instance. Forward substitution with the unit lower factor, then
// backward with the upper one, 64 rows at a time: lane l reads row c0 + l
// (its factor values and right-hand side) while the previous 64 rows are
// being solved, the rows go to LDS, and every lane then runs the 64
// sequential steps from LDS (the same values in every lane; lane u keeps the
// solution of step u and writes it). In each step the terms of the older
// solution values are added first, so a step waits on the previous one for a
// single FMA. Instances with ok == 0 get out = in.
template <int BW>
__global__ void __launch_bounds__(64) k_band_solve(int n_inst, int n, const double* __restrict__ F,
                                                   const int* __restrict__ ok,
                                                   const int* __restrict__ act,
                                                   const double* __restrict__ in,
                                                   double* __restrict__ out) {
  constexpr int HB = 2 * BW + 1, W = 2 * HB + 1, NV = HB + 2;
  __shared__ double buf[WAVE][NV];
  const int inst = blockIdx.x;
  if (act && !act[inst]) return;  // the whole workgroup (one wavefront)
  const int lane = threadIdx.x;
  const int N = 2 * n;
  const double* Fi = F + (size_t)inst * N * W;
  const double* vi = in + (size_t)inst * N;
  double* xo = out + (size_t)inst * N;
  auto at = [&](int r) { return (r & 1) * n + (r >> 1); };  // interleaved -> [A | B]
  if (!ok[inst]) {
    for (int r = lane; r < N; r += WAVE) xo[r] = vi[r];
    return;
  }
  double y[HB], pf[NV];
  // forward: row r: pf[q - 1] = L[r][r - q] (q = 1..HB), pf[HB] = in[r]
  auto fetch_f = [&](int c0) {
    const int r = c0 + lane;
    if (r < N) {
#pragma unroll
      for (int q = 1; q <= HB; ++q) pf[q - 1] = Fi[(size_t)r * W + HB - q];
      pf[HB] = vi[at(r)];
    }
  };
#pragma unroll
  for (int q = 0; q < HB; ++q) y[q] = 0.0;  // y[q]: solution at r - 1 - q
  fetch_f(0);
  for (int c0 = 0; c0 < N; c0 += WAVE) {
#pragma unroll
    for (int k = 0; k < HB + 1; ++k) buf[lane][k] = pf[k];
    __syncthreads();
    fetch_f(c0 + WAVE);  // the next rows' reads overlap this chunk's steps
    const int cnt = min(WAVE, N - c0);
    double xv = 0.0;
#pragma unroll 8
    for (int u = 0; u < cnt; ++u) {
      double x = buf[u][HB];
#pragma unroll
      for (int q = HB; q >= 1; --q) x = fma(-buf[u][q - 1], y[q - 1], x);
#pragma unroll
      for (int q = HB - 1; q > 0; --q) y[q] = y[q - 1];
      y[0] = x;
      xv = lane == u ? x : xv;
    }
    if (lane < cnt) xo[at(c0 + lane)] = xv;
    __syncthreads();
  }
  // backward: row r: pf[q - 1] = U[r][r + q] (q = 1..HB), pf[HB] = 1/U[r][r],
  // pf[HB + 1] = forward solution at r
  auto fetch_b = [&](int c0) {
    const int r = c0 - lane;
    if (r >= 0) {
#pragma unroll
      for (int q = 0; q <= HB; ++q) pf[q == 0 ? HB : q - 1] = Fi[(size_t)r * W + HB + q];
      pf[HB + 1] = xo[at(r)];
    }
  };
#pragma unroll
  for (int q = 0; q < HB; ++q) y[q] = 0.0;  // y[q]: solution at r + 1 + q
  fetch_b(N - 1);
  for (int c0 = N - 1; c0 >= 0; c0 -= WAVE) {
#pragma unroll
    for (int k = 0; k < NV; ++k) buf[lane][k] = pf[k];
    __syncthreads();
    fetch_b(c0 - WAVE);
    const int cnt = min(WAVE, c0 + 1);
    double xv = 0.0;
#pragma unroll 8
    for (int u = 0; u < cnt; ++u) {
      double x = buf[u][HB + 1];
#pragma unroll
      for (int q = HB; q >= 1; --q) x = fma(-buf[u][q - 1], y[q - 1], x);
      x *= buf[u][HB];
#pragma unroll
      for (int q = HB - 1; q > 0; --q) y[q] = y[q - 1];
      y[0] = x;
      xv = lane == u ? x : xv;
    }
    if (lane < cnt) xo[at(c0 - lane)] = xv;
    __syncthreads();
  }
}

}  // namespace

hipError_t launch_jband(hipStream_t st, int n_inst, int n, int nq, int ldk, int bw,
                        const InstDev* inst, const double* K, size_t kstride, const int* lo,
                        const double* sw, const double* s, const double* t, const double* nodes,
                        const double* x, double* D, double* out, int minor) {
  const long rows = (long)n_inst * n;
  hipLaunchKernelGGL(k_jdiag, dim3((unsigned)((rows + 3) / 4)), dim3(256), 0, st, n_inst, n, nq,
                     ldk, inst, K, kstride, s, t, nodes, D);
  const long tot = rows * (2 * bw + 1);
  hipLaunchKernelGGL(k_jband, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, n_inst, n, nq,
                     ldk, bw, inst, K, kstride, lo, sw, s, t, nodes, x, D, out, minor);
  return hipGetLastError();
}

hipError_t launch_band_lu(hipStream_t st, int n_inst, int n, const double* Jb, double* F, int* ok) {
  hipLaunchKernelGGL(k_band_lu<kPrecBand>, dim3(n_inst), dim3(64), 0, st, n_inst, n, Jb, F, ok);
  return hipGetLastError();
}

hipError_t launch_band_solve(hipStream_t st, int n_inst, int n, const double* F, const int* ok,
                             const int* act, const double* in, double* out) {
  hipLaunchKernelGGL(k_band_solve<kPrecBand>, dim3(n_inst), dim3(64), 0, st, n_inst, n, F, ok, act,
                     in, out);
  return hipGetLastError();
}

}  // namespace qdse
