// qdse_mfma.hip -- batched sweeps on the matrix cores (MFMA) for many
// instances that share one set of angular-integrated kernel matrices (same
// grid and omega; D and m are per instance).
//
// The direct-difference form of the sweep (qdse_kernels.hip) is not a matrix
// product because each row subtracts its own A_i, B_i. Splitting every
// difference, e.g. sum_j K_ij sigma_j (B_j - B_i) = (K sigma B)_i - B_i (K sigma)_i,
// turns the sweep of b instances into products of five fixed matrices with
// node columns. With K_2 = (s_i + t_j) K_T:
//   A'_i - 1 = pref [ M1 c0 + A_i M2 c1 - 2 M3 c2 + 2 B_i M3 c3 ]_i
//   B'_i - m = pref [ M4 c5 + A_i M5 c3 - 2 s_i M3 c4 + 2 s_i B_i M3 c1 ]_i
//   M1 = K_3 - K_2, M2 = K_3 + K_2, M3 = K_T, M4 = K_0 + 2 s_i K_T,
//   M5 = K_0 - 2 s_i K_T,
//   c0 = sigma_V A(t), c1 = sigma_V, c2 = sigma_S B(t), c3 = sigma_S,
//   c4 = sigma_V B(t), c5 = sigma_S A(t)     (functions of loop node j).
// Eight products per instance, 16 N (N+1) flops.
//
// Two element types share one kernel template:
//  * FP32 (v_mfma_f32_16x16x4_f32, FP32 accumulation): the split form cancels
//    where A_j ~ A_i near the singular diagonal of K_T, so FP32 sweeps are
//    followed by FP64 sweeps (the refinement) until the FP64 test passes;
//  * FP64 (v_mfma_f64_16x16x4_f64): the same products in FP64, whose
//    cancellation error (~1e-15 relative) is far below the FP64 targets.
// Node functions (with the denominator t A^2 + B^2), the combination above,
// the update and the test statistic are FP64 in both.
//
// Tiling: a workgroup (4 wavefronts) owns 64 rows x 32 instances; per stage of
// 16 loop nodes it stages the five matrix tiles and the six column tiles in
// LDS (coalesced global reads), then each wavefront runs 16 rows x 32
// instances (two 16x16 blocks) for the eight products from LDS.
//
// Layouts (zero padded): MT[x][j][ldi] (x = 0..4, transposed: rows contiguous),
// C[y][inst][ldj] (y = 0..5, loop nodes contiguous); ldi a multiple of 64, ldj a
// multiple of 16, the instance extent a multiple of 32.
#include "qdse_internal.h"

namespace qdse {

namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

constexpr double kMassFloorM = 1e-8;  // GeV, as in the FP64 sweep
constexpr int TM = 64, TN = 32, TK = 16;
constexpr int APAD = 4;  // LDS row padding against bank conflicts

template <class T> struct Mfma;
template <> struct Mfma<float> {
  typedef floatx4 acc_t;
  __device__ static acc_t zero() { return floatx4{0.f, 0.f, 0.f, 0.f}; }
  __device__ static acc_t mac(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};
template <> struct Mfma<double> {
  typedef doublex4 acc_t;
  __device__ static acc_t zero() { return doublex4{0.0, 0.0, 0.0, 0.0}; }
  __device__ static acc_t mac(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};

template <class T>
__global__ void k_build_m(int n, int nq, int ldk, int ldi, const double* __restrict__ K,
                          const double* __restrict__ s_, const double* __restrict__ t_,
                          T* __restrict__ MT, size_t mstride) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)n * nq) return;
  const int j = (int)(idx / n), i = (int)(idx % n);  // i fastest: coalesced writes
  const size_t mat = (size_t)n * ldk;
  const double kT = K[(size_t)i * ldk + j], k3 = K[mat + (size_t)i * ldk + j],
               k0 = K[2 * mat + (size_t)i * ldk + j];
  const double s = s_[i], t = t_[j];
  const double k2 = (s + t) * kT;
  const size_t o = (size_t)j * ldi + i;
  MT[o] = (T)(k3 - k2);
  MT[mstride + o] = (T)(k3 + k2);
  MT[2 * mstride + o] = (T)kT;
  MT[3 * mstride + o] = (T)(k0 + 2.0 * s * kT);
  MT[4 * mstride + o] = (T)(k0 - 2.0 * s * kT);
}

__device__ inline double bits2d(unsigned long long b) { return __longlong_as_double((long long)b); }

// Masked-run decision at the start of sweep k (same rule as the FP64 sweep).
__device__ inline int decide_mm(SolveState* st, const SolveCtl* ctl, int k, bool writer) {
  SolveState& S = *st;
  int status = S.status;
  const int done = S.sweeps_slot[(k + 2) % 3];
  const double prev = bits2d(S.metric[(k + 2) % 3]);
  if (status == 0) {
    if (done > 0) {
      if (!(prev <= 1.7976931348623157e308)) status = 3;
      else if (prev < ctl->tol) status = 1;
    }
    if (status == 0 && done >= ctl->max_iter) status = 2;
  }
  if (writer) {
    if (status != 0 && S.status == 0) S.resid = prev;
    S.status = status;
    const int now = done + (status == 0 ? 1 : 0);
    S.sweeps_slot[k % 3] = now;
    S.sweeps = now;
    S.metric[(k + 1) % 3] = 0ull;
  }
  return status;
}

// Node columns of every instance (FP64 arithmetic, stored as T), with the
// masked-run decision of the previous sweep. Threads run over loop nodes j,
// which are contiguous in C.
template <class T>
__global__ void k_nodes_mm(int n, int nq, int ldj, const int* __restrict__ lo,
                           const double* __restrict__ sw, const double* __restrict__ t,
                           const double* __restrict__ x, T* __restrict__ C, size_t cstride,
                           SolveState* state, const SolveCtl* ctl, int k) {
  const int inst = blockIdx.y;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (state && decide_mm(state + inst, ctl, k, blockIdx.x == 0 && threadIdx.x == 0)) return;
  if (j >= nq) return;
  const double* xA = x + (size_t)inst * 2 * n;
  const int b = lo[j];
  const double* w = sw + 4 * j;
  double Aq = 0.0, Bq = 0.0;
#pragma unroll
  for (int l = 0; l < 4; ++l) {
    Aq = fma(w[l], xA[b + l], Aq);
    Bq = fma(w[l], xA[n + b + l], Bq);
  }
  const double Dl = t[j] * Aq * Aq + Bq * Bq;
  const double sV = Aq / Dl, sS = Bq / Dl;
  const size_t o = (size_t)inst * ldj + j;
  C[o] = (T)(sV * Aq);
  C[cstride + o] = (T)sV;
  C[2 * cstride + o] = (T)(sS * Bq);
  C[3 * cstride + o] = (T)sS;
  C[4 * cstride + o] = (T)(sV * Bq);
  C[5 * cstride + o] = (T)(sS * Aq);
}

template <class T>
__global__ void __launch_bounds__(256) k_mm_sweep(
    int n_inst, int n, int nq_pad, int ldi, int ldj, const T* __restrict__ MT, size_t mstride,
    const T* __restrict__ C, size_t cstride, const InstDev* __restrict__ inst_,
    const double* __restrict__ s_, const double* __restrict__ x_in, double* __restrict__ x_out,
    SolveState* state, const SolveCtl* ctl, int k) {
  typedef typename Mfma<T>::acc_t acc_t;
  __shared__ T As[5][TK][TM + APAD];
  __shared__ T Bs[6][TK][TN + APAD];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int i0 = blockIdx.x * TM;
  const int b0 = blockIdx.y * TN;
  const int lr = lane & 15, lk = lane >> 4;
  acc_t acc[8][2];
#pragma unroll
  for (int p = 0; p < 8; ++p) acc[p][0] = acc[p][1] = Mfma<T>::zero();

  for (int k0 = 0; k0 < nq_pad; k0 += TK) {
    __syncthreads();
    // stage the matrix tiles: 5 x TK x TM, rows contiguous in MT
    for (int e = tid; e < 5 * TK * TM; e += 256) {
      const int x = e / (TK * TM), r = e % (TK * TM);
      const int jj = r / TM, ii = r % TM;
      As[x][jj][ii] = MT[(size_t)x * mstride + (size_t)(k0 + jj) * ldi + i0 + ii];
    }
    // stage the column tiles: 6 x TN x TK, loop nodes contiguous in C
    for (int e = tid; e < 6 * TN * TK; e += 256) {
      const int y = e / (TN * TK), r = e % (TN * TK);
      const int nn = r / TK, jj = r % TK;
      Bs[y][jj][nn] = C[(size_t)y * cstride + (size_t)(b0 + nn) * ldj + k0 + jj];
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < TK; kk += 4) {
      const int kr = kk + lk, ar = wave * 16 + lr;
      const T a1 = As[0][kr][ar], a2 = As[1][kr][ar], a3 = As[2][kr][ar], a4 = As[3][kr][ar],
              a5 = As[4][kr][ar];
#pragma unroll
      for (int cb = 0; cb < 2; ++cb) {
        const int bc = cb * 16 + lr;
        const T c0 = Bs[0][kr][bc], c1 = Bs[1][kr][bc], c2 = Bs[2][kr][bc], c3 = Bs[3][kr][bc],
                c4 = Bs[4][kr][bc], c5 = Bs[5][kr][bc];
        acc[0][cb] = Mfma<T>::mac(a1, c0, acc[0][cb]);
        acc[1][cb] = Mfma<T>::mac(a2, c1, acc[1][cb]);
        acc[2][cb] = Mfma<T>::mac(a3, c2, acc[2][cb]);
        acc[3][cb] = Mfma<T>::mac(a3, c3, acc[3][cb]);
        acc[4][cb] = Mfma<T>::mac(a3, c4, acc[4][cb]);
        acc[5][cb] = Mfma<T>::mac(a3, c1, acc[5][cb]);
        acc[6][cb] = Mfma<T>::mac(a4, c5, acc[6][cb]);
        acc[7][cb] = Mfma<T>::mac(a5, c3, acc[7][cb]);
      }
    }
  }
  // Epilogue: each 16x16 result block holds row 4*(lane/16)+e, column lane%16.
#pragma unroll
  for (int cb = 0; cb < 2; ++cb) {
    const int inst = b0 + cb * 16 + lr;
    const bool inst_ok = inst < n_inst;
    int status = 1;
    InstDev P{};
    if (inst_ok) {
      status = state ? state[inst].status : 0;
      P = inst_[inst];
    }
    double worst = 0.0;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int i = i0 + wave * 16 + 4 * lk + e;
      if (!inst_ok || i >= n) continue;
      const double* xi = x_in + (size_t)inst * 2 * n;
      double* xo = x_out + (size_t)inst * 2 * n;
      const double Ai = xi[i], Bi = xi[n + i];
      if (status != 0) {
        xo[i] = Ai;
        xo[n + i] = Bi;
        continue;
      }
      const double s = s_[i];
      const double p0 = acc[0][cb][e], p1 = acc[1][cb][e], p2 = acc[2][cb][e], p3 = acc[3][cb][e];
      const double p4 = acc[4][cb][e], p5 = acc[5][cb][e], p6 = acc[6][cb][e], p7 = acc[7][cb][e];
      const double An = 1.0 + P.pref * (p0 + Ai * p1 - 2.0 * p2 + 2.0 * Bi * p3);
      const double Bn = P.m + P.pref * (p6 + Ai * p7 - 2.0 * s * p4 + 2.0 * s * Bi * p5);
      xo[i] = An;
      xo[n + i] = Bn;
      if (state) {
        double r;
        const double dA = fabs(An - Ai);
        if (ctl->mode == QDSE_CONV_ABS) {
          r = fmax(dA, fabs(Bn - Bi));
        } else {
          const double Mn = Bn / An, Mo = Bi / Ai;
          r = fmax(dA, fabs(Mn - Mo) / fmax(fabs(Mn), kMassFloorM));
        }
        worst = (isnan(r) || isnan(worst)) ? __longlong_as_double(0x7ff8000000000000ll)
                                            : fmax(worst, r);
      }
    }
    if (state && inst_ok && status == 0) {
      // lanes lr, lr+16, lr+32, lr+48 hold the same instance
      const unsigned long long bits = (unsigned long long)__double_as_longlong(worst);
      atomicMax(&state[inst].metric[k % 3], bits);
    }
  }
}

}  // namespace

MmLayout mm_layout(int n, int nq, int n_inst) {
  MmLayout L;
  L.nq_pad = (nq + TK - 1) / TK * TK;
  L.ldi = (n + TM - 1) / TM * TM;
  L.ldj = L.nq_pad;
  L.inst_pad = (n_inst + TN - 1) / TN * TN;
  L.mstride = (size_t)L.nq_pad * L.ldi;
  L.cstride = (size_t)L.inst_pad * L.ldj;
  return L;
}

template <class T>
hipError_t launch_build_mm(hipStream_t st, int n, int nq, int ldk, const MmLayout& L,
                           const double* K, const double* s, const double* t, T* MT) {
  const long tot = (long)n * nq;
  hipLaunchKernelGGL(k_build_m<T>, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, n, nq,
                     ldk, L.ldi, K, s, t, MT, L.mstride);
  return hipGetLastError();
}

template <class T>
hipError_t launch_sweep_mm(hipStream_t st, int n_inst, int n, int nq, const MmLayout& L,
                           const T* MT, T* C, const InstDev* inst, const int* lo, const double* sw,
                           const double* t, const double* s, const double* x_in, double* x_out,
                           SolveState* state, const SolveCtl* ctl, int k, bool nodes) {
  if (nodes)
    hipLaunchKernelGGL(k_nodes_mm<T>, dim3((nq + 255) / 256, n_inst), dim3(256), 0, st, n, nq,
                       L.ldj, lo, sw, t, x_in, C, L.cstride, state, ctl, k);
  hipLaunchKernelGGL(k_mm_sweep<T>, dim3(L.ldi / TM, L.inst_pad / TN), dim3(256), 0, st, n_inst, n,
                     L.nq_pad, L.ldi, L.ldj, MT, L.mstride, C, L.cstride, inst, s, x_in, x_out,
                     state, ctl, k);
  return hipGetLastError();
}

template hipError_t launch_build_mm<float>(hipStream_t, int, int, int, const MmLayout&,
                                           const double*, const double*, const double*, float*);
template hipError_t launch_build_mm<double>(hipStream_t, int, int, int, const MmLayout&,
                                            const double*, const double*, const double*, double*);
template hipError_t launch_sweep_mm<float>(hipStream_t, int, int, int, const MmLayout&,
                                           const float*, float*, const InstDev*, const int*,
                                           const double*, const double*, const double*,
                                           const double*, double*, SolveState*, const SolveCtl*,
                                           int, bool);
template hipError_t launch_sweep_mm<double>(hipStream_t, int, int, int, const MmLayout&,
                                            const double*, double*, const InstDev*, const int*,
                                            const double*, const double*, const double*,
                                            const double*, double*, SolveState*, const SolveCtl*,
                                            int, bool);

}  // namespace qdse
