// qdse_mfma.hip -- batched FP32 sweep on the matrix cores (MFMA) for many
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
// Eight products per instance, 16 N (N+1) flops. The matrices and columns are
// FP32, the products accumulate in FP32 (v_mfma_f32_16x16x4_f32); node
// functions (with the denominator t A^2 + B^2), the combination above, the
// update and the test statistic are FP64. The split form cancels where A_j ~ A_i
// near the singular diagonal of K_T, so FP32 sweeps are followed by FP64
// direct-difference sweeps (the refinement) until the FP64 test passes.
//
// Layouts (FP32, zero padded): MT[x][j][ldi], x = 0..4 (transposed so a
// lane group reads consecutive rows), C[y][j][ldb], y = 0..5; ldi and ldb are
// multiples of 32, the j extent a multiple of 4.
#include "qdse_internal.h"

namespace qdse {

namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr double kMassFloorM = 1e-8;  // GeV, as in the FP64 sweep

__global__ void k_build_m32(int n, int nq, int ldk, int ldi, const double* __restrict__ K,
                            const double* __restrict__ s_, const double* __restrict__ t_,
                            float* __restrict__ MT, size_t mstride) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)n * nq) return;
  const int j = (int)(idx / n), i = (int)(idx % n);  // i fastest: coalesced writes
  const size_t mat = (size_t)n * ldk;
  const double kT = K[(size_t)i * ldk + j], k3 = K[mat + (size_t)i * ldk + j],
               k0 = K[2 * mat + (size_t)i * ldk + j];
  const double s = s_[i], t = t_[j];
  const double k2 = (s + t) * kT;
  const size_t o = (size_t)j * ldi + i;
  MT[o] = (float)(k3 - k2);
  MT[mstride + o] = (float)(k3 + k2);
  MT[2 * mstride + o] = (float)kT;
  MT[3 * mstride + o] = (float)(k0 + 2.0 * s * kT);
  MT[4 * mstride + o] = (float)(k0 - 2.0 * s * kT);
}

// Node columns of every instance (FP64 arithmetic, FP32 results), with the
// masked-run decision of the previous sweep.
__global__ void k_nodes32(int n, int nq, int ldb, const int* __restrict__ lo,
                          const double* __restrict__ sw, const double* __restrict__ t,
                          const double* __restrict__ x, float* __restrict__ C, size_t cstride,
                          SolveState* state, const SolveCtl* ctl, int k);

__device__ inline double bits2d(unsigned long long b) { return __longlong_as_double((long long)b); }

// Masked-run decision at the start of sweep k (same rule as the FP64 sweep).
__device__ inline int decide32(SolveState* st, const SolveCtl* ctl, int k, bool writer) {
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

__global__ void k_nodes32(int n, int nq, int ldb, const int* __restrict__ lo,
                          const double* __restrict__ sw, const double* __restrict__ t,
                          const double* __restrict__ x, float* __restrict__ C, size_t cstride,
                          SolveState* state, const SolveCtl* ctl, int k) {
  const int inst = blockIdx.y;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (state && decide32(state + inst, ctl, k, blockIdx.x == 0 && threadIdx.x == 0)) return;
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
  const size_t o = (size_t)j * ldb + inst;
  C[o] = (float)(sV * Aq);
  C[cstride + o] = (float)sV;
  C[2 * cstride + o] = (float)(sS * Bq);
  C[3 * cstride + o] = (float)sS;
  C[4 * cstride + o] = (float)(sV * Bq);
  C[5 * cstride + o] = (float)(sS * Aq);
}

// One workgroup = 4 wavefronts = 32 rows x 64 instances; each wavefront owns
// 32 rows x 16 instances as two 16x16 blocks per product, eight products.
// Operands come straight from L2/L1 in the transposed layouts (a 16-lane group
// reads 64 contiguous bytes); the four wavefronts share the matrix operands.
__global__ void __launch_bounds__(256) k_mfma_sweep(
    int n_inst, int n, int nq4, int ldi, int ldb, const float* __restrict__ MT, size_t mstride,
    const float* __restrict__ C, size_t cstride, const InstDev* __restrict__ inst_,
    const double* __restrict__ s_, const double* __restrict__ x_in, double* __restrict__ x_out,
    SolveState* state, const SolveCtl* ctl, int k) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int i0 = blockIdx.x * 32;
  const int b0 = blockIdx.y * 64 + wave * 16;
  const int lr = lane & 15, lk = lane >> 4;  // operand row/col within a block, k slot
  floatx4 acc[8][2];
#pragma unroll
  for (int p = 0; p < 8; ++p) acc[p][0] = acc[p][1] = floatx4{0.f, 0.f, 0.f, 0.f};

  const float* M1 = MT;
  const float* M2 = MT + mstride;
  const float* M3 = MT + 2 * mstride;
  const float* M4 = MT + 3 * mstride;
  const float* M5 = MT + 4 * mstride;
  for (int k0 = 0; k0 < nq4; k0 += 4) {
    const size_t ra = (size_t)(k0 + lk) * ldi + i0 + lr;  // A[m][k] = MT[k][m]
    const size_t cb = (size_t)(k0 + lk) * ldb + b0 + lr;  // B[k][n] = C[k][n]
    float a1[2], a2[2], a3[2], a4[2], a5[2];
#pragma unroll
    for (int rb = 0; rb < 2; ++rb) {
      a1[rb] = M1[ra + rb * 16];
      a2[rb] = M2[ra + rb * 16];
      a3[rb] = M3[ra + rb * 16];
      a4[rb] = M4[ra + rb * 16];
      a5[rb] = M5[ra + rb * 16];
    }
    const float c0 = C[cb], c1 = C[cstride + cb], c2 = C[2 * cstride + cb],
                c3 = C[3 * cstride + cb], c4 = C[4 * cstride + cb], c5 = C[5 * cstride + cb];
#pragma unroll
    for (int rb = 0; rb < 2; ++rb) {
      acc[0][rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1[rb], c0, acc[0][rb], 0, 0, 0);
      acc[1][rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a2[rb], c1, acc[1][rb], 0, 0, 0);
      acc[2][rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a3[rb], c2, acc[2][rb], 0, 0, 0);
      acc[3][rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a3[rb], c3, acc[3][rb], 0, 0, 0);
      acc[4][rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a3[rb], c4, acc[4][rb], 0, 0, 0);
      acc[5][rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a3[rb], c1, acc[5][rb], 0, 0, 0);
      acc[6][rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a4[rb], c5, acc[6][rb], 0, 0, 0);
      acc[7][rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a5[rb], c3, acc[7][rb], 0, 0, 0);
    }
  }
  // Epilogue: the 16x16 result block holds row 4*(lane/16)+e, column lane%16.
  const int inst = b0 + lr;
  const bool inst_ok = inst < n_inst;
  int status = 1;
  InstDev P{};
  if (inst_ok) {
    status = state ? state[inst].status : 0;
    P = inst_[inst];
  }
  double worst = 0.0;
#pragma unroll
  for (int rb = 0; rb < 2; ++rb) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int i = i0 + rb * 16 + 4 * lk + e;
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
      const double p0 = acc[0][rb][e], p1 = acc[1][rb][e], p2 = acc[2][rb][e], p3 = acc[3][rb][e];
      const double p4 = acc[4][rb][e], p5 = acc[5][rb][e], p6 = acc[6][rb][e], p7 = acc[7][rb][e];
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
  }
  if (state && inst_ok && status == 0) {
    // lanes lane, lane+16, lane+32, lane+48 hold the same instance
    unsigned long long bits = (unsigned long long)__double_as_longlong(worst);
    atomicMax(&state[inst].metric[k % 3], bits);
  }
}

}  // namespace

hipError_t launch_build_m32(hipStream_t st, int n, int nq, int ldk, int ldi, const double* K,
                            const double* s, const double* t, float* MT, size_t mstride) {
  const long tot = (long)n * nq;
  hipLaunchKernelGGL(k_build_m32, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, n, nq, ldk,
                     ldi, K, s, t, MT, mstride);
  return hipGetLastError();
}

hipError_t launch_sweep_fp32(hipStream_t st, int n_inst, int n, int nq, int ldi, int ldb,
                             const float* MT, size_t mstride, float* C, size_t cstride,
                             const InstDev* inst, const int* lo, const double* sw, const double* t,
                             const double* s, const double* x_in, double* x_out,
                             SolveState* state, const SolveCtl* ctl, int k) {
  hipLaunchKernelGGL(k_nodes32, dim3((nq + 255) / 256, n_inst), dim3(256), 0, st, n, nq, ldb, lo,
                     sw, t, x_in, C, cstride, state, ctl, k);
  const int nq4 = (nq + 3) & ~3;
  hipLaunchKernelGGL(k_mfma_sweep, dim3((n + 31) / 32, (n_inst + 63) / 64), dim3(256), 0, st,
                     n_inst, n, nq4, ldi, ldb, MT, mstride, C, cstride, inst, s, x_in, x_out, state,
                     ctl, k);
  return hipGetLastError();
}

hipError_t launch_mfma_only(hipStream_t st, int n_inst, int n, int nq, int ldi, int ldb,
                            const float* MT, size_t mstride, const float* C, size_t cstride,
                            const InstDev* inst, const double* s, const double* x_in,
                            double* x_out) {
  const int nq4 = (nq + 3) & ~3;
  hipLaunchKernelGGL(k_mfma_sweep, dim3((n + 31) / 32, (n_inst + 63) / 64), dim3(256), 0, st,
                     n_inst, n, nq4, ldi, ldb, MT, mstride, C, cstride, inst, s, x_in, x_out,
                     (SolveState*)nullptr, (const SolveCtl*)nullptr, 1);
  return hipGetLastError();
}

}  // namespace qdse
