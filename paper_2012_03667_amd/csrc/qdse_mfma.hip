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
//    where A_j ~ A_i near the singular diagonal of K_T (~1e-5 relative), so
//    a solve contracts in FP32 only the node-column differences from a
//    reference iterate, whose products an FP64 sweep stores (the rounding
//    error then scales with the differences; see k_mm_sweep);
//  * FP64 (v_mfma_f64_16x16x4_f64): the same products in FP64, whose
//    cancellation error (~1e-15 relative) is far below the FP64 targets.
// Node functions (with the denominator t A^2 + B^2), the combination above,
// the update and the test statistic are FP64 in both.
//
// Tiling: a workgroup of four wavefronts owns 32 rows x 32 instances: two row
// groups of 16 rows (they read the same node-column panel, the second read
// served from the CU's L1), each split over the loop nodes in two halves
// (four quarters, with eight wavefronts, when the grid underfills the device)
// whose partial products are added through LDS before the FP64 epilogue; a
// wavefront accumulates 16 rows x 32 instances in blocks of 16 x 16, eight
// products each (one 16-row block per wavefront measured fastest for both
// element types; four row groups per workgroup measured no faster). Operands
// are read straight from L2/L1 in layouts where a 16-lane group reads one
// contiguous run, with the following k-steps prefetched.
//
// Layouts (zero padded), VW loop nodes per lane and load (FP32 1, FP64 2):
// MT[x][j / VW][ldi][j % VW] (x = 0..4), C[y][j / VW][ldb][j % VW]
// (y = 0..5); ldi and ldb multiples of 32, the loop-node extent nq_pad a
// multiple of 16. For FP64 a lane's two loop nodes come with one 16-byte
// load (83-85 against 88 us per 1024-instance contraction); FP32 with two
// nodes per load measured slower (59.5 against 56 us) and keeps one.
#include "qdse_internal.h"

namespace qdse {

namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

constexpr double kMassFloorM = 1e-8;  // GeV, as in the FP64 sweep
constexpr int TM_MAX = 32, TN = 32, KSPLIT = 2, KSTEP = 4;
// When the grid underfills the device: k-steps in flight, and the loop nodes
// split four ways between the wavefronts of a row group instead of two (8
// grid classes of 117-142 instances: FP32 + refinement 6.37 -> 5.72 ms, FP64
// 6.24 -> 5.00 ms; at 1024 instances four ways measured slower, FP32 61
// against 56 us and FP64 109 against 83 us). kMinGroupsDeep: load groups a
// quarter of the loop nodes must hold for the four-way split.
constexpr int kDeepPD = 2, kDeepKS = 4, kMinGroupsDeep = 4;

template <class T> struct Mfma;
// Output layout of one 16x16 block: register e of lane l holds row
// row(l / 16, e), column l % 16 (FP32: 4 (l/16) + e; FP64: l/16 + 4 e).
// PD: k-steps of operands in flight ahead of the running one, in rotating
// register sets; 0: the next step's operands load into a staging set that is
// copied after the step (measured faster for FP32 at three wavefronts per
// SIMD: 56 against 70-75 us at 1024 instances; FP64, one wavefront per SIMD,
// gains from two steps in flight: 88 against 92 us). This is the depth for a
// grid that fills the device; with fewer workgroups than compute units (small
// batches) a wavefront's load latency is exposed and FP32 also takes two
// steps in flight (kDeepPD; 8 grid classes of 117-142 instances: batch
// 7.36 -> 6.43 ms).
// VW: consecutive loop nodes a lane reads with one load (its k values of VW
// successive MFMA steps).
typedef float floatx1 __attribute__((ext_vector_type(1)));
typedef double doublex2 __attribute__((ext_vector_type(2)));
template <> struct Mfma<float> {
  typedef floatx4 acc_t;
  typedef floatx1 vec_t;
  static constexpr int RB = 1;  // 16-row blocks per wavefront
  static constexpr int PD = 0;
  static constexpr int VW = 1;
  __device__ static int row(int g, int e) { return 4 * g + e; }
  __device__ static acc_t zero() { return floatx4{0.f, 0.f, 0.f, 0.f}; }
  __device__ static acc_t mac(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};
template <> struct Mfma<double> {
  typedef doublex4 acc_t;
  typedef doublex2 vec_t;
  static constexpr int RB = 1;
  static constexpr int PD = 2;
  static constexpr int VW = 2;
  __device__ static int row(int g, int e) { return g + 4 * e; }
  __device__ static acc_t zero() { return doublex4{0.0, 0.0, 0.0, 0.0}; }
  __device__ static acc_t mac(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};

template <class T>
__global__ void k_build_m(int n, int nq, int ldk, int ldi, const double* __restrict__ K,
                          const double* __restrict__ s_, const double* __restrict__ t_,
                          T* __restrict__ MT, size_t mstride) {
  constexpr int VW = Mfma<T>::VW;
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long nqv = (long)(nq + VW - 1) / VW * VW;
  if (idx >= (long)n * nqv) return;
  // stored order: loop-node block, row, node within the block (coalesced writes)
  const int jv = (int)(idx % VW), i = (int)((idx / VW) % n), j = (int)(idx / ((long)VW * n)) * VW + jv;
  if (j >= nq) return;
  const size_t mat = (size_t)n * ldk;
  const double kT = K[(size_t)i * ldk + j], k3 = K[mat + (size_t)i * ldk + j],
               k0 = K[2 * mat + (size_t)i * ldk + j];
  const double s = s_[i], t = t_[j];
  const double k2 = (s + t) * kT;
  const size_t o = ((size_t)(j / VW) * ldi + i) * VW + jv;
  MT[o] = (T)(k3 - k2);
  MT[mstride + o] = (T)(k3 + k2);
  MT[2 * mstride + o] = (T)kT;
  MT[3 * mstride + o] = (T)(k0 + 2.0 * s * kT);
  MT[4 * mstride + o] = (T)(k0 - 2.0 * s * kT);
}

__device__ inline double bits2d(unsigned long long b) { return __longlong_as_double((long long)b); }

// The statistic of one sweep slot: the max over its lanes.
__device__ inline unsigned long long slot_max(const SolveState& S, int slot) {
  unsigned long long m = S.metric[slot][0];
#pragma unroll
  for (int l = 1; l < kMetricLanes; ++l) m = S.metric[slot][l] > m ? S.metric[slot][l] : m;
  return m;
}

// Masked-run decision at the start of sweep k (same rule as the FP64 sweep).
__device__ inline int decide_mm(SolveState* st, const SolveCtl* ctl, int k, bool writer) {
  SolveState& S = *st;
  int status = S.status;
  const int done = S.sweeps_slot[(k + 2) % 3];
  const double prev = bits2d(slot_max(S, (k + 2) % 3));
  if (status == 0) {
    if (done > 0) {
      if (!(prev <= 1.7976931348623157e308)) status = 3;
      else if (prev < ctl->tol) status = 1;
    }
    if (status == 0 && done >= ctl->max_iter) status = 2;
  }
  if (writer) {
    const unsigned long long before = slot_max(S, (k + 1) % 3);  // sweep k-2, cleared below
    if (status != 0 && S.status == 0) S.resid = prev;
    S.status = status;
    const int now = done + (status == 0 ? 1 : 0);
    S.sweeps_slot[k % 3] = now;
    S.sweeps = now;
#pragma unroll
    for (int l = 0; l < kMetricLanes; ++l) S.metric[(k + 1) % 3][l] = 0ull;
    if (ctl->mirror && k % 6 == 0) {  // host mirror (see SolveCtl)
      SolveState* m = ctl->mirror + (st - ctl->base);
      m->sweeps = now;
      m->resid = S.resid;
      m->metric[0][0] = slot_max(S, (k + 2) % 3);
      m->metric[1][0] = before;
      m->status = status;
    }
  }
  return status;
}

// Node columns of every instance (FP64 arithmetic, stored as T), with the
// masked-run decision of the previous sweep. A block covers 32 loop nodes x
// 32 instances: threads compute with j fastest (the interpolation stencils
// read the iterate contiguously), the six columns pass through LDS, and the
// stores run in C's order (contiguous runs of 32 VW values). With x_ref, the
// columns are the differences c(x) - c(x_ref), formed in FP64 before the
// conversion to T.
template <class T>
__global__ void __launch_bounds__(256) k_nodes_mm(int n_inst, int n, int nq, int ldb,
                                                  const int* __restrict__ lo,
                                                  const double* __restrict__ sw,
                                                  const double* __restrict__ t,
                                                  const double* __restrict__ x,
                                                  const double* __restrict__ x_ref,
                                                  T* __restrict__ C, size_t cstride,
                                                  SolveState* state, const SolveCtl* ctl, int k) {
  __shared__ T tile[6][32][33];
  __shared__ int frozen[32];
  const int j0 = blockIdx.x * 32, b0 = blockIdx.y * 32;
  const int tid = threadIdx.x;
  if (tid < 32) {
    const int inst = b0 + tid;
    int st = 1;
    if (inst < n_inst)
      st = state ? decide_mm(state + inst, ctl, k, blockIdx.x == 0) : 0;
    frozen[tid] = st;
  }
  __syncthreads();
  for (int e = tid; e < 32 * 32; e += 256) {
    const int jj = e % 32, bb = e / 32;
    const int j = j0 + jj, inst = b0 + bb;
    if (j >= nq || inst >= n_inst || frozen[bb]) continue;
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
    double cy[6] = {sV * Aq, sV, sS * Bq, sS, sV * Bq, sS * Aq};
    if (x_ref) {
      const double* xR = x_ref + (size_t)inst * 2 * n;
      double Ar = 0.0, Br = 0.0;
#pragma unroll
      for (int l = 0; l < 4; ++l) {
        Ar = fma(w[l], xR[b + l], Ar);
        Br = fma(w[l], xR[n + b + l], Br);
      }
      const double Dr = t[j] * Ar * Ar + Br * Br;
      const double rV = Ar / Dr, rS = Br / Dr;
      const double cr[6] = {rV * Ar, rV, rS * Br, rS, rV * Br, rS * Ar};
#pragma unroll
      for (int y = 0; y < 6; ++y) cy[y] -= cr[y];
    }
#pragma unroll
    for (int y = 0; y < 6; ++y) tile[y][bb][jj] = (T)cy[y];
  }
  __syncthreads();
  // stored order C[y][j / VW][inst][j % VW]: node within the block fastest,
  // then instance (contiguous runs of 32 VW values)
  constexpr int VW = Mfma<T>::VW;
  for (int e = tid; e < 32 * 32; e += 256) {
    const int jv = e % VW, bb = (e / VW) % 32, jj = (e / (VW * 32)) * VW + jv;
    const int j = j0 + jj, inst = b0 + bb;
    if (j >= nq || inst >= n_inst || frozen[bb]) continue;
    const size_t o = ((size_t)(j / VW) * ldb + inst) * VW + jv;
#pragma unroll
    for (int y = 0; y < 6; ++y) C[(size_t)y * cstride + o] = tile[y][bb][jj];
  }
}

// RH: row groups of 16 rows per workgroup (they share the node-column panel);
// 1 or 2, chosen per context (MmLayout::rh, qdse_autotune). PD: k-steps of
// operands in flight (Mfma<T>::PD, or kDeepPD for a grid smaller than the
// device). KS: wavefronts per row group, each taking a contiguous range of
// whole load groups of the loop nodes (KSPLIT, or kDeepKS for a small grid);
// their partial products are added in the fixed order 0 + 1 + ... + KS-1.
// Refinement by differences: rq_out (FP64 sweep at the reference iterate)
// receives, per row and instance, the six coefficients that make the update
// affine in the row's own A_i, B_i at the reference products P:
//   A' = a0 + A_i a1 + B_i a2,  a0 = 1 + pref (P0 - 2 P2), a1 = pref P1,
//   a2 = 2 pref P3;  B' = b0 + A_i b1 + B_i b2,  b0 = m + pref (P6 - 2 s_i P4),
//   b1 = pref P7, b2 = 2 s_i pref P5,
// stored rq[v][i][ldb] (v = a0 a1 a2 b0 b1 b2), and with xr_out the row's
// input A_i, B_i into xr_out (the new reference iterate). With rq (node columns of
// differences from the reference), the products p of the differences are
// added: A' = a0 + A_i a1 + B_i a2 + pref (p0 + A_i p1 - 2 p2 + 2 B_i p3), and
// likewise B'. This is the same map, with T's rounding error now scaled by
// the size of the differences instead of the columns themselves.
template <class T, int RH, int PD, int KS>
__global__ void __launch_bounds__(64 * KS * RH) k_mm_sweep(
    int n_inst, int n, int nq_pad, int ldi, int ldb, const T* __restrict__ MT, size_t mstride,
    const T* __restrict__ C, size_t cstride, const InstDev* __restrict__ inst_,
    const double* __restrict__ s_, const double* __restrict__ x_in, double* __restrict__ x_out,
    SolveState* state, const SolveCtl* ctl, int k, const double* __restrict__ rq,
    double* __restrict__ rq_out, double* __restrict__ xr_out) {
  typedef typename Mfma<T>::acc_t acc_t;
  constexpr int RB = Mfma<T>::RB, TM = 16 * RB;
  __shared__ acc_t part[RH][8][RB][2][64];  // partial products of the second K half
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform: scalar loop
  const int kh = wave % KS, rh = wave / KS;
  // XCD-aware order: workgroups are dispatched round-robin over the 8 XCDs
  // (workgroup w to XCD w % 8). When the instance blocks divide evenly, XCD x
  // owns the instance blocks ib = x (mod 8) and walks their row blocks, so a
  // node-column panel is fetched into one XCD's L2 and reused from there.
  const int n_rb = ldi / (TM * RH), n_ib = ldb / TN;
  const int w = blockIdx.x;
  int rb, ib;
  if (n_ib % 8 == 0) {
    const int xcd = w % 8, kth = w / 8;
    ib = (kth / n_rb) * 8 + xcd;
    rb = kth % n_rb;
  } else {
    rb = w % n_rb;
    ib = w / n_rb;
  }
  const int ib0 = rb * TM * RH;  // first row of the workgroup
  const int i0 = ib0 + rh * TM, b0 = ib * TN;
  if (state) {
    // every instance of this column block frozen (or absent): carry the
    // iterate along and skip the contraction (all wavefronts agree)
    bool frozen = true;
    if (lane < TN) frozen = b0 + lane >= n_inst || state[b0 + lane].status != 0;
    if (__all(frozen)) {
      for (int e = threadIdx.x; e < TM * RH * TN; e += 64 * KS * RH) {
        const int inst = b0 + e / (TM * RH), i = ib0 + e % (TM * RH);
        if (inst < n_inst && i < n) {
          const size_t o = (size_t)inst * 2 * n;
          x_out[o + i] = x_in[o + i];
          x_out[o + n + i] = x_in[o + n + i];
        }
      }
      return;
    }
  }
  const int lr = lane & 15, lk = lane >> 4;
  constexpr int VW = Mfma<T>::VW, KG = KSTEP * VW;  // loop nodes per load group
  typedef typename Mfma<T>::vec_t vec_t;
  int kb, ke;
  if constexpr (KS == 2) {
    const int half = nq_pad / 2;  // a multiple of KG
    kb = kh * half;
    ke = kb + half;
  } else {
    const int ng = nq_pad / KG;  // load groups
    kb = (kh * ng / KS) * KG;
    ke = ((kh + 1) * ng / KS) * KG;
  }
  acc_t acc[8][RB][2];
#pragma unroll
  for (int p = 0; p < 8; ++p)
#pragma unroll
    for (int r = 0; r < RB; ++r) acc[p][r][0] = acc[p][r][1] = Mfma<T>::zero();
  const T* M1 = MT;
  const T* M2 = MT + mstride;
  const T* M3 = MT + 2 * mstride;
  const T* M4 = MT + 3 * mstride;
  const T* M5 = MT + 4 * mstride;
  // operand sets of PD + 1 consecutive k-steps (two for PD = 0), used in
  // rotation (indices known at compile time, so the sets stay in registers)
  vec_t a[PD + 1 + (PD == 0)][5][RB], c[PD + 1 + (PD == 0)][6][2];
  // One load group: lane (lk, lr) reads loop nodes k0 + VW lk .. + VW - 1 of
  // row i0 + lr (A = MT[x][k / VW][row][k % VW]) and of instance b0 + lr
  // (B = C[y][k / VW][inst][k % VW]): 16 lanes read one contiguous run; MFMA
  // step v of the group then takes k = k0 + VW lk + v in both operands.
  auto load = [&](int k0, vec_t (&A)[5][RB], vec_t (&B)[6][2]) {
    const size_t ra = ((size_t)(k0 / VW + lk) * ldi + i0 + lr) * VW;
    const size_t rc = ((size_t)(k0 / VW + lk) * ldb + b0 + lr) * VW;
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      const size_t o = ra + (size_t)16 * r * VW;
      A[0][r] = *(const vec_t*)(M1 + o);
      A[1][r] = *(const vec_t*)(M2 + o);
      A[2][r] = *(const vec_t*)(M3 + o);
      A[3][r] = *(const vec_t*)(M4 + o);
      A[4][r] = *(const vec_t*)(M5 + o);
    }
#pragma unroll
    for (int y = 0; y < 6; ++y)
#pragma unroll
      for (int cb = 0; cb < 2; ++cb)
        B[y][cb] = *(const vec_t*)(C + (size_t)y * cstride + rc + (size_t)16 * cb * VW);
  };
  auto mma = [&](const vec_t (&A)[5][RB], const vec_t (&B)[6][2]) {
#pragma unroll
    for (int v = 0; v < VW; ++v)
#pragma unroll
      for (int r = 0; r < RB; ++r)
#pragma unroll
        for (int cb = 0; cb < 2; ++cb) {
          acc[0][r][cb] = Mfma<T>::mac(A[0][r][v], B[0][cb][v], acc[0][r][cb]);
          acc[1][r][cb] = Mfma<T>::mac(A[1][r][v], B[1][cb][v], acc[1][r][cb]);
          acc[2][r][cb] = Mfma<T>::mac(A[2][r][v], B[2][cb][v], acc[2][r][cb]);
          acc[3][r][cb] = Mfma<T>::mac(A[2][r][v], B[3][cb][v], acc[3][r][cb]);
          acc[4][r][cb] = Mfma<T>::mac(A[2][r][v], B[4][cb][v], acc[4][r][cb]);
          acc[5][r][cb] = Mfma<T>::mac(A[2][r][v], B[1][cb][v], acc[5][r][cb]);
          acc[6][r][cb] = Mfma<T>::mac(A[3][r][v], B[5][cb][v], acc[6][r][cb]);
          acc[7][r][cb] = Mfma<T>::mac(A[4][r][v], B[3][cb][v], acc[7][r][cb]);
        }
  };
  // software pipeline
  if constexpr (PD == 0) {
    // one step ahead through the staging set a[1], c[1], copied after each
    // step; the last step is peeled so the loop body has no branch
    load(kb, a[0], c[0]);
    for (int k0 = kb; k0 + KG < ke; k0 += KG) {
      load(k0 + KG, a[1], c[1]);
      mma(a[0], c[0]);
#pragma unroll
      for (int q = 0; q < 5; ++q)
#pragma unroll
        for (int r = 0; r < RB; ++r) a[0][q][r] = a[1][q][r];
#pragma unroll
      for (int q = 0; q < 6; ++q) c[0][q][0] = c[1][q][0], c[0][q][1] = c[1][q][1];
    }
    mma(a[0], c[0]);
  } else {
    // while step j runs, the operands of steps j + 1 .. j + PD are in flight;
    // step j uses set j mod (PD + 1) and the load of step j + PD goes to the
    // set step j - 1 used, so no register is copied (a copy would wait for
    // the load it copies)
    const int nst = (ke - kb) / KG;
#pragma unroll
    for (int p = 0; p < PD; ++p)
      if (p < nst) load(kb + p * KG, a[p], c[p]);
    int j0 = 0;
    for (; j0 + 2 * PD < nst; j0 += PD + 1) {
#pragma unroll
      for (int p = 0; p <= PD; ++p) {
        load(kb + (j0 + p + PD) * KG, a[(p + PD) % (PD + 1)], c[(p + PD) % (PD + 1)]);
        mma(a[p], c[p]);
      }
    }
#pragma unroll
    for (int p = 0; p <= 2 * PD; ++p) {
      const int j = j0 + p;
      if (j < nst) {
        if (j + PD < nst)
          load(kb + (j + PD) * KG, a[(p + PD) % (PD + 1)], c[(p + PD) % (PD + 1)]);
        mma(a[p % (PD + 1)], c[p % (PD + 1)]);
      }
    }
  }
  // add the other ranges' partial products, one range at a time through the
  // same LDS buffer (fixed order: range 0 + 1 + ... + KS-1)
  if constexpr (KS == 2) {
    if (kh == 1) {
#pragma unroll
      for (int p = 0; p < 8; ++p)
#pragma unroll
        for (int r = 0; r < RB; ++r)
#pragma unroll
          for (int cb = 0; cb < 2; ++cb) part[rh][p][r][cb][lane] = acc[p][r][cb];
    }
    __syncthreads();
    if (kh == 1) return;
#pragma unroll
    for (int p = 0; p < 8; ++p)
#pragma unroll
      for (int r = 0; r < RB; ++r)
#pragma unroll
        for (int cb = 0; cb < 2; ++cb) acc[p][r][cb] += part[rh][p][r][cb][lane];
  } else {
  for (int h = 1; h < KS; ++h) {
    if (kh == h) {
#pragma unroll
      for (int p = 0; p < 8; ++p)
#pragma unroll
        for (int r = 0; r < RB; ++r)
#pragma unroll
          for (int cb = 0; cb < 2; ++cb) part[rh][p][r][cb][lane] = acc[p][r][cb];
    }
    __syncthreads();
    if (kh == 0) {
#pragma unroll
      for (int p = 0; p < 8; ++p)
#pragma unroll
        for (int r = 0; r < RB; ++r)
#pragma unroll
          for (int cb = 0; cb < 2; ++cb) acc[p][r][cb] += part[rh][p][r][cb][lane];
    }
    if (h + 1 < KS) __syncthreads();  // before range h + 1 overwrites the buffer
  }
  if (kh != 0) return;
  }
  // Epilogue (FP64)
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
    for (int r = 0; r < RB; ++r) {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int i = i0 + 16 * r + Mfma<T>::row(lk, e);
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
        const double p0 = acc[0][r][cb][e], p1 = acc[1][r][cb][e], p2 = acc[2][r][cb][e],
                     p3 = acc[3][r][cb][e], p4 = acc[4][r][cb][e], p5 = acc[5][r][cb][e],
                     p6 = acc[6][r][cb][e], p7 = acc[7][r][cb][e];
        double An, Bn;
        if (rq) {
          const size_t vs = (size_t)ldi * ldb, o = (size_t)i * ldb + inst;
          An = rq[o] + Ai * rq[vs + o] + Bi * rq[2 * vs + o] +
               P.pref * (p0 + Ai * p1 - 2.0 * p2 + 2.0 * Bi * p3);
          Bn = rq[3 * vs + o] + Ai * rq[4 * vs + o] + Bi * rq[5 * vs + o] +
               P.pref * (p6 + Ai * p7 - 2.0 * s * p4 + 2.0 * s * Bi * p5);
        } else {
          An = 1.0 + P.pref * (p0 + Ai * p1 - 2.0 * p2 + 2.0 * Bi * p3);
          Bn = P.m + P.pref * (p6 + Ai * p7 - 2.0 * s * p4 + 2.0 * s * Bi * p5);
          if (rq_out) {
            const size_t vs = (size_t)ldi * ldb, o = (size_t)i * ldb + inst;
            rq_out[o] = 1.0 + P.pref * (p0 - 2.0 * p2);
            rq_out[vs + o] = P.pref * p1;
            rq_out[2 * vs + o] = 2.0 * P.pref * p3;
            rq_out[3 * vs + o] = P.m + P.pref * (p6 - 2.0 * s * p4);
            rq_out[4 * vs + o] = P.pref * p7;
            rq_out[5 * vs + o] = 2.0 * s * P.pref * p5;
            if (xr_out) {
              xr_out[(size_t)inst * 2 * n + i] = Ai;
              xr_out[(size_t)inst * 2 * n + n + i] = Bi;
            }
          }
        }
        xo[i] = An;
        xo[n + i] = Bn;
        if (state) {
          double rr;
          const double dA = fabs(An - Ai);
          if (ctl->mode == QDSE_CONV_ABS) {
            rr = fmax(dA, fabs(Bn - Bi));
          } else {
            const double Mn = Bn / An, Mo = Bi / Ai;
            rr = fmax(dA, fabs(Mn - Mo) / fmax(fabs(Mn), kMassFloorM));
          }
          worst = (isnan(rr) || isnan(worst)) ? __longlong_as_double(0x7ff8000000000000ll)
                                              : fmax(worst, rr);
        }
      }
    }
    if (state) {
      // lanes lr, lr+16, lr+32, lr+48 hold the same instance: maximum of the
      // statistic bits (NaN above +inf) over them, then one atomic
      unsigned long long bits = (unsigned long long)__double_as_longlong(worst);
      unsigned long long o = __shfl_xor(bits, 16, 64);
      bits = o > bits ? o : bits;
      o = __shfl_xor(bits, 32, 64);
      bits = o > bits ? o : bits;
      if (lk == 0 && inst_ok && status == 0)
        atomicMax(&state[inst].metric[k % 3][blockIdx.x % kMetricLanes], bits);
    }
  }
}

}  // namespace

MmLayout mm_layout(int n, int nq, int n_inst) {
  MmLayout L;
  // each K half a whole number of load groups of either element type
  constexpr int Q = KSPLIT * KSTEP * (Mfma<float>::VW > Mfma<double>::VW ? Mfma<float>::VW
                                                                          : Mfma<double>::VW);
  L.nq_pad = (nq + Q - 1) / Q * Q;
  L.ldi = (n + TM_MAX - 1) / TM_MAX * TM_MAX;
  L.ldb = (n_inst + TN - 1) / TN * TN;
  L.mstride = (size_t)L.nq_pad * L.ldi;
  L.cstride = (size_t)L.nq_pad * L.ldb;
  return L;
}

template <class T>
hipError_t launch_build_mm(hipStream_t st, int n, int nq, int ldk, const MmLayout& L,
                           const double* K, const double* s, const double* t, T* MT) {
  const long tot = (long)n * ((nq + Mfma<T>::VW - 1) / Mfma<T>::VW * Mfma<T>::VW);
  hipLaunchKernelGGL(k_build_m<T>, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, n, nq,
                     ldk, L.ldi, K, s, t, MT, L.mstride);
  return hipGetLastError();
}

template <class T>
hipError_t launch_sweep_mm(hipStream_t st, int n_inst, int n, int nq, const MmLayout& L,
                           const T* MT, T* C, const InstDev* inst, const int* lo, const double* sw,
                           const double* t, const double* s, const double* x_in, double* x_out,
                           SolveState* state, const SolveCtl* ctl, int k, bool nodes,
                           hipEvent_t ev0, hipEvent_t ev1, const MmDelta* delta) {
  const double* x_ref = delta ? delta->x_ref : nullptr;
  const double* rq = delta ? delta->rq : nullptr;
  double* rq_out = delta ? delta->rq_out : nullptr;
  double* xr_out = delta ? delta->x_ref_out : nullptr;
  if ((x_ref == nullptr) != (rq == nullptr) || (rq && rq_out) || (xr_out && !rq_out) ||
      (xr_out && (xr_out == x_in || xr_out == x_out)))
    return hipErrorInvalidValue;
  if (nodes)
    hipLaunchKernelGGL(k_nodes_mm<T>, dim3((nq + 31) / 32, L.ldb / 32), dim3(256), 0, st, n_inst,
                       n, nq, L.ldb, lo, sw, t, x_in, x_ref, C, L.cstride, state, ctl, k);
  auto launch = [&](auto kern, int RH, int KS) {
    const dim3 grid((L.ldi / (16 * Mfma<T>::RB * RH)) * (L.ldb / TN));
    if (ev0)
      hipExtLaunchKernelGGL(kern, grid, dim3(64 * KS * RH), 0, st, ev0, ev1, 0, n_inst, n,
                            L.nq_pad, L.ldi, L.ldb, MT, L.mstride, (const T*)C, L.cstride, inst, s,
                            x_in, x_out, state, ctl, k, rq, rq_out, xr_out);
    else
      hipLaunchKernelGGL(kern, grid, dim3(64 * KS * RH), 0, st, n_inst, n, L.nq_pad, L.ldi,
                         L.ldb, MT, L.mstride, (const T*)C, L.cstride, inst, s, x_in, x_out, state,
                         ctl, k, rq, rq_out, xr_out);
  };
  const int RH = L.rh == 1 ? 1 : 2;
  const bool deep = (L.ldi / (16 * Mfma<T>::RB * RH)) * (L.ldb / TN) < L.cus;
  const bool split4 =
      deep && L.nq_pad / (KSTEP * Mfma<T>::VW) >= kDeepKS * kMinGroupsDeep;
  if (RH == 1) {
    if (split4)
      launch(k_mm_sweep<T, 1, kDeepPD, kDeepKS>, 1, kDeepKS);
    else if (deep)
      launch(k_mm_sweep<T, 1, kDeepPD, KSPLIT>, 1, KSPLIT);
    else
      launch(k_mm_sweep<T, 1, Mfma<T>::PD, KSPLIT>, 1, KSPLIT);
  } else {
    if (split4)
      launch(k_mm_sweep<T, 2, kDeepPD, kDeepKS>, 2, kDeepKS);
    else if (deep)
      launch(k_mm_sweep<T, 2, kDeepPD, KSPLIT>, 2, KSPLIT);
    else
      launch(k_mm_sweep<T, 2, Mfma<T>::PD, KSPLIT>, 2, KSPLIT);
  }
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
                                           int, bool, hipEvent_t, hipEvent_t, const MmDelta*);
template hipError_t launch_sweep_mm<double>(hipStream_t, int, int, int, const MmLayout&,
                                            const double*, double*, const InstDev*, const int*,
                                            const double*, const double*, const double*,
                                            const double*, double*, SolveState*, const SolveCtl*,
                                            int, bool, hipEvent_t, hipEvent_t, const MmDelta*);

}  // namespace qdse
