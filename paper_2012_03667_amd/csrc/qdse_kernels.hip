// qdse_kernels.hip -- gfx950 kernels of the Ball-Chiu quark gap-equation
// solver (arXiv:2012.03667, Sec. II eqs. dsesys/dsesys2, Sec. III).
//
// Every sweep of the successive approximation evaluates, for each external
// node p^2 = s_i, a radial x angular Gauss-Legendre sum over loop nodes
// q^2 = t_j and angles z_a. Nothing in the angular sum depends on the unknowns
// A, B, so it is done once per (grid, omega) by k_precompute; a sweep is then
// an O(N^2) contraction of three angular-integrated matrices with per-loop-node
// functions of the interpolated A(t_j), B(t_j).
//
// Angular algebra. With r = sqrt(s t), k^2 = (sqrt s - sqrt t)^2 + 2 r (1 - z)
// and P = p + q, the transverse projector of the Landau-gauge gluon makes the
// bracketed factors of eq. dsesys2 collapse to
//   I_A1 factor  2 t (1-z^2)/k^2,           I_A2 factor  t (s+t)(1-z^2)/k^2,
//   I_A3 factor  [3 r z (s+t) - 2 s t (1+2z^2)]/(s k^2),
//   I_B1 factor = I_B3 factor = 2 s t (1-z^2)/k^2,   I_B2 factor 1,
// so three angular sums per (i, j) suffice:
//   S_T = sum_a w_a sqrt(1-z_a^2) E (1-z_a^2)/k^2,
//   S_3 = sum_a w_a sqrt(1-z_a^2) E [3 r z (s+t) - 2 s t (1+2 z^2)]/k^2,
//   S_0 = sum_a w_a sqrt(1-z_a^2) E,              E = exp(-k^2/omega^2).
// Stored matrices (radial weight W_j = w_j t_j^2 and L_ij = 1/(t_j - s_i),
// the singular kernel of Sec. II, folded in):
//   K_T = W t L S_T,   K_3 = W S_3 / (2 s),   K_0 = 3 W S_0 / 2.
// With sigma_V = A(t)/Delta, sigma_S = B(t)/Delta, Delta = t A(t)^2 + B(t)^2:
//   A'_i = 1 + pref [ -sum_j K_T (2 sigma_S dB + (s_i+t_j) sigma_V dA)
//                     + sum_j K_3 sigma_V sA ]
//   B'_i = m + pref [ 2 s_i sum_j K_T (sigma_S dA - sigma_V dB)
//                     + sum_j K_0 sigma_S sA ]
// where dA = A(t_j) - A(s_i), dB = B(t_j) - B(s_i), sA = A(t_j) + A(s_i)
// (the Ball-Chiu difference quotients and sigma_A, eq. (2)), and
// pref = C_F/(8 pi^3) * 8 pi^2 D/omega^4. The differences are formed directly
// in FP64 before they multiply the singular kernel.

#include "qdse_internal.h"
#include "qdse_sweep_row.h"

namespace qdse {

namespace {

using namespace sweep;

// Ultraviolet term of the Qin-Chang interaction, the part Sec. II leaves out:
// 8 pi^2 gamma_m F(k^2) / ln[tau + (1 + k^2/L^2)^2] with F(k^2) =
// (1 - exp(-k^2/(4 m_t^2)))/k^2, gamma_m = 12/25 (four flavours),
// L = 0.234 GeV, tau = e^2 - 1, m_t = 0.5 GeV; at large k^2 it is 4 pi times
// the one-loop running coupling.
__device__ inline double g_uv_qc(double k2) {
  constexpr double kPi = 3.14159265358979323846;
  constexpr double kGammaM = 12.0 / 25.0;
  constexpr double kInvL2 = 1.0 / (0.234 * 0.234);
  constexpr double kInv4Mt2 = 1.0 / (4.0 * 0.5 * 0.5);
  constexpr double kTau = 6.38905609893065022723;  // e^2 - 1
  const double ff = -expm1(-k2 * kInv4Mt2) / k2;
  const double q = fma(k2, kInvL2, 1.0);
  return 8.0 * kPi * kPi * kGammaM * ff / log(fma(q, q, kTau));
}

// ---------------------------------------------------------------- precompute
// One thread per (i, j); the angular sum runs over a in registers. Writes the
// three matrices (and optionally their omega derivatives) of one omega class,
// zero in the padding columns j >= nq.
__global__ void k_precompute(int n, int nq, int na, int ldk, const double* __restrict__ s_,
                             const double* __restrict__ t_, const double* __restrict__ W_,
                             const double* __restrict__ z_, const double* __restrict__ wz_,
                             double omega, int with_domega, double gir, int uv,
                             double* __restrict__ K, double* __restrict__ dK) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)n * ldk) return;
  const int i = (int)(idx / ldk), j = (int)(idx % ldk);
  const size_t mat = (size_t)n * ldk;
  const size_t o = (size_t)i * ldk + j;
  if (j >= nq) {
    K[o] = 0.0;
    K[mat + o] = 0.0;
    K[2 * mat + o] = 0.0;
    if (with_domega) {
      dK[o] = 0.0;
      dK[mat + o] = 0.0;
      dK[2 * mat + o] = 0.0;
    }
    return;
  }
  const double s = s_[i], t = t_[j];
  const double rs = sqrt(s), rt = sqrt(t), r = rs * rt;
  const double d0 = (rs - rt) * (rs - rt);
  const double inv_om2 = 1.0 / (omega * omega);
  double sT = 0.0, s3 = 0.0, s0 = 0.0, dT = 0.0, d3 = 0.0, dd0 = 0.0;
  for (int a = 0; a < na; ++a) {
    const double z = z_[a], w = wz_[a];
    const double omz = 1.0 - z, opz = 1.0 + z;
    const double k2 = fma(2.0 * r, omz, d0);
    const double E = uv ? w * fma(gir, exp(-k2 * inv_om2), g_uv_qc(k2)) : w * exp(-k2 * inv_om2);
    const double tr = omz * opz / k2;
    const double f3 = (3.0 * r * z * (s + t) - 2.0 * s * t * (1.0 + 2.0 * z * z)) / k2;
    sT = fma(E, tr, sT);
    s3 = fma(E, f3, s3);
    s0 += E;
    if (with_domega) {  // d/domega exp(-k^2/omega^2) = 2 k^2/omega^3 exp(...)
      const double g = E * k2;
      dT = fma(g, tr, dT);
      d3 = fma(g, f3, d3);
      dd0 += g;
    }
  }
  const double W = W_[j], L = 1.0 / (t - s);
  K[o] = W * t * L * sT;
  K[mat + o] = W * s3 / (2.0 * s);
  K[2 * mat + o] = 1.5 * W * s0;
  if (with_domega) {
    const double c = 2.0 / (omega * omega * omega);
    dK[o] = c * W * t * L * dT;
    dK[mat + o] = c * W * d3 / (2.0 * s);
    dK[2 * mat + o] = c * 1.5 * W * dd0;
  }
}

// ---------------------------------------------------------------- masked runs
__device__ inline double bits_to_double(unsigned long long b) { return __longlong_as_double((long long)b); }

// The statistic of one sweep slot: the max over its lanes.
__device__ inline unsigned long long metric_max(const SolveState* st, int slot) {
  unsigned long long m = st->metric[slot][0];
#pragma unroll
  for (int l = 1; l < kMetricLanes; ++l) m = st->metric[slot][l] > m ? st->metric[slot][l] : m;
  return m;
}

__device__ inline void mirror_state(const SolveCtl* ctl, const SolveState* st, int status, int now,
                                    double resid, unsigned long long last,
                                    unsigned long long before) {
  SolveState* m = ctl->mirror + (st - ctl->base);
  m->sweeps = now;
  m->resid = resid;
  m->metric[0][0] = last;
  m->metric[1][0] = before;
  m->status = status;
}

// Status of an instance at the start of sweep k (1-based within a chunk whose
// length is a multiple of 6), from the test statistic of sweep k-1. Every
// block evaluates it the same way; the writer block records it and clears the
// slot that sweep k+1 will fill.
// Inputs of the masked-run decision of sweep k, written only by earlier
// launches: the status (a frozen instance stays frozen; within a launch every
// block derives the same status from the same inputs), the sweep count of slot
// (k-1)%3 and the statistic of sweep k-1, with the run's tolerance, iteration
// cap and test mode. Loaded apart from decide_with so that a kernel can issue
// these reads first and take the decision later.
struct DecideIn {
  int status, done, max_iter, mode;
  double prev, tol;
};
__device__ inline DecideIn decide_inputs(const SolveState* st, const SolveCtl* ctl, int k) {
  DecideIn d;
  d.status = st->status;
  d.done = st->sweeps_slot[(k + 2) % 3];
  d.prev = bits_to_double(metric_max(st, (k + 2) % 3));
  d.tol = ctl->tol;
  d.max_iter = ctl->max_iter;
  d.mode = ctl->mode;
  return d;
}

__device__ inline int decide_with(SolveState* st, const SolveCtl* ctl, int k, bool writer,
                                  const DecideIn& in) {
  SolveState& S = *st;
  int status = in.status;
  const int done = in.done;
  const double prev = in.prev;
  if (status == 0) {
    if (done > 0) {
      if (!(prev <= 1.7976931348623157e308)) status = 3;  // NaN or inf
      else if (prev < in.tol) status = 1;
    }
    if (status == 0 && done >= in.max_iter) status = 2;
  }
  if (writer && threadIdx.x == 0) {
    const unsigned long long before = metric_max(&S, (k + 1) % 3);  // sweep k-2, cleared below
    if (status != 0 && S.status == 0) S.resid = prev;
    S.status = status;
    const int now = done + (status == 0 ? 1 : 0);
    S.sweeps_slot[k % 3] = now;
    S.sweeps = now;
#pragma unroll
    for (int l = 0; l < kMetricLanes; ++l) S.metric[(k + 1) % 3][l] = 0ull;
    if (ctl->mirror && k % 6 == 0)
      mirror_state(ctl, st, status, now, S.resid, metric_max(&S, (k + 2) % 3), before);
  }
  return status;
}

__device__ inline int decide(SolveState* st, const SolveCtl* ctl, int k, bool writer) {
  return decide_with(st, ctl, k, writer, decide_inputs(st, ctl, k));
}

// Start of a masked run: fresh per-instance states, the run's controls (when
// ctl is given) and the starting iterate copied into the run's buffer (when
// x_src is given), in one launch.
__global__ void k_solve_init(int n_inst, SolveState* st, SolveCtl* ctl, SolveCtl v,
                             const double* __restrict__ x_src, double* __restrict__ x_dst,
                             long xlen) {
  const long e0 = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (ctl && e0 == 0) *ctl = v;
  if (x_src)
    for (long e = e0; e < xlen; e += (long)gridDim.x * blockDim.x) x_dst[e] = x_src[e];
  if (e0 >= n_inst) return;
  const int k = (int)e0;
  st[k].status = 0;
  st[k].sweeps = 0;
  st[k].sweeps_slot[0] = st[k].sweeps_slot[1] = st[k].sweeps_slot[2] = 0;
  st[k].resid = __longlong_as_double(0x7ff0000000000000ll);
  for (int l = 0; l < kMetricLanes; ++l) {
    st[k].metric[0][l] = 0x7ff0000000000000ull;  // +inf: no sweep yet
    st[k].metric[1][l] = 0ull;                   // filled by sweep 1
    st[k].metric[2][l] = 0ull;
  }
}


template <class T>
__device__ inline void node_values(int n, int j, const int* lo, const double* sw, double tj,
                                   const double* xA, const double* xB, const double* vA,
                                   const double* vB, T* out) {
  const int b = lo[j];
  double w[4];
  T xa[4], xb[4];
#pragma unroll
  for (int l = 0; l < 4; ++l) {
    w[l] = sw[4 * j + l];
    xa[l] = make<T>(xA[b + l], vA ? vA[b + l] : 0.0);
    xb[l] = make<T>(xB[b + l], vB ? vB[b + l] : 0.0);
  }
  node_core<T>(w, xa, xb, tj, out);
}

__global__ void k_nodes(int n, int nq, int ldk, const int* __restrict__ lo,
                        const double* __restrict__ sw, const double* __restrict__ t,
                        const double* __restrict__ x, double* __restrict__ nodes,
                        SolveState* state, const SolveCtl* ctl, int k) {
  const int inst = blockIdx.y;
  if (state && decide(state + inst, ctl, k, blockIdx.x == 0)) return;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nq) return;
  const double* xA = x + (size_t)inst * 2 * n;
  double v[5];
  node_values<double>(n, j, lo, sw, t[j], xA, xA + n, nullptr, nullptr, v);
  double* o = nodes + (size_t)inst * 5 * ldk;
#pragma unroll
  for (int c = 0; c < 5; ++c) o[(size_t)c * ldk + j] = v[c];
}

__global__ void k_nodes_dual(int n, int nq, int ldk, const int* __restrict__ lo,
                             const double* __restrict__ sw, const double* __restrict__ t,
                             const double* __restrict__ x, const double* __restrict__ vdir,
                             double* __restrict__ nodes, const int* __restrict__ act) {
  const int inst = blockIdx.y;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nq || (act && !act[inst])) return;
  const double* xA = x + (size_t)inst * 2 * n;
  const double* vA = vdir + (size_t)inst * 2 * n;
  Dual v[5];
  node_values<Dual>(n, j, lo, sw, t[j], xA, xA + n, vA, vA + n, v);
  double* o = nodes + (size_t)inst * 10 * ldk;
#pragma unroll
  for (int c = 0; c < 5; ++c) {
    o[(size_t)c * ldk + j] = v[c].v;
    o[(size_t)(5 + c) * ldk + j] = v[c].d;
  }
}

// ---------------------------------------------------------------- contraction
// One 64-lane wavefront per (instance, external row i): lanes stride over
// loop nodes j (coalesced K rows), accumulate the four sums of the direct
// difference form, reduce across the wave, and lane 0 applies the update.
template <class T>
__device__ inline void row_accumulate(int nq, int ldk, size_t mat, const double* Ki,
                                      const double* nd, const double* ndt, double s, T Ai, T Bi,
                                      int lane, T acc[4]) {
  for (int j = lane; j < nq; j += WAVE) {
    const double kT = Ki[j], k3 = Ki[mat + j], k0 = Ki[2 * mat + j];
    const T Aq = make<T>(nd[j], ndt ? ndt[j] : 0.0);
    const T Bq = make<T>(nd[ldk + j], ndt ? ndt[ldk + j] : 0.0);
    const T sV = make<T>(nd[2 * ldk + j], ndt ? ndt[2 * ldk + j] : 0.0);
    const T sS = make<T>(nd[3 * ldk + j], ndt ? ndt[3 * ldk + j] : 0.0);
    const T tsV = make<T>(nd[4 * ldk + j], ndt ? ndt[4 * ldk + j] : 0.0);
    const T dA = Aq - Ai, dB = Bq - Bi, sA = Aq + Ai;
    const T sc = make<T>(s, 0.0);
    // 2 sigma_S dB + (s + t) sigma_V dA
    const T e = make<T>(2.0, 0.0) * sS * dB + (sc * sV + tsV) * dA;
    acc[0] = acc[0] + make<T>(kT, 0.0) * e;
    acc[1] = acc[1] + make<T>(k3, 0.0) * (sV * sA);
    acc[2] = acc[2] + make<T>(kT, 0.0) * (sS * dA - sV * dB);
    acc[3] = acc[3] + make<T>(k0, 0.0) * (sS * sA);
  }
#pragma unroll
  for (int c = 0; c < 4; ++c) acc[c] = wave_sum(acc[c]);
}


// Specialised FP64 body for the hot sweep: lane sums, then wave sums.
template <int U = 6>
__device__ inline void row_accumulate_f64(int nq, int ldk, size_t mat, const double* __restrict__ Ki,
                                          const double* __restrict__ nd, double s, double Ai,
                                          double Bi, int lane, double acc[4]) {
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  row_stream_f64<U>(lane, nq, ldk, mat, Ki, nd, s, Ai, Bi, a0, a1, a2, a3);
  wave_sum4(a0, a1, a2, a3);
  acc[0] = a0;
  acc[1] = a1;
  acc[2] = a2;
  acc[3] = a3;
}


__global__ void __launch_bounds__(256) k_sweep(int n_inst, int n, int nq, int ldk,
                                               const InstDev* __restrict__ inst_,
                                               const double* __restrict__ K, size_t kstride,
                                               const double* __restrict__ s_,
                                               const double* __restrict__ nodes,
                                               const double* __restrict__ x_in,
                                               double* __restrict__ x_out, SolveState* state,
                                               const SolveCtl* ctl, int k, int add_f0) {
  const int lane = threadIdx.x & (WAVE - 1);
  const long row = (long)blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE;
  if (row >= (long)n_inst * n) return;
  const int inst = (int)(row / n), i = (int)(row % n);
  const double* xi = x_in + (size_t)inst * 2 * n;
  double* xo = x_out + (size_t)inst * 2 * n;
  if (state && state[inst].status != 0) {  // frozen: carry the iterate along
    if (lane == 0) {
      xo[i] = xi[i];
      xo[n + i] = xi[n + i];
    }
    return;
  }
  const InstDev P = inst_[inst];
  const size_t mat = (size_t)n * ldk;
  const double* Ki = K + (size_t)P.kblock * kstride + (size_t)i * ldk;
  const double* nd = nodes + (size_t)inst * 5 * ldk;
  const double s = s_[i];
  const double Ai = xi[i], Bi = xi[n + i];
  double acc[4];
  row_accumulate_f64(nq, ldk, mat, Ki, nd, s, Ai, Bi, lane, acc);
  if (lane == 0) {
    const double An = (add_f0 ? 1.0 : 0.0) + P.pref * (acc[1] - acc[0]);
    const double Bn = (add_f0 ? P.m : 0.0) + P.pref * fma(2.0 * s, acc[2], acc[3]);
    xo[i] = An;
    xo[n + i] = Bn;
    if (state) {
      const double r = test_stat(ctl->mode, An, Bn, Ai, Bi);
      const unsigned long long bits = (unsigned long long)__double_as_longlong(isnan(r) ? __longlong_as_double(0x7ff8000000000000ll) : r);
      atomicMax(&state[inst].metric[k % 3][blockIdx.x % kMetricLanes], bits);
    }
  }
}

// Fused sweep: one workgroup = (instance, ROWS consecutive rows); the node
// functions of the instance are rebuilt in LDS by every workgroup (O(N) work
// against O(ROWS N) for the rows), then each wavefront contracts ROWS / 4 rows
// with exactly the per-row arithmetic of k_sweep. Fewer rows per workgroup
// spread a small batch over more compute units.
template <int ROWS>
__global__ void __launch_bounds__(256) k_sweep_fused(
    int n_inst, int n, int nq, int ldk, const InstDev* __restrict__ inst_,
    const double* __restrict__ K, size_t kstride, const int* __restrict__ lo,
    const double* __restrict__ sw, const double* __restrict__ t_, const double* __restrict__ s_,
    const double* __restrict__ x_in, double* __restrict__ x_out, SolveState* state,
    const SolveCtl* ctl, int k, int add_f0) {
  extern __shared__ double nd[];  // [5][ldk]
  const int inst = blockIdx.y;
  const int lane = threadIdx.x & (WAVE - 1), wave = threadIdx.x / WAVE;
  const double* xi = x_in + (size_t)inst * 2 * n;
  double* xo = x_out + (size_t)inst * 2 * n;
  const int r0 = blockIdx.x * ROWS;
  if (state && decide(state + inst, ctl, k, blockIdx.x == 0)) {  // frozen: carry along
    for (int r = threadIdx.x; r < ROWS; r += blockDim.x) {
      const int i = r0 + r;
      if (i < n) {
        xo[i] = xi[i];
        xo[n + i] = xi[n + i];
      }
    }
    return;
  }
  for (int j = threadIdx.x; j < nq; j += blockDim.x) {
    double v[5];
    node_values<double>(n, j, lo, sw, t_[j], xi, xi + n, nullptr, nullptr, v);
#pragma unroll
    for (int c = 0; c < 5; ++c) nd[(size_t)c * ldk + j] = v[c];
  }
  __syncthreads();
  const InstDev P = inst_[inst];
  const size_t mat = (size_t)n * ldk;
  // test statistic as the bits of a non-negative double (NaN above +inf),
  // maximised over the workgroup's rows and folded in with one atomic
  __shared__ unsigned long long wmax[4];
  unsigned long long mine = 0ull;
  for (int rr = 0; rr < ROWS / 4; ++rr) {
    const int i = r0 + wave * (ROWS / 4) + rr;
    if (i >= n) break;
    const double* Ki = K + (size_t)P.kblock * kstride + (size_t)i * ldk;
    const double s = s_[i];
    const double Ai = xi[i], Bi = xi[n + i];
    double acc[4];
    row_accumulate_f64<2>(nq, ldk, mat, Ki, nd, s, Ai, Bi, lane, acc);
    if (lane == 0) {
      const double An = (add_f0 ? 1.0 : 0.0) + P.pref * (acc[1] - acc[0]);
      const double Bn = (add_f0 ? P.m : 0.0) + P.pref * fma(2.0 * s, acc[2], acc[3]);
      xo[i] = An;
      xo[n + i] = Bn;
      if (state) {
        const double r = test_stat(ctl->mode, An, Bn, Ai, Bi);
        const unsigned long long bits = (unsigned long long)__double_as_longlong(
            isnan(r) ? __longlong_as_double(0x7ff8000000000000ll) : r);
        mine = bits > mine ? bits : mine;
      }
    }
  }
  if (state) {
    if (lane == 0) wmax[wave] = mine;
    __syncthreads();
    if (threadIdx.x == 0) {
      unsigned long long m = wmax[0];
      for (int w = 1; w < 4; ++w) m = wmax[w] > m ? wmax[w] : m;
      atomicMax(&state[inst].metric[k % 3][blockIdx.x % kMetricLanes], m);
    }
  }
}

// Small-batch sweep, one row per wavefront (four rows per workgroup). With
// about one workgroup per compute unit a launch lasts as long as one
// workgroup's chain of reads, so they are ordered for latency: the iterate
// values and stencil weights of all of a thread's nodes go out first (vector
// reads complete in issue order), then the row's kernel entries (held in
// registers) and its own values; the node functions are built while the
// kernel entries are still arriving, then the masked-run decision is taken.
// After the barrier the contraction consumes the registers (nodes
// beyond ROW_PF lane strides are streamed as in k_sweep). Same per-row
// arithmetic and order as k_sweep.
constexpr int ROW_PF = 9;   // lane strides held in registers: nq <= 576 in one pass
constexpr int NODE_PT = 3;  // nodes per thread per pass of the node build
//
// QC = true is the renormalised mode's sums kernel: the matrices have n + 1
// rows, row n (p^2 = zeta^2) takes A and B interpolated with the stencil of
// zp, and each wavefront writes its row's loop sums times pref (without the
// inhomogeneous terms) to sig[inst][i], sig[inst][(n+1) + i] for the update
// kernel; frozen instances write nothing.
template <bool QC>
__global__ void __launch_bounds__(256) k_sweep_row(
    int n_inst, int n, int nq, int ldk, const InstDev* __restrict__ inst_,
    const double* __restrict__ K, size_t kstride, const int* __restrict__ lo,
    const double* __restrict__ sw, const double* __restrict__ t_, const double* __restrict__ s_,
    const double* __restrict__ x_in, double* __restrict__ x_out, SolveState* state,
    const SolveCtl* ctl, int k, int add_f0, QcPoint zp, double* __restrict__ sig) {
  extern __shared__ double nd[];  // [5][ldk] and one spare slot
  const int inst = blockIdx.y;
  const int lane = threadIdx.x & (WAVE - 1), wave = threadIdx.x / WAVE;
  const double* xi = x_in + (size_t)inst * 2 * n;
  double* xo = x_out + (size_t)inst * 2 * n;
  const int rows = QC ? n + 1 : n;
  const int i = blockIdx.x * 4 + wave;
  const int ic = i < rows ? i : rows - 1;  // rows past the last read it and write nothing
  // Loop node j lies between external nodes j - 1 and j (the loop grid
  // interleaves the external one), so its 4-point stencil starts at
  // clamp(j - 2, 0, n - 4), the base the grid's stencil table holds: the
  // iterate reads need no table read first.
  // the masked-run inputs (scalar reads) go out before everything else
  DecideIn din{};
  if (state) din = decide_inputs(state + inst, ctl, k);
  double w[NODE_PT][4], tj[NODE_PT], xa[NODE_PT][4], xb[NODE_PT][4];
  auto node_reads = [&](int jb) {
#pragma unroll
    for (int q = 0; q < NODE_PT; ++q) {
      const int j = min(jb + q * 256, nq - 1);
      const int b = min(max(j - 2, 0), n - 4);
#pragma unroll
      for (int l = 0; l < 4; ++l) {
        xa[q][l] = xi[b + l];
        xb[q][l] = xi[n + b + l];
      }
    }
#pragma unroll
    for (int q = 0; q < NODE_PT; ++q) {
      const int j = min(jb + q * 256, nq - 1);
      tj[q] = t_[j];
#pragma unroll
      for (int l = 0; l < 4; ++l) w[q][l] = sw[4 * j + l];
    }
  };
  node_reads(threadIdx.x);
  __builtin_amdgcn_sched_barrier(0);  // keep these reads ahead of the kernel-row reads
  const InstDev P = inst_[inst];
  const size_t mat = (size_t)rows * ldk;
  const double* Ki = K + (size_t)P.kblock * kstride + (size_t)ic * ldk;
  double kT[ROW_PF], k3[ROW_PF], k0[ROW_PF];
  load_row_regs<ROW_PF>(lane, nq, mat, Ki, kT, k3, k0);
  double s, Ai, Bi;
  if (QC && ic == n) {  // the renormalisation point
    s = zp.s;
    Ai = 0.0;
    Bi = 0.0;
#pragma unroll
    for (int l = 0; l < 4; ++l) {
      Ai = fma(zp.w[l], xi[zp.base + l], Ai);
      Bi = fma(zp.w[l], xi[n + zp.base + l], Bi);
    }
  } else {
    s = s_[ic];
    Ai = xi[ic];
    Bi = xi[n + ic];
  }
  __builtin_amdgcn_sched_barrier(0);
  // Every node of the pass is computed and stored, the clamped ones into one
  // spare slot past the five columns, so that no read can be moved into a
  // conditional block behind the kernel-row reads.
  auto nodes = [&](int jb) {
#pragma unroll
    for (int q = 0; q < NODE_PT; ++q) {
      double v[5];
      node_core<double>(w[q], xa[q], xb[q], tj[q], v);
      const int j = jb + q * 256;
#pragma unroll
      for (int c = 0; c < 5; ++c) nd[j < nq ? c * ldk + j : 5 * ldk] = v[c];
    }
  };
  // the first pass outside the loop, so that its waits count only its own reads
  nodes(threadIdx.x);
  for (int jb = threadIdx.x + NODE_PT * 256; jb < nq; jb += NODE_PT * 256) {
    node_reads(jb);
    nodes(jb);
  }
  // (after the node build; its inputs were read at the start)
  const int status = state ? decide_with(state + inst, ctl, k, blockIdx.x == 0, din) : 0;
  __syncthreads();
  if (status != 0) {  // frozen (the same for every wavefront): carry along
    if (!QC && lane == 0 && i < n) {
      xo[i] = Ai;
      xo[n + i] = Bi;
    }
    return;
  }
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  row_regs<ROW_PF>(lane, nq, ldk, nd, kT, k3, k0, s, Ai, Bi, a0, a1, a2, a3);
  row_stream_f64(lane + ROW_PF * WAVE, nq, ldk, mat, Ki, nd, s, Ai, Bi, a0, a1, a2, a3);
  wave_sum4(a0, a1, a2, a3);
  const double acc0 = a0, acc1 = a1, acc2 = a2, acc3 = a3;
  if (QC) {
    if (lane == 0 && i < rows) {
      double* sg = sig + (size_t)inst * 2 * rows;
      sg[i] = P.pref * (acc1 - acc0);
      sg[rows + i] = P.pref * fma(2.0 * s, acc2, acc3);
    }
    return;
  }
  __shared__ unsigned long long wmax[4];
  unsigned long long mine = 0ull;
  if (lane == 0 && i < n) {
    const double An = (add_f0 ? 1.0 : 0.0) + P.pref * (acc1 - acc0);
    const double Bn = (add_f0 ? P.m : 0.0) + P.pref * fma(2.0 * s, acc2, acc3);
    xo[i] = An;
    xo[n + i] = Bn;
    if (state) {
      const double r = test_stat(din.mode, An, Bn, Ai, Bi);
      mine = (unsigned long long)__double_as_longlong(
          isnan(r) ? __longlong_as_double(0x7ff8000000000000ll) : r);
    }
  }
  if (state) {
    if (lane == 0) wmax[wave] = mine;
    __syncthreads();
    if (threadIdx.x == 0) {
      unsigned long long m = wmax[0];
      for (int w = 1; w < 4; ++w) m = wmax[w] > m ? wmax[w] : m;
      atomicMax(&state[inst].metric[k % 3][blockIdx.x % kMetricLanes], m);
    }
  }
}

// ---------------------------------------------------------------- renormalised mode
// Update with the renormalisation constants of this sweep: Z_2 = 1/(1 +
// Sigma_A(zeta^2)) makes A(zeta^2) = 1 and Z_4 m = m - Z_2 Sigma_B(zeta^2)
// makes B(zeta^2) = m (no mass term at m = 0); then A = Z_2 (1 + Sigma_A),
// B = Z_4 m + Z_2 Sigma_B (vertex constant Z_1 = Z_2). One workgroup per
// instance; in a masked run frozen instances carry their iterate and the
// others fold their test statistic in with one atomic.
__global__ void __launch_bounds__(256) k_qc_update(int n_inst, int n,
                                                   const InstDev* __restrict__ inst_,
                                                   const double* __restrict__ sig,
                                                   const double* __restrict__ x_in,
                                                   double* __restrict__ x_out, SolveState* state,
                                                   const SolveCtl* ctl, int k) {
  const int inst = blockIdx.x;
  const double* xi = x_in + (size_t)inst * 2 * n;
  double* xo = x_out + (size_t)inst * 2 * n;
  if (state && state[inst].status != 0) {
    for (int i = threadIdx.x; i < 2 * n; i += blockDim.x) xo[i] = xi[i];
    return;
  }
  const int rows = n + 1;
  const double* sg = sig + (size_t)inst * 2 * rows;
  const double m = inst_[inst].m;
  const double Z2 = 1.0 / (1.0 + sg[n]);
  const double Z4m = m == 0.0 ? 0.0 : m - Z2 * sg[rows + n];
  unsigned long long mine = 0ull;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const double An = Z2 * (1.0 + sg[i]);
    const double Bn = Z4m + Z2 * sg[rows + i];
    xo[i] = An;
    xo[n + i] = Bn;
    if (state) {
      const double r = test_stat(ctl->mode, An, Bn, xi[i], xi[n + i]);
      const unsigned long long b = (unsigned long long)__double_as_longlong(
          isnan(r) ? __longlong_as_double(0x7ff8000000000000ll) : r);
      mine = b > mine ? b : mine;
    }
  }
  if (!state) return;
#pragma unroll
  for (int o = WAVE / 2; o > 0; o >>= 1) {
    const unsigned long long v = __shfl_xor(mine, o, WAVE);
    mine = v > mine ? v : mine;
  }
  __shared__ unsigned long long wmax[4];
  const int lane = threadIdx.x & (WAVE - 1), wave = threadIdx.x / WAVE;
  if (lane == 0) wmax[wave] = mine;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long mm = wmax[0];
    for (int w = 1; w < 4; ++w) mm = wmax[w] > mm ? wmax[w] : mm;
    atomicMax(&state[inst].metric[k % 3][0], mm);
  }
}

// Tangent sweep: jv = dF/dx v, the same arithmetic in dual numbers.
__global__ void __launch_bounds__(256) k_sweep_dual(int n_inst, int n, int nq, int ldk,
                                                    const InstDev* __restrict__ inst_,
                                                    const double* __restrict__ K, size_t kstride,
                                                    const double* __restrict__ s_,
                                                    const double* __restrict__ nodes,
                                                    const double* __restrict__ x,
                                                    const double* __restrict__ vdir,
                                                    double* __restrict__ jv,
                                                    const int* __restrict__ act) {
  const int lane = threadIdx.x & (WAVE - 1);
  const long row = (long)blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE;
  if (row >= (long)n_inst * n) return;
  const int inst = (int)(row / n), i = (int)(row % n);
  if (act && !act[inst]) return;  // (one row per wavefront: the exit is wave-uniform)
  const InstDev P = inst_[inst];
  const size_t mat = (size_t)n * ldk;
  const double* Ki = K + (size_t)P.kblock * kstride + (size_t)i * ldk;
  const double* nd = nodes + (size_t)inst * 10 * ldk;
  const double* xi = x + (size_t)inst * 2 * n;
  const double* vi = vdir + (size_t)inst * 2 * n;
  const Dual Ai{xi[i], vi[i]}, Bi{xi[n + i], vi[n + i]};
  Dual acc[4] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}};
  row_accumulate<Dual>(nq, ldk, mat, Ki, nd, nd + 5 * ldk, s_[i], Ai, Bi, lane, acc);
  if (lane == 0) {
    const double s = s_[i];
    jv[(size_t)inst * 2 * n + i] = P.pref * (acc[1].d - acc[0].d);
    jv[(size_t)inst * 2 * n + n + i] = P.pref * fma(2.0 * s, acc[2].d, acc[3].d);
  }
}

// ---------------------------------------------------------------- reverse mode
// Adjoint of one sweep. With abar_i = pref wA_i and bbar_i = pref wB_i the
// accumulators of row i carry adjoints (-abar, abar, 2 s_i bbar, bbar).
// Row part: d/dA_i and d/dB_i through dA, dB, sA (one wavefront per row).
__global__ void __launch_bounds__(256) k_vjp_rows(int n_inst, int n, int nq, int ldk,
                                                  const InstDev* __restrict__ inst_,
                                                  const double* __restrict__ K, size_t kstride,
                                                  const double* __restrict__ s_,
                                                  const double* __restrict__ t_,
                                                  const double* __restrict__ nodes,
                                                  const double* __restrict__ w,
                                                  double* __restrict__ out,
                                                  const int* __restrict__ act) {
  const int lane = threadIdx.x & (WAVE - 1);
  const long row = (long)blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE;
  if (row >= (long)n_inst * n) return;
  const int inst = (int)(row / n), i = (int)(row % n);
  if (act && !act[inst]) return;
  const InstDev P = inst_[inst];
  const size_t mat = (size_t)n * ldk;
  const double* Ki = K + (size_t)P.kblock * kstride + (size_t)i * ldk;
  const double* nd = nodes + (size_t)inst * 5 * ldk;
  const double s = s_[i];
  const double ab = P.pref * w[(size_t)inst * 2 * n + i];
  const double bb = P.pref * w[(size_t)inst * 2 * n + n + i];
  double gA = 0.0, gB = 0.0;
  for (int j = lane; j < nq; j += WAVE) {
    const double kT = Ki[j], k3 = Ki[mat + j], k0 = Ki[2 * mat + j];
    const double sV = nd[2 * ldk + j], sS = nd[3 * ldk + j], t = t_[j];
    // dF/ddA = -ab kT (s+t) sV + 2 s bb kT sS ; dF/dsA = ab k3 sV + bb k0 sS
    const double gdA = kT * (2.0 * s * bb * sS - ab * (s + t) * sV);
    const double gsA = ab * k3 * sV + bb * k0 * sS;
    // dF/ddB = -2 ab kT sS - 2 s bb kT sV
    const double gdB = -2.0 * kT * (ab * sS + s * bb * sV);
    gA += gsA - gdA;
    gB -= gdB;
  }
  gA = wave_sum(gA);
  gB = wave_sum(gB);
  if (lane == 0) {
    out[(size_t)inst * 2 * n + i] = gA;
    out[(size_t)inst * 2 * n + n + i] = gB;
  }
}

// Column part: per loop node j, partial sums over a chunk of rows of the
// adjoints of A(t_j), B(t_j) (through dA, dB, sA) and of sigma_V, sigma_S.
// One thread per (instance, j, chunk); lanes over j read K rows coalesced.
__global__ void k_vjp_cols(int n_inst, int n, int nq, int ldk, int nchunk,
                           const InstDev* __restrict__ inst_, const double* __restrict__ K,
                           size_t kstride, const double* __restrict__ s_,
                           const double* __restrict__ t_, const double* __restrict__ nodes,
                           const double* __restrict__ x, const double* __restrict__ w,
                           double* __restrict__ part, const int* __restrict__ act) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int chunk = blockIdx.y, inst = blockIdx.z;
  if (j >= nq || (act && !act[inst])) return;
  const InstDev P = inst_[inst];
  const size_t mat = (size_t)n * ldk;
  const double* Kb = K + (size_t)P.kblock * kstride;
  const double* nd = nodes + (size_t)inst * 5 * ldk;
  const double* xi = x + (size_t)inst * 2 * n;
  const double* wi = w + (size_t)inst * 2 * n;
  const double Aq = nd[j], Bq = nd[ldk + j], sV = nd[2 * ldk + j], sS = nd[3 * ldk + j];
  const double t = t_[j];
  const int r0 = (int)((long)n * chunk / nchunk), r1 = (int)((long)n * (chunk + 1) / nchunk);
  double gAq = 0.0, gBq = 0.0, gsV = 0.0, gsS = 0.0;
  for (int i = r0; i < r1; ++i) {
    const double kT = Kb[(size_t)i * ldk + j], k3 = Kb[mat + (size_t)i * ldk + j],
                 k0 = Kb[2 * mat + (size_t)i * ldk + j];
    const double s = s_[i], Ai = xi[i], Bi = xi[n + i];
    const double ab = P.pref * wi[i], bb = P.pref * wi[n + i];
    const double dA = Aq - Ai, dB = Bq - Bi, sA = Aq + Ai;
    const double gdA = kT * (2.0 * s * bb * sS - ab * (s + t) * sV);
    const double gsA = ab * k3 * sV + bb * k0 * sS;
    const double gdB = -2.0 * kT * (ab * sS + s * bb * sV);
    gAq += gdA + gsA;
    gBq += gdB;
    gsS += kT * (2.0 * s * bb * dA - 2.0 * ab * dB) + bb * k0 * sA;
    gsV += ab * k3 * sA - kT * (ab * (s + t) * dA + 2.0 * s * bb * dB);
  }
  double* o = part + (((size_t)inst * nchunk + chunk) * 4) * ldk;
  o[j] = gAq;
  o[ldk + j] = gBq;
  o[2 * ldk + j] = gsV;
  o[3 * ldk + j] = gsS;
}

// Row and column parts in one pass over the kernel matrices: a wavefront owns
// one row chunk; lanes run over loop nodes j = lane + 64 u (u < SLOTS), keep
// the chunk's column partials in registers, and reduce the row sums across
// the wavefront row by row. Node functions of the instance sit in LDS. Every
// sum runs in the same order as in k_vjp_rows and k_vjp_cols, so the result
// is bitwise the same with half the matrix traffic.
template <int SLOTS>
__global__ void __launch_bounds__(256) k_vjp_fused(int n_inst, int n, int nq, int ldk, int nchunk,
                                                   const InstDev* __restrict__ inst_,
                                                   const double* __restrict__ K, size_t kstride,
                                                   const double* __restrict__ s_,
                                                   const double* __restrict__ t_,
                                                   const double* __restrict__ nodes,
                                                   const double* __restrict__ x,
                                                   const double* __restrict__ w,
                                                   double* __restrict__ out,
                                                   double* __restrict__ part,
                                                   const int* __restrict__ act) {
  extern __shared__ double ndl[];  // [5][ldk]: A, B, sigma_V, sigma_S, t
  const int inst = blockIdx.y;
  if (act && !act[inst]) return;  // the whole workgroup: before the barrier
  const double* nd = nodes + (size_t)inst * 5 * ldk;
  for (int j = threadIdx.x; j < nq; j += blockDim.x) {
    ndl[j] = nd[j];
    ndl[ldk + j] = nd[ldk + j];
    ndl[2 * ldk + j] = nd[2 * ldk + j];
    ndl[3 * ldk + j] = nd[3 * ldk + j];
    ndl[4 * ldk + j] = t_[j];
  }
  __syncthreads();
  const int lane = threadIdx.x & (WAVE - 1);
  const int chunk = blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE;
  if (chunk >= nchunk) return;
  const InstDev P = inst_[inst];
  const size_t mat = (size_t)n * ldk;
  const double* Kb = K + (size_t)P.kblock * kstride;
  const double* xi = x + (size_t)inst * 2 * n;
  const double* wi = w + (size_t)inst * 2 * n;
  double* oi = out + (size_t)inst * 2 * n;
  const int r0 = (int)((long)n * chunk / nchunk), r1 = (int)((long)n * (chunk + 1) / nchunk);
  double cA[SLOTS], cB[SLOTS], cV[SLOTS], cS[SLOTS];
#pragma unroll
  for (int u = 0; u < SLOTS; ++u) cA[u] = cB[u] = cV[u] = cS[u] = 0.0;
  for (int i = r0; i < r1; ++i) {
    const double s = s_[i], Ai = xi[i], Bi = xi[n + i];
    const double ab = P.pref * wi[i], bb = P.pref * wi[n + i];
    const double* Ki = Kb + (size_t)i * ldk;
    double gA = 0.0, gB = 0.0;
    // all kernel-matrix loads of the row first (clamped, zero beyond nq)
    double kTs[SLOTS], k3s[SLOTS], k0s[SLOTS];
#pragma unroll
    for (int u = 0; u < SLOTS; ++u) {
      const int j = lane + WAVE * u;
      const int jj = j < nq ? j : nq - 1;
      kTs[u] = Ki[jj];
      k3s[u] = Ki[mat + jj];
      k0s[u] = Ki[2 * mat + jj];
      if (j >= nq) kTs[u] = k3s[u] = k0s[u] = 0.0;
    }
#pragma unroll
    for (int u = 0; u < SLOTS; ++u) {
      const int j = lane + WAVE * u;
      const int jj = j < nq ? j : nq - 1;
      {
        const double kT = kTs[u], k3 = k3s[u], k0 = k0s[u];
        const double Aq = ndl[jj], Bq = ndl[ldk + jj], sV = ndl[2 * ldk + jj],
                     sS = ndl[3 * ldk + jj], t = ndl[4 * ldk + jj];
        const double dA = Aq - Ai, dB = Bq - Bi, sA = Aq + Ai;
        const double gdA = kT * (2.0 * s * bb * sS - ab * (s + t) * sV);
        const double gsA = ab * k3 * sV + bb * k0 * sS;
        const double gdB = -2.0 * kT * (ab * sS + s * bb * sV);
        gA += gsA - gdA;
        gB -= gdB;
        cA[u] += gdA + gsA;
        cB[u] += gdB;
        cS[u] += kT * (2.0 * s * bb * dA - 2.0 * ab * dB) + bb * k0 * sA;
        cV[u] += ab * k3 * sA - kT * (ab * (s + t) * dA + 2.0 * s * bb * dB);
      }
    }
    gA = wave_sum(gA);
    gB = wave_sum(gB);
    if (lane == 0) {
      oi[i] = gA;
      oi[n + i] = gB;
    }
  }
  double* o = part + (((size_t)inst * nchunk + chunk) * 4) * ldk;
#pragma unroll
  for (int u = 0; u < SLOTS; ++u) {
    const int j = lane + WAVE * u;
    if (j < nq) {
      o[j] = cA[u];
      o[ldk + j] = cB[u];
      o[2 * ldk + j] = cV[u];
      o[3 * ldk + j] = cS[u];
    }
  }
}

// The same reverse sweep with the loop nodes of a row split between two
// wavefronts: a workgroup holds two row chunks, wavefront h of a chunk takes
// the lane strides u = h SH .. h SH + SH - 1 (j = lane + 64 u), so each
// wavefront keeps half the column partials and half a row's matrix values in
// registers (one wavefront of the one-wavefront form needs all 256 registers
// at 513 loop nodes and runs alone on its SIMD). Each half's row sums go to
// LDS and are added half 0 + half 1 after the chunk; the column partials are
// those of the one-wavefront form.
template <int SH>
__global__ void __launch_bounds__(256) k_vjp_split(int n_inst, int n, int nq, int ldk, int nchunk,
                                                   int rmax, const InstDev* __restrict__ inst_,
                                                   const double* __restrict__ K, size_t kstride,
                                                   const double* __restrict__ s_,
                                                   const double* __restrict__ t_,
                                                   const double* __restrict__ nodes,
                                                   const double* __restrict__ x,
                                                   const double* __restrict__ w,
                                                   double* __restrict__ out,
                                                   double* __restrict__ part,
                                                   const int* __restrict__ act) {
  extern __shared__ double ndl[];  // [5][ldk]: A, B, sigma_V, sigma_S, t; then row sums
  const int inst = blockIdx.y;
  if (act && !act[inst]) return;  // the whole workgroup: before the barriers
  const double* nd = nodes + (size_t)inst * 5 * ldk;
  for (int j = threadIdx.x; j < nq; j += blockDim.x) {
    ndl[j] = nd[j];
    ndl[ldk + j] = nd[ldk + j];
    ndl[2 * ldk + j] = nd[2 * ldk + j];
    ndl[3 * ldk + j] = nd[3 * ldk + j];
    ndl[4 * ldk + j] = t_[j];
  }
  __syncthreads();
  double* rs = ndl + 5 * ldk;  // [chunk in block 2][half 2][A, B][rmax]
  const int lane = threadIdx.x & (WAVE - 1), wave = threadIdx.x / WAVE;
  const int cl = wave >> 1, h = wave & 1;
  const int chunk = blockIdx.x * 2 + cl;
  const InstDev P = inst_[inst];
  const size_t mat = (size_t)n * ldk;
  const double* Kb = K + (size_t)P.kblock * kstride;
  const double* xi = x + (size_t)inst * 2 * n;
  const double* wi = w + (size_t)inst * 2 * n;
  double* oi = out + (size_t)inst * 2 * n;
  if (chunk < nchunk) {
    const int r0 = (int)((long)n * chunk / nchunk), r1 = (int)((long)n * (chunk + 1) / nchunk);
    double* rA = rs + ((cl * 2 + h) * 2 + 0) * rmax;
    double* rB = rs + ((cl * 2 + h) * 2 + 1) * rmax;
    double cA[SH], cB[SH], cV[SH], cS[SH];
#pragma unroll
    for (int u = 0; u < SH; ++u) cA[u] = cB[u] = cV[u] = cS[u] = 0.0;
#pragma unroll 1
    for (int i = r0; i < r1; ++i) {
      // node values are read from LDS for every row (a compiler-only barrier
      // keeps them out of registers across rows)
      asm volatile("" ::: "memory");
      const double s = s_[i], Ai = xi[i], Bi = xi[n + i];
      const double ab = P.pref * wi[i], bb = P.pref * wi[n + i];
      const double* Ki = Kb + (size_t)i * ldk;
      double gA = 0.0, gB = 0.0;
      double kTs[SH], k3s[SH], k0s[SH];
#pragma unroll
      for (int u = 0; u < SH; ++u) {
        const int j = lane + WAVE * (h * SH + u);
        const int jj = j < nq ? j : nq - 1;
        kTs[u] = Ki[jj];
        k3s[u] = Ki[mat + jj];
        k0s[u] = Ki[2 * mat + jj];
        if (j >= nq) kTs[u] = k3s[u] = k0s[u] = 0.0;
      }
#pragma unroll
      for (int u = 0; u < SH; ++u) {
        const int j = lane + WAVE * (h * SH + u);
        const int jj = j < nq ? j : nq - 1;
        const double kT = kTs[u], k3 = k3s[u], k0 = k0s[u];
        const double Aq = ndl[jj], Bq = ndl[ldk + jj], sV = ndl[2 * ldk + jj],
                     sS = ndl[3 * ldk + jj], t = ndl[4 * ldk + jj];
        const double dA = Aq - Ai, dB = Bq - Bi, sA = Aq + Ai;
        const double gdA = kT * (2.0 * s * bb * sS - ab * (s + t) * sV);
        const double gsA = ab * k3 * sV + bb * k0 * sS;
        const double gdB = -2.0 * kT * (ab * sS + s * bb * sV);
        gA += gsA - gdA;
        gB -= gdB;
        cA[u] += gdA + gsA;
        cB[u] += gdB;
        cS[u] += kT * (2.0 * s * bb * dA - 2.0 * ab * dB) + bb * k0 * sA;
        cV[u] += ab * k3 * sA - kT * (ab * (s + t) * dA + 2.0 * s * bb * dB);
      }
      gA = wave_sum(gA);
      gB = wave_sum(gB);
      if (lane == 0) {
        rA[i - r0] = gA;
        rB[i - r0] = gB;
      }
    }
    double* o = part + (((size_t)inst * nchunk + chunk) * 4) * ldk;
#pragma unroll
    for (int u = 0; u < SH; ++u) {
      const int j = lane + WAVE * (h * SH + u);
      if (j < nq) {
        o[j] = cA[u];
        o[ldk + j] = cB[u];
        o[2 * ldk + j] = cV[u];
        o[3 * ldk + j] = cS[u];
      }
    }
  }
  __syncthreads();
  for (int q = threadIdx.x; q < 2 * rmax; q += blockDim.x) {
    const int c2 = q / rmax, rr = q % rmax, ch = blockIdx.x * 2 + c2;
    if (ch >= nchunk) continue;
    const int r0 = (int)((long)n * ch / nchunk), r1 = (int)((long)n * (ch + 1) / nchunk);
    if (rr >= r1 - r0) continue;
    const double* h0 = rs + (c2 * 2 + 0) * 2 * rmax;
    const double* h1 = rs + (c2 * 2 + 1) * 2 * rmax;
    oi[r0 + rr] = h0[rr] + h1[rr];
    oi[n + r0 + rr] = h0[rmax + rr] + h1[rmax + rr];
  }
}

// Sum the row chunks in a fixed order and push the adjoints of sigma_V,
// sigma_S through sigma = (A or B)/Delta, Delta = t A^2 + B^2: adjoints of
// A(t_j), B(t_j) into gq[inst][2][ldk].
__global__ void k_vjp_nodes(int n_inst, int nq, int ldk, int nchunk, const double* __restrict__ t_,
                            const double* __restrict__ nodes, const double* __restrict__ part,
                            double* __restrict__ gq, const int* __restrict__ act) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int inst = blockIdx.y;
  if (j >= nq || (act && !act[inst])) return;
  double g[4] = {0.0, 0.0, 0.0, 0.0};
  for (int c = 0; c < nchunk; ++c) {
    const double* o = part + (((size_t)inst * nchunk + c) * 4) * ldk;
#pragma unroll
    for (int k = 0; k < 4; ++k) g[k] += o[(size_t)k * ldk + j];
  }
  const double* nd = nodes + (size_t)inst * 5 * ldk;
  const double Aq = nd[j], Bq = nd[ldk + j], sV = nd[2 * ldk + j], sS = nd[3 * ldk + j];
  const double t = t_[j];
  const double Dl = t * Aq * Aq + Bq * Bq;
  const double gD = -(g[2] * sV + g[3] * sS) / Dl;
  gq[(size_t)inst * 2 * ldk + j] = g[0] + g[2] / Dl + gD * 2.0 * t * Aq;
  gq[(size_t)inst * 2 * ldk + ldk + j] = g[1] + g[3] / Dl + gD * 2.0 * Bq;
}

// Transpose of the interpolation: external node l gathers the adjoints of
// every loop node whose stencil contains it; adds the row part in place.
__global__ void k_vjp_scatter(int n_inst, int n, int nq, int ldk, const int* __restrict__ lo,
                              const double* __restrict__ sw, const double* __restrict__ gq,
                              double* __restrict__ out, const int* __restrict__ act) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  const int inst = blockIdx.y;
  if (l >= n || (act && !act[inst])) return;
  double gA = 0.0, gB = 0.0;
  const int j0 = l - 4 < 0 ? 0 : l - 4, j1 = l + 4 > nq - 1 ? nq - 1 : l + 4;
  for (int j = j0; j <= j1; ++j) {
    const int b = lo[j];
    if (l >= b && l < b + 4) {
      const double wl = sw[4 * j + (l - b)];
      gA += wl * gq[(size_t)inst * 2 * ldk + j];
      gB += wl * gq[(size_t)inst * 2 * ldk + ldk + j];
    }
  }
  out[(size_t)inst * 2 * n + l] += gA;
  out[(size_t)inst * 2 * n + n + l] += gB;
}

// ---------------------------------------------------------------- small vector ops
// out[inst * nvec + v] = sum_k a[v][inst][k] b[inst][k], one block per
// (instance, vector), fixed reduction order; instances with act[inst] == 0
// are skipped (act may be null).
__global__ void k_batched_dot(int len, const double* __restrict__ a, size_t lda,
                              const double* __restrict__ b, size_t ldb, int nvec,
                              double* __restrict__ out, const int* __restrict__ act) {
  const int inst = blockIdx.x, v = blockIdx.y;
  if (act && !act[inst]) return;  // the whole block: before the barrier
  const double* av = a + (size_t)v * lda + (size_t)inst * len;
  const double* bv = b + (size_t)inst * ldb;
  double acc = 0.0;
  for (int k = threadIdx.x; k < len; k += blockDim.x) acc = fma(av[k], bv[k], acc);
  __shared__ double red[256 / WAVE];
  acc = wave_sum(acc);
  if ((threadIdx.x & (WAVE - 1)) == 0) red[threadIdx.x / WAVE] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double sacc = 0.0;
    for (int k = 0; k < (int)(blockDim.x / WAVE); ++k) sacc += red[k];
    out[(size_t)inst * nvec + v] = sacc;
  }
}

__global__ void k_gs_update(int n_inst, int len, const double* __restrict__ V, size_t ldv, int nvec,
                            const double* __restrict__ h, int hstride, double* __restrict__ w,
                            const int* __restrict__ act) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)n_inst * len) return;
  const int inst = (int)(e / len);
  if (act && !act[inst]) return;
  double acc = w[e];
  for (int v = 0; v < nvec; ++v) acc -= h[(size_t)inst * hstride + v] * V[(size_t)v * ldv + e];
  w[e] = acc;
}

__global__ void k_combine(int n_inst, int len, const double* __restrict__ V, size_t ldv, int nvec,
                          const double* __restrict__ y, int ystride, double beta,
                          double* __restrict__ out) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)n_inst * len) return;
  const int inst = (int)(e / len);
  double acc = beta == 0.0 ? 0.0 : beta * out[e];
  for (int v = 0; v < nvec; ++v) {  // a zero coefficient contributes 0 (never 0 * inf)
    const double yv = y[(size_t)inst * ystride + v];
    if (yv != 0.0) acc += yv * V[(size_t)v * ldv + e];
  }
  out[e] = acc;
}

__global__ void k_axpby(int n_inst, int len, double alpha, const double* __restrict__ a,
                        const double* __restrict__ scale, const double* __restrict__ b,
                        double* __restrict__ dst) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)n_inst * len) return;
  const double sc = scale ? scale[e / len] : 1.0;
  dst[e] = (alpha == 0.0 ? 0.0 : alpha * a[e]) + (sc == 0.0 ? 0.0 : sc * b[e]);
}

// dst[inst][:] = src[inst][:] for the instances with sel[inst] != 0.
__global__ void k_select(int n_inst, int len, const int* __restrict__ sel,
                         const double* __restrict__ src, double* __restrict__ dst) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)n_inst * len) return;
  if (sel[e / len]) dst[e] = src[e];
}

// The test statistic of Sec. II eq. jifenab2 between two iterates of every
// instance (one workgroup each): mode 0 max_i max(|A'-A|, |B'-B|); mode 1
// max_i max(|M'-M| / max(|M'|, kMassFloor), |A'-A|) with M = B/A.
__global__ void k_conv_stat(int n, int mode, const double* __restrict__ xo,
                            const double* __restrict__ xn, double* __restrict__ out) {
  __shared__ double red[256 / WAVE];
  const int inst = blockIdx.x;
  const double* a = xo + (size_t)inst * 2 * n;
  const double* b = xn + (size_t)inst * 2 * n;
  double r = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const double dA = fabs(b[i] - a[i]);
    double v;
    if (mode == 0) {
      const double dB = fabs(b[n + i] - a[n + i]);
      v = (dA != dA || dB != dB) ? dA + dB : (dA > dB ? dA : dB);
    } else {
      const double Mo = a[n + i] / a[i], Mn = b[n + i] / b[i];
      const double den = fabs(Mn) > kMassFloor ? fabs(Mn) : kMassFloor;
      const double dM = fabs(Mn - Mo) / den;
      v = (dA != dA || dM != dM) ? dA + dM : (dA > dM ? dA : dM);
    }
    r = (r != r || v != v) ? __longlong_as_double(0x7ff8000000000000ll) : (v > r ? v : r);
  }
  r = block_max_nan(r, red);
  if (threadIdx.x == 0) out[inst] = r;
}

// Branch certificate of an iterate, one workgroup per instance
// (certify_block).
__global__ void k_certify(int n, int check_a, const double* __restrict__ x,
                          int* __restrict__ flags) {
  __shared__ double red[1024 / WAVE];
  __shared__ int bits;
  const double* A = x + (size_t)blockIdx.x * 2 * n;
  const int b = certify_block(n, check_a, A, A + n, red, &bits);
  if (threadIdx.x == 0) flags[blockIdx.x] = b;
}

}  // namespace

// ---------------------------------------------------------------- launchers
hipError_t launch_precompute(hipStream_t st, int n, int nq, int na, int ldk, const double* s,
                             const double* t, const double* W, const double* z, const double* wz,
                             double omega, int with_domega, double* K, double* dK, double gir,
                             int uv) {
  const long total = (long)n * ldk;
  const int bs = 256;
  hipLaunchKernelGGL(k_precompute, dim3((unsigned)((total + bs - 1) / bs)), dim3(bs), 0, st, n, nq,
                     na, ldk, s, t, W, z, wz, omega, with_domega, gir, uv, K, dK);
  return hipGetLastError();
}

hipError_t launch_qc_sweep(hipStream_t st, int n_inst, int n, int nq, int ldk,
                           const InstDev* inst, const double* K, size_t kstride, const int* lo,
                           const double* sw, const double* t, const double* s, const QcPoint& zp,
                           const double* x_in, double* x_out, double* sig,
                           SolveState* state, const SolveCtl* ctl, int k, hipEvent_t ev0,
                           hipEvent_t ev1) {
  const size_t lds = ((size_t)5 * ldk + 1) * sizeof(double);
  const dim3 grid((n + 1 + 3) / 4, n_inst);
  if (ev0)
    hipExtLaunchKernelGGL(k_sweep_row<true>, grid, dim3(256), (uint32_t)lds, st, ev0, ev1, 0,
                          n_inst, n, nq, ldk, inst, K, kstride, lo, sw, t, s, x_in, x_out, state,
                          ctl, k, 0, zp, sig);
  else
    hipLaunchKernelGGL(k_sweep_row<true>, grid, dim3(256), lds, st, n_inst, n, nq, ldk, inst, K,
                       kstride, lo, sw, t, s, x_in, x_out, state, ctl, k, 0, zp, sig);
  hipLaunchKernelGGL(k_qc_update, dim3(n_inst), dim3(256), 0, st, n_inst, n, inst,
                     (const double*)sig, x_in, x_out, state, ctl, k);
  return hipGetLastError();
}

hipError_t launch_solve_init(hipStream_t st, int n_inst, SolveState* state, SolveCtl* ctl,
                             SolveCtl v, const double* x_src, double* x_dst, long xlen) {
  long threads = n_inst;
  if (x_src && xlen > threads) threads = xlen < (1l << 20) ? xlen : (1l << 20);
  hipLaunchKernelGGL(k_solve_init, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, st,
                     n_inst, state, ctl, v, x_src, x_dst, xlen);
  return hipGetLastError();
}

hipError_t launch_sweep_fp64(hipStream_t st, int n_inst, int n, int nq, int ldk,
                             const InstDev* inst, const double* K, size_t kstride, const int* lo,
                             const double* sw, const double* t, const double* s,
                             const double* x_in, double* x_out, double* nodes, SolveState* state,
                             const SolveCtl* ctl, int k, int add_f0) {
  hipLaunchKernelGGL(k_nodes, dim3((nq + 255) / 256, n_inst), dim3(256), 0, st, n, nq, ldk, lo,
                     sw, t, x_in, nodes, state, ctl, k);
  const long rows = (long)n_inst * n;
  hipLaunchKernelGGL(k_sweep, dim3((unsigned)((rows + 3) / 4)), dim3(256), 0, st, n_inst, n, nq,
                     ldk, inst, K, kstride, s, nodes, x_in, x_out, state, ctl, k, add_f0);
  return hipGetLastError();
}

hipError_t launch_sweep_fused(hipStream_t st, int n_inst, int n, int nq, int ldk,
                              const InstDev* inst, const double* K, size_t kstride, const int* lo,
                              const double* sw, const double* t, const double* s,
                              const double* x_in, double* x_out, SolveState* state,
                              const SolveCtl* ctl, int k, int add_f0, int rows, hipEvent_t ev0,
                              hipEvent_t ev1) {
  const size_t lds = ((size_t)5 * ldk + 1) * sizeof(double);
  if (rows != 4 && rows != 8 && rows != 16) return hipErrorInvalidValue;
  // (one slot-templated variant that loads a whole row at once measured
  // slower here: more registers, lower occupancy)
  const dim3 grid((n + rows - 1) / rows, n_inst);
  if (rows == 4) {
    const QcPoint none{};
    if (ev0)
      hipExtLaunchKernelGGL(k_sweep_row<false>, grid, dim3(256), (uint32_t)lds, st, ev0, ev1, 0,
                            n_inst, n, nq, ldk, inst, K, kstride, lo, sw, t, s, x_in, x_out,
                            state, ctl, k, add_f0, none, (double*)nullptr);
    else
      hipLaunchKernelGGL(k_sweep_row<false>, grid, dim3(256), lds, st, n_inst, n, nq, ldk, inst,
                         K, kstride, lo, sw, t, s, x_in, x_out, state, ctl, k, add_f0, none,
                         (double*)nullptr);
    return hipGetLastError();
  }
  auto kern = rows == 8 ? k_sweep_fused<8> : k_sweep_fused<16>;
  if (ev0)
    hipExtLaunchKernelGGL(kern, grid, dim3(256), (uint32_t)lds, st, ev0, ev1, 0, n_inst, n, nq,
                          ldk, inst, K, kstride, lo, sw, t, s, x_in, x_out, state, ctl, k, add_f0);
  else
    hipLaunchKernelGGL(kern, grid, dim3(256), lds, st, n_inst, n, nq, ldk, inst, K, kstride, lo,
                       sw, t, s, x_in, x_out, state, ctl, k, add_f0);
  return hipGetLastError();
}

hipError_t launch_contraction_only(hipStream_t st, int n_inst, int n, int nq, int ldk,
                                  const InstDev* inst, const double* K, size_t kstride,
                                  const double* s, const double* x_in, double* x_out,
                                  const double* nodes) {
  const long rows = (long)n_inst * n;
  hipLaunchKernelGGL(k_sweep, dim3((unsigned)((rows + 3) / 4)), dim3(256), 0, st, n_inst, n, nq,
                     ldk, inst, K, kstride, s, nodes, x_in, x_out, (SolveState*)nullptr,
                     (const SolveCtl*)nullptr, 1, 1);
  return hipGetLastError();
}

hipError_t launch_nodes_only(hipStream_t st, int n_inst, int n, int nq, int ldk, const int* lo,
                             const double* sw, const double* t, const double* x, double* nodes) {
  hipLaunchKernelGGL(k_nodes, dim3((nq + 255) / 256, n_inst), dim3(256), 0, st, n, nq, ldk, lo,
                     sw, t, x, nodes, (SolveState*)nullptr, (const SolveCtl*)nullptr, 1);
  return hipGetLastError();
}

hipError_t launch_jvp(hipStream_t st, int n_inst, int n, int nq, int ldk, const InstDev* inst,
                      const double* K, size_t kstride, const int* lo, const double* sw,
                      const double* t, const double* s, const double* x, const double* v,
                      double* jv, double* nodes, const int* act) {
  hipLaunchKernelGGL(k_nodes_dual, dim3((nq + 255) / 256, n_inst), dim3(256), 0, st, n, nq, ldk,
                     lo, sw, t, x, v, nodes, act);
  const long rows = (long)n_inst * n;
  hipLaunchKernelGGL(k_sweep_dual, dim3((unsigned)((rows + 3) / 4)), dim3(256), 0, st, n_inst, n,
                     nq, ldk, inst, K, kstride, s, nodes, x, v, jv, act);
  return hipGetLastError();
}

hipError_t launch_vjp(hipStream_t st, int n_inst, int n, int nq, int ldk, const InstDev* inst,
                      const double* K, size_t kstride, const int* lo, const double* sw,
                      const double* t, const double* s, const double* x, const double* w,
                      double* out, double* nodes, double* part, double* gq, int nchunk,
                      const int* act, bool nodes_ready) {
  if (!nodes_ready)
    hipLaunchKernelGGL(k_nodes, dim3((nq + 255) / 256, n_inst), dim3(256), 0, st, n, nq, ldk, lo,
                       sw, t, x, nodes, (SolveState*)nullptr, (const SolveCtl*)nullptr, 1);
  const int slots = (nq + WAVE - 1) / WAVE;
  const dim3 fgrid((nchunk + 3) / 4, n_inst);
  const size_t flds = (size_t)5 * ldk * sizeof(double);
  const int rmax = (n + nchunk - 1) / nchunk;
  const dim3 sgrid((nchunk + 1) / 2, n_inst);
  const size_t slds = ((size_t)5 * ldk + 8 * (size_t)rmax) * sizeof(double);
  if (slots <= 4) {
    hipLaunchKernelGGL(k_vjp_fused<4>, fgrid, dim3(256), flds, st, n_inst, n, nq, ldk, nchunk,
                       inst, K, kstride, s, t, nodes, x, w, out, part, act);
  } else if (slots <= 10) {
    hipLaunchKernelGGL(k_vjp_split<5>, sgrid, dim3(256), slds, st, n_inst, n, nq, ldk, nchunk,
                       rmax, inst, K, kstride, s, t, nodes, x, w, out, part, act);
  } else if (slots <= 18) {
    hipLaunchKernelGGL(k_vjp_split<9>, sgrid, dim3(256), slds, st, n_inst, n, nq, ldk, nchunk,
                       rmax, inst, K, kstride, s, t, nodes, x, w, out, part, act);
  } else {  // large grids: row and column parts as two passes
    const long rows = (long)n_inst * n;
    hipLaunchKernelGGL(k_vjp_rows, dim3((unsigned)((rows + 3) / 4)), dim3(256), 0, st, n_inst, n,
                       nq, ldk, inst, K, kstride, s, t, nodes, w, out, act);
    hipLaunchKernelGGL(k_vjp_cols, dim3((nq + 63) / 64, nchunk, n_inst), dim3(64), 0, st, n_inst,
                       n, nq, ldk, nchunk, inst, K, kstride, s, t, nodes, x, w, part, act);
  }
  hipLaunchKernelGGL(k_vjp_nodes, dim3((nq + 255) / 256, n_inst), dim3(256), 0, st, n_inst, nq,
                     ldk, nchunk, t, nodes, part, gq, act);
  hipLaunchKernelGGL(k_vjp_scatter, dim3((n + 255) / 256, n_inst), dim3(256), 0, st, n_inst, n, nq,
                     ldk, lo, sw, gq, out, act);
  return hipGetLastError();
}

hipError_t launch_conv_stat(hipStream_t st, int n_inst, int n, int mode, const double* x_old,
                            const double* x_new, double* out) {
  hipLaunchKernelGGL(k_conv_stat, dim3(n_inst), dim3(256), 0, st, n, mode, x_old, x_new, out);
  return hipGetLastError();
}

hipError_t launch_select(hipStream_t st, int n_inst, int len, const int* sel, const double* src,
                         double* dst) {
  const long tot = (long)n_inst * len;
  hipLaunchKernelGGL(k_select, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, n_inst, len,
                     sel, src, dst);
  return hipGetLastError();
}

hipError_t launch_certify(hipStream_t st, int n_inst, int n, int check_a, const double* x,
                          int* flags) {
  hipLaunchKernelGGL(k_certify, dim3(n_inst), dim3(256), 0, st, n, check_a, x, flags);
  return hipGetLastError();
}

hipError_t launch_batched_dot(hipStream_t st, int n_inst, int len, const double* a, size_t lda,
                              const double* b, size_t ldb, int nvec, double* out, const int* act) {
  hipLaunchKernelGGL(k_batched_dot, dim3(n_inst, nvec), dim3(256), 0, st, len, a, lda, b, ldb, nvec,
                     out, act);
  return hipGetLastError();
}

hipError_t launch_gs_update(hipStream_t st, int n_inst, int len, const double* V, size_t ldv,
                            int nvec, const double* h, int hstride, double* w, const int* act) {
  const long tot = (long)n_inst * len;
  hipLaunchKernelGGL(k_gs_update, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, n_inst, len,
                     V, ldv, nvec, h, hstride, w, act);
  return hipGetLastError();
}

hipError_t launch_combine(hipStream_t st, int n_inst, int len, const double* V, size_t ldv,
                          int nvec, const double* y, int ystride, double beta, double* out) {
  const long tot = (long)n_inst * len;
  hipLaunchKernelGGL(k_combine, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, n_inst, len, V,
                     ldv, nvec, y, ystride, beta, out);
  return hipGetLastError();
}

hipError_t launch_axpby(hipStream_t st, int n_inst, int len, double alpha, const double* a,
                        const double* scale, const double* b, double* dst) {
  const long tot = (long)n_inst * len;
  hipLaunchKernelGGL(k_axpby, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, n_inst, len,
                     alpha, a, scale, b, dst);
  return hipGetLastError();
}

}  // namespace qdse
