// qdse_sweep_row.h -- device building blocks of the FP64 sweep of the
// projected gap equations (Sec. II eqs. dsesys/dsesys2): the wavefront sum,
// the loop-node functions (interpolated A, B and sigma_V, sigma_S, eq. (2)),
// one loop node's contribution to a row's four sums, and the per-point test
// of Sec. II eq. jifenab2. Shared by the kernel-per-sweep driver and the
// single-launch solve so that both compute every row with the same
// arithmetic in the same order.
#pragma once

#include "qdse_internal.h"

namespace qdse {
namespace sweep {

constexpr int WAVE = 64;
// Floor (GeV) of the relative mass-function test, where M = B/A vanishes.
constexpr double kMassFloor = 1e-8;

// A 64-bit value moved across lanes by a DPP control (two 32-bit halves);
// lanes of rows outside ROWS receive 0.
template <int CTRL, int ROWS>
__device__ inline double dpp_move(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, ROWS, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROWS, 0xF, false);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// Sum over the 64 lanes (all active), returned in every lane: butterflies
// inside each row of 16 lanes (two quad permutations, the half-row and row
// mirrors), then the broadcasts of lanes 15 and 31 gather the four row sums
// in lane 63, which is read back as a scalar. Register-to-register moves
// only, no LDS round trips.
__device__ inline double wave_sum(double v) {
  v += dpp_move<0xB1, 0xF>(v);   // quad_perm [1,0,3,2]
  v += dpp_move<0x4E, 0xF>(v);   // quad_perm [2,3,0,1]
  v += dpp_move<0x141, 0xF>(v);  // row_half_mirror
  v += dpp_move<0x140, 0xF>(v);  // row_mirror: the row sum in every lane of the row
  v += dpp_move<0x142, 0xA>(v);  // row_bcast:15 into rows 1 and 3
  v += dpp_move<0x143, 0xC>(v);  // row_bcast:31 into rows 2 and 3: the total in row 3
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, 63);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// 64-bit lane exchanges of gfx950: permlane32_swap(x, y) swaps lanes 32-63
// of x with lanes 0-31 of y, permlane16_swap(x, y) rows 1 and 3 of x with
// rows 0 and 2 of y (rows of 16 lanes); each 32-bit half moves on its own.
__device__ inline void swap_halves32(double& x, double& y) {
  const long long bx = __double_as_longlong(x), by = __double_as_longlong(y);
  const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)bx, (unsigned)by, false, false);
  const auto hi =
      __builtin_amdgcn_permlane32_swap((unsigned)(bx >> 32), (unsigned)(by >> 32), false, false);
  x = __longlong_as_double((long long)(((unsigned long long)hi[0] << 32) | lo[0]));
  y = __longlong_as_double((long long)(((unsigned long long)hi[1] << 32) | lo[1]));
}
__device__ inline void swap_rows16(double& x, double& y) {
  const long long bx = __double_as_longlong(x), by = __double_as_longlong(y);
  const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)bx, (unsigned)by, false, false);
  const auto hi =
      __builtin_amdgcn_permlane16_swap((unsigned)(bx >> 32), (unsigned)(by >> 32), false, false);
  x = __longlong_as_double((long long)(((unsigned long long)hi[0] << 32) | lo[0]));
  y = __longlong_as_double((long long)(((unsigned long long)hi[1] << 32) | lo[1]));
}

// The four sums over the 64 lanes of a0..a3 (a row's four loop sums),
// returned in every lane. Transpose and add: an exchange of lanes 32-63 of
// (a0, a2) with lanes 0-31 of (a1, a3) lets every lane add one value over
// the two half-waves, an exchange at distance 16 halves again, leaving one
// partial sum per lane (row 0: a0, row 1: a2, row 2: a1, row 3: a3), which
// the butterflies of wave_sum finish inside each row; the totals are read
// from lanes 0, 32, 16 and 48. Every value goes through the same tree of
// additions (pairs at distance 32, then 16, then the row butterflies).
__device__ inline void wave_sum4(double& a0, double& a1, double& a2, double& a3) {
  swap_halves32(a0, a1);
  swap_halves32(a2, a3);
  double w01 = a0 + a1, w23 = a2 + a3;  // lanes 0-31: a0 | a2; 32-63: a1 | a3
  swap_rows16(w01, w23);
  double v = w01 + w23;  // row 0: a0, row 1: a2, row 2: a1, row 3: a3
  v += dpp_move<0xB1, 0xF>(v);   // quad_perm [1,0,3,2]
  v += dpp_move<0x4E, 0xF>(v);   // quad_perm [2,3,0,1]
  v += dpp_move<0x141, 0xF>(v);  // row_half_mirror
  v += dpp_move<0x140, 0xF>(v);  // row_mirror: the row's total in every lane of the row
  const long long b = __double_as_longlong(v);
  auto lane_value = [&](int l) {
    const int lo = __builtin_amdgcn_readlane((int)b, l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
  };
  a0 = lane_value(0);
  a2 = lane_value(16);
  a1 = lane_value(32);
  a3 = lane_value(48);
}

// Forward-mode dual number: value and directional derivative.
struct Dual {
  double v, d;
  __device__ Dual() = default;
  __device__ constexpr Dual(double a, double b) : v(a), d(b) {}
};
__device__ inline Dual operator+(Dual a, Dual b) { return {a.v + b.v, a.d + b.d}; }
__device__ inline Dual operator-(Dual a, Dual b) { return {a.v - b.v, a.d - b.d}; }
__device__ inline Dual operator*(Dual a, Dual b) { return {a.v * b.v, a.d * b.v + a.v * b.d}; }
__device__ inline Dual operator*(double a, Dual b) { return {a * b.v, a * b.d}; }
__device__ inline Dual operator/(Dual a, Dual b) {
  const double q = a.v / b.v;
  return {q, (a.d - q * b.d) / b.v};
}
__device__ inline Dual dual_fma(Dual a, Dual b, Dual c) { return a * b + c; }
__device__ inline double dual_fma(double a, double b, double c) { return fma(a, b, c); }
__device__ inline Dual wave_sum(Dual x) { return {wave_sum(x.v), wave_sum(x.d)}; }

template <class T> __device__ inline T make(double v, double d);
template <> __device__ inline double make<double>(double v, double) { return v; }
template <> __device__ inline Dual make<Dual>(double v, double d) { return {v, d}; }
__device__ inline double val(double x) { return x; }
__device__ inline double val(Dual x) { return x.v; }
__device__ inline double tan_(Dual x) { return x.d; }

// ---------------------------------------------------------------- node functions
// Interpolated A, B at the loop nodes (4-point stencil with a base index known
// from the interleaving, eq. chazhiresult and its cubic analogue) and the
// functions the contraction needs: nodes[inst][5][ldk] =
// {A(t), B(t), sigma_V, sigma_S, t sigma_V}, plus their tangents for Dual.
template <class T>
__device__ inline void node_core(const double w[4], const T xa[4], const T xb[4], double tj,
                                 T* out) {
  T Aq = make<T>(0.0, 0.0), Bq = make<T>(0.0, 0.0);
#pragma unroll
  for (int l = 0; l < 4; ++l) {
    const T wl = make<T>(w[l], 0.0);
    Aq = Aq + wl * xa[l];
    Bq = Bq + wl * xb[l];
  }
  const T tt = make<T>(tj, 0.0);
  const T Dl = tt * Aq * Aq + Bq * Bq;
  const T rD = make<T>(1.0, 0.0) / Dl;  // one division for both
  const T sV = Aq * rD, sS = Bq * rD;
  out[0] = Aq;
  out[1] = Bq;
  out[2] = sV;
  out[3] = sS;
  out[4] = tt * sV;
}

// One loop node's contribution to the four row sums (explicit FMAs).
__device__ inline void row_term(double kT, double k3, double k0, double Aq, double Bq, double sV,
                                double sS, double tsV, double s, double Ai, double Bi, double& a0,
                                double& a1, double& a2, double& a3) {
  const double dA = Aq - Ai, dB = Bq - Bi, sA = Aq + Ai;
  const double e = fma(2.0 * sS, dB, fma(s, sV, tsV) * dA);
  a0 = fma(kT, e, a0);
  a1 = fma(k3, sV * sA, a1);
  a2 = fma(kT, fma(sS, dA, -(sV * dB)), a2);
  a3 = fma(k0, sS * sA, a3);
}

// Lane sums over the lane strides u < U whose kernel entries the wavefront
// holds in registers (loop node j = lane + 64 u): the five node values of
// stride u + 1 are read before the arithmetic of stride u. A stride past the
// last loop node carries zero kernel entries (load_row_regs), so its terms
// add zero without a branch or a select; its node values are read at an
// index clamped to the last loop node (CLAMP), or, where the caller's node
// array holds finite values (its own nodes, or zeros) up to 4 ldk + 64 U,
// at the stride's own index, which saves the per-stride address arithmetic.
// (A loop node with a non-finite value makes the row's sum non-finite either
// way.) Accumulation order per lane: u = 0, 1, ...
template <int U, bool CLAMP = true>
__device__ inline void row_regs(int lane, int nq, int ldk, const double* nd,
                                const double (&kT)[U], const double (&k3)[U],
                                const double (&k0)[U], double s, double Ai, double Bi,
                                double& a0, double& a1, double& a2, double& a3) {
  double c[2][5];  // strides alternate between the two sets (no copies once unrolled)
  auto rd = [&](int u, double(&v)[5]) {
    const int jc = CLAMP ? min(lane + u * WAVE, nq - 1) : lane + u * WAVE;
#pragma unroll
    for (int f = 0; f < 5; ++f) v[f] = nd[f * ldk + jc];
  };
  rd(0, c[0]);
#pragma unroll
  for (int u = 0; u < U; ++u) {
    if (u + 1 < U) rd(u + 1, c[(u + 1) & 1]);
    const double(&v)[5] = c[u & 1];
    row_term(kT[u], k3[u], k0[u], v[0], v[1], v[2], v[3], v[4], s, Ai, Bi, a0, a1, a2, a3);
  }
}

// The kernel entries of row Ki (three matrices `mat` apart) for the lane
// strides u < U of row_regs, zero past the last loop node.
template <int U>
__device__ inline void load_row_regs(int lane, int nq, size_t mat, const double* Ki, double (&kT)[U],
                                     double (&k3)[U], double (&k0)[U]) {
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int j = lane + u * WAVE, jc = min(j, nq - 1);
    const double t = Ki[jc], t3 = Ki[mat + jc], t0 = Ki[2 * mat + jc];
    kT[u] = j < nq ? t : 0.0;
    k3[u] = j < nq ? t3 : 0.0;
    k0[u] = j < nq ? t0 : 0.0;
  }
}

// Lane sums of the FP64 hot sweep over j = j0, j0 + 64, ... < nq.
template <int U = 6>
__device__ inline void row_stream_f64(int j0, int nq, int ldk, size_t mat,
                                      const double* __restrict__ Ki, const double* __restrict__ nd,
                                      double s, double Ai, double Bi, double& a0, double& a1,
                                      double& a2, double& a3) {
  // Loads of U consecutive lane strides are issued before any arithmetic so
  // that a wavefront has ~8 U loads in flight; the accumulation order per lane
  // is still j = j0, j0 + 64, ... whatever U. U = 6 (two load rounds per row
  // at 513 loop nodes) measured fastest among 4, 5, 6, 8 for small batches;
  // the many-workgroup large-batch sweep prefers U = 2 (more resident
  // wavefronts).
  for (int jb = j0; jb < nq; jb += U * WAVE) {
    double kT[U], k3[U], k0[U], Aq[U], Bq[U], sV[U], sS[U], tsV[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int j = jb + u * WAVE;
      if (j < nq) {
        kT[u] = Ki[j];
        k3[u] = Ki[mat + j];
        k0[u] = Ki[2 * mat + j];
        Aq[u] = nd[j];
        Bq[u] = nd[ldk + j];
        sV[u] = nd[2 * ldk + j];
        sS[u] = nd[3 * ldk + j];
        tsV[u] = nd[4 * ldk + j];
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (jb + u * WAVE < nq)
        row_term(kT[u], k3[u], k0[u], Aq[u], Bq[u], sV[u], sS[u], tsV[u], s, Ai, Bi, a0, a1, a2,
                 a3);
  }
}

__device__ inline double test_stat(int mode, double An, double Bn, double Ao, double Bo) {
  const double dA = fabs(An - Ao);
  if (mode == QDSE_CONV_ABS) return fmax(dA, fabs(Bn - Bo));
  const double Mn = Bn / An, Mo = Bo / Ao;
  return fmax(dA, fabs(Mn - Mo) / fmax(fabs(Mn), kMassFloor));
}

// Max over the 64 lanes, in every lane; a NaN in any lane gives NaN.
__device__ inline double wave_max_nan(double v) {
  for (int o = 32; o > 0; o >>= 1) {
    const double w = __shfl_xor(v, o, WAVE);
    v = (v != v || w != w) ? __longlong_as_double(0x7ff8000000000000ll) : (w > v ? w : v);
  }
  return v;
}

// Block-wide (256 threads) max with NaN propagation; result in every thread.
__device__ inline double block_max_nan(double v, double* red) {
  v = wave_max_nan(v);
  if ((threadIdx.x & (WAVE - 1)) == 0) red[threadIdx.x / WAVE] = v;
  __syncthreads();
  double m = red[0];
  for (int k = 1; k < (int)(blockDim.x / WAVE); ++k) {
    const double w = red[k];
    m = (m != m || w != w) ? __longlong_as_double(0x7ff8000000000000ll) : (w > m ? w : m);
  }
  __syncthreads();
  return m;
}

// Branch certificate of an iterate A, B (n points), evaluated by a whole
// workgroup (every thread calls it; red holds blockDim.x / 64 doubles, bits
// one int, both in LDS); the bits are returned in every thread: bit 1 if
// A <= 0 (or A or B not finite) at some node, bit 2 if A < 1 - 1e-9 at some
// node, bit 4 if the mass function M = B/A rises from one node to the next
// by more than 1e-6 max|M| where |M| exceeds 1e-3 max|M| (in the chiral
// limit the far tail of B changes sign at the 1e-6 level of its infrared
// value, and is not looked at). The physical (Nambu) solution of the
// unrenormalised equation has A = 1 + Sigma_A >= 1 (with a maximum at
// intermediate p^2 for the Ball-Chiu vertex) and M falling with p^2 for
// m >= 0; the other fixed points the drivers can reach (successive
// approximation's with A < 0 in the infrared, Newton's with A << 1 and M of
// several GeV, the negative-mass partner, the grid-scale oscillations near
// the end of the branch) fail one of these.
// check_a = 0 skips bit 2 (renormalised setting: A = 1 at p^2 = zeta^2,
// and A may fall below 1 beyond it).
__device__ inline int certify_block(int n, int check_a, const double* A, const double* B,
                                    double* red, int* bits) {
  if (threadIdx.x == 0) *bits = 0;
  double mmax = 0.0;
  int b = 0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    if (!(A[i] > 0.0) || !(A[i] <= 1.7976931348623157e308) || !(fabs(B[i]) <= 1.7976931348623157e308))
      b |= 1;
    if (check_a && !(A[i] >= 1.0 - 1e-9)) b |= 2;
    const double m = fabs(B[i] / A[i]);
    mmax = (mmax != mmax || m != m) ? __longlong_as_double(0x7ff8000000000000ll) : (m > mmax ? m : mmax);
  }
  mmax = block_max_nan(mmax, red);  // contains a barrier: *bits is initialised
  const double rise = 1e-6 * mmax, floor_m = 1e-3 * mmax;
  for (int i = threadIdx.x; i + 1 < n; i += blockDim.x) {
    const double m0 = B[i] / A[i], m1 = B[i + 1] / A[i + 1];
    if (m1 - m0 > rise && (fabs(m0) > floor_m || fabs(m1) > floor_m)) b |= 4;
  }
  if (b) atomicOr(bits, b);
  __syncthreads();
  const int r = *bits;
  __syncthreads();
  return r;
}

}  // namespace sweep
}  // namespace qdse
