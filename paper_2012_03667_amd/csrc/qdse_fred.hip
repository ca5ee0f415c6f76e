// qdse_fred.hip -- the general system the paper starts from (Sec. I, eqs.
// jifen1, jifen3): two nonlinear integral equations of the second kind on
// [a, b] with regular kernels K1, K2 (caller's matrices at (x_i, t_j)) and the
// singular kernel Kbar(x, t) = |x - t|^-alpha (0 < alpha < 1) or 1/(x - t)
// (alpha = 1), solved by successive approximation (eq. jifen12) on the
// quark equation's discretisation: unknowns on GL(n) nodes x_i, integrals on
// the interlaced GL(n+1) nodes t_j, u(t_j) and v(t_j) by Lagrange stencils.
//
// One sweep = two kernels: the node values G[4][nq] = w_j F_k(u(t_j), v(t_j))
// (k = 11, 12, 21, 22), then the rows (two per wavefront) contracting K1, K2
// and the singular kernel (computed in registers) against them.
#include "qdse_internal.h"

namespace qdse {

namespace {

constexpr int FW = 64;

__device__ inline double quad_f(const double* c, double u, double v) {
  return fma(c[5] * v, v, fma(c[4] * u, v, fma(c[3] * u, u, fma(c[2], v, fma(c[1], u, c[0])))));
}

__global__ void __launch_bounds__(256) k_fred_nodes(int n, int nq, const int* __restrict__ lo,
                                                    const double* __restrict__ sw,
                                                    const double* __restrict__ w,
                                                    const double* __restrict__ coef,
                                                    const double* __restrict__ uv,
                                                    double* __restrict__ G) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nq) return;
  const int b = lo[j];
  double u = 0.0, v = 0.0;
#pragma unroll
  for (int l = 0; l < 4; ++l) {
    u = fma(sw[4 * j + l], uv[b + l], u);
    v = fma(sw[4 * j + l], uv[n + b + l], v);
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) G[(size_t)k * nq + j] = w[j] * quad_f(coef + 6 * k, u, v);
}

__device__ inline double fred_wave_sum(double v) {
#pragma unroll
  for (int o = FW / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, FW);
  return v;
}

// Two rows per wavefront (i0 = 2 w, i0 + 1: they share the loop-node reads
// of t and G), lanes striding over j; the reads of U lane strides go out
// before their arithmetic. Per-lane order j = lane, lane + 64, ... . stat:
// max |uv' - uv| of the sweep as the bits of a non-negative double (NaN
// above +inf), one atomic per workgroup.
constexpr int FR = 2;  // rows per wavefront
__global__ void __launch_bounds__(256) k_fred_rows(
    int n, int nq, double alpha, const double* __restrict__ x, const double* __restrict__ t,
    const double* __restrict__ K1, const double* __restrict__ K2, const double* __restrict__ G,
    const double* __restrict__ f, const double* __restrict__ uv_in, double* __restrict__ uv_out,
    unsigned long long* stat) {
  const int lane = threadIdx.x & (FW - 1), wave = threadIdx.x / FW;
  const int i0 = (blockIdx.x * (blockDim.x / FW) + wave) * FR;
  __shared__ unsigned long long wmax[4];
  unsigned long long mine = 0ull;
  if (i0 < n) {
    constexpr int U = 4;
    const int mode = alpha == 1.0 ? 1 : alpha == 0.5 ? 2 : 0;
    double xi[FR];
    const double *k1[FR], *k2[FR];
#pragma unroll
    for (int r = 0; r < FR; ++r) {
      const int i = min(i0 + r, n - 1);  // a missing last row repeats row n - 1, unwritten
      xi[r] = x[i];
      k1[r] = K1 + (size_t)i * nq;
      k2[r] = K2 + (size_t)i * nq;
    }
    double s1[FR], s2[FR];
#pragma unroll
    for (int r = 0; r < FR; ++r) s1[r] = s2[r] = 0.0;
    for (int jb = lane; jb < nq; jb += U * FW) {
      double a1[FR][U], a2[FR][U], tj[U], g0[U], g1[U], g2[U], g3[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int j = min(jb + u * FW, nq - 1);
#pragma unroll
        for (int r = 0; r < FR; ++r) {
          a1[r][u] = k1[r][j];
          a2[r][u] = k2[r][j];
        }
        tj[u] = t[j];
        g0[u] = G[j];
        g1[u] = G[nq + j];
        g2[u] = G[2 * nq + j];
        g3[u] = G[3 * nq + j];
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (jb + u * FW < nq) {
#pragma unroll
          for (int r = 0; r < FR; ++r) {
            const double d = xi[r] - tj[u];
            const double kb = mode == 1   ? 1.0 / d
                              : mode == 2 ? 1.0 / sqrt(fabs(d))
                                          : exp(-alpha * log(fabs(d)));
            s1[r] = fma(a1[r][u], g0[u], fma(kb, g1[u], s1[r]));
            s2[r] = fma(a2[r][u], g2[u], fma(kb, g3[u], s2[r]));
          }
        }
      }
    }
#pragma unroll
    for (int r = 0; r < FR; ++r) {
      const double t1 = fred_wave_sum(s1[r]), t2 = fred_wave_sum(s2[r]);
      const int i = i0 + r;
      if (lane == 0 && i < n) {
        const double un = f[i] + t1, vn = f[n + i] + t2;
        uv_out[i] = un;
        uv_out[n + i] = vn;
        const double rr = fmax(fabs(un - uv_in[i]), fabs(vn - uv_in[n + i]));
        const unsigned long long bits = (unsigned long long)__double_as_longlong(
            isnan(rr) ? __longlong_as_double(0x7ff8000000000000ll) : rr);
        mine = bits > mine ? bits : mine;
      }
    }
  }
  if (!stat) return;
  if (lane == 0) wmax[wave] = mine;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long m = wmax[0];
    for (int q = 1; q < 4; ++q) m = wmax[q] > m ? wmax[q] : m;
    atomicMax(stat, m);
  }
}

}  // namespace

hipError_t launch_fred_sweep(hipStream_t st, int n, double alpha, const double* x,
                             const double* t, const double* w, const int* lo, const double* sw,
                             const double* coef, const double* K1, const double* K2,
                             const double* f, const double* uv_in, double* uv_out, double* G,
                             unsigned long long* stat, hipEvent_t ev0, hipEvent_t ev1) {
  const int nq = n + 1;
  hipLaunchKernelGGL(k_fred_nodes, dim3((nq + 255) / 256), dim3(256), 0, st, n, nq, lo, sw, w,
                     coef, uv_in, G);
  const dim3 grid((n + 4 * FR - 1) / (4 * FR));
  if (ev0)
    hipExtLaunchKernelGGL(k_fred_rows, grid, dim3(256), 0, st, ev0, ev1, 0, n, nq, alpha, x, t,
                          K1, K2, (const double*)G, f, uv_in, uv_out, stat);
  else
    hipLaunchKernelGGL(k_fred_rows, grid, dim3(256), 0, st, n, nq, alpha, x, t, K1, K2,
                       (const double*)G, f, uv_in, uv_out, stat);
  return hipGetLastError();
}

}  // namespace qdse
