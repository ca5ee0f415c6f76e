// qdse_persistent.hip -- the whole successive-approximation solve of a few
// instances in one cooperative launch (Sec. I eq. jifen12 with the per-point
// test of Sec. II eq. jifenab2 or its mass-function form).
//
// A few-instance solve at N = 512 does ~7 MFLOP per sweep: launch latency,
// not arithmetic or bandwidth, bounds a kernel-per-sweep driver. Here each of
// G workgroups (all co-resident: cooperative launch) owns the external rows
// i = g, g + G, ... for every instance, keeps the three kernel-matrix rows of
// those i in LDS for the whole solve, and per sweep
//   1. decides from the previous sweep's global test statistics which
//      instances are frozen (all workgroups decide identically),
//   2. copies the current iterate of a group of instances into LDS (coalesced
//      coherent loads) and rebuilds their loop-node functions there
//      (redundantly per workgroup: O(N) work),
//   3. contracts its rows against them (FP64 direct-difference form, the same
//      arithmetic as k_sweep) and writes the new iterate rows,
//   4. folds its rows' test statistics into a per-instance global maximum,
//   5. meets the other workgroups at a grid barrier.
// Iterate and statistics travel through coherent (agent-scope) atomic loads,
// stores and read-modify-writes, which reach the level shared by all L2
// caches; a workgroup arrives at the barrier only after every one of its
// memory operations has been acknowledged (s_waitcnt 0), so no cache
// write-back or invalidation is needed. Arrivals are spread over NCTR
// counters on separate cache lines (workgroup g adds to counter g % NCTR),
// and wavefront 0 polls all of them at once. A plain variant (ordinary
// accesses, release on arrival, acquire after the wait) is kept for checks.
// The barrier wait is bounded: a workgroup that waits too long raises an error
// flag and every workgroup leaves the loop, so the grid always drains.
#include "qdse_internal.h"

namespace qdse {

namespace {

constexpr int PBLOCK = 256;
constexpr int PWAVES = PBLOCK / 64;
constexpr int MAX_RPW = 8;           // rows per workgroup held in LDS
constexpr long SPIN_LIMIT = 1l << 24;  // ~0.5 s of polling before giving up
constexpr double kMassFloorP = 1e-8;   // GeV, as in the kernel-per-sweep path
constexpr int NCTR = 8;                // arrival counters
constexpr int CTR_STRIDE = 32;         // unsigned ints between counters (128 bytes)

__device__ inline double wsum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ inline double stat_p(int mode, double An, double Bn, double Ao, double Bo) {
  const double dA = fabs(An - Ao);
  if (mode == QDSE_CONV_ABS) return fmax(dA, fabs(Bn - Bo));
  const double Mn = Bn / An, Mo = Bo / Ao;
  return fmax(dA, fabs(Mn - Mo) / fmax(fabs(Mn), kMassFloorP));
}

__device__ inline unsigned long long stat_bits(double r) {
  if (isnan(r)) return 0x7ff8000000000000ull;
  return (unsigned long long)__double_as_longlong(r);
}

// Grid-wide barrier number k (1-based) on NCTR monotonically increasing
// counters. Returns false if the wait timed out or another workgroup raised
// the error flag.
__device__ bool grid_sync(unsigned int* ctr, int G, unsigned int k, int* err,
                          bool coherent_data) {
  __shared__ int ok;
  if (coherent_data) __builtin_amdgcn_s_waitcnt(0);  // this thread's accesses acknowledged
  __syncthreads();
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    if (lane == 0) {
      ok = 1;
      unsigned int* mine = ctr + (blockIdx.x % NCTR) * CTR_STRIDE;
      if (coherent_data)
        __hip_atomic_fetch_add(mine, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      else  // release: this workgroup's plain stores before the arrival
        __hip_atomic_fetch_add(mine, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
    // arrivals expected on counter `lane`: k times the workgroups g < G with
    // g % NCTR == lane
    const unsigned int target =
        lane < NCTR ? k * (unsigned int)((G - lane + NCTR - 1) / NCTR) : 0u;
    long spins = 0;
    bool good = true;
    for (;;) {
      bool reached = true;
      if (lane < NCTR)
        reached = __hip_atomic_load(ctr + lane * CTR_STRIDE, __ATOMIC_RELAXED,
                                    __HIP_MEMORY_SCOPE_AGENT) >= target;
      if (__all(reached)) break;
      int bad = 0;
      if (lane == 0) {
        if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) bad = 1;
        if (++spins > SPIN_LIMIT) {
          __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          bad = 1;
        }
      }
      if (__shfl(bad, 0, 64)) {
        good = false;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    if (lane == 0) {
      if (!good) ok = 0;
      if (!coherent_data)  // agent-wide acquire: other workgroups' plain stores
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
  }
  __syncthreads();
  return ok != 0;
}

// Iterate exchange between workgroups. With coherent = 1 every load and store
// of the iterate is an agent-scope relaxed atomic (coherent across the XCDs'
// L2 caches without invalidating them); ordering comes from the release on
// barrier arrival. With coherent = 0 plain accesses plus an agent-scope
// acquire after the barrier are used.
__device__ inline double ld_x(const double* p, int coherent) {
  return coherent ? __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : *p;
}
__device__ inline void st_x(double* p, double v, int coherent) {
  if (coherent)
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  else
    *p = v;
}

struct PArgs {
  int n_inst, n, nq, rpw, G, gsz;  // gsz: instances whose node functions share LDS
  int coherent;  // 1: iterate exchanged with agent-scope atomic loads/stores
  const InstDev* inst;
  const double* K;  // kernel block shared by every instance
  int ldk;
  const int* lo;
  const double* sw;
  const double* t;
  const double* s;
  double* xbuf0;
  double* xbuf1;
  SolveState* state;
  const SolveCtl* ctl;
  unsigned long long* slots;  // [3][n_inst] bits of the per-sweep maxima
  unsigned int* barrier;
  int* flags;  // [0] error, [1] buffer index of the final iterate
};

__global__ void __launch_bounds__(PBLOCK) k_persistent(PArgs a) {
  extern __shared__ double lds[];
  const int n = a.n, nq = a.nq, rpw = a.rpw, G = a.G, g = blockIdx.x;
  double* Kl = lds;                            // [rpw][3][nq]
  double* xs = Kl + (size_t)rpw * 3 * nq;      // [gsz][2n] iterate of a group
  double* nd = xs + (size_t)a.gsz * 2 * n;     // [gsz][4][nq] node functions
  __shared__ int st_status[64];
  __shared__ int st_sweeps[64];
  __shared__ double st_resid[64];
  __shared__ double red[PWAVES][MAX_RPW][4];
  __shared__ unsigned long long wgmax;
  __shared__ int all_frozen;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const SolveCtl ctl = *a.ctl;

  // rows of this workgroup: i = g + r * G
  int nrows = 0;
  for (int r = 0; r < rpw; ++r)
    if (g + r * G < n) nrows = r + 1;
  for (int r = 0; r < nrows; ++r) {
    const int i = g + r * G;
    for (int c = 0; c < 3; ++c)
      for (int j = tid; j < nq; j += PBLOCK)
        Kl[((size_t)r * 3 + c) * nq + j] = a.K[(size_t)c * n * a.ldk + (size_t)i * a.ldk + j];
  }
  for (int q = tid; q < a.n_inst; q += PBLOCK) {
    st_status[q] = 0;
    st_sweeps[q] = 0;
    st_resid[q] = __longlong_as_double(0x7ff0000000000000ll);
  }
  __syncthreads();

  int k = 1;
  bool fine = true;
  for (;; ++k) {
    const double* xc = (k & 1) ? a.xbuf0 : a.xbuf1;  // sweep k reads buf[(k-1)%2]
    double* xn = (k & 1) ? a.xbuf1 : a.xbuf0;
    // 1. decisions from the statistics of sweep k-1
    if (tid == 0) all_frozen = 1;
    __syncthreads();
    for (int q = tid; q < a.n_inst; q += PBLOCK) {
      int stq = st_status[q];
      if (stq == 0) {
        if (st_sweeps[q] > 0) {
          const double prev = __longlong_as_double((long long)__hip_atomic_load(
              &a.slots[(size_t)((k - 1) % 3) * a.n_inst + q], __ATOMIC_RELAXED,
              __HIP_MEMORY_SCOPE_AGENT));
          if (!(prev <= 1.7976931348623157e308)) stq = 3;
          else if (prev < ctl.tol) stq = 1;
          if (stq) st_resid[q] = prev;
        }
        if (stq == 0 && st_sweeps[q] >= ctl.max_iter) {
          stq = 2;
          st_resid[q] = __longlong_as_double((long long)__hip_atomic_load(
              &a.slots[(size_t)((k - 1) % 3) * a.n_inst + q], __ATOMIC_RELAXED,
              __HIP_MEMORY_SCOPE_AGENT));
        }
        st_status[q] = stq;
      }
      if (stq == 0) all_frozen = 0;
      if (g == 0)
        __hip_atomic_store(&a.slots[(size_t)((k + 1) % 3) * a.n_inst + q], 0ull, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    if (all_frozen) break;

    for (int q0 = 0; q0 < a.n_inst; q0 += a.gsz) {
      const int q1 = min(a.n_inst, q0 + a.gsz);
      // 2. iterate of the group into LDS, then the node functions of its
      //    running instances
      for (int e = tid; e < (q1 - q0) * 2 * n; e += PBLOCK) {
        const int q = q0 + e / (2 * n);
        if (st_status[q] == 0) xs[e] = ld_x(xc + (size_t)q0 * 2 * n + e, a.coherent);
      }
      __syncthreads();
#pragma unroll 4
      for (int e = tid; e < (q1 - q0) * nq; e += PBLOCK) {
        const int q = q0 + e / nq, j = e % nq;
        if (st_status[q] != 0) continue;
        const double* xq = xs + (size_t)(q - q0) * 2 * n;
        const int b = a.lo[j];
        const double* w = a.sw + 4 * j;
        double Aq = 0.0, Bq = 0.0;
#pragma unroll
        for (int l = 0; l < 4; ++l) {
          Aq = fma(w[l], xq[b + l], Aq);
          Bq = fma(w[l], xq[n + b + l], Bq);
        }
        const double tj = a.t[j];
        const double Dl = tj * Aq * Aq + Bq * Bq;
        double* ndq = nd + (size_t)(q - q0) * 4 * nq;
        ndq[j] = Aq;
        ndq[nq + j] = Bq;
        ndq[2 * nq + j] = Aq / Dl;
        ndq[3 * nq + j] = Bq / Dl;
      }
      __syncthreads();
      for (int q = q0; q < q1; ++q) {
        const double* xq = xc + (size_t)q * 2 * n;
        double* xo = xn + (size_t)q * 2 * n;
        if (st_status[q] != 0) {  // frozen: carry the iterate forward
          for (int r = tid; r < nrows; r += PBLOCK) {
            const int i = g + r * G;
            st_x(xo + i, ld_x(xq + i, a.coherent), a.coherent);
            st_x(xo + n + i, ld_x(xq + n + i, a.coherent), a.coherent);
          }
          continue;
        }
        const double* ndq = nd + (size_t)(q - q0) * 4 * nq;
        const double* xsq = xs + (size_t)(q - q0) * 2 * n;
        if (tid == 0) wgmax = 0ull;
        // 3. contraction of this workgroup's rows
        const InstDev P = a.inst[q];
        double acc[MAX_RPW][4];
        double Ai[MAX_RPW], Bi[MAX_RPW], si[MAX_RPW];
#pragma unroll
        for (int r = 0; r < MAX_RPW; ++r) {
          acc[r][0] = acc[r][1] = acc[r][2] = acc[r][3] = 0.0;
          if (r < nrows) {
            const int i = g + r * G;
            Ai[r] = xsq[i];
            Bi[r] = xsq[n + i];
            si[r] = a.s[i];
          }
        }
        for (int j = tid; j < nq; j += PBLOCK) {
          const double Aq = ndq[j], Bq = ndq[nq + j], sV = ndq[2 * nq + j], sS = ndq[3 * nq + j];
          const double tsV = a.t[j] * sV;
#pragma unroll
          for (int r = 0; r < MAX_RPW; ++r) {
            if (r < nrows) {
              const double* Kr = Kl + (size_t)r * 3 * nq;
              const double kT = Kr[j], k3 = Kr[nq + j], k0 = Kr[2 * nq + j];
              const double dA = Aq - Ai[r], dB = Bq - Bi[r], sA = Aq + Ai[r];
              const double e = fma(2.0 * sS, dB, fma(si[r], sV, tsV) * dA);
              acc[r][0] = fma(kT, e, acc[r][0]);
              acc[r][1] = fma(k3, sV * sA, acc[r][1]);
              acc[r][2] = fma(kT, fma(sS, dA, -(sV * dB)), acc[r][2]);
              acc[r][3] = fma(k0, sS * sA, acc[r][3]);
            }
          }
        }
#pragma unroll
        for (int r = 0; r < MAX_RPW; ++r) {
          if (r < nrows) {
#pragma unroll
            for (int c = 0; c < 4; ++c) {
              const double v = wsum(acc[r][c]);
              if (lane == 0) red[wave][r][c] = v;
            }
          }
        }
        __syncthreads();
        if (tid < nrows) {
          const int r = tid, i = g + r * G;
          double c4[4];
          for (int c = 0; c < 4; ++c) {
            double v = 0.0;
            for (int w = 0; w < PWAVES; ++w) v += red[w][r][c];
            c4[c] = v;
          }
          const double An = 1.0 + P.pref * (c4[1] - c4[0]);
          const double Bn = P.m + P.pref * fma(2.0 * si[r], c4[2], c4[3]);
          st_x(xo + i, An, a.coherent);
          st_x(xo + n + i, Bn, a.coherent);
          atomicMax(&wgmax, stat_bits(stat_p(ctl.mode, An, Bn, Ai[r], Bi[r])));
        }
        __syncthreads();
        // 4. this workgroup's contribution to the instance's test statistic
        if (tid == 0) {
          atomicMax(&a.slots[(size_t)(k % 3) * a.n_inst + q], wgmax);
          st_sweeps[q] += 1;
        }
      }
      __syncthreads();
    }
    // 5. grid barrier k
    if (!grid_sync(a.barrier, G, (unsigned int)k, a.flags, a.coherent != 0)) {
      fine = false;
      break;
    }
  }
  if (g == 0) {
    for (int q = tid; q < a.n_inst; q += PBLOCK) {
      a.state[q].status = fine ? st_status[q] : 3;
      a.state[q].sweeps = st_sweeps[q];
      a.state[q].resid = st_resid[q];
    }
    if (tid == 0) a.flags[1] = (k - 1) & 1;  // the last completed sweep wrote buf[(k-1)%2]
  }
}

__global__ void k_persistent_reset(unsigned long long* slots, int nslots, unsigned int* barrier,
                                   int* flags) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < nslots) slots[t] = 0ull;
  if (t < NCTR) barrier[t * CTR_STRIDE] = 0u;
  if (t == 0) {
    flags[0] = 0;
    flags[1] = 0;
  }
}

}  // namespace

size_t persistent_lds_bytes(int rpw, int n, int nq, int gsz) {
  return ((size_t)rpw * 3 * nq + (size_t)gsz * (2 * n + 4 * nq)) * sizeof(double);
}

size_t persistent_barrier_words() { return (size_t)NCTR * CTR_STRIDE; }

// Launches the persistent solve; G workgroups, each holding rpw rows. The
// caller has checked that every instance uses kernel block 0, that G
// workgroups of this size are co-resident, and that n_inst <= 64.
hipError_t launch_persistent(hipStream_t st, int n_inst, int n, int nq, int ldk,
                             const InstDev* inst, const double* K, const int* lo,
                             const double* sw, const double* t, const double* s, double* xbuf0,
                             double* xbuf1, SolveState* state, const SolveCtl* ctl,
                             unsigned long long* slots, unsigned int* barrier, int* flags, int G,
                             int rpw, int gsz, int coherent) {
  if (rpw > MAX_RPW || n_inst > 64 || (long)G * rpw < n || gsz < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_persistent_reset, dim3((3 * n_inst + 255) / 256), dim3(256), 0, st, slots,
                     3 * n_inst, barrier, flags);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  PArgs a{n_inst, n, nq, rpw, G, gsz, coherent, inst, K, ldk, lo, sw, t, s, xbuf0, xbuf1, state,
          ctl, slots, barrier, flags};
  const size_t lds = persistent_lds_bytes(rpw, n, nq, gsz);
  e = hipFuncSetAttribute((const void*)k_persistent, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)lds);
  if (e != hipSuccess) return e;
  void* args[] = {&a};
  return hipLaunchCooperativeKernel((const void*)k_persistent, dim3(G), dim3(PBLOCK), args, lds, st);
}

hipError_t persistent_max_blocks(int rpw, int n, int nq, int gsz, int* max_blocks) {
  int dev = 0, ncu = 0, occ = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  const size_t lds = persistent_lds_bytes(rpw, n, nq, gsz);
  e = hipFuncSetAttribute((const void*)k_persistent, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)lds);
  if (e != hipSuccess) return e;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, (const void*)k_persistent, PBLOCK, lds);
  if (e != hipSuccess) return e;
  *max_blocks = occ * ncu;
  return hipSuccess;
}

}  // namespace qdse
