// qdse_persistent.hip -- the whole successive-approximation solve of a few
// instances in one launch (Sec. I eq. jifen12, stopped by the per-point test
// of Sec. II eq. jifenab2 or its mass-function form).
//
// A few-instance sweep at N = 512 is ~7 MFLOP and ~6 MB of kernel matrices:
// with one launch per sweep, launch latency costs more than the sweep's work.
// Here one launch runs every sweep. Each wavefront owns one external row i
// (ceil(n / 8) workgroups of eight wavefronts, all co-resident) and keeps the
// row's three kernel-matrix entries per lane stride in registers for the
// whole solve. The instances take turns, one sweep per turn, in the same
// order in every workgroup; a turn of instance q
//   1. gathers the full iterate x_k of q that its previous turn published
//      (it travelled while the other instances took their turns),
//   2. evaluates the test statistic of sweep k over all rows (from x_{k-1}
//      and x_k in LDS; every workgroup holds the same statistic, so every
//      workgroup takes the same decision) and the loop-node functions of x_k,
//   3. decides whether q stops, and if not
//   4. contracts its rows (the arithmetic and summation order of the
//      kernel-per-sweep row kernel, so both drivers produce the same bits)
//      and publishes x_{k+1}.
// Exchange without a separate barrier: every value travels as two 64-bit
// words, each holding half of the value's bits and the sweep's 32-bit tag,
// written and read with agent-scope atomic stores and loads (single-copy
// atomic, coherent across the caches of the eight XCDs). A reader takes a
// value once both of its words carry the tag of the sweep it waits for, so
// the data is its own arrival flag: one store and one load per value and
// sweep, no counters and no cache write-back or invalidation. Words are
// double-buffered per instance by the parity of k; a workgroup can publish
// sweep k + 2 of q only after every workgroup has published sweep k + 1 of
// q, which each does only after it has finished reading sweep k of q. Tags
// are tag0 + k; the host raises tag0 above every tag of the previous solve,
// so words left from earlier solves never match.
// At the end every workgroup writes its rows of the final iterates, and
// workgroup 0 the outcome and the branch certificate of every instance into
// pinned host memory (one synchronisation and no copies for the host).
// The renormalised mode (template argument QC, below) exchanges the rows'
// loop sums instead and renormalises after the gather.
// Every wait is bounded: a workgroup that polls too long stores the solve's
// tag0 into the error word and every workgroup leaves the loop at its next
// poll, so the grid always drains (an older value in the error word belongs
// to an earlier solve and is ignored).
// Co-residency: the host launches only grids that fit the device at once
// (persistent_fits: ceil(n / 8) workgroups against occupancy x compute
// units). The launch is an ordinary one: work of
// other streams can delay the dispatch of some workgroups but not prevent it,
// since nothing it waits for depends on this kernel. (A cooperative launch
// gives the same guarantee, but after one the HIP runtime ran the later
// multi-stream work of the process markedly slower: 8.4 against 5.1 ms for a
// batch of eight grid classes on their own streams.)
#include "qdse_internal.h"
#include "qdse_sweep_row.h"

namespace qdse {

namespace {

using namespace sweep;

constexpr int PBLOCK = 512;                 // eight wavefronts, one row each
constexpr int PROWS = PBLOCK / WAVE;
constexpr int PMAX_INST = 4;                // instances of one solve
constexpr int ROW_REG = 9;                  // lane strides of the row held in registers
constexpr int GATHER_PT = 2;                // values per thread per gather round
constexpr long SPIN_LIMIT = 1l << 20;       // default: polls (each ~1-2 us) before giving up
constexpr int ERR_CHECK_EVERY = 16;         // polls between reads of the error word
// Divergence of successive approximation: from sweep DIVERGE_AFTER on, a
// statistic above DIVERGE_FACTOR times the smallest one seen so far marks
// the instance (reported as diverged if it ends without passing the test).
constexpr double DIVERGE_FACTOR = 100.0;
constexpr int DIVERGE_AFTER = 30;

struct PArgs {
  int n_inst, n, nq, ldk;
  const InstDev* inst;
  const double* K;   // kernel block shared by every instance: [3][rows][ldk]
  const double* sw;  // stencil weights [nq][4]; base clamp(j - 2, 0, n - 4)
  const double* t;   // loop nodes
  const double* s;   // external nodes
  double* x;         // [n_inst][2n]: starting iterate in, solution out
  unsigned long long* xw;  // [2][n_inst][2n][2] tagged words
  PersistOut* out;   // per-instance outcome and branch certificate (host-mapped)
  double tol;
  int max_iter, mode;
  unsigned tag0;
  unsigned* err;
  long spin_limit;  // failed polls of one gather round before the solve is abandoned
  QcPoint zp;       // renormalised mode: the renormalisation point's node and stencil
};

__device__ inline unsigned long long tagged(unsigned half, unsigned tag) {
  return ((unsigned long long)tag << 32) | half;
}

__device__ inline unsigned long long bits_of(double v) {
  return (unsigned long long)__double_as_longlong(v);
}
__device__ inline double from_bits(unsigned long long b) { return __longlong_as_double((long long)b); }

// Max over the 64 lanes of non-negative values, in every lane (v_max_f64
// through the butterflies and row broadcasts of wave_sum; lanes a row
// broadcast leaves out receive 0, which is neutral). NaN is the caller's.
__device__ inline double wave_max_nonneg(double v) {
  v = fmax(v, dpp_move<0xB1, 0xF>(v));
  v = fmax(v, dpp_move<0x4E, 0xF>(v));
  v = fmax(v, dpp_move<0x141, 0xF>(v));
  v = fmax(v, dpp_move<0x140, 0xF>(v));
  v = fmax(v, dpp_move<0x142, 0xA>(v));
  v = fmax(v, dpp_move<0x143, 0xC>(v));
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, 63);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// The test statistic of one row (test_stat) with M_old = Bo/Ao supplied (the
// value the previous sweep's statistic computed for the row); M_new = Bn/An
// is returned for the next sweep. Same operations, same bits.
__device__ inline double test_stat_m(int mode, double An, double Bn, double Ao, double Bo,
                                     double Mo, double& Mn) {
  const double dA = fabs(An - Ao);
  if (mode == QDSE_CONV_ABS) {
    Mn = 0.0;
    return fmax(dA, fabs(Bn - Bo));
  }
  Mn = Bn / An;
  return fmax(dA, fabs(Mn - Mo) / fmax(fabs(Mn), kMassFloor));
}

// Doubles per instance of the node-function block: five columns of ldk, and
// room for the unclamped reads of row_regs (up to 4 ldk + 64 ROW_REG).
__host__ __device__ inline size_t node_block(int ldk) {
  const size_t need = (size_t)4 * ldk + (size_t)ROW_REG * WAVE;
  return need > (size_t)5 * ldk ? need : (size_t)5 * ldk;
}

// QC: the renormalised mode (Qin-Chang interaction with its ultraviolet term,
// renormalisation at zeta). The kernel matrices have n + 1 rows, row n at
// p^2 = zeta^2 with A and B interpolated there (the stencil of zp); a
// wavefront publishes its row's loop sums times pref, sigma_A and sigma_B
// (row n's two after the 2n of the others), and a workgroup that has gathered
// them forms Z_2 = 1 / (1 + sigma_A(zeta)), Z_4 m = m - Z_2 sigma_B(zeta) (0 at
// m = 0), A = Z_2 (1 + sigma_A), B = Z_4 m + Z_2 sigma_B: the arithmetic of the
// kernel-per-sweep renormalised sweep, so both drivers give the same bits.
template <bool QC>
__global__ void __launch_bounds__(PBLOCK) k_persistent(PArgs a) {
  extern __shared__ double lds[];
  const int n = a.n, nq = a.nq, ldk = a.ldk, nI = a.n_inst;
  const int tid = threadIdx.x, lane = tid & (WAVE - 1), wave = tid / WAVE;
  const int i = blockIdx.x * PROWS + wave;
  const int rows = QC ? n + 1 : n;
  const bool row_ok = i < rows;
  const int ic = row_ok ? i : rows - 1;  // rows past the last compute and publish nothing
  const bool zrow = QC && ic == n;       // the renormalisation point's row
  const int xl = 2 * n;
  const int xlw = xl + (QC ? 2 : 0);  // exchanged values per instance (QC: + sigma(zeta))
  // node functions of one instance: five columns, then zeros up to the last
  // index the register-held strides read (row_regs without clamping)
  const size_t ndl = node_block(ldk);
  double* xs = lds;                          // [2][nI][2n]: x_k of instance q at parity k & 1
  double* ms = xs + (size_t)2 * nI * xlw;    // [2][nI][n]: M = B/A of the same iterates
  double* nd = ms + (size_t)2 * nI * n;      // [nI][5][ldk] node functions
  double* wsl = nd + (size_t)nI * ndl;       // [nq][4] stencil weights
  double* tl = wsl + (size_t)4 * nq;         // [nq] loop nodes
  __shared__ unsigned long long st_max[PMAX_INST][2];
  __shared__ double s_pref[PMAX_INST], s_m[PMAX_INST];
  __shared__ double red[PBLOCK / WAVE];
  __shared__ int ok, cbits;

  // the row's kernel entries, for the whole solve
  const size_t mat = (size_t)rows * ldk;
  const double* Ki = a.K + (size_t)ic * ldk;
  double kT[ROW_REG], k3[ROW_REG], k0[ROW_REG];
  load_row_regs<ROW_REG>(lane, nq, mat, Ki, kT, k3, k0);
  const double s = zrow ? a.zp.s : a.s[ic];
  for (int e = tid; e < 4 * nq; e += PBLOCK) wsl[e] = a.sw[e];
  for (int e = tid; e < nq; e += PBLOCK) tl[e] = a.t[e];
  if constexpr (QC) {
    for (int e = tid; e < nI * xl; e += PBLOCK) xs[(e / xl) * xlw + e % xl] = a.x[e];
  } else {
    for (int e = tid; e < nI * xl; e += PBLOCK) xs[e] = a.x[e];  // x_0 at parity 0
  }
  // node blocks zeroed: the padding between and after the columns is read by
  // the unclamped strides of row_regs (with zero kernel entries)
  for (size_t e = tid; e < (size_t)nI * ndl; e += PBLOCK) nd[e] = 0.0;
  if (tid < nI) {
    s_pref[tid] = a.inst[tid].pref;
    s_m[tid] = a.inst[tid].m;
  }
  if (tid < 2 * PMAX_INST) st_max[tid / 2][tid % 2] = 0ull;
  if (tid == 0) ok = 1;
  __syncthreads();

  // Node functions of loop node j of instance q's iterate x at parity p.
  auto node = [&](int q, int p, int j) {
    const double* xq = xs + ((size_t)p * nI + q) * xlw;
    const int b = min(max(j - 2, 0), n - 4);
    double w[4], xa[4], xb[4], v[5];
#pragma unroll
    for (int l = 0; l < 4; ++l) {
      w[l] = wsl[4 * j + l];
      xa[l] = xq[b + l];
      xb[l] = xq[n + b + l];
    }
    node_core<double>(w, xa, xb, tl[j], v);
    double* ndq = nd + (size_t)q * ndl;
#pragma unroll
    for (int c = 0; c < 5; ++c) ndq[c * ldk + j] = v[c];
  };
  for (int q = 0; q < nI; ++q) {
    const double* x0 = xs + (size_t)q * xlw;
    for (int j = tid; j < nq; j += PBLOCK) node(q, 0, j);
    for (int ii = tid; ii < n; ii += PBLOCK) ms[(size_t)q * n + ii] = x0[n + ii] / x0[ii];
  }
  __syncthreads();

  // Solve state of instance q in lane q of every wavefront (the same in every
  // workgroup): status (0 running, 1 converged, 2 sweep cap, 3 not finite),
  // the sweeps whose iterate the workgroup holds, the deciding statistic.
  int st_v = lane < nI ? (a.max_iter <= 0 ? 2 : 0) : 4;
  int done_v = 0, div_v = 0;
  double resid_v = __longlong_as_double(0x7ff0000000000000ll);  // +inf: no sweep yet
  double rmin_v = resid_v;
  unsigned run = (unsigned)__ballot(st_v == 0);

  // Instances take turns, one sweep per turn, in the same order in every
  // workgroup: a turn of instance q gathers the iterate its previous turn
  // published (in flight meanwhile, behind the other instances' turns),
  // evaluates the test statistic and the node functions, decides, and, if q
  // still runs, contracts and publishes the next iterate.
  unsigned pend = 0;  // instances with a published sweep not yet gathered
  int q = 0;
  // The next turn's instance pf_q: its words are loaded during this turn's
  // contraction and taken into LDS before this turn publishes (so that the
  // wait for them does not queue behind this turn's stores); pf_pend marks
  // this thread's values that did not yet carry the tag.
  int pf_q = -1;
  unsigned pf_pend = 0;
  // one round of loads of the tagged words of the values still pending
  auto load_round = [&](const unsigned long long* wk, int v0, unsigned long long(&lo)[GATHER_PT],
                        unsigned long long(&hi)[GATHER_PT], unsigned mask) {
#pragma unroll
    for (int g = 0; g < GATHER_PT; ++g) {
      if (mask & (1u << g)) {
        const int e = v0 + g * PBLOCK + tid;
        lo[g] = __hip_atomic_load(wk + 2 * e, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        hi[g] = __hip_atomic_load(wk + 2 * e + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
  };
  // the next running instance with a sweep in flight: its first gather round
  // goes out during this turn
  int y = -1, ky = 0;
  unsigned long long pf_lo[GATHER_PT], pf_hi[GATHER_PT];
  unsigned pf_mask = 0;
  auto issue_prefetch = [&]() {
    y = -1;
    pf_mask = 0;
#pragma unroll
    for (int d = 1; d < PMAX_INST; ++d) {
      const int c = (q + d) % PMAX_INST;
      if (y < 0 && ((run >> c) & 1u) && ((pend >> c) & 1u)) y = c;
    }
    if (y >= 0) {
      ky = __builtin_amdgcn_readlane(done_v, y);
#pragma unroll
      for (int g = 0; g < GATHER_PT; ++g)
        if (g * PBLOCK + tid < xlw) pf_mask |= 1u << g;
      load_round(a.xw + ((size_t)((ky + 1) & 1) * nI + y) * xlw * 2, 0, pf_lo, pf_hi, pf_mask);
    }
  };
  while (run) {
    while (!((run >> q) & 1u)) q = (q + 1) % PMAX_INST;
    int k = __builtin_amdgcn_readlane(done_v, q);  // sweeps of q held before this turn
    bool issued = false;
    if ((pend >> q) & 1u) {
      // gather x_{k+1} of q
      const unsigned tag = a.tag0 + (unsigned)(k + 1);
      const unsigned long long* wk = a.xw + ((size_t)((k + 1) & 1) * nI + q) * xlw * 2;
      double* xn = xs + ((size_t)((k + 1) & 1) * nI + q) * xlw;
      bool good = true;
      long spins = 0;
      for (int v0 = 0; v0 < xlw && good; v0 += GATHER_PT * PBLOCK) {
        unsigned long long lo[GATHER_PT], hi[GATHER_PT];
        unsigned pending = 0;
#pragma unroll
        for (int g = 0; g < GATHER_PT; ++g)
          if (v0 + g * PBLOCK + tid < xlw) pending |= 1u << g;
        if (v0 == 0 && pf_q == q) pending &= pf_pend;  // the rest is in LDS already
        while (pending) {
          load_round(wk, v0, lo, hi, pending);
#pragma unroll
          for (int g = 0; g < GATHER_PT; ++g) {
            if ((pending & (1u << g)) && (unsigned)(lo[g] >> 32) == tag &&
                (unsigned)(hi[g] >> 32) == tag) {
              xn[v0 + g * PBLOCK + tid] =
                  from_bits(((hi[g] & 0xffffffffull) << 32) | (lo[g] & 0xffffffffull));
              pending &= ~(1u << g);
            }
          }
          if (!pending) break;
          ++spins;
          if (spins % ERR_CHECK_EVERY == 0 &&
              __hip_atomic_load(a.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == a.tag0) {
            good = false;
            break;
          }
          if (spins > a.spin_limit) {
            __hip_atomic_store(a.err, a.tag0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            good = false;
            break;
          }
          __builtin_amdgcn_s_sleep(1);
        }
      }
      if (!good) ok = 0;
      pf_q = -1;
      __syncthreads();
      if (!ok) break;
      if constexpr (QC) {
        // the gathered sums of sweep k + 1 into A and B (every thread the
        // values it gathered, Z_2 and Z_4 m from the two at the end)
        const double Z2 = 1.0 / (1.0 + xn[xl]);
        const double mq = s_m[q];
        const double Z4m = mq == 0.0 ? 0.0 : mq - Z2 * xn[xl + 1];
        for (int e = tid; e < xl; e += PBLOCK) xn[e] = e < n ? Z2 * (1.0 + xn[e]) : Z4m + Z2 * xn[e];
        __syncthreads();
      }
      k += 1;
      pend &= ~(1u << q);
      // statistic of sweep k over all rows (M of x_k kept for the next one)
      // and the node functions of x_k (built before the decision: for an
      // instance that stops here they are not used)
      const double* xo = xs + ((size_t)((k - 1) & 1) * nI + q) * xlw;
      const double* xq = xs + ((size_t)(k & 1) * nI + q) * xlw;
      const double* mo = ms + ((size_t)((k - 1) & 1) * nI + q) * n;
      double* mn = ms + ((size_t)(k & 1) * nI + q) * n;
      if (tid == 0) st_max[q][(k + 1) & 1] = 0ull;  // last read at sweep k - 1
      // (the maximum by value with a separate NaN flag: the same result as
      // the maximum of the statistics' bit patterns with NaN above inf)
      double m = 0.0;
      bool bad = false;
      for (int t = tid; t < nq; t += PBLOCK) {
        if (t < n) {
          double Mn;
          const double r = test_stat_m(a.mode, xq[t], xq[n + t], xo[t], xo[n + t], mo[t], Mn);
          bad = bad || !(r == r);
          m = fmax(m, r);
          mn[t] = Mn;
        }
        node(q, k & 1, t);
      }
      const bool wave_bad = __ballot(bad) != 0;
      m = wave_max_nonneg(m);
      if (lane == 0)
        atomicMax(&st_max[q][k & 1], wave_bad ? 0x7ff8000000000000ull : bits_of(m));
      __syncthreads();
      issue_prefetch();
      issued = true;
      // decision (every thread alike)
      const double st = from_bits(st_max[q][k & 1]);
      int sq = 0;
      if (!(st <= 1.7976931348623157e308)) sq = 3;  // NaN or inf
      else if (st < a.tol) sq = 1;
      if (sq == 0 && k >= a.max_iter) sq = 2;
      if (lane == q) {
        done_v = k;
        if (st < rmin_v) rmin_v = st;
        if (k >= DIVERGE_AFTER && st > DIVERGE_FACTOR * rmin_v) div_v = 1;
        if (sq != 0) {
          st_v = sq;
          resid_v = st;
        }
      }
      if (sq != 0) {
        run &= ~(1u << q);
        q = (q + 1) % PMAX_INST;
        continue;
      }
    }
    if (!issued) issue_prefetch();
    // contraction of this wavefront's row of q from x_k: x_{k+1}, published
    // tagged (lanes 0-3: the halves of A_i and B_i)
    {
      const double* xq = xs + ((size_t)(k & 1) * nI + q) * xlw;
      const double* ndq = nd + (size_t)q * ndl;
      double Ai, Bi;
      if (zrow) {  // A and B interpolated at the renormalisation point
        Ai = 0.0;
        Bi = 0.0;
#pragma unroll
        for (int l = 0; l < 4; ++l) {
          Ai = fma(a.zp.w[l], xq[a.zp.base + l], Ai);
          Bi = fma(a.zp.w[l], xq[n + a.zp.base + l], Bi);
        }
      } else {
        Ai = xq[ic];
        Bi = xq[n + ic];
      }
      double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
      row_regs<ROW_REG, false>(lane, nq, ldk, ndq, kT, k3, k0, s, Ai, Bi, a0, a1, a2, a3);
      if (nq > ROW_REG * WAVE)
        row_stream_f64(lane + ROW_REG * WAVE, nq, ldk, mat, Ki, ndq, s, Ai, Bi, a0, a1, a2, a3);
      wave_sum4(a0, a1, a2, a3);
      // published: A and B, or (QC) the sums times pref
      const double An = (QC ? 0.0 : 1.0) + s_pref[q] * (a1 - a0);
      const double Bn = (QC ? 0.0 : s_m[q]) + s_pref[q] * fma(2.0 * s, a2, a3);
      if (y >= 0) {  // take the next instance's words that have arrived
        const unsigned tag = a.tag0 + (unsigned)(ky + 1);
        double* xy = xs + ((size_t)((ky + 1) & 1) * nI + y) * xlw;
        pf_pend = pf_mask;
#pragma unroll
        for (int g = 0; g < GATHER_PT; ++g) {
          if ((pf_mask & (1u << g)) && (unsigned)(pf_lo[g] >> 32) == tag &&
              (unsigned)(pf_hi[g] >> 32) == tag) {
            xy[g * PBLOCK + tid] =
                from_bits(((pf_hi[g] & 0xffffffffull) << 32) | (pf_lo[g] & 0xffffffffull));
            pf_pend &= ~(1u << g);
          }
        }
        pf_q = y;
      }
      if (row_ok && lane < 4) {
        const unsigned tag = a.tag0 + (unsigned)(k + 1);
        unsigned long long* wk = a.xw + ((size_t)((k + 1) & 1) * nI + q) * xlw * 2;
        const unsigned long long bits = bits_of(lane < 2 ? An : Bn);
        const unsigned half = (lane & 1) ? (unsigned)(bits >> 32) : (unsigned)bits;
        const int e = zrow ? (lane < 2 ? xl : xl + 1) : (lane < 2 ? i : n + i);
        __hip_atomic_store(wk + 2 * e + (lane & 1), tagged(half, tag), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
      }
      pend |= 1u << q;
    }
    q = (q + 1) % PMAX_INST;
  }

  if (!ok) return;  // the host reports the error; x is left as it was
  // the final iterate of every instance: this workgroup's rows
  for (int e = tid; e < nI * PROWS * 2; e += PBLOCK) {
    const int qq = e / (PROWS * 2), r = e % (PROWS * 2);
    const int ii = blockIdx.x * PROWS + (r >> 1);
    int kq = 0;
#pragma unroll
    for (int b = 0; b < PMAX_INST; ++b) {
      const int db = __builtin_amdgcn_readlane(done_v, b);
      if (b == qq) kq = db;
    }
    if (ii < n) {
      const int col = (r & 1) ? n + ii : ii;
      a.x[(size_t)qq * xl + col] = xs[((size_t)(kq & 1) * nI + qq) * xlw + col];
    }
  }
  if (blockIdx.x != 0) return;
  // outcome and branch certificate of every instance (workgroup 0)
  for (int qq = 0; qq < nI; ++qq) {
    const int kq = __builtin_amdgcn_readlane(done_v, qq);
    const double* xf = xs + ((size_t)(kq & 1) * nI + qq) * xlw;
    const int cb = certify_block(n, QC ? 0 : 1, xf, xf + n, red, &cbits);
    if (tid == 0) a.out->cert[qq] = cb;
  }
  if (tid < nI) {
    a.out->status[tid] = st_v;
    a.out->sweeps[tid] = done_v;
    a.out->resid[tid] = resid_v;
    a.out->diverged[tid] = div_v;
  }
  __syncthreads();
  if (tid == 0) {
    __atomic_thread_fence(__ATOMIC_RELEASE);
    a.out->tag = a.tag0;
  }
}

}  // namespace

size_t persistent_lds_bytes(int n_inst, int n, int ldk, bool qc) {
  const size_t nq = (size_t)n + 1;
  return ((size_t)2 * n_inst * (3 * n + (qc ? 2 : 0)) + (size_t)n_inst * node_block(ldk) + 5 * nq) *
         sizeof(double);
}

size_t persistent_words(int n_inst, int n, bool qc) {
  return (size_t)2 * n_inst * (2 * n + (qc ? 2 : 0)) * 2;
}

int persistent_blocks(int n, bool qc) { return (n + (qc ? 1 : 0) + PROWS - 1) / PROWS; }

int persistent_max_inst() { return PMAX_INST; }

// Whether the single-launch solve of n_inst instances on an n-row grid fits:
// LDS within the device's limit and ceil(rows / 8) workgroups co-resident
// (rows = n, or n + 1 in the renormalised mode).
hipError_t persistent_fits(int n_inst, int n, int ldk, bool qc, bool* fits) {
  *fits = false;
  if (n_inst < 1 || n_inst > PMAX_INST || n < 4) return hipSuccess;
  int dev = 0, ncu = 0, occ = 0, lds_max = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  e = hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
  if (e != hipSuccess) return e;
  const size_t lds = persistent_lds_bytes(n_inst, n, ldk, qc);
  if (lds + 1024 > (size_t)lds_max) return hipSuccess;
  const void* kern = qc ? (const void*)k_persistent<true> : (const void*)k_persistent<false>;
  e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, PBLOCK, lds);
  if (e != hipSuccess) return e;
  *fits = (long)occ * ncu >= persistent_blocks(n, qc);
  return hipSuccess;
}

// Launches the solve. The caller has checked persistent_fits,
// that every instance uses kernel block 0, that xw holds persistent_words
// zero-initialised or older-tagged words, and that no tag in
// (tag0, tag0 + max_iter + 1] was used before on xw or err.
hipError_t launch_persistent(hipStream_t st, int n_inst, int n, int nq, int ldk,
                             const InstDev* inst, const double* K, const double* sw,
                             const double* t, const double* s, double* x,
                             unsigned long long* xw, PersistOut* out, double tol, int max_iter,
                             int mode, unsigned tag0, unsigned* err, hipEvent_t ev0,
                             hipEvent_t ev1, long spin_limit, const QcPoint* zp) {
  if (n_inst < 1 || n_inst > PMAX_INST || n < 4 || nq != n + 1 || max_iter < 0)
    return hipErrorInvalidValue;
  const bool qc = zp != nullptr;
  if (qc && (zp->base < 0 || zp->base > n - 4)) return hipErrorInvalidValue;
  PArgs a{n_inst, n, nq, ldk, inst, K, sw, t, s, x, xw, out, tol, max_iter, mode, tag0, err,
          spin_limit < 0 ? SPIN_LIMIT : spin_limit, qc ? *zp : QcPoint{}};
  const size_t lds = persistent_lds_bytes(n_inst, n, ldk, qc);
  const void* kern = qc ? (const void*)k_persistent<true> : (const void*)k_persistent<false>;
  hipError_t e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  void* args[] = {&a};
  // events (may be null) recorded on the stream just before and after the
  // launch: the kernel's span plus the two markers. (Events carried on the
  // dispatch packet itself cost 16-24 us of host time per launch here,
  // against 4-5 us for the launch and two records; a launch without events
  // was reported complete by the stream ~30 us after its end.)
  if (ev0) {
    e = hipEventRecord(ev0, st);
    if (e != hipSuccess) return e;
  }
  e = hipLaunchKernel(kern, dim3(persistent_blocks(n, qc)), dim3(PBLOCK), args, lds, st);
  if (e != hipSuccess || !ev1) return e;
  return hipEventRecord(ev1, st);
}

}  // namespace qdse
