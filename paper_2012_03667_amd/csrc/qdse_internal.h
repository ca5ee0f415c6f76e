// qdse_internal.h -- shared declarations of the gfx950 gap-equation library
// (host grid construction, kernel launchers and the context layout).
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <vector>

#include "../../include/qdse.h"

namespace qdse {

// Host copy of one discretisation (see qdse_grid.cpp).
struct HostGrid {
  int n = 0, nq = 0, na = 0, ldk = 0;
  std::vector<double> u, s;       // external nodes: ln p^2 and p^2        [n]
  std::vector<double> uq, t, W;   // loop nodes: ln q^2, q^2, weight t^2 du [nq]
  std::vector<double> z, wz;      // angular nodes and w_a sqrt(1 - z_a^2)  [na]
  std::vector<int> lo;            // stencil base index                     [nq]
  std::vector<double> sw;         // stencil weights                        [nq][4]
};

void gauss_legendre(int n, double* x, double* w);
// The n-point rule on [a, b]: x = RN(a + (b - a)(x_GL + 1)/2), w = RN((b - a)/2 w_GL).
void gl_mapped(int n, double a, double b, double* x, double* w);
int build_grid(const qdse_grid& g, HostGrid* hg);
void build_stencils(int n, int order, const double* u, const double* uq, int* lo, double* sw);

// Host copy of a finite-mu discretisation.
struct HostMuGrid {
  int ns = 0, n4 = 0, nqs = 0, nq4 = 0, na = 0;
  std::vector<double> us, ps, v4, p4;          // external nodes and grid variables
  std::vector<double> uqs, qs, wqs;            // loop |q|, weight |q|^2 d|q|
  std::vector<double> vq4, q4, wq4;            // loop |q4|, weight dq4
  std::vector<double> z, wz;                   // angle, flat weight
  std::vector<int> lo_s, lo_4;                 // stencil bases per direction
  std::vector<double> sw_s, sw_4;              // stencil weights per direction
};
int build_mu_grid(const qdse_mu_grid& g, HostMuGrid* h);

// Fixed device workspace of the entry points that allocate nothing
// (qdse_noalloc.hip): kScratchDoubles doubles per device, shared by every
// call on that device. noalloc_scratch returns its device address on
// `device`, looked up once per device.
constexpr size_t kScratchDoubles = (size_t)4 << 20;  // 32 MiB
hipError_t noalloc_scratch(int device, double** ptr);

// Per-instance constants on the device.
struct InstDev {
  double pref;   // C_F/(8 pi^3) * 8 pi^2 D / omega^4: multiplies every loop sum
  double m;      // current mass
  double D;      // interaction strength (for parameter derivatives)
  double omega;  // interaction range
  int kblock;    // which kernel-matrix block (omega class) the instance uses
  int pad;
};

// Per-instance state of a masked run (device).
constexpr int kMetricLanes = 8;
struct SolveState {
  int status;                   // 0 running, 1 converged, 2 max_iter, 3 non-finite
  int sweeps;                   // sweeps done while running (for the host)
  int sweeps_slot[3];           // the same count per sweep slot: sweep k reads slot
                                // (k-1)%3 and writes slot k%3, so no block of a
                                // launch sees a value written in that launch
  int pad;
  double resid;                 // test statistic of the deciding sweep
  // bits of the non-negative max over rows; sweep k uses slot k%3, reads slot
  // (k-1)%3, clears slot (k+1)%3. Each slot has kMetricLanes words that
  // different workgroups fold into with atomic max (workgroup w into lane
  // w % kMetricLanes: one word for every workgroup of an instance serialises
  // their atomics) and that readers reduce with max. In the host mirror,
  // metric[0][0] and metric[1][0] hold the reduced statistics.
  unsigned long long metric[3][kMetricLanes];
};

// Controls of a masked successive-approximation run (device copy).
struct SolveCtl {
  double tol;
  int mode;      // QDSE_CONV_ABS or QDSE_CONV_MASS
  int max_iter;
  // Optional host mirror (pinned, device-visible): the deciding block of
  // every sixth sweep (k a multiple of 6, so the last sweep of every chunk)
  // writes the instance's new status, sweep count and resid, and the test
  // statistics of the two previous sweeps (metric[0]: sweep `sweeps` - 1,
  // metric[1]: sweeps - 2), at mirror[state - base].
  SolveState* mirror;
  const SolveState* base;
};

// Matrices per kernel block: K_T, K_3, K_0 (see qdse_kernels.hip).
constexpr int NKER = 3;

// ---- launchers (qdse_kernels.hip); all asynchronous on `st` --------------
// Kernel matrices of one interaction class for n external rows. gir and uv
// select the interaction: uv = 0: exp(-k^2/omega^2) (D/omega^4 stays in the
// instance's pref); uv = 1: gir exp(-k^2/omega^2) + the ultraviolet term of
// the Qin-Chang interaction (pref without D).
hipError_t launch_precompute(hipStream_t st, int n, int nq, int na, int ldk, const double* s,
                             const double* t, const double* W, const double* z, const double* wz,
                             double omega, int with_domega, double* K, double* dK,
                             double gir = 1.0, int uv = 0);

// Renormalisation point of the renormalised mode: p^2 = s and the 4-point
// stencil (base, weights) that interpolates the iterate there.
struct QcPoint {
  double s;
  double w[4];
  int base;
  int pad;
};
QcPoint qc_point(const HostGrid& g, int order, double s);
// One sweep with renormalisation at zp (two kernels: the sums of the n + 1
// rows into sig [n_inst][2 (n + 1)] with the masked-run decision, then the
// update). K has n + 1 rows per matrix; ev0/ev1 time the sums kernel.
hipError_t launch_qc_sweep(hipStream_t st, int n_inst, int n, int nq, int ldk,
                           const InstDev* inst, const double* K, size_t kstride, const int* lo,
                           const double* sw, const double* t, const double* s, const QcPoint& zp,
                           const double* x_in, double* x_out, double* sig,
                           SolveState* state, const SolveCtl* ctl, int k,
                           hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
// Fresh solve states; optionally also the controls (ctl, v) and a copy of the
// starting iterate x_src -> x_dst (xlen doubles).
hipError_t launch_solve_init(hipStream_t st, int n_inst, SolveState* state,
                             SolveCtl* ctl = nullptr, SolveCtl v = SolveCtl{},
                             const double* x_src = nullptr, double* x_dst = nullptr,
                             long xlen = 0);
// One FP64 sweep: node functions, then the contraction and update (two
// kernels). With state != nullptr the run is masked (frozen instances carry
// their iterate); k is the 1-based sweep index inside a chunk (a multiple of 6
// sweeps). add_f0 = 0 drops the inhomogeneous terms (1, m) from the output.
hipError_t launch_sweep_fp64(hipStream_t st, int n_inst, int n, int nq, int ldk,
                             const InstDev* inst, const double* K, size_t kstride, const int* lo,
                             const double* sw, const double* t, const double* s,
                             const double* x_in, double* x_out, double* nodes, SolveState* state,
                             const SolveCtl* ctl, int k, int add_f0);
// The same sweep as one kernel: each workgroup rebuilds the node functions of
// its instance in LDS and contracts `rows` rows (bitwise the same arithmetic).
// With ev0/ev1 the launch carries start/stop events on its dispatch packet
// (kernel duration only).
hipError_t launch_sweep_fused(hipStream_t st, int n_inst, int n, int nq, int ldk,
                              const InstDev* inst, const double* K, size_t kstride, const int* lo,
                              const double* sw, const double* t, const double* s,
                              const double* x_in, double* x_out, SolveState* state,
                              const SolveCtl* ctl, int k, int add_f0, int rows,
                              hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
hipError_t launch_contraction_only(hipStream_t st, int n_inst, int n, int nq, int ldk,
                                  const InstDev* inst, const double* K, size_t kstride,
                                  const double* s, const double* x_in, double* x_out,
                                  const double* nodes);
hipError_t launch_nodes_only(hipStream_t st, int n_inst, int n, int nq, int ldk, const int* lo,
                             const double* sw, const double* t, const double* x, double* nodes);
// Tangent and adjoint sweeps. act (nullable, device, one int per instance):
// instances whose flag is 0 are skipped and their outputs left as they were.
// nodes_ready: the node functions of x are already in `nodes` (the adjoint
// reuses them while x stays fixed).
hipError_t launch_jvp(hipStream_t st, int n_inst, int n, int nq, int ldk, const InstDev* inst,
                      const double* K, size_t kstride, const int* lo, const double* sw,
                      const double* t, const double* s, const double* x, const double* v,
                      double* jv, double* nodes, const int* act = nullptr);
hipError_t launch_vjp(hipStream_t st, int n_inst, int n, int nq, int ldk, const InstDev* inst,
                      const double* K, size_t kstride, const int* lo, const double* sw,
                      const double* t, const double* s, const double* x, const double* w,
                      double* out, double* nodes, double* part, double* gq, int nchunk,
                      const int* act = nullptr, bool nodes_ready = false);
hipError_t launch_batched_dot(hipStream_t st, int n_inst, int len, const double* a, size_t lda,
                              const double* b, size_t ldb, int nvec, double* out,
                              const int* act = nullptr);
// w[inst][:] -= sum_v h[inst * hstride + v] V[v][inst][:]  (Gram-Schmidt step)
hipError_t launch_gs_update(hipStream_t st, int n_inst, int len, const double* V, size_t ldv,
                            int nvec, const double* h, int hstride, double* w,
                            const int* act = nullptr);
// Near-diagonal band of the sweep Jacobian at x (qdse_band.hip): D receives
// the direct derivatives [n_inst][n][4]; out the blocks {AA, AB, BA, BB} of
// J[(a,i),(b,l)] for l = i - bw .. i + bw (zero outside the grid), layout
// [inst][i][2bw+1][4], or [i][2bw+1][4][inst] when minor != 0. nodes holds the
// node functions of x.
hipError_t launch_jband(hipStream_t st, int n_inst, int n, int nq, int ldk, int bw,
                        const InstDev* inst, const double* K, size_t kstride, const int* lo,
                        const double* sw, const double* s, const double* t, const double* nodes,
                        const double* x, double* D, double* out, int minor);
// Banded preconditioner of the adjoint solve: band half-width kPrecBand nodes.
// launch_band_lu factors M = I - band(J)^T per instance from the
// instance-minor band (F: [n_inst][2n][4 kPrecBand + 3]; ok[inst] = 0 if a
// pivot was unsafe); launch_band_solve applies M^{-1} (act may be null; in
// and out distinct).
constexpr int kPrecBand = 2;
hipError_t launch_band_lu(hipStream_t st, int n_inst, int n, const double* Jb, double* F, int* ok);
hipError_t launch_band_solve(hipStream_t st, int n_inst, int n, const double* F, const int* ok,
                             const int* act, const double* in, double* out);
// out[inst] = the test statistic (mode QDSE_CONV_ABS or QDSE_CONV_MASS) of the
// change x_old -> x_new of every instance ([n_inst][2n] each); NaN propagates.
hipError_t launch_conv_stat(hipStream_t st, int n_inst, int n, int mode, const double* x_old,
                            const double* x_new, double* out);
// flags[inst] = branch certificate bits of x ([n_inst][2n]): 1 A <= 0 or not
// finite somewhere, 2 A increases with p^2 (checked if check_a), 4 M = B/A
// increases with p^2 (see k_certify).
hipError_t launch_certify(hipStream_t st, int n_inst, int n, int check_a, const double* x,
                          int* flags);
// dst[inst][:] = src[inst][:] (len doubles) where sel[inst] != 0.
hipError_t launch_select(hipStream_t st, int n_inst, int len, const int* sel, const double* src,
                         double* dst);
// out[inst][:] = beta * out[inst][:] + sum_v y[inst * ystride + v] V[v][inst][:]
hipError_t launch_combine(hipStream_t st, int n_inst, int len, const double* V, size_t ldv,
                          int nvec, const double* y, int ystride, double beta, double* out);
// dst[inst][:] = alpha * a[inst][:] + scale[inst] * b[inst][:] (scale may be null: 1)
hipError_t launch_axpby(hipStream_t st, int n_inst, int len, double alpha, const double* a,
                        const double* scale, const double* b, double* dst);

// Matrix-core sweeps (qdse_mfma.hip): five transposed matrices [5][nq_pad][ldi]
// per kernel block and six node columns [6][nq_pad][ldb], element type float
// (FP32 MFMA) or double (FP64 MFMA).
struct MmLayout {
  int nq_pad = 0, ldi = 0, ldb = 0;
  size_t mstride = 0, cstride = 0;
  int rh = 2;  // row groups of 16 rows per workgroup of the contraction (1 or 2)
  int cus = 256;  // compute units of the device (a smaller grid takes deeper prefetch)
};
MmLayout mm_layout(int n, int nq, int n_inst);
template <class T>
hipError_t launch_build_mm(hipStream_t st, int n, int nq, int ldk, const MmLayout& L,
                           const double* K, const double* s, const double* t, T* MT);
// Refinement by differences from a reference iterate x_ref ([n_inst][2n]):
// rq ([6][ldi][ldb] doubles) holds the FP64 products at x_ref in the form that
// makes a row's update affine in its own A_i, B_i. A sweep with rq_out set
// (x_ref, rq null) writes them, and with x_ref_out also copies its input
// iterate there (every running instance; a buffer apart from x_in and x_out);
// a sweep with x_ref and rq set contracts only the node-column differences
// c(x) - c(x_ref) and adds them.
struct MmDelta {
  const double* x_ref = nullptr;
  const double* rq = nullptr;
  double* rq_out = nullptr;
  double* x_ref_out = nullptr;
};
// nodes = false skips the node-column kernel (columns already built); ev0/ev1
// time the contraction kernel's dispatch as in launch_sweep_fused; delta as
// above (nullptr: the plain sweep). hipErrorInvalidValue for an inconsistent
// delta (x_ref without rq or the reverse, rq with rq_out, x_ref_out without
// rq_out or equal to x_in or x_out).
template <class T>
hipError_t launch_sweep_mm(hipStream_t st, int n_inst, int n, int nq, const MmLayout& L,
                           const T* MT, T* C, const InstDev* inst, const int* lo, const double* sw,
                           const double* t, const double* s, const double* x_in, double* x_out,
                           SolveState* state, const SolveCtl* ctl, int k, bool nodes,
                           hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr,
                           const MmDelta* delta = nullptr);

// Finite-mu sweep (qdse_mu.hip); x, L complex interleaved.
// Per-instance constants of a finite-mu sweep: mu, the interaction's
// prefactor 8 pi^2 D / omega^4 and 1 / omega^2, the current mass.
struct MuInst {
  double mu, gnorm, inv_om2, m;
};
// One finite-mu sweep of n_inst instances in one launch (act: nullptr, or
// per instance 0 = copy the iterate forward).
hipError_t launch_mu_sweep(hipStream_t st, int n_inst, int ns, int n4, int nqs, int nq4, int na,
                           const double* ps, const double* p4, const double* qs, const double* q4,
                           const double* wqs, const double* wq4, const double* z, const double* wz,
                           const int* lo_s, const double* sw_s, const int* lo_4,
                           const double* sw_4, const MuInst* inst, const int* act,
                           const double* x_in, double* x_out, double* L);
hipError_t launch_mu_stat(hipStream_t st, int n_inst, int ne, const double* x_old,
                          const double* x_new, unsigned long long* stat);

// General second-kind system (qdse_fred.hip): one sweep on n external and
// n + 1 loop nodes; K1, K2 [n][n+1] row-major, coef [4][6], G [4][n+1]
// workspace, stat (optional) receives max |uv' - uv| as double bits.
hipError_t launch_fred_sweep(hipStream_t st, int n, double alpha, const double* x,
                             const double* t, const double* w, const int* lo, const double* sw,
                             const double* coef, const double* K1, const double* K2,
                             const double* f, const double* uv_in, double* uv_out, double* G,
                             unsigned long long* stat, hipEvent_t ev0 = nullptr,
                             hipEvent_t ev1 = nullptr);
void gl_nodes_on(int n, double a, double b, double* x, double* w);

// Outcome of a single-launch solve, written by its workgroup 0 into pinned
// host memory at the end: per instance the status (0 running, 1 converged,
// 2 sweep cap, 3 not finite), sweeps, deciding statistic, branch
// certificate bits and divergence mark; tag last (the solve's tag0).
struct PersistOut {
  unsigned tag;
  int pad;
  int status[4], sweeps[4];
  double resid[4];
  int cert[4], diverged[4];
};

// Single-launch solve of up to persistent_max_inst() instances
// sharing kernel block 0 (qdse_persistent.hip).
// qc: the renormalised mode (n + 1 kernel-matrix rows, launch with zp).
size_t persistent_lds_bytes(int n_inst, int n, int ldk, bool qc);
size_t persistent_words(int n_inst, int n, bool qc);
int persistent_blocks(int n, bool qc);
int persistent_max_inst();
hipError_t persistent_fits(int n_inst, int n, int ldk, bool qc, bool* fits);
hipError_t launch_persistent(hipStream_t st, int n_inst, int n, int nq, int ldk,
                             const InstDev* inst, const double* K, const double* sw,
                             const double* t, const double* s, double* x,
                             unsigned long long* xw, PersistOut* out, double tol, int max_iter,
                             int mode, unsigned tag0, unsigned* err, hipEvent_t ev0,
                             hipEvent_t ev1, long spin_limit,  // < 0: the default
                             const QcPoint* zp = nullptr);     // renormalised mode

}  // namespace qdse
