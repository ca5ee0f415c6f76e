/* qdse.h -- C ABI of the MI355X (gfx950) solver for the vacuum quark gap
 * equation with the Ball-Chiu vertex (Huang, Duan, Hu, Chen, arXiv:2012.03667).
 *
 * The library evaluates, on one GPU, the successive-approximation map of the
 * projected gap equations (Sec. II, eqs. dsesys, dsesys2; Sec. I, eq. jifen12)
 *     A'(p^2) = 1 + C_F int d^4q/(2pi)^4 g(k^2) I_A / (q^2 A(q^2)^2 + B(q^2)^2)
 *     B'(p^2) = m + C_F int d^4q/(2pi)^4 g(k^2) I_B / (q^2 A(q^2)^2 + B(q^2)^2)
 * with g(k^2) = (8 pi^2 / omega^4) D exp(-k^2/omega^2) (eq. IRGsQC), C_F = 4/3,
 * Gauss-Legendre quadrature in u = ln p^2 (radial) and in z = cos(theta)
 * (angular), external nodes p^2 = s_i (N-point rule) interleaved with loop nodes
 * q^2 = t_j ((N+1)-point rule on the same interval; Sec. III A, eq.
 * pqrelationship), and Lagrange interpolation of A, B at the loop nodes with a
 * bracket known in advance (Sec. III A, eq. chazhiresult; 2-point as in the
 * paper or 4-point).
 *
 * Besides the paper's vacuum setting: batched matrix-core sweeps
 * (precision), Newton-Krylov solves, tangent/adjoint sweeps and implicit
 * gradients (qdse_jvp, qdse_vjp, qdse_jacobian_band, qdse_grad), a launch-shape autotuner
 * (qdse_autotune), the renormalised setting with the full Qin-Chang
 * interaction (qdse_setup_qc), finite chemical potential and temperature
 * (qdse_mu_*), and the general two-equation system of Sec. I (qdse_fred_*).
 *
 * Conventions for every entry point:
 *  - Pointers named d_* are DEVICE pointers (HIP device memory of the GPU that
 *    was current at qdse_setup); all others are host pointers. The caller owns
 *    every array it passes; the library never frees caller memory.
 *  - The unknown vector of one instance is x = [A(s_0..s_{N-1}) | B(s_0..s_{N-1})],
 *    FP64, N = n_radial. A batch is instance-major: x[inst * 2N + k].
 *  - All device work is enqueued on the HIP stream given to qdse_setup.
 *    qdse_iterate, qdse_jvp and qdse_vjp return without synchronising;
 *    qdse_solve and qdse_grad synchronise the stream before they return
 *    because they report convergence to the host.
 *  - Return value: QDSE_OK (0), QDSE_NOT_CONVERGED (1, outputs hold the last
 *    iterate), or a negative error code (outputs unspecified, except that
 *    QDSE_EDIVERGED and QDSE_ESPURIOUS from a solve leave the last iterate
 *    in the caller's array). Arguments are validated before any HIP call.
 *    qdse_strerror names every code. A batch returns its most severe
 *    per-instance outcome (QDSE_ENAN, then QDSE_EDIVERGED, QDSE_ESPURIOUS,
 *    QDSE_NOT_CONVERGED, QDSE_OK); qdse_solve_status gives each instance's.
 *  - A context is not thread-safe; distinct contexts are independent.
 */
#ifndef QDSE_H
#define QDSE_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct qdse_ctx qdse_ctx; /* opaque: grids, kernel matrices, workspaces */

/* Discretisation shared by every instance of a context (Sec. IV: N external
 * momenta, M Gauss-Legendre nodes). */
typedef struct {
  int n_radial;      /* N >= 4 external nodes p^2 = s_i                         */
  int n_angle;       /* M >= 1 angular nodes in z = cos(theta)                   */
  int interp_order;  /* 1: 2-point (eq. chazhiresult), 3: 4-point Lagrange in u  */
  double s_min;      /* p^2 range in GeV^2, 0 < s_min < s_max                    */
  double s_max;
} qdse_grid;

/* Per-instance physics parameters (Sec. II eq. IRGsQC; Sec. IV). */
typedef struct {
  double D;      /* interaction strength, GeV^2, D >= 0   */
  double omega;  /* interaction range, GeV, omega > 0     */
  double m;      /* current-quark mass, GeV                */
} qdse_params;

enum {
  QDSE_OK = 0,
  QDSE_NOT_CONVERGED = 1,
  QDSE_EINVAL = -1,   /* bad argument (size, range, null pointer)            */
  QDSE_ENOMEM = -2,   /* device or host allocation failed                    */
  QDSE_EDEVICE = -3,  /* a HIP call failed (message via qdse_last_error)     */
  QDSE_ENAN = -4,     /* an iterate became NaN or infinite                   */
  QDSE_ENOTSUP = -5,  /* option not available for this context              */
  QDSE_EDIVERGED = -6, /* successive approximation ended without passing
                          its test after the test statistic had risen above
                          100 times its smallest value (checked from sweep
                          30 on, at the host's reads of the solve state):
                          the sweep does not contract near the iterate (the
                          paper's iteration assumes it does)             */
  QDSE_ESPURIOUS = -7  /* the test of eq. jifenab2 passed at a fixed point
                          that fails the branch certificate: A <= 0 at some
                          node, A < 1 - 1e-9 at some node (not checked in
                          the renormalised setting), or M = B/A rising from
                          one node to the next by more than 1e-6 max|M|
                          where |M| > 1e-3 max|M|;
                          the physical (Nambu) solution has A = 1 +
                          Sigma_A >= 1 and a mass function falling with
                          p^2 (m >= 0)                                   */
};

/* Driver of qdse_solve (set at qdse_setup). */
enum {
  QDSE_PICARD = 0,  /* successive approximation, Sec. I eq. jifen12 (the paper's)  */
  QDSE_NEWTON = 1,  /* Newton's method on F(x) - x from the initial functions:
                       each step solves (I - J) dx = F(x) - x by restarted GMRES
                       with Jacobian-vector products; at most 40 steps        */
  QDSE_AUTO = 2     /* successive approximation, then Newton from the initial
                       functions for every instance that did not end at a
                       certified fixed point (not converged, diverged,
                       spurious or non-finite)                               */
};

/* Arithmetic of the contraction over loop nodes, the only O(N^2) step. */
enum {
  QDSE_FP64 = 0,         /* FP64 throughout (direct difference form)          */
  QDSE_FP32_REFINE = 1,  /* FP32 MFMA contraction with FP32 accumulation of
                            the node-column differences from a reference
                            iterate, added to the FP64 products there; an
                            FP64 matrix-core sweep renews the reference
                            every sixth sweep, one phase until the test
                            holds. Environment QDSE_REFINE=phased: FP32
                            sweeps to 1e-5, one FP64 reference sweep, then
                            sweeps of differences from it; =fp64: FP32
                            sweeps to 1e-5, then FP64 matrix-core sweeps    */
  QDSE_FP64_MATRIX = 2   /* FP64 MFMA contraction (split form) for batches    */
};

/* Convergence test of qdse_solve. */
enum {
  QDSE_CONV_ABS = 0,  /* max_i |A'-A| < tol and max_i |B'-B| < tol (eq. jifenab2) */
  QDSE_CONV_MASS = 1  /* max_i |M'-M|/max(|M'|, 1e-8 GeV) < tol and
                         max_i |A'-A| < tol, M = B/A                           */
};

/* Builds the grids, the interpolation stencils and the angular-integrated
 * kernel matrices for n_inst instances that share `grid` and have their own
 * `params[inst]` (instances with equal omega share one set of matrices).
 * precision: QDSE_FP64, QDSE_FP32_REFINE or QDSE_FP64_MATRIX (the last two
 * build the matrices of the matrix-core sweeps and need one common omega:
 * QDSE_ENOTSUP otherwise). solver: QDSE_PICARD, QDSE_NEWTON or QDSE_AUTO,
 * the driver of qdse_solve (Newton steps always use FP64 sweeps).
 * hip_stream: a hipStream_t (NULL = the null stream). On success *out owns all
 * device memory of the context until qdse_destroy.
 * Errors: QDSE_EINVAL (grid or params out of range, n_inst < 1, unknown
 * precision or solver, out == NULL), QDSE_ENOMEM, QDSE_EDEVICE. */
int qdse_setup(const qdse_grid* grid, const qdse_params* params, int n_inst,
               int precision, int solver, void* hip_stream, qdse_ctx** out);

/* Picks the launch shape of the context's sweep by timing the candidates on
 * its own batch (reps timed launches each, the kernels as a solve runs them):
 * rows per workgroup of the FP64 sweep (4: one row per wavefront, 8 or 16)
 * for QDSE_FP64 contexts, row groups of 16 rows per workgroup of the
 * matrix-core contraction (1 or 2; timed on the FP32 kernel for
 * QDSE_FP32_REFINE, which uses it for its FP64 refinement too) otherwise.
 * cache_path (may be NULL): a JSON object of earlier winners keyed by device,
 * path, grid and batch size; a hit sets the shape without timing, a miss
 * times and adds the winner (the file is rewritten). Outputs (each may be
 * NULL): the chosen fused_rows and mm_row_groups, from_cache = 1 on a hit.
 * Renormalised contexts have one shape (nothing is timed). Overwrites the
 * context's work buffers; synchronises the stream.
 * Errors: QDSE_EINVAL (ctx NULL, reps < 1, cache file not writable),
 * QDSE_EDEVICE. */
int qdse_autotune(qdse_ctx* ctx, int reps, const char* cache_path, int* fused_rows,
                  int* mm_row_groups, int* from_cache);

/* Renormalised setting with the full Qin-Chang interaction, beyond the
 * paper: Sec. II (after eq. IRGsQC) keeps only the infrared Gaussian of the
 * Qin-Chang interaction and sets the renormalisation constants to 1. Here
 *  - uv = 1 adds its ultraviolet term, g_UV(k^2) = 8 pi^2 gamma_m
 *    (1 - exp(-k^2/(4 m_t^2))) / (k^2 ln[tau + (1 + k^2/L^2)^2]) with
 *    gamma_m = 12/25, L = 0.234 GeV, tau = e^2 - 1, m_t = 0.5 GeV (4 pi times
 *    the one-loop running coupling at large k^2); the top of the radial grid
 *    is the regulator;
 *  - every sweep is renormalised at p^2 = zeta^2: with the vertex constant
 *    Z_1 = Z_2 (the Ward-Takahashi identity of the Ball-Chiu vertex),
 *    A = Z_2 (1 + Sigma_A), B = Z_4 m + Z_2 Sigma_B, where Sigma are the loop
 *    sums of eq. dsesys at the current iterate and Z_2, Z_4 follow from
 *    A(zeta^2) = 1 and B(zeta^2) = m (params[].m is the current mass at zeta;
 *    m = 0: no mass term). A and B at zeta^2 are interpolated from the
 *    iterate like the loop values. */
typedef struct {
  int uv;       /* 0 or 1: the ultraviolet term of the interaction          */
  double zeta;  /* renormalisation point in GeV, s_min < zeta^2 < s_max     */
} qdse_qc;

/* qdse_setup for the renormalised setting above (FP64 sweeps only). The
 * context supports qdse_iterate, qdse_solve, qdse_solve_group,
 * qdse_solve_stats, qdse_dims, qdse_nodes and qdse_time_contraction (which =
 * 0 times the sums kernel); the other entry points return QDSE_ENOTSUP.
 * Errors: as qdse_setup, and QDSE_EINVAL for qc == NULL, uv not 0 or 1,
 * zeta^2 outside (s_min, s_max) or equal to a loop node, or a grid whose node
 * functions do not fit one workgroup's LDS (about N > 4080 on gfx950). */
int qdse_setup_qc(const qdse_grid* grid, const qdse_params* params, int n_inst,
                  const qdse_qc* qc, void* hip_stream, qdse_ctx** out);

/* Releases every resource of ctx (NULL is allowed). */
void qdse_destroy(qdse_ctx* ctx);

/* Number of external nodes N, loop nodes N+1, angular nodes M, instances. */
int qdse_dims(const qdse_ctx* ctx, int* n_radial, int* n_loop, int* n_angle, int* n_inst);

/* Host copies of the grid: s[N] external p^2, t[N+1] loop q^2 (GeV^2). Either
 * pointer may be NULL. */
int qdse_nodes(const qdse_ctx* ctx, double* s, double* t);

/* Host-only (no HIP call): the grid a context with `grid` would use. Any
 * pointer may be NULL. s[N], u[N]: external p^2 and ln p^2; t[N+1], W[N+1]:
 * loop q^2 and the radial weight (Gauss-Legendre weight in ln q^2 times t^2);
 * z[M], wz[M]: angular nodes and w_a sqrt(1 - z_a^2). Gauss-Legendre nodes and
 * weights are correctly rounded to FP64. Errors: QDSE_EINVAL. */
int qdse_grid_nodes(const qdse_grid* grid, double* s, double* u, double* t, double* W,
                    double* z, double* wz);

/* One sweep x_out = F(x_in) of the successive approximation (Sec. I eq.
 * jifen12) for every instance, in FP64. d_x_in, d_x_out: [n_inst][2N] device,
 * distinct buffers. d_resid (device [n_inst], may be NULL): the paper's
 * per-point test statistic of this sweep (Sec. II eq. jifenab2),
 * max_i max(|A_out - A_in|, |B_out - B_in|), per instance (NaN if any value
 * is NaN). Asynchronous. */
int qdse_iterate(qdse_ctx* ctx, const double* d_x_in, double* d_x_out, double* d_resid);

/* Same sweep with the FP32 MFMA contraction (context set up with
 * QDSE_FP32_REFINE, else QDSE_ENOTSUP). Asynchronous. */
int qdse_iterate_fp32(qdse_ctx* ctx, const double* d_x_in, double* d_x_out);

/* Same sweep with the FP64 MFMA contraction in split form (contexts set up
 * with QDSE_FP32_REFINE or QDSE_FP64_MATRIX, else QDSE_ENOTSUP). Asynchronous. */
int qdse_iterate_fp64_matrix(qdse_ctx* ctx, const double* d_x_in, double* d_x_out);

/* Solve from the initial functions in d_x (Sec. II eq. jifenab1 gives
 * A0 = B0 = 1; any start is accepted) with the context's driver.
 * QDSE_PICARD: successive approximation until the test `conv_mode` holds with
 * tolerance tol (Sec. II eq. jifenab2) or max_iter sweeps are done; each
 * instance stops at its own first passing sweep. QDSE_NEWTON: Newton steps
 * (at most min(max_iter, 40)) until the same test, applied to the sweep
 * x -> F(x) at the current iterate, holds. QDSE_AUTO: successive
 * approximation, then Newton from the initial functions for the instances
 * whose outcome is not QDSE_OK. Every converged instance is checked against
 * the branch certificate (QDSE_ESPURIOUS). d_x is overwritten with the last
 * iterate of every instance. iters[n_inst] (host, may be NULL): evaluations
 * per instance (sweeps, plus Newton's sweeps and Jacobian-vector products,
 * each about one sweep of work); resid[n_inst] (host, may be NULL): the last
 * test statistic. Returns the most severe per-instance outcome: QDSE_OK,
 * QDSE_NOT_CONVERGED (max_iter reached), QDSE_ESPURIOUS, QDSE_EDIVERGED or
 * QDSE_ENAN (qdse_solve_status lists them). Synchronises the stream.
 * Drivers of QDSE_PICARD: with FP64 precision, one kernel block, up to four
 * instances and the iterates, node functions and stencils of all instances
 * within one workgroup's LDS (N = 512: up to three instances), the whole
 * solve runs as one launch, also in the renormalised mode of qdse_setup_qc
 * (same arithmetic, same results bit for bit as the kernel-per-sweep driver,
 * which serves every other case);
 * the environment variable QDSE_PERSISTENT=0 selects the kernel-per-sweep
 * driver, QDSE_PERSISTENT=1 makes the single launch a requirement
 * (QDSE_ENOTSUP where it does not apply). The single launch's waits for the
 * other workgroups are bounded (about a second of polling; QDSE_PERSIST_SPIN
 * sets the number of failed polls, 0 forces the error path in tests): a wait
 * that runs out ends every workgroup and the solve returns QDSE_EDEVICE with
 * d_x unchanged. */
int qdse_solve(qdse_ctx* ctx, double* d_x, double tol, int max_iter, int conv_mode,
               int* iters, double* resid);

/* Per-instance outcome of the last qdse_solve, qdse_solve_group or
 * qdse_newton of ctx: status[n_inst] (host) receives QDSE_OK,
 * QDSE_NOT_CONVERGED, QDSE_ESPURIOUS, QDSE_EDIVERGED or QDSE_ENAN
 * (QDSE_NOT_CONVERGED before any solve). Errors: QDSE_EINVAL. */
int qdse_solve_status(const qdse_ctx* ctx, int* status);

/* The same solve for several contexts at once (for example one per grid
 * class of a mixed batch): ctxs[n_ctx] distinct contexts, d_x[q] the device
 * unknowns of context q, iters[q] / resid[q] host arrays of its n_inst
 * entries (the outer arrays may be NULL, or any entry). Each context runs its
 * own phases on its own stream; the contexts' work overlaps only if their
 * streams differ (set at qdse_setup). QDSE_AUTO contexts hand their
 * uncertified instances to Newton afterwards, one context at a time;
 * QDSE_NEWTON contexts are refused (QDSE_ENOTSUP: call qdse_solve). Returns
 * the most severe outcome of any instance; outputs as for qdse_solve.
 * Synchronises every context's stream. */
int qdse_solve_group(qdse_ctx** ctxs, int n_ctx, double** d_x, double tol, int max_iter,
                     int conv_mode, int** iters, double** resid);

/* Newton's method on the fixed-point residual R(x) = F(x) - x for every
 * instance, for fixed points where successive approximation does not contract:
 * each step solves (I - J) dx = R by restarted GMRES with Jacobian-vector
 * products (to ||.||_2 relative tolerance lin_tol) and sets x += dx. An
 * instance stops when max_i |R_i| < tol (the norm is reduced on the device),
 * when that norm has grown 1e4-fold above its smallest value from the third
 * step on (QDSE_EDIVERGED), or after max_newton steps; converged instances
 * are checked against the branch certificate. d_x: in initial guess, out last iterate. steps[n_inst],
 * resid[n_inst] (host, may be NULL): Newton steps and final max|R|. The
 * Krylov workspace is allocated by the context on its first Newton or
 * adjoint solve and reused afterwards. Returns QDSE_OK, QDSE_NOT_CONVERGED,
 * QDSE_ESPURIOUS, QDSE_EDIVERGED or QDSE_ENAN. Synchronises the stream. */
int qdse_newton(qdse_ctx* ctx, double* d_x, double tol, int max_newton, double lin_tol,
                int* steps, double* resid);

/* Duration in microseconds of the single-launch kernel of the last
 * qdse_solve on this context (HIP events recorded on the context's stream
 * just before and after the launch); QDSE_ENOTSUP if the last solve used
 * another driver. us must not be NULL. */
int qdse_solve_kernel_us(const qdse_ctx* ctx, double* us);

/* Sweep counts of the last qdse_solve per instance (host arrays [n_inst], may
 * be NULL). QDSE_FP32_REFINE in its default form: FP32 sweeps of differences
 * and FP64 reference sweeps; in the phased and fp64 forms: sweeps of the
 * FP32 phase, which stops at max(tol, 1e-5) on the same test, and of the
 * refinement that then runs to tol (its FP64 reference sweep included).
 * Other contexts: 0 and every sweep. */
int qdse_solve_stats(const qdse_ctx* ctx, int* sweeps_fp32, int* sweeps_fp64);

/* Jacobian-vector product d_jv = (dF/dx)(d_x) d_v for every instance (FP64,
 * forward mode through interpolation, node functions and contraction).
 * All [n_inst][2N] device. Asynchronous. */
int qdse_jvp(qdse_ctx* ctx, const double* d_x, const double* d_v, double* d_jv);

/* Transposed product d_out = (dF/dx)(d_x)^T d_w (reverse mode). Asynchronous. */
int qdse_vjp(qdse_ctx* ctx, const double* d_x, const double* d_w, double* d_out);

/* qdse_vjp for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same kernels and result bit for bit, with the reverse sweep's workspace in
 * a fixed device array of 4 Mi doubles (32 MiB) that the library holds on
 * every GPU it runs on until the process ends, instead of buffers the
 * context allocates on its first qdse_vjp. The call itself allocates
 * nothing. A batch needs n_inst * 66 * ldk doubles, ldk = N + 1 rounded up
 * to a multiple of 8 (at N = 512 up to 122 instances); larger batches get
 * QDSE_EINVAL before any device work. Calls on one GPU share the array:
 * calls that overlap in time on one GPU (two streams, or two host threads)
 * race and give undefined results; calls ordered on one stream are safe.
 * Nothing in the array needs to start at zero. Asynchronous. */
int qdse_vjp_noalloc(qdse_ctx* ctx, const double* d_x, const double* d_w, double* d_out);

/* Near-diagonal band of the sweep Jacobian J = dF/dx at d_x (the derivative of
 * the map of Sec. II eqs. dsesys, dsesys2 in the direct-difference form):
 * d_out[inst][i][o][4] (device, FP64, n_inst * N * (2 bw + 1) * 4 values)
 * holds, for l = i - bw + o, the blocks {dF^A_i/dA_l, dF^A_i/dB_l,
 * dF^B_i/dA_l, dF^B_i/dB_l}; entries with l outside [0, N) are zero. Row i
 * depends on A_l, B_l through A_i, B_i themselves (l = i) and through the
 * interpolation stencils of the loop nodes. 0 <= bw < N (QDSE_EINVAL
 * otherwise); QDSE_ENOTSUP for a renormalised context. Asynchronous. The
 * adjoint solve of qdse_grad factors I - band^T (bw = 2) per instance as its
 * preconditioner. */
int qdse_jacobian_band(qdse_ctx* ctx, const double* d_x, int bw, double* d_out);

/* Gradient of a loss L(x*) through the fixed point x* = F(x*; theta), theta =
 * (D, omega, m) per instance, by implicit differentiation: solves
 * (I - J)^T lambda = d_g (J = dF/dx at d_xstar, d_g = dL/dx*) and returns
 * theta_bar = lambda^T dF/dtheta in theta_bar[n_inst][3] (host). The linear
 * solve (restarted GMRES, right-preconditioned by a banded LU of I - band(J)^T,
 * see qdse_jacobian_band; environment QDSE_BAND_PREC=0 switches the
 * preconditioner off) runs until ||residual||_2 < tol ||d_g||_2 for every
 * instance or max_iter Krylov steps. Requires D > 0 for every instance
 * (QDSE_EINVAL otherwise).
 * Returns QDSE_NOT_CONVERGED if the adjoint solve did not reach tol.
 * Synchronises the stream. */
int qdse_grad(qdse_ctx* ctx, const double* d_xstar, const double* d_g, double tol,
              int max_iter, double* theta_bar);

/* Device copy of the three angular-integrated kernel matrices of instance inst,
 * FP64 [3][N][N+1] into d_K (for inspection and tests). With E = exp(-k^2/omega^2),
 * k^2 = p^2 + q^2 - 2 |p||q| z, the angular weight w_a sqrt(1 - z_a^2) (the
 * d^4q measure), W_j = (radial weight in ln q^2) * t_j^2 and L = 1/(t_j - s_i):
 *   K[0][i][j] = W_j t_j L sum_a w_a sqrt(1-z_a^2) E (1 - z_a^2)/k^2
 *   K[1][i][j] = W_j/(2 s_i) sum_a w_a sqrt(1-z_a^2) E [3 r z (s_i+t_j) - 2 s_i t_j (1+2 z^2)]/k^2
 *   K[2][i][j] = (3/2) W_j sum_a w_a sqrt(1-z_a^2) E,      r = sqrt(s_i t_j).
 * These are the angular integrals of the bracketed factors of eq. dsesys2
 * after the transverse-projector algebra (see the kernel source). */
int qdse_kernel_matrices(qdse_ctx* ctx, int inst, double* d_K);

/* Diagnostics: average device duration in milliseconds of one sweep kernel at
 * d_x over `reps` launches on the context's stream; each launch carries a
 * start and a stop HIP event on its own dispatch packet, so the figure is the
 * kernel's execution time without launch gaps. The kernels run exactly as in
 * a solve (masked-run decision, per-instance test statistics) against a
 * private solve state whose tolerance is never met. which = 0: the fused FP64
 * sweep kernel (node functions and the O(N^2) contraction in one launch;
 * QDSE_ENOTSUP on grids whose node functions do not fit one workgroup's LDS,
 * about N > 4080 on gfx950, where sweeps use a node kernel plus a contraction
 * kernel with the same arithmetic);
 * 1: the FP32 matrix-core contraction kernel alone; 2: the FP64 matrix-core
 * contraction kernel alone (node columns are built once before; 1 and 2 need
 * a context with the matrix-core data, else QDSE_ENOTSUP). d_out [n_inst][2N]
 * receives the sweep. Allocates the private state on first use; synchronises
 * the stream. */
int qdse_time_contraction(qdse_ctx* ctx, int which, const double* d_x, double* d_out, int reps,
                          double* avg_ms);

/* ---------------------------------------------------------------------------
 * Finite chemical potential mu, at T = 0 or at finite temperature (the
 * extensions named in Sec. II and V of the paper). Unknowns A(p~), B(p~), C(p~) are complex, p~ = (p_vec, p4 + i mu):
 *   S^-1(p~) = i gamma_vec.p_vec A + i gamma_4 (p4 + i mu) C + B,
 * on an external grid |p_vec| (n_space Gauss-Legendre nodes in ln|p_vec| on
 * [r_min, r_max]) x p4 > 0 (n_time Gauss-Legendre nodes in v, p4 = lam4 sinh v,
 * v in [0, asinh(p4_max/lam4)]); values at p4 < 0 follow from
 * F(|p|, -p4) = F(|p|, p4)^*. The loop grid has one more node per direction on
 * the same intervals (interleaved, so brackets are known in advance), q4 of
 * both signs, and n_angle Gauss-Legendre nodes in the cosine of the angle
 * between p_vec and q_vec (flat weight). The vertex is the Ball-Chiu vertex
 * written with p~, q~ (Sigma_A on the spatial gammas, Sigma_C on gamma_4,
 * difference quotients over q~^2 - p~^2), which satisfies the Ward-Takahashi
 * identity with S^-1(p~); interaction and colour factor as in the vacuum.
 * Unknown layout per instance: complex128 [3][n_space][n_time] (A, B, C),
 * |p_vec|-major; a batch is instance-major. All instances share the grid.
 * ------------------------------------------------------------------------- */
typedef struct qdse_mu_ctx qdse_mu_ctx;

typedef struct {
  int n_space;      /* >= 4 external |p_vec| nodes                          */
  int n_time;       /* >= 4 external p4 > 0 nodes                           */
  int n_angle;      /* 1..256 angular nodes                                 */
  int interp_order; /* 1 or 3 (per direction of the 2-D tensor stencil)    */
  double r_min, r_max;   /* |p_vec| range, GeV, 0 < r_min < r_max           */
  double p4_max, lam4;   /* p4 range [0, p4_max] and sinh-map scale, GeV    */
  double T;              /* temperature, GeV: 0 gives the T = 0 grid above;
                            T > 0 replaces p4 by the fermion Matsubara
                            frequencies w_n = (2n+1) pi T, n < n_time, and
                            the q4 integral by the sum over the same
                            frequencies with weight 2 pi T (int dq4/(2pi) ->
                            T sum_n); no interpolation in the time direction;
                            p4_max and lam4 are then unused               */
} qdse_mu_grid;

typedef struct {
  double D, omega, m; /* as qdse_params                                    */
  double mu;          /* quark chemical potential, GeV, >= 0               */
} qdse_mu_params;

/* Builds a finite-mu context for n_inst instances. Errors as qdse_setup. */
int qdse_mu_setup(const qdse_mu_grid* grid, const qdse_mu_params* params, int n_inst,
                  void* hip_stream, qdse_mu_ctx** out);
void qdse_mu_destroy(qdse_mu_ctx* ctx);

/* Host-only grid arrays (any pointer may be NULL): external ps[n_space],
 * p4[n_time]; loop qs[n_space+1], q4[n_time+1] (q4[n_time] when T > 0) with
 * measure weights wqs = |q|^2 d|q| and wq4 = dq4 per node (2 pi T when
 * T > 0); angular z[n_angle], wz[n_angle]. */
int qdse_mu_grid_nodes(const qdse_mu_grid* grid, double* ps, double* p4, double* qs,
                       double* q4, double* wqs, double* wq4, double* z, double* wz);

/* One finite-mu sweep for every instance (complex128 device arrays, distinct),
 * all instances in one launch with their own mu, m and interaction.
 * Asynchronous. */
int qdse_mu_iterate(qdse_mu_ctx* ctx, const double* d_x_in, double* d_x_out);

/* Successive approximation from d_x until max |F' - F| over the three
 * functions and the grid (complex modulus) < tol for every instance, or
 * max_iter sweeps. iters, resid: host [n_inst] (may be NULL). Returns QDSE_OK,
 * QDSE_NOT_CONVERGED or QDSE_ENAN. Synchronises the stream. */
int qdse_mu_solve(qdse_mu_ctx* ctx, double* d_x, double tol, int max_iter, int* iters,
                  double* resid);

/* The same successive approximation for several finite-mu contexts at once
 * (for example the grid classes of a mixed batch, each context holding the
 * instances of one grid with their own mu, m and interaction): every round
 * enqueues one sweep of each unfinished context on that context's stream,
 * then reads their statistics, so the classes' sweeps overlap when their
 * streams differ. ctxs[n_ctx] distinct; d_x[q], iters[q], resid[q] as for
 * qdse_mu_solve on context q (the outer arrays may be NULL). Returns the
 * most severe code of any context. Synchronises every context's stream. */
int qdse_mu_solve_group(qdse_mu_ctx** ctxs, int n_ctx, double** d_x, double tol, int max_iter,
                        int** iters, double** resid);

/* The same fixed point found with Anderson mixing of depth `depth` (0..16;
 * 0 is plain successive approximation): with g = F(x) and f = g - x at the
 * current iterate, the next iterate is g - dG gamma, where dG, dF hold the
 * differences of the last `depth` images and residuals and gamma minimises
 * |f - dF gamma| (real coefficients on the real and imaginary parts). The
 * stopping test and outputs are those of qdse_mu_solve (iters counts sweeps);
 * a converged instance returns F(x) of its last iterate. The paper iterates
 * plainly; the mixing only reaches the same fixed point in fewer sweeps where
 * successive approximation contracts slowly. Allocates its history on the
 * device per call; synchronises the stream. */
int qdse_mu_solve_anderson(qdse_mu_ctx* ctx, double* d_x, double tol, int max_iter, int depth,
                           int* iters, double* resid);

/* ---- the general system the paper starts from (Sec. I) ------------------
 * Two nonlinear integral equations of the second kind on [a, b] (eq. jifen1):
 *   u(x) = f1(x) + int [K1(x,t) F11(u,v)(t) + Kbar(x,t) F12(u,v)(t)] dt
 *   v(x) = f2(x) + int [K2(x,t) F21(u,v)(t) + Kbar(x,t) F22(u,v)(t)] dt
 * (eq. jifen1 prints F21 twice; the second is read as F22), with the
 * singular kernel of eq. jifen3 taken as Kbar = |x - t|^-alpha for
 * 0 < alpha < 1 and as 1/(x - t) for alpha = 1, solved by successive
 * approximation (eq. jifen12) on the quark equation's discretisation:
 * unknowns at the n Gauss-Legendre nodes x_i of [a, b], integrals on the
 * n + 1 Gauss-Legendre nodes t_j (weights w_j; the two sets interlace, so
 * x_i != t_j), u(t_j) and v(t_j) by Lagrange interpolation on the x grid
 * (2- or 4-point, as eq. chazhiresult and its cubic analogue). The
 * nonlinearities are quadratics F(u, v) = c0 + c1 u + c2 v + c3 u^2 +
 * c4 u v + c5 v^2. */
typedef struct qdse_fred_ctx qdse_fred_ctx;

typedef struct {
  int n;             /* external nodes, 4 <= n <= 65536                       */
  int interp_order;  /* 1 or 3                                                */
  double a, b;       /* the interval, a < b                                   */
  double alpha;      /* singular exponent, 0 < alpha <= 1                     */
} qdse_fred_grid;

typedef struct {
  double c[6];       /* F(u, v) = c0 + c1 u + c2 v + c3 u^2 + c4 u v + c5 v^2 */
} qdse_fred_poly;

/* Host arrays x [n], t [n+1], w [n+1] of the discretisation (no device use).
 * Errors: QDSE_EINVAL. */
int qdse_fred_nodes(const qdse_fred_grid* grid, double* x, double* t, double* w);

/* F: host [4] = F11, F12, F21, F22. d_K1, d_K2: device [n][n+1] row-major,
 * K(x_i, t_j); d_f: device [2n] = f1(x_i) | f2(x_i). The three device arrays
 * stay owned by the caller and are read by every later call (keep them
 * alive and unchanged). Unknowns: device [2n] = u(x_i) | v(x_i).
 * Errors: QDSE_EINVAL (grid out of range, NULL pointer, non-finite
 * coefficient), QDSE_ENOMEM, QDSE_EDEVICE. */
int qdse_fred_setup(const qdse_fred_grid* grid, const qdse_fred_poly* F, const double* d_K1,
                    const double* d_K2, const double* d_f, void* hip_stream,
                    qdse_fred_ctx** out);
void qdse_fred_destroy(qdse_fred_ctx* ctx);

/* One sweep of eq. jifen12, asynchronous on the context's stream. */
int qdse_fred_iterate(qdse_fred_ctx* ctx, const double* d_in, double* d_out);

/* Successive approximation from d_uv (in place) until max |uv' - uv| < tol
 * (the test of eq. jifenab2 on u and v) or max_iter sweeps; *iters = sweeps
 * done, *resid = the last change (either may be NULL). Returns QDSE_OK,
 * QDSE_NOT_CONVERGED or QDSE_ENAN; synchronises the stream. */
int qdse_fred_solve(qdse_fred_ctx* ctx, double* d_uv, double tol, int max_iter, int* iters,
                    double* resid);

/* Average duration of the row kernel over `reps` sweeps d_in -> d_out (events
 * on its dispatch packet), in ms. */
int qdse_fred_time_sweep(qdse_fred_ctx* ctx, const double* d_in, double* d_out, int reps,
                         double* avg_ms);

/* The floor under a latency-bound launch, measured on the current device
 * with events on each dispatch packet (as qdse_time_contraction times its
 * kernels), averaged over 50 launches of `workgroups` x 256 threads:
 * empty_us for a kernel that does nothing, read_us for one that streams
 * read_bytes (rounded up to whole doubles per workgroup) once, coalesced, and
 * writes one value per workgroup. Each output may be NULL. Allocates and
 * frees its own buffers; synchronises hip_stream. Errors: QDSE_EINVAL
 * (workgroups < 1, read_bytes < 0), QDSE_ENOMEM, QDSE_EDEVICE. */
int qdse_measure_launch_floor(void* hip_stream, int workgroups, long long read_bytes,
                              double* empty_us, double* read_us);

/* The ceilings quoted by the rooflines, measured on the current device:
 * copy_gbs: read + write bandwidth of a 1 GiB streaming copy (larger than
 * the Infinity Cache); read_gbs: bandwidth of a read-only streaming pass over
 * 4 GiB (sixteen times the Infinity Cache; the ceiling of read-dominated
 * kernels); mfma32_tflops / mfma64_tflops: dense rate of back-to-back
 * v_mfma_f32_16x16x4f32 / v_mfma_f64_16x16x4f64 with independent
 * accumulators on every compute unit. Each output may be NULL (skipped).
 * Allocates and frees its own buffers; synchronises hip_stream.
 * Errors: QDSE_ENOMEM, QDSE_EDEVICE. */
int qdse_measure_peaks(void* hip_stream, double* copy_gbs, double* mfma32_tflops,
                       double* mfma64_tflops, double* read_gbs);

/* Human-readable name of a status code. */
const char* qdse_strerror(int code);

/* Text of the last HIP failure seen by this thread (empty if none). */
const char* qdse_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* QDSE_H */
