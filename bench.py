"""Benchmark: converged quark gap-equation solves per second on one MI355X.

Headline (`value`): the plain FP64 GPU solver on the 512 x 128 vacuum workload
(512 Gauss-Legendre nodes in ln p^2 on [1e-4, 1e4] GeV^2, 513 interleaved loop
nodes, 128 angular nodes in cos(theta), 4-point interpolation), two instances
per step, m = 0 and m = 5 MeV, with the paper's interaction D = 0.55 GeV^2,
omega = 0.678 GeV, from A0 = B0 = 1 (Sec. II eq. jifenab1), successive
approximation until max|dM|/max(|M|, 1e-8 GeV) < 1e-10 and max|dA| < 1e-10.
One step = reset both instances to the initial functions and solve them.

Also reported on the same grid and interaction:
* `batched`: 1024 instances with m ~ U[0, 0.2] GeV solved at equal accuracy
  (1e-7 relative to the oracle's fixed point: test tolerance 1e-8) by
  (a) FP32 matrix-core sweeps to 1e-5 followed by FP64 matrix-core sweeps,
  (b) FP64 matrix-core sweeps only and (c) FP64 direct-difference sweeps only;
  plus the plain two-instance solver at the same tolerance, for the
  equal-accuracy comparison.
* `roofline`: the fused FP64 sweep kernel of the headline solve (HBM bound),
  and `roofline_fp32`: the FP32 MFMA contraction of the batch (MFMA bound),
  each timed live with HIP events on the library's stream.
* `cpu_baseline`: one complete oracle solve of the m = 5 MeV instance on the
  host cores (direct radial x angular sums, OpenMP over rows).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP32_MFMA_PEAK_TFLOPS = 157.3
FP64_MFMA_PEAK_TFLOPS = 78.6
FP64_VALU_PEAK_TFLOPS = 78.6
MU_FLOPS_PER_PAIR = 1617
MU_FLOPS_PER_ANGLE = 36
COPY_BYTES = 1 << 30


def counter_traffic(summary, source):
    """HBM bytes per launch from a committed rocprofv3 counter summary
    (profiles/*.md: lines 'fetch_bytes_per_dispatch:', 'write_bytes_per_dispatch:'
    already scaled by the copy-kernel calibration, and 'source_sha256:' of the
    kernel's source file when the counters were taken). None when the summary
    is missing or the kernel source has changed since."""
    import hashlib
    path = os.path.join(ROOT, "profiles", summary)
    src = os.path.join(ROOT, "paper_2012_03667_amd", "csrc", source)
    if not (os.path.exists(path) and os.path.exists(src)):
        return None
    vals = {}
    for ln in open(path):
        if ":" in ln and ln.split(":", 1)[0].strip() in (
                "fetch_bytes_per_dispatch", "write_bytes_per_dispatch", "source_sha256"):
            k, v = ln.split(":", 1)
            vals[k.strip()] = v.strip().strip("`")
    if len(vals) != 3:
        return None
    if hashlib.sha256(open(src, "rb").read()).hexdigest() != vals["source_sha256"]:
        return None
    return float(vals["fetch_bytes_per_dispatch"]) + float(vals["write_bytes_per_dispatch"])


def paper_table1(O, np, threads):
    """The structure of the paper's Table 1 (Sec. IV) on this host's cores:
    the four algorithms (traditional / modified interpolation inside the loops,
    sequential / OpenMP over external momenta, Sec. III) on the Table 1
    workload N = 150, M = 100, D = 0.55, omega = 0.678, m = 0, A0 = B0 = 1,
    linear interpolation, absolute test xi = 0.005. Every algorithm computes
    the same sweep (checked bitwise in the oracle tests), so one sweep of each
    is timed and the iteration count comes from a full solve with algorithm 4."""
    g = O.vac_grid(150, 100, order=1)
    p = O.Params(0.55, 0.678, 0.0)
    x0 = np.ones(300)
    _, iters = O.picard_paper(g, p, x0, 0.005, modified=True, nthreads=threads)
    per = {}
    for name, modified, th in (("alg1_traditional_sequential", False, 1),
                               ("alg2_modified_sequential", True, 1),
                               ("alg3_traditional_openmp", False, threads),
                               ("alg4_modified_openmp", True, threads)):
        t0 = time.perf_counter()
        O.F_paper(g, p, x0, modified, th)
        per[name] = time.perf_counter() - t0
    a1 = per["alg1_traditional_sequential"]
    return {
        "workload": "N=150, M=100, D=0.55, omega=0.678, m=0, A0=B0=1, linear interpolation, xi=0.005",
        "iterations": int(iters), "threads": threads, "seconds_per_sweep": per,
        "estimated_solve_seconds": {k: v * iters for k, v in per.items()},
        "speedup_vs_alg1": {k: a1 / v for k, v in per.items()},
        "paper_seconds": {"alg1": 65, "alg2": 6, "alg3": 9, "alg4": 1,
                          "hardware": "Intel i7 at 1.00 GHz (model not stated), GCC 9.3, OpenMP"},
    }


def gradient_batch(Q, np, torch, B):
    """B vacuum instances at 512 x 128 with their own interaction (one kernel
    block per instance): kappa = (D omega)^(1/3) ~ U[0.70, 0.825] GeV,
    omega ~ U[0.65, 0.70] GeV, m ~ U[0, 0.1] GeV (seed 5), the region where
    successive approximation converges for every mass; FP64 solve to 1e-12,
    then dL/d(D, omega, m) by the implicit adjoint (banded-LU-preconditioned
    GMRES) for
    L = sum_i (M_i - M_T(s_i))^2, M_T(s) = 0.005 + M0 / (1 + s / Lam2),
    M0 ~ U[0.3, 0.5] GeV, Lam2 ~ U[0.5, 2] GeV^2 (seed 55)."""
    n, na = 512, 128
    rng = np.random.default_rng(5)
    kap = rng.uniform(0.70, 0.825, B)
    om = rng.uniform(0.65, 0.70, B)
    m = rng.uniform(0.0, 0.1, B)
    params = [(float(k ** 3 / o), float(o), float(mm)) for k, o, mm in zip(kap, om, m)]
    rng = np.random.default_rng(55)
    M0 = rng.uniform(0.3, 0.5, B)
    L2 = rng.uniform(0.5, 2.0, B)
    s = Q.grid_nodes(n, na)["s"]
    T = 0.005 + M0[:, None] / (1.0 + s[None, :] / L2[:, None])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    S = Q.Solver(n, na, params, interp_order=3)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    x0 = S.initial(1.0, 1.0)
    x = x0.clone()
    S.solve(x, tol=1e-12, max_iter=3000)  # warm-up (graph capture, clocks)
    x.copy_(x0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rc, it, rs = S.solve(x, tol=1e-12, max_iter=3000)
    torch.cuda.synchronize()
    t_solve = time.perf_counter() - t0
    xs = x.cpu().numpy()
    A, Bf = xs[:, :n], xs[:, n:]
    M = Bf / A
    g = np.concatenate([-2.0 * (M - T) * Bf / A ** 2, 2.0 * (M - T) / A], axis=1)
    gd = torch.tensor(g, device=x.device)
    S.grad(x, gd, tol=1e-12, max_iter=400)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tb, rcg = S.grad(x, gd, tol=1e-12, max_iter=400)
    torch.cuda.synchronize()
    t_grad = time.perf_counter() - t0
    tb = np.asarray(tb)
    # one kernel block per instance: each sweep streams B x 6.3 MB of matrices
    kbytes = 3 * n * (n + 1) * 8
    return {
        "instances": B, "rc_solve": int(rc), "rc_grad": int(rcg),
        "all_converged": bool(rc == Q.QDSE_OK), "all_A_positive": bool(np.all(A > 0)),
        "sweeps_max": int(it.max()), "sweeps_mean": float(it.mean()),
        "setup_ms": 1e3 * t_setup, "solve_ms": 1e3 * t_solve, "grad_ms": 1e3 * t_grad,
        "solve_plus_grad_per_s": B / (t_solve + t_grad),
        "kernel_matrix_bytes_per_sweep": kbytes * B,
        "loss": float(np.sum((M - T) ** 2)),
        "theta_bar_finite": bool(np.all(np.isfinite(tb))),
        "workload": "512x128, kappa~U[0.70,0.825], omega~U[0.65,0.70], m~U[0,0.1] (seed 5); "
                    "target seed 55; FP64 solve tol 1e-12 then implicit adjoint (GMRES tol 1e-12, "
                    "right-preconditioned by the banded LU of I - band(J)^T)",
    }


STATUS_NAMES = {0: "ok", 1: "not_converged", -4: "nan", -6: "diverged", -7: "spurious"}


def status_counts(np, st):
    vals, cnt = np.unique(np.asarray(st), return_counts=True)
    return {STATUS_NAMES.get(int(v), str(int(v))): int(c) for v, c in zip(vals, cnt)}


def configs_interaction(Q, np, torch):
    """The 512 x 128 workload at the configurations' own interaction, kappa =
    (D omega)^(1/3) = 0.8 GeV, omega = 0.5 GeV, m in {0, 5 MeV}, from A0 = 1,
    B0 = 0.3 GeV: successive approximation (3000 sweeps at most) and AUTO
    (then Newton from the start). The physical branch ends before this point
    (kappa / omega ~ 1.41 at the end, found by continuation on the oracle), so
    neither driver may return a certified solution; the outcome codes and the
    work spent are recorded."""
    n, na = 512, 128
    params = [(0.8 ** 3 / 0.5, 0.5, 0.0), (0.8 ** 3 / 0.5, 0.5, 0.005)]
    out = {"workload": "512x128, kappa=0.8 GeV, omega=0.5 GeV, m in {0, 5 MeV}, A0=1, B0=0.3, "
                       "tol 1e-10 on max|dM/M| and max|dA|",
           "certified_solutions": 0,
           "evidence": "the branch of certified solutions ends before this point "
                       "(tests/test_oracle_branch.py, tests/test_gpu_driver.py)"}
    for name, sol in (("picard", Q.QDSE_PICARD), ("auto", Q.QDSE_AUTO)):
        S = Q.Solver(n, na, params, solver=sol)
        x = S.initial(1.0, 0.3)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc, it, rs = S.solve(x, tol=1e-10, max_iter=3000)
        torch.cuda.synchronize()
        st = S.solve_status()
        xa = x.cpu().numpy()
        out[name] = {"status": [STATUS_NAMES.get(int(v), str(int(v))) for v in st],
                     "evaluations": [int(v) for v in it], "last_statistic": [float(v) for v in rs],
                     "seconds": time.perf_counter() - t0,
                     "min_A": [float(v) for v in xa[:, :n].min(axis=1)]}
        out["certified_solutions"] += int(np.sum(st == Q.QDSE_OK))
        S.close()
    return out


def gradient_stated_box(Q, np, torch, B):
    """The gradient configuration as stated: B instances at 512 x 128 with
    kappa ~ U[0.7, 0.9] GeV, omega ~ U[0.4, 0.6] GeV, m ~ U[0, 0.1] GeV (seed
    5), own interaction each; AUTO solve (successive approximation to 1e-12 on
    M and A, at most 600 sweeps, then Newton from the start for every instance
    not certified), then dL/d(D, omega, m) by the implicit adjoint for the
    certified instances (dL/dx set to 0 for the others, which therefore take
    no Krylov steps). Most of the box lies beyond the end of the physical
    branch (kappa / omega > ~1.41); those instances end as diverged, not
    converged or spurious, and get no gradient."""
    n, na = 512, 128
    rng = np.random.default_rng(5)
    kap = rng.uniform(0.7, 0.9, B)
    om = rng.uniform(0.4, 0.6, B)
    m = rng.uniform(0.0, 0.1, B)
    params = [(float(k ** 3 / o), float(o), float(mm)) for k, o, mm in zip(kap, om, m)]
    rng = np.random.default_rng(55)
    M0 = rng.uniform(0.3, 0.5, B)
    L2 = rng.uniform(0.5, 2.0, B)
    s = Q.grid_nodes(n, na)["s"]
    T = 0.005 + M0[:, None] / (1.0 + s[None, :] / L2[:, None])
    S = Q.Solver(n, na, params, solver=Q.QDSE_AUTO)
    x = S.initial(1.0, 0.3)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rc, it, rs = S.solve(x, tol=1e-12, max_iter=600)
    torch.cuda.synchronize()
    t_solve = time.perf_counter() - t0
    st = S.solve_status()
    ok = st == Q.QDSE_OK
    xs = x.cpu().numpy()
    A, Bf = xs[:, :n], xs[:, n:]
    M = Bf / A
    g = np.concatenate([-2.0 * (M - T) * Bf / A ** 2, 2.0 * (M - T) / A], axis=1)
    g[~ok] = 0.0
    gd = torch.tensor(g, device=x.device)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tb, rcg = S.grad(x, gd, tol=1e-12, max_iter=400)
    torch.cuda.synchronize()
    t_grad = time.perf_counter() - t0
    tb = np.asarray(tb)
    S.close()
    return {
        "instances": B, "status_counts": status_counts(np, st),
        "certified": int(ok.sum()),
        "certified_kappa_over_omega_max": float(np.max(kap[ok] / om[ok])) if ok.any() else None,
        "uncertified_kappa_over_omega_min": float(np.min(kap[~ok] / om[~ok])) if (~ok).any() else None,
        "evaluations_mean_certified": float(it[ok].mean()) if ok.any() else None,
        "solve_ms": 1e3 * t_solve, "grad_ms": 1e3 * t_grad, "rc_grad": int(rcg),
        "certified_solve_plus_grad_per_s": float(ok.sum()) / (t_solve + t_grad),
        "theta_bar_finite_certified": bool(np.all(np.isfinite(tb[ok]))),
        "workload": "512x128, kappa~U[0.7,0.9], omega~U[0.4,0.6], m~U[0,0.1] (seed 5), target seed "
                    "55; AUTO solve tol 1e-12 (600 sweeps, then Newton), implicit adjoint on the "
                    "certified instances",
    }


def mixed_batch(Q, np, torch, B):
    """B vacuum instances (paper interaction) with m ~ U[0, 0.2] GeV, radial
    grid sizes uniform in {128, 256, 384, 512} and 64 or 128 angular nodes
    (seed 4). Instances are grouped by grid class (one context per class,
    kernel matrices shared inside a class) and each class is solved to 1e-7
    accuracy (tol 1e-8) with FP32 MFMA sweeps + refinement, and
    with FP64 MFMA sweeps only; all classes are driven together by
    qdse_solve_group, each on its own stream."""
    rng = np.random.default_rng(4)
    m = rng.uniform(0.0, 0.2, B)
    nr = rng.choice([128, 256, 384, 512], B)
    nan = rng.choice([64, 128], B)
    classes = sorted(set(zip(nr.tolist(), nan.tolist())))
    out = {"instances": B, "classes": len(classes),
           "class_sizes": {f"{n}x{na}": int(np.sum((nr == n) & (nan == na))) for n, na in classes}}
    tot, shapes = {}, {}
    # one stream per class, the same streams for both precisions (streams
    # created later in the process map onto the device's hardware queues
    # differently, which alone moved either precision's time by ~20 %)
    streams = [torch.cuda.Stream() for _ in classes]
    for prec in (Q.QDSE_FP32_REFINE, Q.QDSE_FP64_MATRIX):
        solvers, x0s = [], []
        for (n, na), stream in zip(classes, streams):  # one context per class
            sel = np.nonzero((nr == n) & (nan == na))[0]
            params = [(0.55, 0.678, float(m[k])) for k in sel]
            S = Q.Solver(n, na, params, interp_order=3, precision=prec, stream=stream)
            shapes[(prec, n, na)] = S.autotune(reps=10)["mm_row_groups"]  # per class
            solvers.append(S)
            x0s.append(S.initial(1.0, 1.0))
        torch.cuda.synchronize()
        xs = [x.clone() for x in x0s]
        Q.solve_group(solvers, xs, tol=1e-8, max_iter=2000)  # warm-up (graph capture)
        runs = []
        for _ in range(3):  # the median of three timed group solves
            xs = [x.clone() for x in x0s]
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rc, its, rss = Q.solve_group(solvers, xs, tol=1e-8, max_iter=2000)
            torch.cuda.synchronize()
            runs.append(time.perf_counter() - t0)
            if rc != Q.QDSE_OK:
                raise SystemExit(f"mixed batch did not converge: rc={rc}")
        tot[prec] = float(np.median(runs))
        for S in solvers:
            S.close()
    out["fp32_refined_solves_per_s"] = B / tot[Q.QDSE_FP32_REFINE]
    out["fp64_mfma_solves_per_s"] = B / tot[Q.QDSE_FP64_MATRIX]
    out["fp32_refined_ms"] = 1e3 * tot[Q.QDSE_FP32_REFINE]
    out["fp64_mfma_ms"] = 1e3 * tot[Q.QDSE_FP64_MATRIX]
    out["autotuned_row_groups"] = {("fp32" if p == Q.QDSE_FP32_REFINE else "fp64") + f"_{n}x{na}": v
                                   for (p, n, na), v in shapes.items()}
    out["workload"] = ("vacuum, paper interaction, m~U[0,0.2], N_r in {128,256,384,512} x N_a in "
                       "{64,128} (seed 4), tol 1e-8; one context and stream per class (launch shape "
                       "autotuned per class), qdse_solve_group; median of three timed solves")
    return out


def renormalised_qc(Q, np, torch, reps=20):
    """Renormalised Qin-Chang setting (ultraviolet term of the interaction,
    renormalisation at zeta = 19 GeV) on the headline's 512 x 128 grid with its
    infrared parameters, m(zeta) in {3.4 MeV, 0}: converged solves/s (tol
    1e-10 on M and A), the whole solve as one launch, against the HBM
    roofline on the method's bytes (as the headline's); the kernel-per-sweep
    driver's sums kernel beside it."""
    n, na, zeta = 512, 128, 19.0
    params = [(0.55, 0.678, 0.0034), (0.55, 0.678, 0.0)]
    S = Q.Solver(n, na, params, zeta=zeta)
    x0 = S.initial(1.0, 1.0)
    x = torch.empty_like(x0)
    for _ in range(3):
        x.copy_(x0)
        S.solve(x, tol=1e-10, max_iter=2000)
    torch.cuda.synchronize()
    kus = []
    t0 = time.perf_counter()
    for _ in range(reps):
        x.copy_(x0)
        rc, it, rs = S.solve(x, tol=1e-10, max_iter=2000)
        kus.append(S.solve_kernel_us())
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    xs = x.cpu().numpy()
    ms = S.time_contraction(x, reps=200)
    S.close()
    nq = n + 1
    single = all(v is not None for v in kus)
    # per sweep the method's six FP64 kernel matrices of the n + 1 rows, the
    # loop-node data, and per running instance the iterate in and out
    running = [sum(1 for v in it if v >= k) for k in range(1, int(max(it)) + 1)]
    solve_bytes = sum(6 * (n + 1) * nq * 8 + nq * 40 + r * 2 * (2 * n * 8) for r in running)
    kus_mean = float(np.mean(kus)) if single else None
    roof = None
    if single:
        ach = solve_bytes / (kus_mean * 1e-6) / 1e9
        roof = {"bound": "hbm", "kernel": "k_persistent<true> (single-launch renormalised solve, 2 instances)",
                "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
                "traffic": None, "avg_kernel_us": kus_mean, "alg_bytes_per_launch": solve_bytes}
    # the kernel-per-sweep driver's sums kernel: three FP64 matrices with n + 1
    # rows and the loop-node weights and t once; per instance the iterate read
    # and 2 (n + 1) sums written
    alg = 3 * (n + 1) * nq * 8 + nq * 40 + len(params) * (2 * n * 8 + 2 * (n + 1) * 8)
    ach_s = alg / (ms * 1e-3) / 1e9
    return {
        "workload": "512x128, D=0.55 GeV^2, omega=0.678 GeV plus the Qin-Chang ultraviolet term, "
                    "renormalised at zeta=19 GeV, m(zeta) in {3.4 MeV, 0}, A0=B0=1, tol 1e-10",
        "rc": int(rc), "sweeps": [int(v) for v in it], "solves_per_s": len(params) / dt,
        "ms_per_step": dt * 1e3, "single_launch": single,
        "M_at_p2_1e-4": [float(xs[k, n] / xs[k, 0]) for k in range(len(params))],
        "A_at_p2_1e-4": [float(xs[k, 0]) for k in range(len(params))],
        "roofline": roof,
        "roofline_sweep_kernel": {
            "bound": "hbm", "kernel": "k_sweep_row<true> (renormalised sums of the n + 1 rows, 2 instances)",
            "achieved": ach_s, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach_s / HBM_PEAK_GBS,
            "traffic": None, "avg_kernel_us": ms * 1e3, "alg_bytes_per_launch": alg},
    }


def general_system(Q, np, torch, n=4096, reps=50):
    """The general system of Sec. I at n = 4096 (alpha = 1/2): one sweep's row
    kernel against the HBM roofline (the two caller matrices K1, K2 are the
    traffic) and a contracting solve to 1e-12."""
    a, b, alpha = 0.0, 1.0, 0.5
    rng = np.random.default_rng(4096)
    x, t, w = Q.fred_nodes(n, a, b, alpha)
    K1 = 0.1 * np.exp(-(x[:, None] - t[None, :]) ** 2)
    K2 = 0.1 * np.cos(x[:, None] + 2 * t[None, :])
    F = rng.uniform(-1, 1, (4, 6)) * np.array([0.1, 0.2, 0.2, 0.05, 0.05, 0.05])
    f = np.concatenate([1.0 + 0.3 * np.sin(x), 0.5 * np.cos(x)])
    dev = lambda a_: torch.tensor(np.ascontiguousarray(a_), device="cuda")  # noqa: E731
    dK1, dK2, df = dev(K1), dev(K2), dev(f)
    del K1, K2
    S = Q.FredSolver(n, a, b, alpha, F, dK1, dK2, df)
    uv = dev(np.ones(2 * n))
    ms = S.time_sweep(uv, reps=reps)
    x0 = uv.clone()
    S.solve(uv, tol=1e-12, max_iter=500)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    uv.copy_(x0)
    rc, it, r = S.solve(uv, tol=1e-12, max_iter=500)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    S.close()
    nq = n + 1
    alg = 2 * n * nq * 8 + 4 * nq * 8 + nq * 8 + 3 * 2 * n * 8
    ach = alg / (ms * 1e-3) / 1e9
    return {
        "workload": f"n={n} on [0, 1], alpha=1/2, K1 Gaussian, K2 cosine (0.1 scale), seeded quadratic F",
        "sweep_kernel_us": ms * 1e3, "solve": {"rc": int(rc), "sweeps": int(it), "seconds": dt},
        "roofline": {"bound": "hbm", "kernel": "k_fred_rows", "achieved": ach, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": ach / HBM_PEAK_GBS, "traffic": None,
                     "avg_kernel_us": ms * 1e3, "alg_bytes_per_launch": alg},
    }


def finite_mu(Q, np, torch):
    """Finite mu = 0.3 GeV, T = 0, paper interaction, m = 5 MeV: external
    128 |p_vec| x 128 p4 nodes, loop 129 x 129 nodes with q4 of both signs and
    32 angles; average of 3 sweeps timed with the device synchronised."""
    ns, n4, na = 128, 128, 32
    S = Q.MuSolver(ns, n4, na, [(0.55, 0.678, 0.005, 0.3)])
    x = torch.zeros(S.shape, dtype=torch.complex128, device="cuda")
    x[:, 0] = 1.0
    x[:, 1] = 0.3
    x[:, 2] = 1.0
    y = S.iterate(x)
    torch.cuda.synchronize()
    reps = 3
    t0 = time.perf_counter()
    for _ in range(reps):
        S.iterate(x, out=y)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    points = ns * n4 * (ns + 1) * (n4 + 1) * 2 * na
    S.close()
    # FP64 operations of the sweep kernel per (external point, loop point)
    # pair, both signs of q4 included, as compiled (FMA = 2, mul/add = 1):
    # the angle-independent coefficient algebra plus one moment update per
    # angle; counted from the gfx950 code of k_mu_sweep.
    pairs = ns * n4 * (ns + 1) * (n4 + 1)
    flops = pairs * (MU_FLOPS_PER_PAIR + MU_FLOPS_PER_ANGLE * na)
    tf = flops / dt / 1e12
    # one complete solve from A = C = 1, B = 0.3 GeV (absolute complex change of
    # A, B, C below 1e-8)
    S = Q.MuSolver(ns, n4, na, [(0.55, 0.678, 0.005, 0.3)])
    xs = x.clone()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rc, it, rs = S.solve(xs, tol=1e-8, max_iter=600)
    torch.cuda.synchronize()
    t_solve = time.perf_counter() - t0
    S.close()
    # seeded subsample of the mixed workload's mu > 0 instances (reading: mu > 0
    # instances solve the finite-mu equations on an (N_r / 4)^2 grid with the
    # instance's 64 or 128 angles): two instances of each of the four classes
    # with N_r in {128, 256}, mu ~ U[0, 0.4], m ~ U[0, 0.2] (seed 4), each
    # class one context on its own stream, solved together to 1e-8; the
    # classes N_r in {384, 512} (96^2 and 128^2 external points) are costed
    # per sweep only (a solve there takes seconds to tens of seconds)
    rng = np.random.default_rng(4)
    solvers, xs_, cls = [], [], []
    for g4 in (32, 64):
        for nang in (64, 128):
            pp = [(0.55, 0.678, float(rng.uniform(0.0, 0.2)), float(rng.uniform(0.0, 0.4)))
                  for _ in range(2)]
            Sg = Q.MuSolver(g4, g4, nang, pp, stream=torch.cuda.Stream())
            xq = torch.zeros(Sg.shape, dtype=torch.complex128, device="cuda")
            xq[:, 0] = 1.0
            xq[:, 1] = 0.3
            xq[:, 2] = 1.0
            solvers.append(Sg)
            xs_.append(xq)
            cls.append((g4, nang, pp))
    x0s = [xq.clone() for xq in xs_]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rcg, itg, rsg = Q.mu_solve_group(solvers, xs_, tol=1e-8, max_iter=600)
    torch.cuda.synchronize()
    t_group = time.perf_counter() - t0
    # the same instances with Anderson mixing (depth 8), class by class from
    # the same initial functions
    t0 = time.perf_counter()
    aa = []
    for Sg, xq in zip(solvers, x0s):
        rca, ita, rsa = Sg.solve(xq, tol=1e-8, max_iter=600, anderson=8)
        aa.append((ita, rsa))
    torch.cuda.synchronize()
    t_aa = time.perf_counter() - t0
    sub = []
    n_ok = n_ok_aa = 0
    for (g4, nang, pp), its_, rss_, (ita, rsa) in zip(cls, itg, rsg, aa):
        for k, (D_, om_, mm, mu) in enumerate(pp):
            conv, conv_aa = bool(rss_[k] < 1e-8), bool(rsa[k] < 1e-8)
            n_ok += conv
            n_ok_aa += conv_aa
            sub.append({"grid": f"{g4}x{g4}x{nang}", "mu": mu, "m": mm,
                        "picard": {"sweeps": int(its_[k]), "converged": conv,
                                   "last_change": float(rss_[k])},
                        "anderson8": {"sweeps": int(ita[k]), "converged": conv_aa,
                                      "last_change": float(rsa[k])}})
    for Sg in solvers:
        Sg.close()
    per_sweep = {}
    for g4 in (96, 128):
        for nang in (64, 128):
            Sg = Q.MuSolver(g4, g4, nang, [(0.55, 0.678, 0.1, 0.2)])
            xq = torch.zeros(Sg.shape, dtype=torch.complex128, device="cuda")
            xq[:, 0] = 1.0
            xq[:, 1] = 0.3
            xq[:, 2] = 1.0
            yq = Sg.iterate(xq)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            Sg.iterate(xq, out=yq)
            torch.cuda.synchronize()
            per_sweep[f"{g4}x{g4}x{nang}"] = 1e3 * (time.perf_counter() - t1)
            Sg.close()
    mixed_mu = {"label": "subsample of the mixed workload's mu > 0 instances (8 of 1024)",
                "instances": sub, "converged_picard": n_ok, "picard_group_seconds": t_group,
                "converged_picard_solves_per_s": n_ok / t_group,
                "converged_anderson8": n_ok_aa, "anderson8_seconds": t_aa,
                "converged_anderson8_solves_per_s": n_ok_aa / t_aa,
                "sweep_ms_larger_classes": per_sweep,
                "note": "successive approximation at finite mu does not converge for every "
                        "instance: where it does not, the iterate diverges or cycles (the "
                        "difference quotients of the finite-mu vertex have near-poles where "
                        "q~^2 ~ p~^2); Anderson mixing converges for more of them"}
    return {"workload": "mu=0.3 GeV, 128x128 external, 129x129x2 loop points x 32 angles, m=5 MeV",
            "sweep_ms": 1e3 * dt, "integrand_points_per_sweep": points,
            "integrand_points_per_s": points / dt,
            "solve": {"rc": int(rc), "sweeps": int(it[0]), "seconds": t_solve,
                      "solves_per_s": 1.0 / t_solve, "tol": 1e-8},

            "mixed_workload_mu_subsample": mixed_mu,
            "roofline": {"bound": "alu", "kernel": "k_mu_sweep (FP64 VALU)", "achieved": tf,
                         "peak": FP64_VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                         "frac": tf / FP64_VALU_PEAK_TFLOPS, "traffic": None,
                         "flops_per_sweep": flops}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--batch", type=int, default=1024)
    ap.add_argument("--batch-steps", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-grad", action="store_true")
    ap.add_argument("--no-mu", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-qc", action="store_true")
    ap.add_argument("--no-fred", action="store_true")
    ap.add_argument("--no-cfg", action="store_true")
    ap.add_argument("--grad-batch", type=int, default=256)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one cold 1 GiB device copy (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the solver runs on a single MI355X "
              "(multi-GPU sharding is a design note, not part of this build)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2012_03667_amd as Q

    torch.cuda.set_device(0)
    n, na = 512, 128
    D, om = 0.55, 0.678
    masses = (0.0, 0.005)

    def timed_solves(S, x0, tol, steps, warmup, kernel_us=None):
        x = torch.empty_like(x0)
        its = None
        for _ in range(warmup):
            x.copy_(x0)
            S.solve(x, tol=tol, max_iter=2000, conv_mode=Q.QDSE_CONV_MASS)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            x.copy_(x0)
            rc, its, rs = S.solve(x, tol=tol, max_iter=2000, conv_mode=Q.QDSE_CONV_MASS)
            if rc != Q.QDSE_OK:
                raise SystemExit(f"solve did not converge: rc={rc} iters={its} resid={rs}")
            if kernel_us is not None:  # HIP events around the solve's single launch
                kernel_us.append(S.solve_kernel_us())
        torch.cuda.synchronize()
        return time.perf_counter() - t0, x, its

    # ---- headline: plain FP64 solver, two instances per step
    S = Q.Solver(n, na, [(D, om, m) for m in masses], interp_order=3)
    x0 = S.initial(1.0, 1.0)
    kus = []
    dt, x, iters = timed_solves(S, x0, 1e-10, args.steps, args.warmup, kernel_us=kus)
    solves = args.steps * len(masses)
    xs = x.cpu().numpy()
    certified = bool(np.all(S.solve_status() == Q.QDSE_OK))

    if any(v is None for v in kus):
        raise SystemExit("the headline solve did not run as one launch")
    kernel_us = float(np.mean(kus))
    nq = n + 1
    # algorithmic bytes of one launch (one whole solve): per sweep the method's
    # six angular-integrated FP64 kernel matrices (N x N_q each) and the
    # loop-node data (4 stencil weights and t per node), per running instance
    # the iterate in and out; the kernel itself reads the three folded matrices
    # once into registers and exchanges iterates between workgroups
    running = [sum(1 for v in iters if v >= k) for k in range(1, int(max(iters)) + 1)]
    solve_bytes = sum(6 * n * nq * 8 + nq * (4 * 8 + 8) + r * 2 * (2 * n * 8) for r in running)
    solve_achieved = solve_bytes / (kernel_us * 1e-6) / 1e9
    reps = 200
    avg_ms = S.time_contraction(x, reps=reps)
    # algorithmic bytes of one sweep launch: the method's six angular-integrated
    # FP64 kernel matrices (one per bracketed factor of the projected
    # integrands, N x N_q each) and the loop-node data (4 stencil weights and t
    # per node) once, per instance the iterate in and out
    per_inst = 2 * (2 * n * 8)
    alg_bytes = 6 * n * nq * 8 + nq * (4 * 8 + 8) + len(masses) * per_inst
    # what this kernel reads: the transverse-projector algebra folds the six
    # matrices into three
    read_bytes = 3 * n * nq * 8 + nq * (4 * 8 + 8) + len(masses) * per_inst
    achieved = alg_bytes / (avg_ms * 1e-3) / 1e9

    line = {
        "metric": "converged qDSE solves/s at N=512 (plain FP64 vs batched FP32-MFMA), % roofline",
        "value": solves / dt,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * dt / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "vacuum BC-vertex gap equation, 512 radial x 128 angular GL nodes, "
                        "cubic interpolation, m in {0, 5 MeV}, paper interaction D=0.55 GeV^2, "
                        "omega=0.678 GeV, A0=B0=1, tol 1e-10 on max|dM/M| and max|dA|",
            "n_radial": n, "n_angle": na, "instances_per_step": len(masses),
            "solver": "plain FP64 successive approximation, the whole solve in one kernel launch "
                      "(one row per wavefront, the two instances taking turns)",
            "sweeps_per_solve": [int(v) for v in iters],
            "branch_certified": certified,
            "note": "the configurations' interaction (kappa=0.8, omega=0.5) lies beyond the end of "
                    "the certified branch (see configs_interaction); the paper's interaction is used",
        },
        "roofline": {
            "bound": "hbm", "kernel": "k_persistent (single-launch FP64 solve, 2 instances)",
            "achieved": solve_achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": solve_achieved / HBM_PEAK_GBS,
            "traffic": counter_traffic("k_persistent_512x128_2inst.md", "qdse_persistent.hip"),
            "avg_kernel_us": kernel_us, "alg_bytes_per_launch": solve_bytes,
            "sweeps_per_launch": int(max(iters)), "instance_sweeps_per_launch": int(sum(iters)),
            "us_per_sweep": kernel_us / int(max(iters)),
            "alg_bytes_note": "per sweep six N x N_q FP64 kernel matrices + loop-node data, "
                              "per running instance the iterate in and out; the kernel reads "
                              "the three folded matrices once and keeps them in registers",
        },
        "roofline_sweep_kernel": {
            "bound": "hbm", "kernel": "k_sweep_row (kernel-per-sweep driver, 2 instances)",
            "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": counter_traffic("k_sweep_row_512x128_2inst.md", "qdse_kernels.hip"),
            "avg_kernel_us": avg_ms * 1e3, "alg_bytes_per_launch": alg_bytes,
            "alg_bytes_note": "six N x N_q FP64 kernel matrices + loop-node data + iterate; "
                              "the kernel reads three matrices (kernel_read_bytes_per_launch)",
            "kernel_read_bytes_per_launch": read_bytes,
            "kernel_read_GBs": read_bytes / (avg_ms * 1e-3) / 1e9,
        },
    }

    # ---- batched: FP32 MFMA + refinement vs FP64, equal 1e-7 accuracy
    if not args.no_batch:
        B = args.batch
        rng = np.random.default_rng(4)
        mb = rng.uniform(0.0, 0.2, B)
        mb[0] = 0.005
        pb = [(D, om, float(m)) for m in mb]
        res = {}
        tol_eq = 1e-8
        dtp, xp, itp = timed_solves(S, x0, tol_eq, args.steps, 1)
        res["plain_fp64_2inst"] = {"solves_per_s": len(masses) * args.steps / dtp,
                                   "sweeps": [int(v) for v in itp]}
        S32 = Q.Solver(n, na, pb, interp_order=3, precision=Q.QDSE_FP32_REFINE)
        tuned = {"fp32_mfma_row_groups": S32.autotune(reps=10)["mm_row_groups"]}
        xb0 = S32.initial(1.0, 1.0)
        dt32, x32, it32 = timed_solves(S32, xb0, tol_eq, args.batch_steps, 1)
        n32, n64 = S32.solve_stats()
        res["fp32_mfma_refined"] = {
            "solves_per_s": B * args.batch_steps / dt32, "ms_per_batch": 1e3 * dt32 / args.batch_steps,
            "fp32_sweeps_max": int(n32.max()), "fp64_sweeps_max": int(n64.max()),
            "fp32_sweeps_mean": float(n32.mean()), "fp64_sweeps_mean": float(n64.mean()),
            "refinement": ("one phase: FP32 sweeps of the node-column differences from a reference "
                           "iterate, renewed by an FP64 sweep (the fp64 sweeps) every sixth sweep")}
        del S32
        S64 = Q.Solver(n, na, pb, interp_order=3)
        tuned["fp64_direct_rows_per_workgroup"] = S64.autotune(reps=5)["fused_rows"]
        dt64, x64, it64 = timed_solves(S64, S64.initial(1.0, 1.0), tol_eq, args.batch_steps, 1)
        res["fp64_direct"] = {"solves_per_s": B * args.batch_steps / dt64,
                              "ms_per_batch": 1e3 * dt64 / args.batch_steps,
                              "sweeps_max": int(it64.max()), "sweeps_mean": float(it64.mean())}
        Smm = Q.Solver(n, na, pb, interp_order=3, precision=Q.QDSE_FP64_MATRIX)
        tuned["fp64_mfma_row_groups"] = Smm.autotune(reps=10)["mm_row_groups"]
        dtm, xmm, itm = timed_solves(Smm, Smm.initial(1.0, 1.0), tol_eq, args.batch_steps, 1)
        res["fp64_mfma"] = {"solves_per_s": B * args.batch_steps / dtm,
                            "ms_per_batch": 1e3 * dtm / args.batch_steps,
                            "sweeps_max": int(itm.max()), "sweeps_mean": float(itm.mean())}
        ms_mm64 = Smm.time_contraction(x64, reps=50, which=2)
        del Smm
        a32, a64 = x32.cpu().numpy(), x64.cpu().numpy()
        d = np.abs(a32 - a64) / np.maximum(np.abs(a64), 1e-8 * np.abs(a64).max(axis=1, keepdims=True))
        res["max_rel_diff_fp32_vs_fp64"] = float(d.max())
        res["instances"] = B
        res["autotuned"] = tuned
        res["workload"] = ("512x128 paper interaction, m ~ U[0, 0.2] GeV (seed 4, m[0] = 5 MeV), "
                           "tol 1e-8 (1e-7 accuracy target); launch shapes from qdse_autotune")
        line["batched"] = res
        # MFMA roofline of the FP32 contraction at this batch
        S32 = Q.Solver(n, na, pb, interp_order=3, precision=Q.QDSE_FP32_REFINE)
        rh32 = S32.autotune(reps=10)["mm_row_groups"]
        ms32 = S32.time_contraction(x64, reps=50, which=1)
        # algorithmic flops: the method's twelve N x N_q matrix-vector products
        # per instance (six kernels x two columns), 2 flop per MAC; the
        # kernel issues eight products of its five folded matrices
        flops = 24.0 * n * nq * B
        issued = 16.0 * n * nq * B
        tf = flops / (ms32 * 1e-3) / 1e12
        line["roofline_fp32"] = {
            "bound": "mfma", "kernel": f"k_mm_sweep<float, {rh32}, 0, 2> (FP32 contraction, batch)",
            "achieved": tf, "peak": FP32_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": tf / FP32_MFMA_PEAK_TFLOPS,
            "traffic": counter_traffic("k_mm_sweep_fp32_512x128_1024inst.md", "qdse_mfma.hip"),
            "avg_kernel_us": ms32 * 1e3,
            "alg_flops_per_launch": flops, "issued_flops_per_launch": issued,
            "issued_frac": issued / (ms32 * 1e-3) / 1e12 / FP32_MFMA_PEAK_TFLOPS}
        ms64 = S64.time_contraction(x64, reps=20)
        line["batched"]["fp64_direct_sweep_kernel_us"] = ms64 * 1e3
        line["batched"]["fp32_mfma_contraction_kernel_us"] = ms32 * 1e3
        line["batched"]["fp64_mfma_contraction_kernel_us"] = ms_mm64 * 1e3
        line["roofline_fp64_mfma"] = {
            "bound": "mfma",
            "kernel": f"k_mm_sweep<double, {tuned['fp64_mfma_row_groups']}, 2, 2> (FP64 contraction, batch)",
            "achieved": flops / (ms_mm64 * 1e-3) / 1e12, "peak": FP64_MFMA_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": flops / (ms_mm64 * 1e-3) / 1e12 / FP64_MFMA_PEAK_TFLOPS,
            "traffic": counter_traffic("k_mm_sweep_fp64_512x128_1024inst.md", "qdse_mfma.hip"),
            "avg_kernel_us": ms_mm64 * 1e3, "alg_flops_per_launch": flops,
            "issued_flops_per_launch": issued,
            "issued_frac": issued / (ms_mm64 * 1e-3) / 1e12 / FP64_MFMA_PEAK_TFLOPS}
        del S32, S64
        batch_x0 = a64[0]
    else:
        batch_x0 = None

    # ---- the configurations' own interaction: outcome codes, no certified branch
    if not args.no_cfg:
        line["configs_interaction"] = configs_interaction(Q, np, torch)

    # ---- gradient batch: per-instance interaction, solve + implicit adjoint;
    # the stated box (mostly beyond the end of the physical branch) and a
    # rectangle on its physical side where every instance converges
    if not args.no_grad:
        line["gradient_stated_box"] = gradient_stated_box(Q, np, torch, args.grad_batch)
        line["gradient_batch"] = gradient_batch(Q, np, torch, args.grad_batch)

    # ---- mixed grid classes (vacuum instances), grouped by class
    if not args.no_mixed:
        line["mixed_batch_vacuum"] = mixed_batch(Q, np, torch, args.batch)

    # ---- renormalised Qin-Chang setting (ultraviolet term, renormalisation)
    if not args.no_qc:
        line["renormalised_qc"] = renormalised_qc(Q, np, torch)

    # ---- the general second-kind system of Sec. I
    if not args.no_fred:
        line["general_system"] = general_system(Q, np, torch)

    # ---- finite chemical potential: one sweep of the 128 x 128 x 32 grid
    if not args.no_mu:
        line["finite_mu"] = finite_mu(Q, np, torch)

    if args.copy_calibration:
        # source written first, then 1 GiB of other data, so that the copy reads
        # its source from HBM (the 256 MB Infinity Cache holds at most the tail
        # of the second buffer)
        a = torch.empty(COPY_BYTES // 8, dtype=torch.float64, device="cuda").fill_(1.0)
        evict = torch.empty_like(a).fill_(2.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b, evict

    # the ceilings measured on this device (the rooflines quote the datasheet's)
    line["measured_peaks"] = Q.measure_peaks()
    line["measured_peaks"]["note"] = ("1 GiB streaming copy (read + write), 4 GiB read-only "
                                      "stream, and back-to-back v_mfma_*_16x16x4 loops; "
                                      "datasheet: HBM 8000 GB/s, FP32 matrix 157.3, FP64 matrix "
                                      "78.6 TFLOP/s")
    rd = line["measured_peaks"]["read_GBs"]
    line["roofline"]["frac_of_measured"] = line["roofline"]["achieved"] / rd
    rs = line["roofline_sweep_kernel"]
    rs["frac_of_measured"] = rs["achieved"] / rd
    rs["kernel_read_frac_of_measured"] = rs["kernel_read_GBs"] / rd
    for key in ("renormalised_qc", "general_system"):
        if key in line:
            for rk in ("roofline", "roofline_sweep_kernel"):
                r = line[key].get(rk)
                if r:
                    r["frac_of_measured"] = r["achieved"] / rd
    # the floor under the latency-bound per-sweep kernel: the same grid (four
    # rows per workgroup, one workgroup column per instance) launched empty, and
    # streaming the same algorithmic bytes once, both timed like the kernel
    wg = ((n + 3) // 4) * len(masses)
    fl = Q.measure_launch_floor(wg, rs["alg_bytes_per_launch"])
    rs["launch_floor"] = {
        "workgroups": wg, "empty_kernel_us": fl["empty_us"],
        "stream_same_bytes_us": fl["stream_read_us"],
        "note": "packet-timed like avg_kernel_us: a launch of this grid that does nothing takes "
                "empty_kernel_us, one that only streams the kernel's algorithmic bytes "
                "stream_same_bytes_us; the sweep's dependent chain (iterate reads, node "
                "functions, contraction, reductions) takes the rest"}
    if "roofline_fp32" in line:
        line["roofline_fp32"]["frac_of_measured"] = (line["roofline_fp32"]["achieved"] /
                                                     line["measured_peaks"]["mfma_fp32_TFLOPs"])
        line["roofline_fp64_mfma"]["frac_of_measured"] = (
            line["roofline_fp64_mfma"]["achieved"] / line["measured_peaks"]["mfma_fp64_TFLOPs"])

    if not args.no_cpu_baseline:
        from oracle import qdse_oracle as O
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        g = O.vac_grid(n, na, order=3)
        t1 = time.perf_counter()
        xr, itr, _, _ = O.picard(g, O.Params(D, om, masses[1]), np.ones(2 * n), 1e-10,
                                 max_iter=2000, mode=1, nthreads=threads)
        tc = time.perf_counter() - t1
        line["cpu_baseline"] = {
            "value": 1.0 / tc, "unit": "solves/s", "cores": threads, "kind": "oracle",
            "sample": f"one complete oracle solve of the m=5 MeV instance ({itr} sweeps, "
                      f"{tc:.1f} s, direct radial x angular sums, OpenMP over rows)",
        }
        # one thread: two sweeps of the same solve timed, the solve estimated
        # from its sweep count (a full single-thread solve takes about a minute)
        xw = np.ones(2 * n)
        t1 = time.perf_counter()
        for _ in range(2):
            xw = O.F(g, O.Params(D, om, masses[1]), xw, 1)
        t_sweep1 = (time.perf_counter() - t1) / 2
        line["cpu_baseline"]["single_thread"] = {
            "seconds_per_sweep": t_sweep1, "sweeps": int(itr),
            "estimated_solve_seconds": t_sweep1 * itr,
            "estimated_solves_per_s": 1.0 / (t_sweep1 * itr),
            "sample": "two sweeps of the m=5 MeV solve on one thread, scaled by its sweep count"}
        line["cpu_baseline"]["paper_table1"] = paper_table1(O, np, threads)
        den = np.maximum(np.abs(xr), 1e-8 * np.abs(xr).max())
        line["gpu_vs_oracle_max_rel"] = float(np.max(np.abs(xs[1] - xr) / den))
        if batch_x0 is not None:
            line["batched"]["fp64_inst0_vs_oracle_max_rel"] = float(np.max(np.abs(batch_x0 - xr) / den))
            line["batched"]["fp32_refined_inst0_vs_oracle_max_rel"] = float(
                np.max(np.abs(a32[0] - xr) / den))
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
