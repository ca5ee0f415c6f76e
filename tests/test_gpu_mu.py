"""Finite chemical potential: the HIP sweep (scalar four-vector algebra)
against the oracle (explicit complex Dirac matrices), through the C ABI.
Tolerance as for the vacuum FP64 path: 1e-12 relative per function (complex
modulus), with a floor of 1e-8 of the largest value."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import qdse_oracle as O  # noqa: E402

RTOL = 1e-12


@pytest.fixture(scope="module")
def Q():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2012_03667_amd as Q
    Q.load()
    return Q


def smooth_mu(g, rng):
    P2 = (g.ps[:, None] ** 2 + g.p4[None, :] ** 2).ravel()
    P4 = np.broadcast_to(g.p4[None, :], (g.ns, g.n4)).ravel()
    a, b = rng.uniform(0.5, 1.2, 2)
    A = 1 + a / (1 + P2 / 0.4) + 0.05j * P4 / (1 + P2)
    B = 0.005 + b / (1 + P2 / 0.5) - 0.03j * P4 / (1 + P2)
    C = 1 + 1.1 * a / (1 + P2 / 0.35) + 0.04j * P4 / (1 + P2)
    return np.stack([A, B, C])


def rel(gpu, ref):
    den = np.maximum(np.abs(ref), 1e-8 * np.max(np.abs(ref)))
    return float(np.max(np.abs(gpu - ref) / den))


@pytest.mark.parametrize("ns,n4,na,order,mu", [(8, 8, 6, 3, 0.3), (10, 7, 5, 1, 0.3),
                                               (9, 12, 8, 3, 0.0), (6, 5, 3, 3, 0.45)])
def test_mu_sweep_matches_oracle(Q, ns, n4, na, order, mu):
    print(f"case mu sweep {ns}x{n4}x{na} order {order} mu {mu}", flush=True)
    rng = np.random.default_rng(ns * 100 + n4)
    kw = dict(r_min=1e-2, r_max=8.0, p4_max=8.0, lam4=0.5)
    params = [(0.55, 0.678, 0.005, mu), (1.024, 0.5, 0.0, mu)]
    S = Q.MuSolver(ns, n4, na, params, interp_order=order, **kw)
    g = O.mu_grid(ns, n4, na, order=order, **kw)
    xs = [smooth_mu(g, rng) for _ in params]
    x = torch.tensor(np.stack(xs), device="cuda")
    y = S.iterate(x).cpu().numpy()
    for k, (D, om, m, mu_) in enumerate(params):
        ref = O.F_mu(g, D, om, m, mu_, xs[k])
        for f in range(3):
            assert rel(y[k, f], ref[f]) < RTOL, (k, f, rel(y[k, f], ref[f]))


def test_mu_full_size_sampled_rows(Q):
    """The 128 x 128 external grid with 129 x 129 x 2 loop points and 32 angles
    at mu = 0.3 GeV: one sweep compared on sampled external points."""
    ns = n4 = 128
    na = 32
    mu = 0.3
    rng = np.random.default_rng(128)
    S = Q.MuSolver(ns, n4, na, [(0.55, 0.678, 0.005, mu)])
    g = O.mu_grid(ns, n4, na)
    x0 = smooth_mu(g, rng)
    y = S.iterate(torch.tensor(x0[None], device="cuda")).cpu().numpy()[0]
    rows = np.sort(rng.choice(g.ne, 6, replace=False))
    ref = O.F_mu(g, 0.55, 0.678, 0.005, mu, x0, rows=rows)
    for f in range(3):
        assert rel(y[f, rows], ref[f]) < RTOL, (f, rel(y[f, rows], ref[f]))


@pytest.mark.parametrize("ns,n4,na,T", [(6, 330, 4, 0.0), (80, 4, 64, 0.0), (5, 340, 3, 0.002)])
def test_mu_sweep_long_grids_sampled_rows(Q, ns, n4, na, T):
    """Grids past the kernel's per-workgroup tables: a loop q4 grid longer than
    the tabulated q4 factors (n4 = 330, 340: the factors evaluated in the
    loop; the last case on Matsubara frequencies) and more loop radii x
    angles than one LDS table holds (81 x 64: the radii in two blocks). One
    sweep against the oracle on sampled external points."""
    print(f"case mu long grid {ns}x{n4}x{na} T {T}", flush=True)
    mu = 0.25
    rng = np.random.default_rng(ns * 1000 + n4)
    kw = dict(r_min=1e-2, r_max=8.0, p4_max=8.0, lam4=0.5)
    if T > 0:
        kw["T"] = T
    S = Q.MuSolver(ns, n4, na, [(0.55, 0.678, 0.005, mu)], **kw)
    g = O.mu_grid(ns, n4, na, **kw)
    x0 = smooth_mu(g, rng)
    y = S.iterate(torch.tensor(x0[None], device="cuda")).cpu().numpy()[0]
    rows = np.sort(rng.choice(g.ne, 5, replace=False))
    ref = O.F_mu(g, 0.55, 0.678, 0.005, mu, x0, rows=rows)
    for f in range(3):
        assert rel(y[f, rows], ref[f]) < RTOL, (f, rel(y[f, rows], ref[f]))


def test_mu_solve_matches_oracle_picard(Q):
    ns, n4, na, mu = 8, 8, 6, 0.25
    kw = dict(r_min=1e-2, r_max=8.0, p4_max=8.0)
    S = Q.MuSolver(ns, n4, na, [(0.55, 0.678, 0.005, mu)], **kw)
    g = O.mu_grid(ns, n4, na, **kw)
    x = torch.zeros(S.shape, dtype=torch.complex128, device="cuda")
    x[0, 0] = 1.0
    x[0, 1] = 0.3
    x[0, 2] = 1.0
    rc, it, rs = S.solve(x, tol=1e-11, max_iter=300)
    assert rc == Q.QDSE_OK, (rc, it, rs)
    xr = np.zeros((3, g.ne), complex)
    xr[0], xr[1], xr[2] = 1.0, 0.3, 1.0
    for k in range(1, 301):
        xn = O.F_mu(g, 0.55, 0.678, 0.005, mu, xr)
        r = np.max(np.abs(xn - xr))
        xr = xn
        if r < 1e-11:
            break
    assert abs(int(it[0]) - k) <= 1
    got = x[0].cpu().numpy()
    for f in range(3):
        assert rel(got[f], xr[f]) < 1e-11


@pytest.mark.parametrize("ns,n4,na,order,mu,T", [(8, 8, 6, 3, 0.3, 0.1), (10, 6, 5, 1, 0.0, 0.05),
                                                  (7, 9, 4, 3, 0.2, 0.15)])
def test_finite_temperature_sweep_matches_oracle(Q, ns, n4, na, order, mu, T):
    """T > 0: Matsubara frequencies in p4 and in the loop (weight 2 pi T, no
    interpolation in time), same integrand; GPU sweep vs oracle sweep."""
    print(f"case finite-T sweep {ns}x{n4}x{na} order {order} mu {mu} T {T}", flush=True)
    rng = np.random.default_rng(ns * 1000 + n4)
    kw = dict(r_min=1e-2, r_max=8.0)
    params = [(0.55, 0.678, 0.005, mu), (0.8, 0.6, 0.02, mu)]
    S = Q.MuSolver(ns, n4, na, params, interp_order=order, T=T, **kw)
    g = O.mu_grid(ns, n4, na, order=order, T=T, **kw)
    xs = [smooth_mu(g, rng) for _ in params]
    x = torch.tensor(np.stack(xs), device="cuda")
    y = S.iterate(x).cpu().numpy()
    for k, (D, om, m, mu_) in enumerate(params):
        ref = O.F_mu(g, D, om, m, mu_, xs[k])
        for f in range(3):
            assert rel(y[k, f], ref[f]) < RTOL, (k, f, rel(y[k, f], ref[f]))


@pytest.mark.parametrize("depth", [0, 5])
def test_mu_anderson_solve_reaches_oracle_fixed_point(Q, depth):
    """Anderson mixing (qdse_mu_solve_anderson) reaches the oracle's Picard
    fixed point; depth 0 is plain successive approximation; depth 5 needs
    fewer sweeps."""
    ns, n4, na, mu = 8, 8, 6, 0.3
    kw = dict(r_min=1e-2, r_max=8.0, p4_max=8.0)
    S = Q.MuSolver(ns, n4, na, [(0.55, 0.678, 0.005, mu), (0.55, 0.678, 0.05, mu)], **kw)
    g = O.mu_grid(ns, n4, na, **kw)
    x = torch.zeros(S.shape, dtype=torch.complex128, device="cuda")
    x[:, 0] = 1.0
    x[:, 1] = 0.3
    x[:, 2] = 1.0
    rc, it, rs = S.solve(x, tol=1e-12, max_iter=400, anderson=depth)
    assert rc == Q.QDSE_OK, (rc, it, rs)
    for k, m in enumerate((0.005, 0.05)):
        xr = np.zeros((3, g.ne), complex)
        xr[0], xr[1], xr[2] = 1.0, 0.3, 1.0
        for n_sw in range(1, 401):
            xn = O.F_mu(g, 0.55, 0.678, m, mu, xr)
            r = np.max(np.abs(xn - xr))
            xr = xn
            if r < 1e-13:
                break
        got = x[k].cpu().numpy()
        for f in range(3):
            assert rel(got[f], xr[f]) < 1e-10, (k, f, rel(got[f], xr[f]))
        if depth:
            assert it[k] < 0.6 * n_sw, (it[k], n_sw)



def test_mu_batch_with_own_parameters_matches_single_instances(Q):
    """One launch sweeps instances with their own mu, m and interaction: the
    result equals, bit for bit, single-instance contexts of the same grid."""
    print("case mu batch vs single instances 8x8x6", flush=True)
    rng = np.random.default_rng(41)
    kw = dict(r_min=1e-2, r_max=8.0, p4_max=8.0, lam4=0.5)
    params = [(0.55, 0.678, 0.005, 0.1), (0.55, 0.678, 0.15, 0.37), (1.024, 0.5, 0.0, 0.25)]
    g = O.mu_grid(8, 8, 6, **kw)
    xs = np.stack([smooth_mu(g, rng) for _ in params])
    S = Q.MuSolver(8, 8, 6, params, **kw)
    y = S.iterate(torch.tensor(xs, device="cuda"))
    for k, p in enumerate(params):
        S1 = Q.MuSolver(8, 8, 6, [p], **kw)
        y1 = S1.iterate(torch.tensor(xs[k:k + 1], device="cuda"))
        assert torch.equal(y[k:k + 1], y1), k
        ref = O.F_mu(g, *p, xs[k])
        for f in range(3):
            assert rel(y[k, f].cpu().numpy(), ref[f]) < RTOL


def test_mu_group_solve_of_ragged_classes_matches_oracle(Q):
    """A ragged batch in the manner of the mixed configuration: three grid
    classes (external grids 6x6, 8x8, 6x8 with 12, 16, 16 angles), each
    context holding instances with their own mu in (0.05, 0.4) and m in
    (0.03, 0.2), solved together by qdse_mu_solve_group on three streams;
    each instance's fixed point matches the oracle's successive approximation
    (same sweep count +-1, values to 1e-11). (Coarser angular rules, and the
    chiral limit at larger mu, make successive approximation cycle or
    diverge on grids this small, on both sides.)"""
    print("case mu group solve of 3 classes", flush=True)
    rng = np.random.default_rng(4)
    kw = dict(r_min=1e-2, r_max=1e2, p4_max=1e2, lam4=0.5)
    classes = [(6, 6, 12), (8, 8, 16), (6, 8, 16)]
    solvers, xs, plist = [], [], []
    for q, (ns, n4, na) in enumerate(classes):
        params = [(0.55, 0.678, float(rng.uniform(0.03, 0.2)), float(rng.uniform(0.05, 0.4)))
                  for _ in range(2 + q % 2)]
        st = torch.cuda.Stream()
        S = Q.MuSolver(ns, n4, na, params, stream=st, **kw)
        x = torch.zeros(S.shape, dtype=torch.complex128, device="cuda")
        x[:, 0] = 1.0
        x[:, 1] = 0.3
        x[:, 2] = 1.0
        solvers.append(S)
        xs.append(x)
        plist.append(params)
    torch.cuda.synchronize()
    rc, its, rss = Q.mu_solve_group(solvers, xs, tol=1e-10, max_iter=300)
    assert rc == Q.QDSE_OK, (rc, its)
    for q, (ns, n4, na) in enumerate(classes):
        g = O.mu_grid(ns, n4, na, **kw)
        got = xs[q].cpu().numpy()
        for k, (D, om, m, mu) in enumerate(plist[q]):
            x = np.zeros((3, g.ne), complex)
            x[0], x[1], x[2] = 1.0, 0.3, 1.0
            for it in range(1, 301):
                xn = O.F_mu(g, D, om, m, mu, x)
                r = np.max(np.abs(xn - x))
                x = xn
                if r < 1e-10:
                    break
            assert abs(int(its[q][k]) - it) <= 1, (q, k, its[q][k], it)
            for f in range(3):
                assert rel(got[k, f], x[f]) < 1e-11, (q, k, f, rel(got[k, f], x[f]))
