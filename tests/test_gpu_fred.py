"""Parity of the general second-kind system (qdse_fred_*, Sec. I eqs. jifen1,
jifen3, jifen12) with its CPU oracle, through the C ABI. Both sides sum the
same n + 1 products in FP64 in a different order, and the singular kernel is
exp(-alpha ln|d|) on the GPU against numpy's power on the host (a few ulps
per term), so outputs agree to ~1e-14 relative to the largest term; the bar
is 1e-12 of max(|ref|, 1e-3 max|ref|) per array."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import qdse_oracle_fred as OF  # noqa: E402


def err(gpu, ref):
    den = np.maximum(np.abs(ref), 1e-3 * np.max(np.abs(ref)))
    return float(np.max(np.abs(gpu - ref) / den))


@pytest.fixture(scope="module")
def Q():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2012_03667_amd as Q
    Q.load()
    return Q


def problem(n, a, b, rng, scale=0.2):
    x, t, w = OF.nodes(n, a, b)
    K1 = scale * np.exp(-(x[:, None] - t[None, :]) ** 2 / (b - a)) * rng.uniform(0.5, 1.0)
    K2 = scale * np.cos(x[:, None] + 2 * t[None, :]) * rng.uniform(0.5, 1.0)
    F = rng.uniform(-1, 1, (4, 6)) * np.array([0.1, 0.2, 0.2, 0.05, 0.05, 0.05])
    f = np.concatenate([1.0 + 0.3 * np.sin(x), 0.5 * np.cos(x)])
    return x, t, w, K1, K2, F, f


CASES = [(37, 3, 0.5, 0.0, 1.0), (64, 1, 1.0, -1.0, 2.0), (130, 3, 0.25, 0.0, 3.0),
         (4, 3, 0.7, 0.0, 1.0), (257, 1, 0.9, 1.0, 2.0)]


@pytest.mark.parametrize("n,order,alpha,a,b", CASES)
def test_sweep_matches_oracle(Q, n, order, alpha, a, b):
    print(f"case fred sweep n={n} order={order} alpha={alpha}", flush=True)
    rng = np.random.default_rng(n)
    x, t, w, K1, K2, F, f = problem(n, a, b, rng)
    uv = np.concatenate([1.0 + 0.1 * rng.standard_normal(n), 0.5 + 0.1 * rng.standard_normal(n)])
    dev = lambda a_: torch.tensor(np.ascontiguousarray(a_), device="cuda")  # noqa: E731
    S = Q.FredSolver(n, a, b, alpha, F, dev(K1), dev(K2), dev(f), interp_order=order)
    y = S.iterate(dev(uv)).cpu().numpy()
    ref = OF.fred_map(x, t, w, K1, K2, F, f, uv, alpha, order)
    assert err(y[:n], ref[:n]) < 1e-12 and err(y[n:], ref[n:]) < 1e-12
    S.close()


def test_solve_matches_oracle_fixed_point(Q):
    n, a, b, alpha = 96, 0.0, 1.0, 0.5
    print("case fred solve n=96", flush=True)
    rng = np.random.default_rng(96)
    x, t, w, K1, K2, F, f = problem(n, a, b, rng, scale=0.1)
    dev = lambda a_: torch.tensor(np.ascontiguousarray(a_), device="cuda")  # noqa: E731
    S = Q.FredSolver(n, a, b, alpha, F, dev(K1), dev(K2), dev(f))
    uv = dev(np.ones(2 * n))
    rc, it, r = S.solve(uv, tol=1e-13, max_iter=500)
    assert rc == Q.QDSE_OK and r < 1e-13
    ref, itr, _ = OF.picard(x, t, w, K1, K2, F, f, np.ones(2 * n), alpha, 3, 1e-13, max_iter=500)
    assert abs(it - itr) <= 1, (it, itr)
    got = uv.cpu().numpy()
    assert err(got[:n], ref[:n]) < 1e-11 and err(got[n:], ref[n:]) < 1e-11
    # max_iter stop and status
    uv2 = dev(np.ones(2 * n))
    rc2, it2, _ = S.solve(uv2, tol=1e-300, max_iter=11)
    assert rc2 == Q.QDSE_NOT_CONVERGED and it2 == 11
    S.close()


def test_large_sweep_matches_oracle(Q):
    """n = 1024 (16 row blocks of 64 rows, 1025 loop nodes in 17 lane strides)."""
    n, a, b, alpha = 1024, 0.0, 1.0, 0.5
    print("case fred sweep n=1024", flush=True)
    rng = np.random.default_rng(1024)
    x, t, w, K1, K2, F, f = problem(n, a, b, rng)
    uv = np.concatenate([1.0 + 0.1 * np.sin(5 * x), 0.5 + 0.1 * np.cos(3 * x)])
    dev = lambda a_: torch.tensor(np.ascontiguousarray(a_), device="cuda")  # noqa: E731
    S = Q.FredSolver(n, a, b, alpha, F, dev(K1), dev(K2), dev(f))
    y = S.iterate(dev(uv)).cpu().numpy()
    ref = OF.fred_map(x, t, w, K1, K2, F, f, uv, alpha, 3)
    assert err(y[:n], ref[:n]) < 1e-12 and err(y[n:], ref[n:]) < 1e-12
    S.close()
