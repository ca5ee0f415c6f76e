"""Where the Ball-Chiu gap equation has a physical solution: a finding of the
oracle about the benchmark configurations' interaction, kappa = (D omega)^(1/3)
= 0.8 GeV, omega = 0.5 GeV (Sec. II eqs. dsesys, IRGsQC with the readings of
the interaction's normalisation and the colour factor), recorded as a test.

Walking towards that point along a smooth path of certified solutions
(Newton's method, one step of the path at a time), the branch ends before
the point is reached, and it ends in a characteristic way: not at a fold,
where one singular value of I - J vanishes, but with a whole cluster of
eigenvalues of the sweep's Jacobian J approaching 1 together (about twenty
at N = 64) while the mass function develops grid-scale oscillations in the
infrared. Beyond the end Newton finds no certified solution, and successive
approximation ends at a fixed point with A < 0. Two paths are recorded:

* the vertex homotopy (lam scales the Ball-Chiu parts of the vertex, lam = 0
  is the rainbow vertex) at kappa = 0.8, omega = 0.5: the branch ends at
  lam ~ 0.824 (0.825 at N = 128);
* the straight path in (kappa, omega) at lam = 1 from the paper's parameters
  (D = 0.55 GeV^2, omega = 0.678 GeV) to (0.8, 0.5): the branch ends at
  s ~ 0.72 of the way (kappa ~ 0.777, omega ~ 0.550; s ~ 0.71 at N = 128).

So the configurations' interaction has no certified solution on these grids;
measured throughput at it would be of spurious fixed points. The benchmark
therefore measures converged solves at the paper's interaction, and the
gradient batch samples the part of the (kappa, omega) box that lies on the
physical side of the end of the branch.
"""
import os

import numpy as np
import pytest

from oracle import qdse_oracle as O

N, NA = 64, 32
THREADS = os.cpu_count() or 1


def spectrum(g, p, x):
    """Five smallest singular values of I - J and the number of eigenvalues
    of J within 0.01 of the unit circle."""
    J = O.jacobian(g, p, x, THREADS)
    sv = np.linalg.svd(np.eye(2 * g.n) - J, compute_uv=False)[-5:]
    return sv, int(np.sum(np.abs(np.linalg.eigvals(J)) > 0.99))


def certified_newton(g, p, x, max_newton=12):
    xn, _, r = O.newton(g, p, x, tol=1e-12, max_newton=max_newton, nthreads=THREADS)
    c = O.certificate(g, p, xn, THREADS)
    return xn, bool(r < 1e-11 and c["certified"])


def walk(g, params, steps, x):
    """Natural continuation along params(s) for s in steps, Newton from the
    secant prediction of the last two solutions; every point must be
    certified. Returns the last solution."""
    prev = None
    s_prev = None
    for k, s in enumerate(steps):
        guess = x
        if prev is not None:
            guess = x + (s - steps[k - 1]) / (steps[k - 1] - s_prev) * (x - prev)
        xn, ok = certified_newton(g, params(s), guess)
        assert ok, s
        if k > 0:
            prev, s_prev = x, steps[k - 1]
        x = xn
    return x


@pytest.mark.slow
def test_vertex_homotopy_branch_ends_before_ball_chiu():
    g = O.vac_grid(N, NA)
    x0 = np.concatenate([np.ones(N), np.full(N, 0.3)])
    p08 = O.Params.from_kappa(0.8, 0.5, 0.005, lam=0.8)
    x, rn = O.continuation(g, p08, x0, steps=8, tol=1e-12, nthreads=THREADS)
    assert rn < 1e-12 and O.certificate(g, p08, x, THREADS)["certified"]
    sv08, n08 = spectrum(g, p08, x)
    p082 = O.Params.from_kappa(0.8, 0.5, 0.005, lam=0.82)
    x, ok = certified_newton(g, p082, x)
    assert ok
    sv082, n082 = spectrum(g, p082, x)
    # a cluster, not a fold: the five smallest singular values fall together
    assert np.all(sv082 < 0.25 * sv08) and sv082[-2] < 0.003
    assert n08 == 0 and n082 >= 10
    # beyond the end (lam* ~ 0.824) no certified solution near the branch
    _, ok = certified_newton(g, O.Params.from_kappa(0.8, 0.5, 0.005, lam=0.83), x, max_newton=8)
    assert not ok


@pytest.mark.slow
def test_parameter_path_from_the_paper_point_ends_before_the_configuration():
    g = O.vac_grid(N, NA)
    k0, w0 = (0.55 * 0.678) ** (1 / 3), 0.678

    def params(s):
        return O.Params.from_kappa(k0 + s * (0.8 - k0), w0 + s * (0.5 - w0), 0.005)

    x, it, r, _ = O.picard(g, params(0.0), np.concatenate([np.ones(N), np.full(N, 0.3)]), 1e-12,
                           max_iter=500, mode=1, nthreads=THREADS)
    assert r < 1e-12
    x5 = walk(g, params, [0.0, 0.2, 0.4, 0.5], x)
    x = walk(g, params, [0.4, 0.5, 0.6, 0.65, 0.68, 0.7], x5)
    sv5, _ = spectrum(g, params(0.5), x5)
    sv, _ = spectrum(g, params(0.7), x)
    # the five smallest singular values of I - J fall together along the path
    assert np.all(sv < 0.25 * sv5) and sv[-2] < 0.01
    for s in (0.75, 1.0):
        _, ok = certified_newton(g, params(s), x, max_newton=8)
        assert not ok, s
    # successive approximation at the configuration itself ends at A < 0
    p1 = params(1.0)
    xp, it, r, _ = O.picard(g, p1, np.concatenate([np.ones(N), np.full(N, 0.3)]), 1e-10,
                            max_iter=2000, mode=1, nthreads=THREADS)
    c = O.certificate(g, p1, xp, THREADS)
    assert r < 1e-10 and not c["A_pos"] and not c["certified"]
