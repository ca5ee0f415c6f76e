"""Pins of the oracle's renormalised Qin-Chang setting (beyond the paper,
whose Sec. II drops the ultraviolet part of the interaction and sets the
renormalisation constants to 1), each against something other than the
oracle's own formulas:

* the ultraviolet term reduces to 4 pi times the textbook one-loop running
  coupling 12 pi / ((33 - 2 N_f) ln(k^2/L^2)) at large k^2, and to its closed
  form at k^2 -> 0;
* the renormalisation conditions A(zeta^2) = 1, B(zeta^2) = m hold for the
  map's output when zeta^2 is a grid node;
* free limit: D = 0 without the ultraviolet term gives (1, m) for any input;
* multiplicative renormalisability: with Z_1 = Z_2 the loop sums are
  invariant under (A, B) -> c (A, B), so the fixed points for two
  renormalisation points are proportional and the mass function B/A is the
  same (exactly, for the discrete map), given the matching current mass;
* the current-mass part of M runs at large p^2 with a log slope near
  -gamma_m = -12/25 (leading-log physics, a loose check).
"""
import math

import numpy as np
import pytest

from oracle import qdse_oracle as O

GAMMA_M = 12.0 / 25.0
LQCD2 = 0.234 ** 2


def test_uv_term_is_the_one_loop_running_coupling_at_large_k2():
    for k2 in (1e3, 1e5, 1e7, 1e9):
        alpha1 = 12.0 * math.pi / (25.0 * math.log(k2 / LQCD2))
        ratio = k2 * O.g_uv(k2) / (4.0 * math.pi * alpha1)
        x = k2 / LQCD2
        # ln[tau + (1 + x)^2] = ln x^2 + 2/x + O(1/x^2); the infrared factor is 1 to exp(-k2)
        assert abs(ratio - 1.0) < 2.0 * (2.0 / x) / math.log(x * x) + 1e-12, (k2, ratio)


def test_uv_term_infrared_limit():
    # k^2 -> 0: F -> 1/(4 m_t^2) and ln[tau + 1] = ln e^2 = 2
    want = 8.0 * math.pi ** 2 * GAMMA_M / (4.0 * 0.25 * 2.0)
    assert O.g_uv(1e-12) == pytest.approx(want, rel=1e-9)


def smooth_x(g, seed=3):
    rng = np.random.default_rng(seed)
    u = (g.u - g.u[0]) / (g.u[-1] - g.u[0])
    A = 1.0 + 0.3 * np.exp(-3 * u) + 0.01 * rng.standard_normal() * u
    B = 0.35 * np.exp(-4 * u) + 0.004
    return np.concatenate([A, B])


@pytest.mark.parametrize("order", [1, 3])
def test_renormalisation_conditions_hold_at_a_grid_node(order):
    n, na = 24, 12
    g = O.vac_grid(n, na, order=order)
    k = 17
    zeta = math.sqrt(g.s[k])
    x = smooth_x(g)
    for m in (0.0034, 0.02):
        y = O.F(g, O.Params(0.55, 0.678, m, 1.0, 1, zeta), x)
        assert abs(y[k] - 1.0) < 1e-13
        assert abs(y[n + k] - m) < 1e-13 * max(1.0, abs(y[n:]).max())
    y0 = O.F(g, O.Params(0.55, 0.678, 0.0, 1.0, 1, zeta), x)
    assert abs(y0[k] - 1.0) < 1e-13


def test_free_limit_without_uv_term():
    n = 16
    g = O.vac_grid(n, 8)
    x = smooth_x(g)
    y = O.F(g, O.Params(0.0, 0.678, 0.005, 1.0, 0, 19.0), x)
    assert np.array_equal(y, np.concatenate([np.ones(n), np.full(n, 0.005)]))


def solve(g, p, tol=1e-14):
    x, it = O.picard(g, p, np.ones(2 * g.n), tol, max_iter=3000, mode=0)[:2]
    assert it < 3000
    return x


@pytest.mark.parametrize("m1", [0.0, 0.0034])
def test_mass_function_does_not_depend_on_the_renormalisation_point(m1):
    n, na = 40, 20
    g = O.vac_grid(n, na)
    x1 = solve(g, O.Params(0.55, 0.678, m1, 1.0, 1, 19.0))
    k = 28  # second point at a grid node: the matching current mass is M1 there
    zeta2 = math.sqrt(g.s[k])
    m2 = x1[n + k] / x1[k] if m1 else 0.0
    x2 = solve(g, O.Params(0.55, 0.678, m2, 1.0, 1, zeta2))
    M1, M2 = x1[n:] / x1[:n], x2[n:] / x2[:n]
    assert np.max(np.abs(M1 - M2) / np.abs(M1)) < 1e-11
    c = x1[:n] / x2[:n]  # the fixed points are proportional
    assert np.ptp(c) < 1e-11 * abs(c[0])
    assert abs(x2[k] - 1.0) < 1e-12


def test_current_mass_runs_with_the_anomalous_dimension():
    n, na = 64, 32
    g = O.vac_grid(n, na)
    xm = solve(g, O.Params(0.55, 0.678, 0.0034, 1.0, 1, 19.0), tol=1e-13)
    x0 = solve(g, O.Params(0.55, 0.678, 0.0, 1.0, 1, 19.0), tol=1e-13)
    dM = xm[n:] / xm[:n] - x0[n:] / x0[:n]
    lnln = np.log(np.log(g.s[g.s > 1.0] / LQCD2))
    d = dM[g.s > 1.0]
    i1 = np.argmin(abs(g.s[g.s > 1.0] - 1e3))
    i2 = np.argmin(abs(g.s[g.s > 1.0] - 5e3))
    slope = (math.log(d[i2]) - math.log(d[i1])) / (lnln[i2] - lnln[i1])
    assert -GAMMA_M - 0.15 < slope < -GAMMA_M + 0.05, slope
