"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these retypes the oracle's discretised map: the integrand is checked
against explicit 4x4 Euclidean gamma-matrix traces of the gap equation, the
measure against the volume of the 3-sphere and a Bessel-function closed form,
the full map against adaptive continuum quadrature, the iteration against the
paper's Table 1, and the rest against exact structural limits.
"""
import json
import os

import numpy as np
import pytest
from scipy import integrate, special

from oracle import qdse_oracle as O

HERE = os.path.dirname(os.path.abspath(__file__))
rng = np.random.default_rng(20120366)


# ---------------------------------------------------------------- gamma algebra
def euclid_gammas():
    """Hermitian Euclidean Dirac matrices (chiral representation)."""
    s1 = np.array([[0, 1], [1, 0]], complex)
    s2 = np.array([[0, -1j], [1j, 0]], complex)
    s3 = np.array([[1, 0], [0, -1]], complex)
    z2, i2 = np.zeros((2, 2)), np.eye(2)
    g = [np.block([[z2, -1j * s], [1j * s, z2]]) for s in (s1, s2, s3)]
    g.append(np.block([[z2, i2], [i2, z2]]).astype(complex))
    return g


G = euclid_gammas()
I4 = np.eye(4, dtype=complex)


def slash(v):
    return sum(v[m] * G[m] for m in range(4))


def sinv(v, A, B):
    """Inverse propagator i gamma.p A + B (Sec. II)."""
    return 1j * slash(v) * A + B * I4


def bc_vertex(q, p, Aq, Ap, Bq, Bp, lam=1.0):
    """Ball-Chiu vertex of eq. bcvtxmu with the coefficients of eq. (2),
    lambda_4 = 0; lam scales its parts beyond the bare vertex gamma_nu."""
    P = p + q
    p2, q2 = p @ p, q @ q
    l1 = (Ap + Aq) / 2
    l2 = -1j * (Bp - Bq) / (p2 - q2)
    l3 = 0.5 * (Ap - Aq) / (p2 - q2)
    return [(1 + lam * (l1 - 1)) * G[nu] + lam * (l2 * P[nu] * I4 + l3 * P[nu] * slash(P))
            for nu in range(4)]


def test_clifford_algebra():
    for m in range(4):
        for n in range(4):
            ac = G[m] @ G[n] + G[n] @ G[m]
            assert np.allclose(ac, 2 * (m == n) * I4)
            assert np.allclose(G[m], G[m].conj().T)


def test_vertex_ward_takahashi():
    """i (q-p).Gamma(q,p) = S^-1(q) - S^-1(p) for the vertex of eq. bcvtxmu."""
    for _ in range(50):
        p, q = rng.normal(size=4), rng.normal(size=4)
        Ap, Aq, Bp, Bq = rng.uniform(0.5, 2, 4)
        Gam = bc_vertex(q, p, Aq, Ap, Bq, Bp)
        lhs = 1j * sum((q - p)[nu] * Gam[nu] for nu in range(4))
        rhs = sinv(q, Aq, Bq) - sinv(p, Ap, Bp)
        assert np.allclose(lhs, rhs, atol=1e-13)


@pytest.mark.parametrize("lam", [1.0, 0.0, 0.37])
def test_integrand_equals_dirac_trace(lam):
    """I_A/Delta_q = tr[-i gamma.p M]/(4p^2) and I_B/Delta_q = tr[M]/4 with
    M = T_mu_nu(k) gamma_mu S(q) Gamma_nu(q,p), k = p - q (eq. gendse with the
    kernel ansatz of eq. KernelAnsatz). p, q in general position."""
    worst = 0.0
    for _ in range(200):
        p, q = rng.normal(size=4) * rng.uniform(0.1, 3), rng.normal(size=4) * rng.uniform(0.1, 3)
        Ap, Aq = rng.uniform(0.8, 2.5, 2)
        Bp, Bq = rng.uniform(-0.2, 0.8, 2)
        k = p - q
        T = np.eye(4) - np.outer(k, k) / (k @ k)
        Sq = np.linalg.inv(sinv(q, Aq, Bq))
        Gam = bc_vertex(q, p, Aq, Ap, Bq, Bp, lam)
        M = sum(T[mu, nu] * G[mu] @ Sq @ Gam[nu] for mu in range(4) for nu in range(4))
        trA = np.trace(-1j * slash(p) @ M) / (4 * (p @ p))
        trB = np.trace(M) / 4
        s, t = p @ p, q @ q
        z = (p @ q) / np.sqrt(s * t)
        IA, IB = O.integrand(s, t, z, Ap, Bp, Aq, Bq, lam)
        Dq = t * Aq ** 2 + Bq ** 2
        for a, b in ((IA / Dq, trA), (IB / Dq, trB)):
            assert abs(b.imag) < 1e-12 * (1 + abs(b))
            worst = max(worst, abs(a - b.real) / (1 + abs(b.real)))
    assert worst < 1e-12, worst


# ---------------------------------------------------------------- quadrature
def test_gauss_legendre_exactness():
    for n in (2, 5, 33, 150):
        x, w = np.polynomial.legendre.leggauss(n)
        for deg in range(0, 2 * n, max(1, (2 * n) // 7)):
            exact = 0.0 if deg % 2 else 2.0 / (deg + 1)
            assert abs(w @ x ** deg - exact) < 1e-13


def test_interleaving():
    """t_0 < s_0 < t_1 < ... < s_{N-1} < t_N, the ordering of eq. pqrelationship."""
    for n in (4, 64, 150, 512):
        g = O.vac_grid(n, 8)
        assert g.nq == n + 1
        merged = np.empty(2 * n + 1)
        merged[0::2], merged[1::2] = g.t, g.s
        assert np.all(np.diff(merged) > 0)


def test_interpolation_reproduces_polynomials_and_brackets():
    g = O.vac_grid(40, 8)
    cubic = 0.3 + 0.2 * g.u - 0.05 * g.u ** 2 + 0.004 * g.u ** 3
    fx, br = O.interp(g.u, cubic, g.uq, 3)
    ref = 0.3 + 0.2 * g.uq - 0.05 * g.uq ** 2 + 0.004 * g.uq ** 3
    assert np.max(np.abs(fx - ref)) < 1e-12 * np.max(np.abs(ref))
    # the searched bracket is the a-priori one of eq. pqrelationship: t_j lies
    # between s_{j-1} and s_j
    assert np.array_equal(br, np.arange(-1, g.n))
    lin = 1.5 - 0.1 * g.u
    fx, _ = O.interp(g.u, lin, g.uq, 1)
    inner = slice(1, g.n)
    assert np.max(np.abs(fx[inner] - (1.5 - 0.1 * g.uq[inner]))) < 1e-13
    # eq. chazhiresult: flat beyond the last node; same below the first
    assert fx[-1] == lin[-1] and fx[0] == lin[0]


def qc_g(k2, D, omega):
    """The Gaussian interaction of eq. IRGsQC, read as G(k^2)/k^2."""
    return 8 * np.pi ** 2 / omega ** 4 * D * np.exp(-k2 / omega ** 2)


def test_measure_at_zero_momentum():
    """A = 1, B = b constant: at p -> 0 the gap equation gives
    B(0) - m = C_F * 3 * int d^4q/(2pi)^4 g(q^2) b/(q^2 + b^2), and
    int d^4q f(q^2) = pi^2 int dt t f(t) (the 3-sphere has area 2 pi^2)."""
    D, om, m, b = 1.024, 0.5, 0.005, 0.35
    # the angular rule for sqrt(1-z^2) converges only as O(M^-3): use many nodes
    g = O.vac_grid(128, 3000, s_min=1e-10, s_max=1e4)
    x = np.concatenate([np.ones(g.n), np.full(g.n, b)])
    _, Bn = O.F_rows(g, O.Params(D, om, m), x, [0])
    f = lambda t: t * qc_g(t, D, om) * b / (t + b * b)
    ref = (4.0 / 3.0) * 3 * np.pi ** 2 / (2 * np.pi) ** 4 * integrate.quad(f, 0, np.inf, epsabs=0, epsrel=1e-13, limit=200)[0]
    assert abs((Bn[0] - m) / ref - 1) < 1e-9


def test_angular_bessel_closed_form():
    """A = 1, B = b constant, any p: the angular integral of the Gaussian is
    int_0^pi sin^2(th) e^{x cos th} dth = pi I_1(x)/x, x = 2 sqrt(st)/omega^2, so
    B(s) - m = 1/(2 pi^2) int dt t g0 e^{-(sqrt s - sqrt t)^2/omega^2} I1e(x)/x b/(t+b^2).
    The angular rule converges algebraically (O(M^-3)), the radial one fast."""
    D, om, m, b = 1.024, 0.5, 0.0, 0.3
    g0 = 8 * np.pi ** 2 / om ** 4 * D
    errs = []
    for na in (64, 512):
        g = O.vac_grid(160, na, s_min=1e-4, s_max=1e3)
        rows = [int(np.argmin(np.abs(g.s - s0))) for s0 in (0.01, 0.3, 3.0)]
        x = np.concatenate([np.ones(g.n), np.full(g.n, b)])
        _, Bn = O.F_rows(g, O.Params(D, om, m), x, rows)
        e = []
        for r, bn in zip(rows, Bn):
            s = g.s[r]

            def f(t):
                xx = 2 * np.sqrt(s * t) / om ** 2
                return t * g0 * np.exp(-(np.sqrt(s) - np.sqrt(t)) ** 2 / om ** 2) * special.i1e(xx) / xx * b / (t + b * b)

            # the discrete problem lives on [s_min, s_max]; the Gaussian is
            # below 1e-60 beyond hi
            hi = (np.sqrt(s) + 12 * om) ** 2
            ref = sum(integrate.quad(f, a, b_, epsabs=0, epsrel=1e-12, limit=400)[0]
                      for a, b_ in ((1e-4, s), (s, hi))) / (2 * np.pi ** 2)
            e.append(abs(bn / ref - 1))
        errs.append(max(e))
    assert errs[1] < 5e-7, errs
    assert errs[1] < errs[0] / 100, errs  # O(M^-3): 8x nodes -> ~500x


def smooth_AB(s):
    return 1 + 0.8 / (1 + s / 0.3), 0.005 + 0.4 / (1 + s / 0.5)


def continuum_row(s, D, om, m, lam=1.0):
    """A'(s), B'(s) of the gap equation for the smooth inputs smooth_AB, by
    adaptive quadrature over |q| and the angle with the measure
    d^4q/(2pi)^4 = 4 pi q^3 dq sin^2(th) dth / (2pi)^4, and the integrand of
    the oracle (pinned above against Dirac traces)."""
    Ap, Bp = smooth_AB(s)

    def inner(th, t, which):
        Aq, Bq = smooth_AB(t)
        z = np.cos(th)
        IA, IB = O.integrand(s, t, z, Ap, Bp, Aq, Bq, lam)
        k2 = s + t - 2 * np.sqrt(s * t) * z
        val = (IA if which == 0 else IB) / (t * Aq ** 2 + Bq ** 2)
        return np.sin(th) ** 2 * qc_g(k2, D, om) * val

    out = []
    for which in (0, 1):
        def radial(lnt):
            t = np.exp(lnt)
            ang = integrate.quad(inner, 0, np.pi, args=(t, which), epsabs=0, epsrel=1e-11, limit=200)[0]
            return 4 * np.pi * 0.5 * t * t * ang / (2 * np.pi) ** 4  # q^3 dq = t^2/2 dln t

        lo, hi = np.log(1e-4), np.log(s) + 2.0 + 6.0 * om / np.sqrt(s) + 6 * om * om / s
        val = integrate.quad(radial, lo, min(hi, np.log(1e4)), points=[np.log(s)], epsabs=1e-13,
                             epsrel=1e-10, limit=400)[0]
        out.append(val)
    cf = 4.0 / 3.0
    return 1 + cf * out[0], m + cf * out[1]


@pytest.mark.slow
def test_map_converges_to_continuum_integral():
    """The discretised sweep (interpolation in ln p^2, Gauss-Legendre radial and
    angular sums, singular difference quotients on the interleaved grid)
    approaches the continuum right-hand side of eq. dsesys as N, M grow."""
    D, om, m = 0.55, 0.678, 0.005
    targets = [0.02, 0.3, 2.0]
    errs = {}
    for n, na in ((48, 48), (192, 192)):
        g = O.vac_grid(n, na)
        A, B = smooth_AB(g.s)
        rows = [int(np.argmin(np.abs(g.s - s))) for s in targets]
        An, Bn = O.F_rows(g, O.Params(D, om, m), np.concatenate([A, B]), rows)
        e = 0.0
        for r, a, b in zip(rows, An, Bn):
            ra, rb = continuum_row(g.s[r], D, om, m)
            e = max(e, abs(a - ra) / abs(ra - 1), abs(b - rb) / abs(rb - m))
        errs[n] = e
    assert errs[192] < 5e-5, errs
    assert errs[192] < errs[48] / 8, errs


# ---------------------------------------------------------------- exact limits
def rand_x(n, wigner=False):
    A = 1 + rng.uniform(0, 1, n)
    B = np.zeros(n) if wigner else rng.uniform(0, 0.5, n)
    return np.concatenate([A, B])


def test_free_limit():
    """D = 0: no interaction, F(x) = (1, m) exactly for any x."""
    g = O.vac_grid(24, 12)
    y = O.F(g, O.Params(0.0, 0.5, 0.005), rand_x(24))
    assert np.all(y[:24] == 1.0) and np.all(y[24:] == 0.005)


def test_wigner_solution():
    """m = 0 and B = 0: every B term carries B(q^2) or a B difference, so B stays 0."""
    g = O.vac_grid(24, 12)
    y = O.F(g, O.Params(1.024, 0.5, 0.0), rand_x(24, wigner=True))
    assert np.all(y[24:] == 0.0)
    assert np.all(np.isfinite(y[:24]))


def test_constant_inputs_kill_difference_terms():
    """A = a, B = b constants: both difference quotients vanish and sigma_A = a,
    so the Ball-Chiu sweep is the bare-vertex sweep scaled by a, and with a = 1
    it does not depend on the vertex homotopy at all."""
    g = O.vac_grid(32, 16)
    for a in (1.0, 1.7):
        x = np.concatenate([np.full(32, a), np.full(32, 0.3)])
        y1 = O.F(g, O.Params(1.024, 0.5, 0.005, 1.0), x)
        y0 = O.F(g, O.Params(1.024, 0.5, 0.005, 0.0), x)
        assert np.allclose(y1[:32] - 1, a * (y0[:32] - 1), rtol=1e-12, atol=1e-15)
        assert np.allclose(y1[32:] - 0.005, a * (y0[32:] - 0.005), rtol=1e-12, atol=1e-15)
        if a == 1.0:
            y5 = O.F(g, O.Params(1.024, 0.5, 0.005, 0.5), x)
            # interpolation weights sum to one only up to rounding, so the
            # difference quotients are rounding-level, not exactly zero
            assert np.allclose(y5, y1, rtol=1e-13, atol=0)


def test_openmp_rows_bitwise_equal_sequential():
    """Rows are independent (Sec. III, Table 1's sequential and OpenMP programs): any thread count gives
    the same bits."""
    g = O.vac_grid(64, 32)
    x = rand_x(64)
    p = O.Params.from_kappa(0.8, 0.5, 0.005)
    assert np.array_equal(O.F(g, p, x, 1), O.F(g, p, x, 8))
    assert np.array_equal(O.F(g, p, x, 3), O.F(g, p, x, 8))
    a, b = O.F_rows(g, p, x, [5, 0, 63], 2)
    full = O.F(g, p, x, 1)
    assert np.array_equal(a, full[[5, 0, 63]]) and np.array_equal(b, full[64 + np.array([5, 0, 63])])


def test_jvp_matches_central_differences():
    g = O.vac_grid(32, 16)
    p = O.Params.from_kappa(0.8, 0.5, 0.005)
    x, v = rand_x(32), rng.normal(size=64)
    jv = O.jvp(g, p, x, v)
    h = 1e-6
    fd = (O.F(g, p, x + h * v) - O.F(g, p, x - h * v)) / (2 * h)
    assert np.max(np.abs(jv - fd)) < 1e-7 * np.max(np.abs(jv))


# ---------------------------------------------------------------- the paper's run
def test_table1_iteration_count():
    """Sec. IV Table 1: N = 150, M = 100, xi = 0.005, D = 0.55, omega = 0.678,
    A0 = B0 = 1: the iteration stops after 11 sweeps."""
    with open(os.path.join(HERE, "golden", "table1.json")) as f:
        ref = json.load(f)
    n = ref["N"]
    g = O.vac_grid(n, ref["M"])
    x0 = np.concatenate([np.full(n, ref["A0"]), np.full(n, ref["B0"])])
    x, it, r, _ = O.picard(g, O.Params(ref["D"], ref["omega"], 0.0), x0, ref["xi"], mode=0)
    assert it == ref["iterations"]
    assert r < ref["xi"]


def test_paper_algorithms_give_the_same_sweep():
    """Table 1's four algorithms (traditional or modified interpolation inside
    the loops, sequential or OpenMP over external momenta, Sec. III) compute
    exactly the same sweep as the oracle map with interpolation hoisted out of
    the loops; the modified bracket of eq. pqrelationship equals the searched
    one on the interleaved grid."""
    rng = np.random.default_rng(31)
    for n, na, order in ((40, 16, 1), (33, 12, 3)):
        g = O.vac_grid(n, na, order=order)
        p = O.Params(0.55, 0.678, 0.005)
        A, B = smooth_AB(g.s)
        x = np.concatenate([A * (1 + 0.05 * rng.standard_normal(n)), B])
        ref = O.F(g, p, x, nthreads=1)
        for modified in (False, True):
            for threads in (1, 4):
                got = O.F_paper(g, p, x, modified, threads)
                assert np.array_equal(got, ref), (n, order, modified, threads)


def test_paper_algorithm_4_table1_iterations():
    """Algorithm 4 of Table 1 (modified interpolation, OpenMP) on the Table 1
    workload stops after 11 sweeps, like the hoisted oracle."""
    with open(os.path.join(HERE, "golden", "table1.json")) as f:
        ref = json.load(f)
    n = ref["N"]
    g = O.vac_grid(n, ref["M"])
    x0 = np.concatenate([np.full(n, ref["A0"]), np.full(n, ref["B0"])])
    x, it = O.picard_paper(g, O.Params(ref["D"], ref["omega"], 0.0), x0, ref["xi"],
                           modified=True, nthreads=4)
    assert it == ref["iterations"]


def test_newton_reaches_picard_fixed_point():
    """At the paper's parameters successive approximation contracts; Newton on
    F(x) - x = 0 from the same start finds the same fixed point."""
    n = 32
    g = O.vac_grid(n, 24)
    p = O.Params(0.55, 0.678, 0.005)
    x0 = np.concatenate([np.ones(n), np.ones(n)])
    xp, it, r, _ = O.picard(g, p, x0, 1e-13, max_iter=500, mode=0)
    xn, steps, rn = O.newton(g, p, x0, tol=1e-13)
    assert rn < 1e-13 and steps < 15
    assert np.max(np.abs(xp - xn)) < 1e-12
    rho, _ = O.spectral_radius(g, p, xn)
    assert rho < 1.0


# ---------------------------------------------------------------- drivers
def rainbow_map(g, D, om, m, x):
    """The Landau-gauge rainbow sweep (bare vertex) written here from the
    textbook form: A(s) = 1 + C_F s^-1 int g(k^2) sigma_V [p.q + 2 (k.p)(k.q)/k^2],
    B(s) = m + 3 C_F int g(k^2) sigma_S, sigma_V = A(t)/Delta, sigma_S =
    B(t)/Delta, Delta = t A(t)^2 + B(t)^2, int d^4q/(2 pi)^4 = (8 pi^3)^-1
    sum_j W_j sum_a w_a sqrt(1 - z_a^2), W_j = GL weight in ln t times t^2 (the grid's W),
    g(k^2) = (8 pi^2 / omega^4) D exp(-k^2 / omega^2); A(t), B(t) from the
    oracle's interpolation (pinned separately by polynomial reproduction)."""
    n = g.n
    Aq, _ = O.interp(g.u, x[:n], g.uq, g.order)
    Bq, _ = O.interp(g.u, x[n:], g.uq, g.order)
    Dl = g.t * Aq ** 2 + Bq ** 2
    s = g.s[:, None, None]
    t = g.t[None, :, None]
    z = g.z[None, None, :]
    r = np.sqrt(s * t)
    k2 = s + t - 2 * r * z
    kp, kq = s - r * z, r * z - t
    wgt = g.W[None, :, None] * (g.wz * np.sqrt(1 - g.z ** 2))[None, None, :]
    gk = 8 * np.pi ** 2 * D / om ** 4 * np.exp(-k2 / om ** 2)
    c = (4 / 3) / (8 * np.pi ** 3)
    a = 1 + c * np.sum(wgt * gk * (Aq / Dl)[None, :, None] * (r * z + 2 * kp * kq / k2), axis=(1, 2)) / g.s
    b = m + 3 * c * np.sum(wgt * gk * (Bq / Dl)[None, :, None], axis=(1, 2))
    return np.concatenate([a, b])


def test_homotopy_start_is_the_rainbow_map():
    """lam = 0 of the vertex homotopy is the bare vertex: the oracle's sweep
    at lam = 0 equals the rainbow sweep written above, at the configurations'
    interaction and at the paper's."""
    g = O.vac_grid(40, 20)
    x = rand_x(40)
    for kap, om in ((0.8, 0.5), ((0.55 * 0.678) ** (1 / 3), 0.678)):
        p = O.Params.from_kappa(kap, om, 0.005, lam=0.0)
        got = O.F(g, p, x)
        ref = rainbow_map(g, p.D, om, 0.005, x)
        assert np.max(np.abs(got - ref) / np.maximum(np.abs(ref), 1e-3)) < 1e-12


def test_continuation_endpoints():
    """continuation(): its lam = 0 stage converges to the fixed point of the
    rainbow sweep written above (iterated here; it contracts), and walking to
    lam = 1 at the paper's parameters ends at successive approximation's
    fixed point of the full Ball-Chiu sweep."""
    n = 32
    g = O.vac_grid(n, 24)
    x0 = np.concatenate([np.ones(n), np.full(n, 0.3)])
    p0 = O.Params.from_kappa(0.8, 0.5, 0.005, lam=0.0)
    xr = x0.copy()
    for _ in range(300):
        xn = rainbow_map(g, p0.D, 0.5, 0.005, xr)
        done = np.max(np.abs(xn - xr)) < 1e-14
        xr = xn
        if done:
            break
    xc, rn = O.continuation(g, p0, x0, steps=1)
    assert rn < 1e-13
    assert np.max(np.abs(xc - xr)) < 1e-12
    assert xr[n] > 0.3  # dynamical mass in the infrared
    p1 = O.Params(0.55, 0.678, 0.005)
    xc1, rn1 = O.continuation(g, p1, x0, steps=4)
    xp, it, r, _ = O.picard(g, p1, x0, 1e-14, max_iter=500, mode=0)
    assert rn1 < 1e-13 and np.max(np.abs(xc1 - xp)) < 1e-12


def test_certificate_flags():
    """certificate(): the residual is max |F(x) - x|; A <= 0 anywhere clears
    A_pos, A < 1 clears A_ge_1, a rise of M with p^2 clears M_falls; a mass
    function whose node-to-node slope changes sign is counted (slope_flips),
    a monotone one gives 0. The Nambu fixed point at the paper's parameters
    is certified (its A has a maximum at intermediate p^2, so A is not
    required to fall)."""
    n = 32
    g = O.vac_grid(n, 24)
    p = O.Params(0.55, 0.678, 0.005)
    x0 = np.concatenate([np.ones(n), np.ones(n)])
    xs, _, _, _ = O.picard(g, p, x0, 1e-14, max_iter=500, mode=0)
    c = O.certificate(g, p, xs)
    assert c["certified"] and c["slope_flips"] == 0 and c["resid"] < 1e-13
    y = xs.copy()
    y[3] = -0.5
    c = O.certificate(g, p, y)
    assert not c["A_pos"] and not c["certified"]
    assert abs(c["resid"] - np.max(np.abs(O.F(g, p, y) - y))) == 0.0
    assert np.any(np.diff(xs[:n]) > 0.01)
    y = xs.copy()
    y[n - 3] = 0.99
    c = O.certificate(g, p, y)
    assert c["A_pos"] and not c["A_ge_1"] and not c["certified"]
    y = xs.copy()
    y[n + 5] *= 1.2  # a bump in B: the slope of M changes sign twice
    c = O.certificate(g, p, y)
    assert c["slope_flips"] == 2 and not c["M_falls"] and not c["certified"]
    y = xs.copy()
    y[n:] = -y[n:]  # the negative-mass partner: M rises towards 0
    assert not O.certificate(g, p, y)["M_falls"]
    y = xs.copy()
    y[n + 4:n + 12] *= 1 + 0.3 * (-1) ** np.arange(8)
    assert O.certificate(g, p, y)["slope_flips"] >= 6
