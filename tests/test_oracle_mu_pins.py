"""Pins of the finite-mu oracle (explicit complex Dirac algebra) against the
pinned vacuum oracle and exact properties."""
import numpy as np
import pytest

from oracle import qdse_oracle as O
from tests.test_oracle_pins import G, I4, slash

rng = np.random.default_rng(2012)


def sinv_mu(v, A, B, C):
    """i gamma_vec.v_vec A + i gamma_4 v_4 C + B for a complex four-vector v."""
    return 1j * (A * sum(v[m] * G[m] for m in range(3)) + C * v[3] * G[3]) + B * I4


def vertex_mu(q, p, fq, fp):
    Aq, Bq, Cq = fq
    Ap, Bp, Cp = fp
    P = p + q
    dq = q @ q - p @ p
    sA, sC = (Aq + Ap) / 2, (Cq + Cp) / 2
    dA, dB, dC = (Aq - Ap) / dq, (Bq - Bp) / dq, (Cq - Cp) / dq
    Pv = sum(P[m] * G[m] for m in range(3))
    return [(sA if nu < 3 else sC) * G[nu] + P[nu] * (dA / 2 * Pv + dC / 2 * P[3] * G[3] - 1j * dB * I4)
            for nu in range(4)]


def test_finite_mu_vertex_ward_takahashi():
    """i (q~ - p~).Gamma = S^-1(q~) - S^-1(p~) with complex p~ = (p_vec, p4 + i mu)."""
    for _ in range(40):
        mu = rng.uniform(0, 0.5)
        p = np.array([*rng.normal(size=3), rng.normal() + 1j * mu])
        q = np.array([*rng.normal(size=3), rng.normal() + 1j * mu])
        fp = rng.uniform(0.5, 2, 3) + 1j * rng.uniform(-.3, .3, 3)
        fq = rng.uniform(0.5, 2, 3) + 1j * rng.uniform(-.3, .3, 3)
        Gam = vertex_mu(q, p, fq, fp)
        lhs = 1j * sum((q - p)[nu] * Gam[nu] for nu in range(4))
        rhs = sinv_mu(q, *fq) - sinv_mu(p, *fp)
        assert np.allclose(lhs, rhs, atol=1e-12)


def test_finite_mu_projections_reduce_to_vacuum_integrand():
    """At mu = 0 with C = A (real), |p_vec|^2 A-proj + p4^2 C-proj is the vacuum
    A projection times p^2 and the B projections agree: the finite-mu algebra
    against the vacuum integrand pinned by the Dirac-trace test."""
    worst = 0.0
    for _ in range(200):
        pabs, qabs = rng.uniform(0.05, 3, 2)
        p4, q4 = rng.uniform(-2, 2, 2)
        z = rng.uniform(-1, 1)
        Ap, Aq = rng.uniform(0.8, 2.5, 2)
        Bp, Bq = rng.uniform(-0.2, 0.8, 2)
        a, b, c = O.mu_projections(pabs, p4, qabs, q4, z, 0.0, (Ap, Bp, Ap), (Aq, Bq, Aq))
        s, t = pabs ** 2 + p4 ** 2, qabs ** 2 + q4 ** 2
        z4 = (pabs * qabs * z + p4 * q4) / np.sqrt(s * t)
        IA, IB = O.integrand(s, t, z4, Ap, Bp, Aq, Bq, 1.0)
        Dq = t * Aq ** 2 + Bq ** 2
        lhs = pabs ** 2 * a + p4 ** 2 * c
        for x, y in ((lhs, s * IA / Dq), (b, IB / Dq)):
            assert abs(x.imag) < 1e-12
            worst = max(worst, abs(x.real - y) / (1 + abs(y)))
    assert worst < 1e-12, worst


def test_finite_mu_free_limit_and_wigner():
    g = O.mu_grid(6, 5, 4, r_max=8, p4_max=8)
    x = np.stack([1.2 + 0.1j * rng.normal(size=g.ne), 0.3 + 0.05j * rng.normal(size=g.ne),
                  1.1 + 0.1j * rng.normal(size=g.ne)])
    y = O.F_mu(g, 0.0, 0.6, 0.005, 0.3, x)
    assert np.all(y[0] == 1.0) and np.all(y[1] == 0.005) and np.all(y[2] == 1.0)
    x[1] = 0.0
    y = O.F_mu(g, 0.55, 0.678, 0.0, 0.3, x)
    assert np.all(y[1] == 0.0)


@pytest.mark.slow
def test_finite_mu_at_zero_mu_approaches_vacuum_continuum():
    """mu = 0 and an O(4)-symmetric input A(p^2) = C(p^2), B(p^2): as the
    (|p_vec|, p4, angle) grid is refined the finite-mu sweep approaches the
    vacuum sweep at p^2 = |p_vec|^2 + p4^2 (the vacuum map on a fine grid,
    itself pinned to continuum quadrature). Pins the finite-mu measure, the
    q4 symmetrisation and the 2-D interpolation."""
    D, om, m = 0.55, 0.678, 0.005
    Af = lambda s: 1 + 0.8 / (1 + s / 0.3)
    Bf = lambda s: 0.005 + 0.4 / (1 + s / 0.5)
    gv = O.vac_grid(256, 256, s_min=1e-4, s_max=64.0)
    xv = np.concatenate([Af(gv.s), Bf(gv.s)])
    yv = O.F(gv, O.Params(D, om, m), xv)
    errs = []
    for ns, na in ((10, 8), (20, 16)):
        g = O.mu_grid(ns, ns, na, r_min=1e-2, r_max=8.0, p4_max=8.0)
        P2 = (g.ps[:, None] ** 2 + g.p4[None, :] ** 2).ravel()
        x = np.stack([Af(P2), Bf(P2), Af(P2)]).astype(complex)
        rows = [e for e in range(g.ne) if 0.05 < P2[e] < 2.0][::3]
        y = O.F_mu(g, D, om, m, 0.0, x, rows=rows)
        refA = np.interp(np.log(P2[rows]), np.log(gv.s), yv[:gv.n])
        refB = np.interp(np.log(P2[rows]), np.log(gv.s), yv[gv.n:])
        assert np.max(np.abs(y.imag)) < 1e-12
        e = max(np.max(np.abs(y[0].real - refA) / np.abs(refA - 1)),
                np.max(np.abs(y[2].real - refA) / np.abs(refA - 1)),
                np.max(np.abs(y[1].real - refB) / np.abs(refB - m)))
        errs.append(e)
    assert errs[1] < errs[0] / 3, errs
    assert errs[1] < 0.03, errs


def test_matsubara_sum_closed_form():
    """Finite temperature: the loop frequencies and weights of the T > 0 grid,
    summed over both signs, reproduce the fermion Matsubara sum
    T sum_n 1 / (w_n^2 + E^2) = tanh(E / 2T) / (2 E), w_n = (2n+1) pi T, i.e.
    sum over the grid of w4 f(q4) = 2 pi x that (int dq4/(2 pi) -> T sum_n).
    A bosonic set 2 n pi T gives coth instead, a weight pi T half the value.
    The truncation error is a 1/n4 tail, removed by Richardson extrapolation
    from n4 = 1000 and 2000."""
    for T, E in ((0.1, 0.5), (0.02, 0.3)):
        exact = 2 * np.pi * np.tanh(E / (2 * T)) / (2 * E)
        S = {}
        for n4 in (1000, 2000):
            g = O.mu_grid(6, n4, 4, T=T)
            S[n4] = 2.0 * np.sum(g.wq4 / (g.q4 ** 2 + E ** 2))  # both signs of q4
        assert abs(S[2000] - exact) < abs(S[1000] - exact) / 1.9
        assert abs(2 * S[2000] - S[1000] - exact) < 1e-8 * exact, (T, E)


def test_finite_temperature_free_limit_and_wigner():
    g = O.mu_grid(6, 5, 4, r_max=8, T=0.1)
    x = np.stack([1.2 + 0.1j * rng.normal(size=g.ne), 0.3 + 0.05j * rng.normal(size=g.ne),
                  1.1 + 0.1j * rng.normal(size=g.ne)])
    y = O.F_mu(g, 0.0, 0.6, 0.005, 0.3, x)
    assert np.all(y[0] == 1.0) and np.all(y[1] == 0.005) and np.all(y[2] == 1.0)
    x[1] = 0.0
    y = O.F_mu(g, 0.55, 0.678, 0.0, 0.3, x)
    assert np.all(y[1] == 0.0)


def test_finite_temperature_approaches_zero_temperature():
    """mu = 0, an O(4)-symmetric input A(p^2) = C(p^2), B(p^2): as T falls (with
    the frequency range held fixed, n4 = 8 / (2 pi T)) the finite-T sweep at
    the lowest frequency approaches the vacuum sweep at p^2 = |p_vec|^2 +
    (pi T)^2: the thermal difference shrinks much faster than T, down to the
    spatial discretisation floor. Pins the Matsubara measure inside the full
    sweep."""
    D, om, m = 0.55, 0.678, 0.005
    Af = lambda s: 1 + 0.8 / (1 + s / 0.3)
    Bf = lambda s: 0.005 + 0.4 / (1 + s / 0.5)
    gv = O.vac_grid(256, 256, s_min=1e-4, s_max=64.0)
    xv = np.concatenate([Af(gv.s), Bf(gv.s)])
    yv = O.F(gv, O.Params(D, om, m), xv)
    errs = []
    for T in (0.08, 0.04, 0.02):
        n4 = int(round(8.0 / (2 * np.pi * T)))
        g = O.mu_grid(32, n4, 32, r_min=1e-2, r_max=8.0, T=T)
        P2 = (g.ps[:, None] ** 2 + g.p4[None, :] ** 2).ravel()
        x = np.stack([Af(P2), Bf(P2), Af(P2)]).astype(complex)
        rows = [e for e in range(g.ne) if e % g.n4 == 0 and 0.05 < P2[e] < 2.0]
        y = O.F_mu(g, D, om, m, 0.0, x, rows=rows)
        refA = np.interp(np.log(P2[rows]), np.log(gv.s), yv[:gv.n])
        refB = np.interp(np.log(P2[rows]), np.log(gv.s), yv[gv.n:])
        assert np.max(np.abs(y.imag)) < 1e-12
        e = max(np.max(np.abs(y[0].real - refA) / np.abs(refA - 1)),
                np.max(np.abs(y[1].real - refB) / np.abs(refB - m)))
        errs.append(e)
    assert errs[1] < errs[0] / 5, errs
    assert errs[2] < errs[1] and errs[2] < 3e-3, errs


def test_finite_temperature_successive_approximation_is_unstable():
    """A finding, recorded so that it is not lost: with the finite-mu
    Ball-Chiu vertex carried over to Matsubara frequencies, successive
    approximation from A = C = 1, B = 0.3 GeV diverges on every tested grid
    (the same growing mode appears with 16 or 128 angles, so it is not the
    angular rule); sweeps themselves are well defined and parity-tested.
    Once A, B, C depend on |p_vec| and p4 separately, the difference
    quotients (F(q~) - F(p~)) / (q~^2 - p~^2) no longer vanish where
    q~^2 = p~^2, and loop points close to that circle enter with large
    weight."""
    g = O.mu_grid(16, 10, 16, r_min=1e-2, r_max=8.0, T=0.1)
    x = np.zeros((3, g.ne), complex)
    x[0], x[1], x[2] = 1.0, 0.3, 1.0
    r = []
    for _ in range(8):
        xn = O.F_mu(g, 0.55, 0.678, 0.005, 0.0, x, nthreads=4)
        r.append(np.max(np.abs(xn - x)))
        x = xn
    assert r[-1] > 100 * r[1], r



# ------------------------------------------------ finite mu != 0, test-side Dirac algebra
def dirac_projections(pv, p4t, qv, q4t, fp, fq):
    """(A, B, C) projections of M = T_mu_nu(k) gamma_mu S(q~) Gamma_nu(q~, p~)
    built here from explicit matrices: p~ = (pv, p4t), q~ = (qv, q4t) with
    complex fourth components, k = p - q real (Re of the difference; the shift
    i mu cancels), S = inverse of sinv_mu, Gamma = vertex_mu (both checked by
    the Ward-Takahashi test above). A = tr[-i gamma_vec.p_vec M]/(4 |p_vec|^2),
    C = tr[-i gamma_4 p~_4 M]/(4 p~_4^2), B = tr[M]/4."""
    p = np.array([*pv, p4t], complex)
    q = np.array([*qv, q4t], complex)
    k = (p - q).real
    assert np.max(np.abs((p - q).imag)) < 1e-14
    T = np.eye(4) - np.outer(k, k) / (k @ k)
    S = np.linalg.inv(sinv_mu(q, *fq))
    Gam = vertex_mu(q, p, fq, fp)
    M = sum(T[a, b] * G[a] @ S @ Gam[b] for a in range(4) for b in range(4))
    pvs = sum(pv[m] * G[m] for m in range(3))
    A = np.trace(-1j * pvs @ M) / (4 * (pv @ pv))
    C = np.trace(-1j * p4t * G[3] @ M) / (4 * p4t * p4t)
    B = np.trace(M) / 4
    return A, B, C


def _random_frame():
    e1 = rng.normal(size=3)
    e1 /= np.linalg.norm(e1)
    e2 = rng.normal(size=3)
    e2 -= (e2 @ e1) * e1
    e2 /= np.linalg.norm(e2)
    return e1, e2


def _cplx3():
    return rng.uniform(0.5, 2, 3) + 1j * rng.uniform(-0.4, 0.4, 3)


@pytest.mark.parametrize("mu", [0.1, 0.3, 0.45])
def test_finite_mu_projections_match_dirac_traces(mu):
    """The oracle's projections at mu != 0 with complex A, B, C against the
    traces built here with p~ = (p_vec, p4 + i mu), q~ = (q_vec, q4 + i mu) in
    a randomly oriented frame (the oracle fixes p_vec along one axis, so this
    also checks rotation invariance). A sign slip in p4 + i mu, a conjugated
    q~^2 or a wrong projector changes these at O(mu)."""
    worst = 0.0
    for _ in range(220):
        pabs, qabs = rng.uniform(0.05, 3, 2)
        p4, q4 = rng.uniform(-2, 2, 2)
        z = rng.uniform(-1, 1)
        fp, fq = _cplx3(), _cplx3()
        e1, e2 = _random_frame()
        pv = pabs * e1
        qv = qabs * (z * e1 + np.sqrt(1 - z * z) * e2)
        ref = dirac_projections(pv, p4 + 1j * mu, qv, q4 + 1j * mu, fp, fq)
        got = O.mu_projections(pabs, p4, qabs, q4, z, mu, tuple(fp), tuple(fq))
        for a, b in zip(got, ref):
            worst = max(worst, abs(a - b) / (1 + abs(b)))
    assert worst < 1e-12, worst


def test_finite_mu_projections_constant_functions_closed_form():
    """A = C = a, B = b constant (complex): the vertex is a gamma_nu and
    S(q~) = (-i a gamma.q~ + b)/(a^2 q~^2 + b^2) with q~^2 = |q|^2 + (q4 + i mu)^2
    (no conjugation). The Dirac algebra (tr of four gammas, T_mu_mu = 3) gives
    B = 3 a b / Delta, A = -a^2 (2 p.T.q~ - 3 p.q~)/(|p|^2 Delta) with p the
    spatial four-vector (p_vec, 0), C = -a^2 (2 (T q~)_4 - 3 q~_4)/(p~_4 Delta).
    A closed form independent of any matrix code; at mu = 0 it is the Landau
    rainbow integrand."""
    worst = 0.0
    for _ in range(200):
        mu = rng.uniform(0.05, 0.5)
        pabs, qabs = rng.uniform(0.05, 3, 2)
        p4, q4 = rng.uniform(-2, 2, 2)
        z = rng.uniform(-1, 1)
        a = complex(rng.uniform(0.6, 2), rng.uniform(-0.3, 0.3))
        b = complex(rng.uniform(0.1, 0.8), rng.uniform(-0.3, 0.3))
        sn = np.sqrt(1 - z * z)
        pt = np.array([0, 0, pabs, p4 + 1j * mu])
        qt = np.array([qabs * sn, 0, qabs * z, q4 + 1j * mu])
        k = (pt - qt).real
        T = np.eye(4) - np.outer(k, k) / (k @ k)
        Dl = a * a * (qt @ qt) + b * b
        ps = np.array([0, 0, pabs, 0])
        Bc = 3 * a * b / Dl
        Ac = -a * a * (2 * ps @ T @ qt - 3 * ps @ qt) / (pabs ** 2 * Dl)
        Cc = -a * a * (2 * (T @ qt)[3] - 3 * qt[3]) / (pt[3] * Dl)
        got = O.mu_projections(pabs, p4, qabs, q4, z, mu, (a, b, a), (a, b, a))
        for x, y in zip(got, (Ac, Bc, Cc)):
            worst = max(worst, abs(x - y) / (1 + abs(y)))
    assert worst < 1e-12, worst


def test_finite_mu_projections_time_reversal_conjugation():
    """p4 -> -p4 and q4 -> -q4 with conjugated A, B, C conjugates all three
    projections (the symmetry behind F(|p|, -p4) = F(|p|, p4)^*): checked
    on the oracle at mu != 0."""
    worst = 0.0
    for _ in range(200):
        mu = rng.uniform(0.05, 0.5)
        pabs, qabs = rng.uniform(0.05, 3, 2)
        p4, q4 = rng.uniform(-2, 2, 2)
        z = rng.uniform(-1, 1)
        fp, fq = _cplx3(), _cplx3()
        a = O.mu_projections(pabs, p4, qabs, q4, z, mu, tuple(fp), tuple(fq))
        b = O.mu_projections(pabs, -p4, qabs, -q4, z, mu, tuple(np.conj(fp)), tuple(np.conj(fq)))
        for x, y in zip(a, b):
            worst = max(worst, abs(x - np.conj(y)) / (1 + abs(x)))
    assert worst < 1e-12, worst


def test_finite_mu_sweep_matches_brute_force_sum():
    """Whole finite-mu sweep at mu = 0.3 on a tiny grid against a sum written
    here from the readings: measure d^4q/(2 pi)^4 = dq4 2 pi |q|^2 d|q| dz /
    (2 pi)^4 over the loop points (q4 of both signs, values at -q4 the
    complex conjugates), C_F g(k^2) with g = (8 pi^2 / omega^4) D exp(-k^2 /
    omega^2), projections from the test-side Dirac algebra. The input A, B, C
    are complex bicubic polynomials in (ln|p|, v), which the 4-point tensor
    stencils reproduce exactly, so the loop values are the polynomials
    themselves. Pins the q4 fold (a dropped conjugation fails), the measure
    and the sign of the i mu shift inside the full sweep."""
    g = O.mu_grid(5, 5, 3, r_min=0.1, r_max=4.0, p4_max=4.0, lam4=0.5, order=3)
    D, om, m, mu = 0.55, 0.678, 0.005, 0.3
    vmax = np.arcsinh(4.0 / 0.5)
    cf = rng.normal(size=(3, 4, 4)) * 0.05 + 1j * rng.normal(size=(3, 4, 4)) * 0.05
    cf[0, 0, 0] += 1.3
    cf[1, 0, 0] += 0.35
    cf[2, 0, 0] += 1.2

    def poly(f, us, v):
        xi, eta = us / 2.0, v / vmax
        return sum(cf[f, a, b] * xi ** a * eta ** b for a in range(4) for b in range(4))

    x = np.stack([np.array([poly(f, us, v) for us in g.us for v in g.v4]) for f in range(3)])
    rows = [0, 7, 12, 24]
    got = O.F_mu(g, D, om, m, mu, x, rows=rows, nthreads=2)
    gn = 8 * np.pi ** 2 * D / om ** 4
    for r_i, e in enumerate(rows):
        ia, ib = divmod(e, g.n4)
        pv = np.array([0.0, 0.0, g.ps[ia]])
        p4t = g.p4[ib] + 1j * mu
        fp = x[:, e]
        acc = np.zeros(3, complex)
        for c in range(len(g.qs)):
            for d in range(len(g.q4)):
                fq0 = np.array([poly(f, g.uqs[c], g.vq4[d]) for f in range(3)])
                for sgn in (1, -1):
                    fq = fq0 if sgn > 0 else np.conj(fq0)
                    q4 = sgn * g.q4[d]
                    for a in range(g.na):
                        z = g.z[a]
                        qv = g.qs[c] * np.array([np.sqrt(1 - z * z), 0.0, z])
                        k2 = np.sum((pv - qv) ** 2) + (g.p4[ib] - q4) ** 2
                        w = (4 / 3) * g.wq4[d] * 2 * np.pi * g.wqs[c] * g.wz[a] / (2 * np.pi) ** 4
                        w *= gn * np.exp(-k2 / om ** 2)
                        acc += w * np.array(dirac_projections(pv, p4t, qv, q4 + 1j * mu, fp, fq))
        ref = np.array([1.0, m, 1.0]) + acc
        err = np.max(np.abs(got[:, r_i] - ref) / (1 + np.abs(ref)))
        assert err < 1e-11, (e, err)
