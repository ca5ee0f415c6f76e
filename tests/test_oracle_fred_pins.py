"""Pins of the oracle for the general system of Sec. I (eqs. jifen1, jifen3,
jifen12), against continuum solutions built independently of it:

* regular kernels, polynomial data: with cubic u*, v*, polynomial kernels and
  quadratic nonlinearities every integrand is a polynomial of degree <= 2n+1
  and the interpolation reproduces cubics, so the discrete fixed point is the
  continuum solution at the nodes to rounding; f is computed from the
  closed-form integrals (numpy polynomial arithmetic);
* the weakly singular kernel |x - t|^(-alpha): f from adaptive quadrature
  with the algebraic weight on both sides of x (scipy quad), the discrete
  solution approaching the continuum one at the rate n^(alpha - 1) of the
  quadrature of the singular factor.
"""
import numpy as np
import pytest
from numpy.polynomial import polynomial as P

from oracle import qdse_oracle_fred as OF

A, B = 0.0, 1.0
U_STAR = np.array([1.0, 0.5, -0.3, 0.2])   # u*(x) = 1 + x/2 - 0.3 x^2 + 0.2 x^3
V_STAR = np.array([0.4, -0.2, 0.1, 0.05])
F = np.array([[0.0, 0.0, 0.0, 0.3, 0.0, 0.0],    # F11 = 0.3 u^2
              [0.0, 0.0, 0.0, 0.0, 0.0, 0.0],    # F12
              [0.1, 0.2, 0.0, 0.0, 0.1, 0.0],    # F21 = 0.1 + 0.2 u + 0.1 u v
              [0.0, 0.0, 0.0, 0.0, 0.0, 0.0]])   # F22


def poly_F(c, pu, pv):
    return P.polyadd(P.polyadd(P.polyadd([c[0]], P.polymul([c[1]], pu)), P.polymul([c[2]], pv)),
                     P.polyadd(P.polyadd(P.polymul([c[3]], P.polymul(pu, pu)),
                                         P.polymul([c[4]], P.polymul(pu, pv))),
                               P.polymul([c[5]], P.polymul(pv, pv))))


def test_polynomial_problem_has_the_continuum_solution_as_discrete_fixed_point():
    # K1(x, t) = 0.5 x t + 0.2, K2(x, t) = 0.3 (x + t): f1(x) = u*(x) - int K1 F11 dt etc.
    g1 = poly_F(F[0], U_STAR, V_STAR)
    g2 = poly_F(F[2], U_STAR, V_STAR)
    I = lambda c: P.polyval(B, P.polyint(c)) - P.polyval(A, P.polyint(c))  # noqa: E731
    # int K1 g1 dt = 0.5 x int t g1 + 0.2 int g1 ; int K2 g2 dt = 0.3 x int g2 + 0.3 int t g2
    m1_t, m1_0 = I(P.polymul([0.0, 1.0], g1)), I(g1)
    m2_0, m2_t = I(g2), I(P.polymul([0.0, 1.0], g2))
    for n in (8, 23):
        x, t, w = OF.nodes(n, A, B)
        K1 = 0.5 * np.outer(x, t) + 0.2
        K2 = 0.3 * (x[:, None] + t[None, :])
        f1 = P.polyval(x, U_STAR) - (0.5 * x * m1_t + 0.2 * m1_0)
        f2 = P.polyval(x, V_STAR) - (0.3 * x * m2_0 + 0.3 * m2_t)
        f = np.concatenate([f1, f2])
        uv, it, r = OF.picard(x, t, w, K1, K2, F, f, np.ones(2 * n), 0.5, 3, 1e-15, max_iter=300)
        want = np.concatenate([P.polyval(x, U_STAR), P.polyval(x, V_STAR)])
        assert np.max(np.abs(uv - want)) < 1e-13, (n, it, np.max(np.abs(uv - want)))


def test_weakly_singular_problem_approaches_the_continuum_solution():
    from scipy.integrate import quad
    alpha = 0.5
    Fs = np.array([[0.0, 0.0, 0.0, 0.2, 0.0, 0.0],    # F11 = 0.2 u^2
                   [0.0, 0.0, 0.1, 0.0, 0.0, 0.0],    # F12 = 0.1 v
                   [0.0, 0.3, 0.0, 0.0, 0.0, 0.0],    # F21 = 0.3 u
                   [0.05, 0.0, 0.0, 0.0, 0.0, 0.05]])  # F22 = 0.05 + 0.05 v^2
    us = lambda x: 1.0 + 0.5 * np.sin(2 * x)  # noqa: E731
    vs = lambda x: np.exp(-x)  # noqa: E731
    k1 = lambda x, t: np.exp(-(x - t) ** 2)  # noqa: E731
    k2 = lambda x, t: 0.5 * np.cos(x + t)  # noqa: E731

    def sing(x, g):  # int_0^1 |x - t|^-alpha g(t) dt, algebraic weight on both sides
        left = quad(g, A, x, weight="alg", wvar=(0.0, -alpha))[0] if x > A else 0.0
        right = quad(g, x, B, weight="alg", wvar=(-alpha, 0.0))[0] if x < B else 0.0
        return left + right

    def f_at(x):
        g11 = lambda t: OF.poly(Fs[0], us(t), vs(t))  # noqa: E731
        g12 = lambda t: OF.poly(Fs[1], us(t), vs(t))  # noqa: E731
        g21 = lambda t: OF.poly(Fs[2], us(t), vs(t))  # noqa: E731
        g22 = lambda t: OF.poly(Fs[3], us(t), vs(t))  # noqa: E731
        f1 = us(x) - quad(lambda t: k1(x, t) * g11(t), A, B, epsabs=1e-13)[0] - sing(x, g12)
        f2 = vs(x) - quad(lambda t: k2(x, t) * g21(t), A, B, epsabs=1e-13)[0] - sing(x, g22)
        return f1, f2

    errs = []
    for n in (16, 64, 256):
        x, t, w = OF.nodes(n, A, B)
        K1, K2 = k1(x[:, None], t[None, :]), k2(x[:, None], t[None, :])
        ff = np.array([f_at(xi) for xi in x])
        f = np.concatenate([ff[:, 0], ff[:, 1]])
        uv, it, r = OF.picard(x, t, w, K1, K2, Fs, f, np.ones(2 * n), alpha, 3, 1e-14, max_iter=500)
        errs.append(max(np.max(np.abs(uv[:n] - us(x))), np.max(np.abs(uv[n:] - vs(x)))))
    # the product of |x - t|^-1/2 with the interlaced Gauss-Legendre rule
    # converges like n^(alpha - 1) = n^-1/2: the error halves per factor 4 in n
    for e0, e1 in zip(errs, errs[1:]):
        assert 1.6 < e0 / e1 < 2.4, errs
    assert errs[-1] < 0.02, errs
