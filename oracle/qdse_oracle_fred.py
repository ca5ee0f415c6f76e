"""Plain FP64 CPU oracle for the general system the paper starts from: two
nonlinear integral equations of the second kind with a regular and a singular
kernel (Sec. I, eqs. jifen1 and jifen3), solved by successive approximation
(Sec. I, eq. jifen12).

TEST INFRASTRUCTURE ONLY: the tests and the benchmark's checks may import this
module; the product path never does. It shares no code with the HIP library.

The system, with x in [a, b]:
    u(x) = f1(x) + int_a^b [K1(x, t) F11(u, v)(t) + Kbar(x, t) F12(u, v)(t)] dt
    v(x) = f2(x) + int_a^b [K2(x, t) F21(u, v)(t) + Kbar(x, t) F22(u, v)(t)] dt

Readings (listed in the design notes too):
* the second equation's second nonlinearity is F22 (eq. jifen1 prints F21
  twice);
* Kbar(x, t) = 1/(x - t)^alpha is taken as |x - t|^(-alpha) for
  0 < alpha < 1 (weakly singular, real for x < t) and as the Cauchy kernel
  1/(x - t) for alpha = 1;
* discretisation as the paper does for the quark equation (Sec. III): the
  unknowns live on the n-point Gauss-Legendre nodes x_i of [a, b], the
  integrals use the (n+1)-point nodes t_j with weights w_j (the two sets
  interlace, so x_i != t_j), and u(t_j), v(t_j) come from Lagrange
  interpolation on the x grid (2- or 4-point, the bracket found by search);
* the nonlinearities are quadratics F(u, v) = c0 + c1 u + c2 v + c3 u^2 +
  c4 u v + c5 v^2 (a family the caller parametrises).
"""
from __future__ import annotations

import numpy as np

from .qdse_oracle import gl_interval


def nodes(n: int, a: float, b: float):
    """External nodes x (GL(n)), integration nodes t and weights w (GL(n+1)),
    correctly rounded: x = RN(a + (b - a)(x_GL + 1)/2), w = RN((b - a)/2 w_GL)."""
    import mpmath
    a_, b_ = mpmath.mpf(a), mpmath.mpf(b)
    x, _ = gl_interval(n, a_, b_)
    t, w = gl_interval(n + 1, a_, b_)
    return x, t, np.array([float(v) for v in w])


def interp(xg: np.ndarray, f: np.ndarray, xq: float, order: int) -> float:
    """Lagrange interpolation of f (given at xg) at xq; bracket xg[b] < xq <=
    xg[b+1] found by search; order 1: the two bracketing nodes (end values
    beyond the grid), order 3: nodes b-1..b+2 shifted into the grid."""
    n = len(xg)
    b = -1
    for i in range(n):
        if xg[i] < xq:
            b = i
    if order == 1:
        if b < 0:
            return float(f[0])
        if b >= n - 1:
            return float(f[n - 1])
        lo, cnt = b, 2
    else:
        lo, cnt = min(max(b - 1, 0), n - 4), 4
    acc = 0.0
    for l in range(lo, lo + cnt):
        w = 1.0
        for k in range(lo, lo + cnt):
            if k != l:
                w *= (xq - xg[k]) / (xg[l] - xg[k])
        acc += w * f[l]
    return acc


def poly(c, u, v):
    return c[0] + c[1] * u + c[2] * v + c[3] * u * u + c[4] * u * v + c[5] * v * v


def kbar(x, t, alpha):
    d = x - t
    return 1.0 / d if alpha == 1.0 else np.abs(d) ** (-alpha)


def fred_map(x, t, w, K1, K2, F, f, uv, alpha, order):
    """One sweep of eq. jifen12 on the discrete system: uv = [u(x_i) | v(x_i)],
    K1, K2 sampled at (x_i, t_j), F = four coefficient rows (F11, F12, F21,
    F22), f = [f1(x_i) | f2(x_i)]."""
    n = len(x)
    u, v = uv[:n], uv[n:]
    uq = np.array([interp(x, u, tj, order) for tj in t])
    vq = np.array([interp(x, v, tj, order) for tj in t])
    out = np.empty(2 * n)
    g11, g12 = w * poly(F[0], uq, vq), w * poly(F[1], uq, vq)
    g21, g22 = w * poly(F[2], uq, vq), w * poly(F[3], uq, vq)
    for i in range(n):
        kb = kbar(x[i], t, alpha)
        out[i] = f[i] + np.sum(K1[i] * g11) + np.sum(kb * g12)
        out[n + i] = f[n + i] + np.sum(K2[i] * g21) + np.sum(kb * g22)
    return out


def picard(x, t, w, K1, K2, F, f, uv0, alpha, order, tol, max_iter=1000):
    """Successive approximation until max |uv' - uv| < tol. Returns (uv,
    sweeps, last change)."""
    uv = np.array(uv0, dtype=np.float64)
    r = np.inf
    for it in range(1, max_iter + 1):
        nx = fred_map(x, t, w, K1, K2, F, f, uv, alpha, order)
        r = float(np.max(np.abs(nx - uv)))
        uv = nx
        if r < tol:
            return uv, it, r
    return uv, max_iter, r
