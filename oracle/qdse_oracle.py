"""Plain FP64 CPU oracle for the vacuum quark gap equation with the Ball-Chiu
vertex (Huang, Duan, Hu, Chen, arXiv:2012.03667).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg of
the benchmark may import this module; the product path never does. It shares no
code with the HIP library.

The map itself (one successive-approximation sweep, Sec. II eqs. dsesys and
dsesys2, evaluated by direct radial x angular Gauss-Legendre sums as in Sec. III
and Table 1) lives in ``qdse_oracle.cpp``; this module builds the grids, loads
that library through ctypes and drives it:

* ``picard``: successive approximation (Sec. I eq. jifen12) with the paper's
  per-point convergence test (Sec. II eq. jifenab2) or the relative test on the
  mass function M = B/A.
* ``newton``: Newton's method on F(x) - x = 0 with Jacobian-vector products by
  the complex step, for fixed points where successive approximation is not a
  contraction; ``continuation`` walks the vertex homotopy lam from the bare
  vertex (lam = 0) to Ball-Chiu (lam = 1).

Grid (readings of Sec. II/III): u = ln p^2 on [ln s_min, ln s_max]; external
nodes are the N-point Gauss-Legendre nodes in u, loop nodes the (N+1)-point ones
on the same interval, so that the two sets interlace strictly (zeros of
consecutive Legendre polynomials interlace), which is the ordering of eq.
pqrelationship; angular nodes are M-point Gauss-Legendre nodes in z = cos(theta).
Gauss-Legendre nodes come from ``numpy.polynomial.legendre.leggauss``, polished
to correct FP64 rounding in extended precision (mpmath).
"""
from __future__ import annotations

import ctypes
import functools
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "qdse_oracle.cpp")
_SRC_MU = os.path.join(_HERE, "qdse_oracle_mu.cpp")
_LIB = os.path.join(_HERE, "libqdse_oracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (portable flags: no -march=native, no FMA
    contraction, IEEE semantics)."""
    if force or not os.path.exists(_LIB):
        cmd = ["g++", "-O2", "-std=c++17", "-fopenmp", "-fPIC", "-shared",
               "-ffp-contract=off", "-fno-fast-math", _SRC, _SRC_MU, "-o", _LIB + ".tmp"]
        subprocess.check_call(cmd)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _Grid(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("nq", ctypes.c_int), ("na", ctypes.c_int),
                ("order", ctypes.c_int)] + [
        (nm, ctypes.POINTER(ctypes.c_double))
        for nm in ("s", "u", "t", "uq", "W", "z", "wz")]


class _Par(ctypes.Structure):
    _fields_ = [("D", ctypes.c_double), ("omega", ctypes.c_double),
                ("m", ctypes.c_double), ("lam", ctypes.c_double),
                ("uv", ctypes.c_int), ("zeta", ctypes.c_double)]


class _MuGrid(ctypes.Structure):
    _fields_ = [(nm, ctypes.c_int) for nm in ("ns", "n4", "nqs", "nq4", "na", "order")] + [
        (nm, ctypes.POINTER(ctypes.c_double))
        for nm in ("ps", "us", "p4", "v4", "qs", "uqs", "wqs", "q4", "vq4", "wq4", "z", "wz")]


class _MuPar(ctypes.Structure):
    _fields_ = [(nm, ctypes.c_double) for nm in ("D", "omega", "m", "mu")]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < max(
                os.path.getmtime(_SRC), os.path.getmtime(_SRC_MU)):
            build()
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        gp, pp = ctypes.POINTER(_Grid), ctypes.POINTER(_Par)
        L.qo_vac_map.argtypes = [gp, pp, dp, dp, ctypes.c_int]
        L.qo_vac_map_rows.argtypes = [gp, pp, dp, ip, ctypes.c_int, dp, ctypes.c_int]
        L.qo_vac_map_paper.argtypes = [gp, pp, dp, dp, ctypes.c_int, ctypes.c_int]
        L.qo_vac_jvp.argtypes = [gp, pp, dp, dp, dp, ctypes.c_int]
        L.qo_vac_map_c.argtypes = [gp, pp, dp, dp, dp, dp, ctypes.c_int]
        L.qo_interp.argtypes = [ctypes.c_int, dp, dp, ctypes.c_int, dp, ctypes.c_int, dp, ip]
        L.qo_integrand.argtypes = [ctypes.c_double] * 8 + [dp, dp]
        L.qo_integrand.restype = None
        L.qo_g_uv.argtypes = [ctypes.c_double]
        L.qo_g_uv.restype = ctypes.c_double
        L.qo_mu_map.argtypes = [ctypes.POINTER(_MuGrid), ctypes.POINTER(_MuPar), dp, dp, ip,
                                ctypes.c_int, dp, dp, ctypes.c_int]
        L.qo_mu_projections.argtypes = [ctypes.c_double] * 6 + [dp, dp, dp]
        L.qo_mu_projections.restype = None
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


@dataclass
class VacGrid:
    """Discretisation of the vacuum problem (all float64 numpy arrays)."""
    n: int
    na: int
    order: int
    s: np.ndarray
    u: np.ndarray
    t: np.ndarray
    uq: np.ndarray
    W: np.ndarray
    z: np.ndarray
    wz: np.ndarray

    @property
    def nq(self):
        return len(self.t)

    def _c(self):
        g = _Grid(self.n, self.nq, self.na, self.order,
                  *[_dp(a) for a in (self.s, self.u, self.t, self.uq, self.W, self.z, self.wz)])
        g._keep = self  # keep arrays alive
        return g


EXACT_NODES_MAX = 1100


@functools.lru_cache(maxsize=None)
def gauss_legendre(n: int):
    """n-point Gauss-Legendre nodes (ascending) and weights on [-1, 1],
    correctly rounded to FP64: numpy's nodes (accurate to ~2 ulp) polished by
    Newton's method on the Legendre three-term recurrence in 34-digit mpmath
    arithmetic. Above EXACT_NODES_MAX points numpy's nodes are used as they are.
    Correct rounding matters because the discrete map at large p^2 is
    sensitive to single-ulp moves of the angular nodes (exp(-k^2/omega^2) with
    k^2 ~ 2|p||q|(1 - z))."""
    x0, w0 = np.polynomial.legendre.leggauss(n)
    if n > EXACT_NODES_MAX or n < 2:
        return x0, w0
    import mpmath
    ctx = mpmath.mp.clone() if hasattr(mpmath.mp, "clone") else mpmath.mp
    ctx.dps = 34

    def legendre_and_derivative(r):
        p0, p1 = ctx.mpf(1), r
        for ell in range(2, n + 1):
            p0, p1 = p1, ((2 * ell - 1) * r * p1 - (ell - 1) * p0) / ell
        return p1, n * (r * p1 - p0) / (r * r - 1)

    x, w = np.empty(n), np.empty(n)
    for k in range(n // 2):  # negative roots; the rule is symmetric
        r = ctx.mpf(float(x0[k]))
        for _ in range(2):
            p, dp = legendre_and_derivative(r)
            r = r - p / dp
        p, dp = legendre_and_derivative(r)
        x[k], x[n - 1 - k] = float(r), -float(r)
        w[k] = w[n - 1 - k] = float(2 / ((1 - r * r) * dp * dp))
    if n % 2:
        _, dp = legendre_and_derivative(ctx.mpf(0))
        x[n // 2] = 0.0
        w[n // 2] = float(2 / (dp * dp))
    return x, w


def _mp():
    """A private 60-digit mpmath context: every grid quantity is an exact
    expression of FP64 inputs, evaluated here and rounded once to FP64."""
    import mpmath
    ctx = mpmath.mp.clone() if hasattr(mpmath.mp, "clone") else mpmath.mp
    ctx.dps = 60
    return ctx


def gl_interval(n: int, a, b, mp=None):
    """n-point Gauss-Legendre rule mapped to [a, b] (a, b exact mpmath numbers):
    nodes RN(a + (b - a)(x + 1)/2) for the FP64 nodes x, and the exact factors
    (b - a)/2 * w of the weights (mpmath numbers, rounded by the caller)."""
    mp = mp or _mp()
    a, b = mp.mpf(a), mp.mpf(b)
    x, w = gauss_legendre(n)
    half = (b - a) / 2
    return (np.array([float(a + (b - a) * (mp.mpf(float(v)) + 1) / 2) for v in x]),
            [half * mp.mpf(float(v)) for v in w])


def vac_grid(n: int, na: int, s_min: float = 1e-4, s_max: float = 1e4,
             order: int = 3, nq: int | None = None) -> VacGrid:
    """External grid GL(n) in u = ln s, loop grid GL(n+1) in u on the same
    interval (interleaved), angular grid GL(na) in z. The grid is defined by
    correctly rounded values (reading of Sec. III A): with a = ln s_min,
    b = ln s_max exact and x, w the correctly rounded Gauss-Legendre rule,
    u = RN(a + (b - a)(x + 1)/2), s = RN(e^u), and the loop weight of the
    measure t dt = t^2 du is W = RN((b - a)/2 w t^2)."""
    mp = _mp()
    a, b = mp.log(mp.mpf(s_min)), mp.log(mp.mpf(s_max))
    u, _ = gl_interval(n, a, b, mp)
    uq, wq = gl_interval(n + 1 if nq is None else nq, a, b, mp)
    z, wz = gauss_legendre(na)
    s = np.array([float(mp.exp(mp.mpf(float(v)))) for v in u])
    t = np.array([float(mp.exp(mp.mpf(float(v)))) for v in uq])
    W = np.array([float(h * mp.mpf(float(tj)) ** 2) for h, tj in zip(wq, t)])
    return VacGrid(n, na, order, s, u, t, uq, W, z.copy(), wz.copy())


@dataclass
class Params:
    """D (GeV^2), omega (GeV), current mass m (GeV), vertex homotopy lam.
    uv = 1 adds the ultraviolet term of the Qin-Chang interaction; zeta > 0
    (GeV) renormalises at p^2 = zeta^2 with A(zeta^2) = 1, B(zeta^2) = m
    (Z_1 = Z_2; see qdse_oracle.cpp). The defaults are the paper's setting."""
    D: float
    omega: float
    m: float
    lam: float = 1.0
    uv: int = 0
    zeta: float = 0.0

    def _c(self):
        return _Par(self.D, self.omega, self.m, self.lam, int(self.uv), float(self.zeta))

    @staticmethod
    def from_kappa(kappa: float, omega: float, m: float, lam: float = 1.0):
        """D from the product D * omega = kappa^3."""
        return Params(kappa ** 3 / omega, omega, m, lam)


def g_uv(k2: float) -> float:
    """Ultraviolet term of the Qin-Chang interaction, g_UV(k^2) (GeV^-2)."""
    return lib().qo_g_uv(float(k2))


def _threads(nthreads):
    return int(nthreads) if nthreads else int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))


def F(g: VacGrid, p: Params, x: np.ndarray, nthreads: int | None = None) -> np.ndarray:
    """One sweep x' = F(x) of the successive approximation, x = [A | B]."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    assert x.shape == (2 * g.n,)
    out = np.empty_like(x)
    gc, pc = g._c(), p._c()
    rc = lib().qo_vac_map(ctypes.byref(gc), ctypes.byref(pc), _dp(x), _dp(out), _threads(nthreads))
    if rc:
        raise ValueError("oracle: bad grid")
    return out


def F_paper(g: VacGrid, p: Params, x: np.ndarray, modified: bool, nthreads: int = 1) -> np.ndarray:
    """One sweep organised as the paper's code (Sec. III): functionA and
    functionB per external momentum, interpolation inside the loops, with the
    traditional bracket search (modified = False) or the bracket from eq.
    pqrelationship (modified = True); nthreads = 1 is sequential, more runs
    OpenMP over external momenta. Table 1's algorithms 1-4 are (False, 1), (True, 1), (False, P),
    (True, P). Same values as F."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    assert x.shape == (2 * g.n,)
    out = np.empty_like(x)
    gc, pc = g._c(), p._c()
    rc = lib().qo_vac_map_paper(ctypes.byref(gc), ctypes.byref(pc), _dp(x), _dp(out),
                                int(bool(modified)), int(nthreads))
    if rc:
        raise ValueError("oracle: bad grid")
    return out


def picard_paper(g: VacGrid, p: Params, x0: np.ndarray, tol: float, modified: bool,
                 nthreads: int = 1, max_iter: int = 1000):
    """Successive approximation with F_paper and the paper's absolute per-point
    test on A and B (Sec. II eq. jifenab2). Returns (x, iterations)."""
    x = np.array(x0, dtype=np.float64)
    for it in range(1, max_iter + 1):
        xn = F_paper(g, p, x, modified, nthreads)
        ok, _ = converged(x, xn, g.n, tol, 0)
        x = xn
        if ok:
            return x, it
    return x, max_iter


def F_rows(g: VacGrid, p: Params, x: np.ndarray, rows, nthreads: int | None = None):
    """A'(rows), B'(rows) of one sweep, computed for the listed rows only."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    rows = np.ascontiguousarray(rows, dtype=np.int32)
    out = np.empty(2 * len(rows))
    gc, pc = g._c(), p._c()
    rc = lib().qo_vac_map_rows(ctypes.byref(gc), ctypes.byref(pc), _dp(x), _ip(rows),
                               len(rows), _dp(out), _threads(nthreads))
    if rc:
        raise ValueError("oracle: bad grid or row index")
    return out[:len(rows)], out[len(rows):]


def F_complex(g: VacGrid, p: Params, x: np.ndarray, nthreads=None) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.complex128)
    xr, xi = np.ascontiguousarray(x.real), np.ascontiguousarray(x.imag)
    orr, oi = np.empty_like(xr), np.empty_like(xr)
    gc, pc = g._c(), p._c()
    rc = lib().qo_vac_map_c(ctypes.byref(gc), ctypes.byref(pc), _dp(xr), _dp(xi), _dp(orr),
                            _dp(oi), _threads(nthreads))
    if rc:
        raise ValueError("oracle: bad grid")
    return orr + 1j * oi


def jvp(g: VacGrid, p: Params, x: np.ndarray, v: np.ndarray, nthreads=None) -> np.ndarray:
    """(dF/dx) v by the complex step."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    v = np.ascontiguousarray(v, dtype=np.float64)
    out = np.empty_like(x)
    gc, pc = g._c(), p._c()
    rc = lib().qo_vac_jvp(ctypes.byref(gc), ctypes.byref(pc), _dp(x), _dp(v), _dp(out),
                          _threads(nthreads))
    if rc:
        raise ValueError("oracle: bad grid")
    return out


def jacobian(g: VacGrid, p: Params, x: np.ndarray, nthreads=None) -> np.ndarray:
    """Dense dF/dx, one complex-step column at a time (small grids only)."""
    n2 = 2 * g.n
    J = np.empty((n2, n2))
    e = np.zeros(n2)
    for k in range(n2):
        e[:] = 0.0
        e[k] = 1.0
        J[:, k] = jvp(g, p, x, e, nthreads)
    return J


def interp(u: np.ndarray, f: np.ndarray, x: np.ndarray, order: int):
    """Interpolated values at x and the searched bracket of each point."""
    u = np.ascontiguousarray(u, dtype=np.float64)
    f = np.ascontiguousarray(f, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64)
    fx = np.empty_like(x)
    br = np.empty(len(x), dtype=np.int32)
    rc = lib().qo_interp(len(u), _dp(u), _dp(f), len(x), _dp(x), order, _dp(fx), _ip(br))
    if rc:
        raise ValueError("oracle: bad interpolation request")
    return fx, br


def integrand(s, t, z, Ap, Bp, Aq, Bq, lam=1.0):
    """(I_A, I_B) of eq. dsesys2 at one point (I_A includes its 1/p^2)."""
    ia, ib = ctypes.c_double(), ctypes.c_double()
    lib().qo_integrand(s, t, z, Ap, Bp, Aq, Bq, lam, ctypes.byref(ia), ctypes.byref(ib))
    return ia.value, ib.value


# --------------------------------------------------------------------------
# Drivers
# --------------------------------------------------------------------------

M_FLOOR = 1e-8  # GeV


def converged(x_old, x_new, n, tol, mode):
    """Convergence test. mode 0: the paper's per-point absolute test on A and B
    (Sec. II eq. jifenab2). mode 1: max |dM|/max(|M|, M_FLOOR) < tol and
    max |dA| < tol, M = B/A; the floor (1e-8 GeV) keeps the test finite where
    the chiral-limit mass function vanishes."""
    Ao, Bo, An, Bn = x_old[:n], x_old[n:], x_new[:n], x_new[n:]
    if mode == 0:
        r = max(np.max(np.abs(An - Ao)), np.max(np.abs(Bn - Bo)))
    else:
        Mo, Mn = Bo / Ao, Bn / An
        r = max(np.max(np.abs(Mn - Mo) / np.maximum(np.abs(Mn), M_FLOOR)),
                np.max(np.abs(An - Ao)))
    return r < tol, r


def picard(g, p, x0, tol, max_iter=1000, mode=0, nthreads=None, history=False):
    """Successive approximation x_{n+1} = F(x_n) (Sec. I eq. jifen12) until the
    convergence test holds. Returns (x, iterations, last residual, hist)."""
    x = np.array(x0, dtype=np.float64)
    hist = []
    r = np.inf
    for it in range(1, max_iter + 1):
        xn = F(g, p, x, nthreads)
        ok, r = converged(x, xn, g.n, tol, mode)
        if history:
            hist.append(xn.copy())
        x = xn
        if not np.all(np.isfinite(x)):
            return x, it, np.nan, hist
        if ok:
            return x, it, r, hist
    return x, max_iter, r, hist


def residual(g, p, x, nthreads=None):
    return F(g, p, x, nthreads) - x


def newton(g, p, x0, tol=1e-13, max_newton=40, dense_max=130, nthreads=None,
           gmres_tol=1e-12):
    """Newton's method on R(x) = F(x) - x: (I - J) dx = R, J = dF/dx. Dense
    solve for small grids, GMRES (scipy) on complex-step products otherwise.
    Returns (x, newton steps, max|R|)."""
    x = np.array(x0, dtype=np.float64)
    n2 = 2 * g.n
    for it in range(max_newton):
        R = residual(g, p, x, nthreads)
        rn = np.max(np.abs(R))
        if not np.isfinite(rn):
            return x, it, np.inf
        if rn < tol:
            return x, it, rn
        if g.n <= dense_max:
            J = jacobian(g, p, x, nthreads)
            dx = np.linalg.solve(np.eye(n2) - J, R)
        else:
            from scipy.sparse.linalg import LinearOperator, gmres
            op = LinearOperator((n2, n2), matvec=lambda v: v - jvp(g, p, x, v, nthreads))
            dx, info = gmres(op, R, rtol=gmres_tol, atol=0.0, restart=200, maxiter=20)
        x = x + dx
    R = residual(g, p, x, nthreads)
    return x, max_newton, np.max(np.abs(R))


def continuation(g, p, x0, steps=10, tol=1e-13, nthreads=None):
    """Walk the vertex homotopy lam = 0 -> p.lam (bare -> Ball-Chiu): solve at
    lam = 0 by Newton from x0, then Newton from the previous solution at each
    of `steps` equally spaced lam values. Returns (x, max|R| at the end)."""
    x = np.array(x0, dtype=np.float64)
    rn = np.inf
    for k in range(steps + 1):
        pk = Params(p.D, p.omega, p.m, p.lam * k / steps)
        x, _, rn = newton(g, pk, x, tol=tol, nthreads=nthreads)
    return x, rn


def certificate(g, p, x, nthreads=None):
    """Physical-branch checks of a fixed point (the reading of a certified
    solution of the unrenormalised equation): residual max|F(x) - x|; A > 0
    at every node; A >= 1 (A = 1 + Sigma_A; up to 1e-9); the mass function
    M = B/A falling with p^2 for m >= 0 (a rise counts if it exceeds 1e-6
    max|M| where |M| exceeds 1e-3 max|M|: the chiral-limit tail of B changes
    sign at the 1e-6 level); and, for information, the number of
    node-to-node sign changes of the slope of M.
    certified = A_pos and A_ge_1 and M_falls."""
    n = g.n
    A, B = x[:n], x[n:]
    M = B / A
    R = residual(g, p, x, nthreads)
    dM = np.diff(M)
    flips = int(np.sum(dM[1:] * dM[:-1] < 0))
    a_pos = bool(np.all(A > 0))
    a_ge_1 = bool(np.all(A >= 1 - 1e-9))
    big = np.maximum(np.abs(M[:-1]), np.abs(M[1:])) > 1e-3 * np.max(np.abs(M))
    m_falls = not bool(np.any((dM > 1e-6 * np.max(np.abs(M))) & big))
    return {"resid": float(np.max(np.abs(R))), "A_pos": a_pos, "A_ge_1": a_ge_1,
            "M_falls": m_falls, "slope_flips": flips,
            "certified": a_pos and a_ge_1 and m_falls}


def spectral_radius(g, p, x, nthreads=None):
    """Largest |eigenvalue| of dF/dx at x (dense; small grids), and the
    eigenvalues themselves."""
    ev = np.linalg.eigvals(jacobian(g, p, x, nthreads))
    return float(np.max(np.abs(ev))), ev


# --------------------------------------------------------------------------
# Finite chemical potential (qdse_oracle_mu.cpp)
# --------------------------------------------------------------------------

@dataclass
class MuGrid:
    """External (|p_vec|, p4 > 0) grid, loop (|q_vec|, |q4|) grid (one more node
    per direction on the same log intervals, interleaved), angular grid in
    cos(theta) with flat weight."""
    ns: int
    n4: int
    na: int
    order: int
    ps: np.ndarray
    us: np.ndarray
    p4: np.ndarray
    v4: np.ndarray
    qs: np.ndarray
    uqs: np.ndarray
    wqs: np.ndarray
    q4: np.ndarray
    vq4: np.ndarray
    wq4: np.ndarray
    z: np.ndarray
    wz: np.ndarray

    @property
    def ne(self):
        return self.ns * self.n4

    def _c(self):
        arrs = [self.ps, self.us, self.p4, self.v4, self.qs, self.uqs, self.wqs, self.q4,
                self.vq4, self.wq4, self.z, self.wz]
        g = _MuGrid(self.ns, self.n4, len(self.qs), len(self.q4), self.na, self.order,
                    *[_dp(a) for a in arrs])
        g._keep = self
        return g


def mu_grid(ns: int, n4: int, na: int, r_min=1e-2, r_max=1e2, p4_max=1e2, lam4=0.5,
            order: int = 3, T: float = 0.0) -> MuGrid:
    """|p_vec| on GL(ns) in ln|p| over [r_min, r_max]; p4 = lam4 sinh(v) with v on
    GL(n4) over [0, asinh(p4_max/lam4)]; loop grids GL(ns+1), GL(n4+1) on the same
    intervals; angle GL(na) in cos(theta) with flat weight. Loop weights carry
    the measure: |q|^2 d|q| = |q|^3 dln|q| and dq4 = lam4 cosh(v) dv.
    T > 0 (finite temperature, the paper's named extension): p4 runs over the
    fermion Matsubara frequencies w_n = (2n+1) pi T, n < n4, the loop over the
    same frequencies (both signs by conjugation) with weight 2 pi T, since
    int dq4/(2 pi) f becomes T sum_n f(w_n); the time grid variable is w_n
    itself, so interpolation in the time direction is at the nodes."""
    mp = _mp()
    a, b = mp.log(mp.mpf(r_min)), mp.log(mp.mpf(r_max))
    us, _ = gl_interval(ns, a, b, mp)
    uqs, wu = gl_interval(ns + 1, a, b, mp)
    z, wz = gauss_legendre(na)
    ps = np.array([float(mp.exp(mp.mpf(float(t)))) for t in us])
    qs = np.array([float(mp.exp(mp.mpf(float(t)))) for t in uqs])
    wqs = np.array([float(w * mp.mpf(float(q)) ** 3) for w, q in zip(wu, qs)])
    if T > 0:
        p4 = np.array([float((2 * n + 1) * mp.pi * mp.mpf(T)) for n in range(n4)])
        v4 = p4.copy()
        q4, vq4 = p4.copy(), p4.copy()
        wq4 = np.full(n4, float(2 * mp.pi * mp.mpf(T)))
    else:
        vmax = mp.asinh(mp.mpf(p4_max) / mp.mpf(lam4))
        v4, _ = gl_interval(n4, mp.mpf(0), vmax, mp)
        vq4, wv = gl_interval(n4 + 1, mp.mpf(0), vmax, mp)
        p4 = np.array([float(mp.mpf(lam4) * mp.sinh(mp.mpf(float(t)))) for t in v4])
        q4 = np.array([float(mp.mpf(lam4) * mp.sinh(mp.mpf(float(t)))) for t in vq4])
        wq4 = np.array([float(w * mp.mpf(lam4) * mp.cosh(mp.mpf(float(t)))) for w, t in zip(wv, vq4)])
    return MuGrid(ns, n4, na, order, ps, us, p4, np.asarray(v4), qs, uqs, wqs, q4,
                  np.asarray(vq4), wq4, z.copy(), wz.copy())


def F_mu(g: MuGrid, D, omega, m, mu, x: np.ndarray, rows=None, nthreads=None):
    """One finite-mu sweep. x: complex [3][ns*n4] (A, B, C), |p_vec|-major.
    Returns complex [3][ne] (or [3][len(rows)])."""
    x = np.ascontiguousarray(x, dtype=np.complex128).reshape(3, g.ne)
    xr, xi = np.ascontiguousarray(x.real), np.ascontiguousarray(x.imag)
    if rows is None:
        rp, cnt = None, g.ne
    else:
        rows = np.ascontiguousarray(rows, dtype=np.int32)
        rp, cnt = _ip(rows), len(rows)
    orr, oi = np.empty(3 * cnt), np.empty(3 * cnt)
    gc = g._c()
    pc = _MuPar(D, omega, m, mu)
    rc = lib().qo_mu_map(ctypes.byref(gc), ctypes.byref(pc), _dp(xr), _dp(xi), rp,
                         0 if rows is None else cnt, _dp(orr), _dp(oi), _threads(nthreads))
    if rc:
        raise ValueError("oracle: bad finite-mu grid")
    return (orr + 1j * oi).reshape(3, cnt)


def mu_projections(pabs, p4, qabs, q4, z, mu, fp, fq):
    """(A, B, C) projections of T gamma S(q~) Gamma(q~, p~) at one point, without
    g(k^2); fp, fq: complex (A, B, C) at p~ and q~."""
    a = np.empty(6)
    fpa = np.array([v for c in fp for v in (c.real, c.imag)])
    fqa = np.array([v for c in fq for v in (c.real, c.imag)])
    lib().qo_mu_projections(pabs, p4, qabs, q4, z, mu, _dp(fpa), _dp(fqa), _dp(a))
    return complex(a[0], a[1]), complex(a[2], a[3]), complex(a[4], a[5])
