"""ctypes binding of libqdse.so: argument marshalling only (see include/qdse.h)."""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIBPATH = os.path.join(_HERE, "libqdse.so")

QDSE_OK, QDSE_NOT_CONVERGED = 0, 1
QDSE_EINVAL, QDSE_ENOMEM, QDSE_EDEVICE, QDSE_ENAN, QDSE_ENOTSUP = -1, -2, -3, -4, -5
QDSE_EDIVERGED, QDSE_ESPURIOUS = -6, -7
QDSE_PICARD, QDSE_NEWTON, QDSE_AUTO = 0, 1, 2
QDSE_FP64, QDSE_FP32_REFINE, QDSE_FP64_MATRIX = 0, 1, 2
QDSE_CONV_ABS, QDSE_CONV_MASS = 0, 1


class QdseError(RuntimeError):
    def __init__(self, code, what):
        self.code = code
        super().__init__(f"{what}: {code} ({_strerror(code)}) {_last_error()}")


class Grid(ctypes.Structure):
    _fields_ = [("n_radial", ctypes.c_int), ("n_angle", ctypes.c_int),
                ("interp_order", ctypes.c_int), ("s_min", ctypes.c_double),
                ("s_max", ctypes.c_double)]


class Params(ctypes.Structure):
    _fields_ = [("D", ctypes.c_double), ("omega", ctypes.c_double), ("m", ctypes.c_double)]


class MuGrid(ctypes.Structure):
    _fields_ = [("n_space", ctypes.c_int), ("n_time", ctypes.c_int), ("n_angle", ctypes.c_int),
                ("interp_order", ctypes.c_int), ("r_min", ctypes.c_double),
                ("r_max", ctypes.c_double), ("p4_max", ctypes.c_double),
                ("lam4", ctypes.c_double), ("T", ctypes.c_double)]


class Qc(ctypes.Structure):
    _fields_ = [("uv", ctypes.c_int), ("zeta", ctypes.c_double)]


class FredGrid(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("interp_order", ctypes.c_int), ("a", ctypes.c_double),
                ("b", ctypes.c_double), ("alpha", ctypes.c_double)]


class FredPoly(ctypes.Structure):
    _fields_ = [("c", ctypes.c_double * 6)]


class MuParams(ctypes.Structure):
    _fields_ = [("D", ctypes.c_double), ("omega", ctypes.c_double), ("m", ctypes.c_double),
                ("mu", ctypes.c_double)]


_lib = None
_vp, _dp, _ip = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int)


def library_path() -> str:
    return _LIBPATH


def load():
    """Loads libqdse.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIBPATH):
        raise RuntimeError(f"{_LIBPATH} is missing: build it with paper_2012_03667_amd/build.py")
    L = ctypes.CDLL(_LIBPATH)
    L.qdse_setup.argtypes = [ctypes.POINTER(Grid), ctypes.POINTER(Params), ctypes.c_int,
                             ctypes.c_int, ctypes.c_int, _vp, ctypes.POINTER(_vp)]
    L.qdse_setup_qc.argtypes = [ctypes.POINTER(Grid), ctypes.POINTER(Params), ctypes.c_int,
                                ctypes.POINTER(Qc), _vp, ctypes.POINTER(_vp)]
    L.qdse_destroy.argtypes = [_vp]
    L.qdse_destroy.restype = None
    L.qdse_dims.argtypes = [_vp, _ip, _ip, _ip, _ip]
    L.qdse_nodes.argtypes = [_vp, _dp, _dp]
    L.qdse_grid_nodes.argtypes = [ctypes.POINTER(Grid)] + [_dp] * 6
    L.qdse_iterate.argtypes = [_vp, _vp, _vp, _vp]
    L.qdse_iterate_fp32.argtypes = [_vp, _vp, _vp]
    L.qdse_iterate_fp64_matrix.argtypes = [_vp, _vp, _vp]
    L.qdse_solve.argtypes = [_vp, _vp, ctypes.c_double, ctypes.c_int, ctypes.c_int, _ip, _dp]
    L.qdse_solve_group.argtypes = [ctypes.POINTER(_vp), ctypes.c_int, ctypes.POINTER(_vp),
                                   ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                   ctypes.POINTER(_ip), ctypes.POINTER(_dp)]
    L.qdse_solve_stats.argtypes = [_vp, _ip, _ip]
    L.qdse_solve_kernel_us.argtypes = [_vp, _dp]
    L.qdse_solve_status.argtypes = [_vp, _ip]
    L.qdse_newton.argtypes = [_vp, _vp, ctypes.c_double, ctypes.c_int, ctypes.c_double, _ip, _dp]
    L.qdse_jvp.argtypes = [_vp, _vp, _vp, _vp]
    L.qdse_vjp.argtypes = [_vp, _vp, _vp, _vp]
    L.qdse_vjp_noalloc.argtypes = [_vp, _vp, _vp, _vp]
    L.qdse_jacobian_band.argtypes = [_vp, _vp, ctypes.c_int, _vp]
    L.qdse_grad.argtypes = [_vp, _vp, _vp, ctypes.c_double, ctypes.c_int, _dp]
    L.qdse_kernel_matrices.argtypes = [_vp, ctypes.c_int, _vp]
    L.qdse_time_contraction.argtypes = [_vp, ctypes.c_int, _vp, _vp, ctypes.c_int, _dp]
    L.qdse_mu_setup.argtypes = [ctypes.POINTER(MuGrid), ctypes.POINTER(MuParams), ctypes.c_int,
                                _vp, ctypes.POINTER(_vp)]
    L.qdse_mu_destroy.argtypes = [_vp]
    L.qdse_mu_destroy.restype = None
    L.qdse_mu_grid_nodes.argtypes = [ctypes.POINTER(MuGrid)] + [_dp] * 8
    L.qdse_mu_iterate.argtypes = [_vp, _vp, _vp]
    L.qdse_mu_solve.argtypes = [_vp, _vp, ctypes.c_double, ctypes.c_int, _ip, _dp]
    L.qdse_mu_solve_anderson.argtypes = [_vp, _vp, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                         _ip, _dp]
    L.qdse_mu_solve_group.argtypes = [ctypes.POINTER(_vp), ctypes.c_int, ctypes.POINTER(_vp),
                                      ctypes.c_double, ctypes.c_int, ctypes.POINTER(_ip),
                                      ctypes.POINTER(_dp)]
    L.qdse_measure_peaks.argtypes = [_vp, _dp, _dp, _dp, _dp]
    L.qdse_measure_launch_floor.argtypes = [_vp, ctypes.c_int, ctypes.c_longlong, _dp, _dp]
    L.qdse_autotune.argtypes = [_vp, ctypes.c_int, ctypes.c_char_p, _ip, _ip, _ip]
    L.qdse_fred_nodes.argtypes = [ctypes.POINTER(FredGrid), _dp, _dp, _dp]
    L.qdse_fred_setup.argtypes = [ctypes.POINTER(FredGrid), ctypes.POINTER(FredPoly), _vp, _vp,
                                  _vp, _vp, ctypes.POINTER(_vp)]
    L.qdse_fred_destroy.argtypes = [_vp]
    L.qdse_fred_destroy.restype = None
    L.qdse_fred_iterate.argtypes = [_vp, _vp, _vp]
    L.qdse_fred_solve.argtypes = [_vp, _vp, ctypes.c_double, ctypes.c_int, _ip, _dp]
    L.qdse_fred_time_sweep.argtypes = [_vp, _vp, _vp, ctypes.c_int, _dp]
    L.qdse_strerror.argtypes = [ctypes.c_int]
    L.qdse_strerror.restype = ctypes.c_char_p
    L.qdse_last_error.argtypes = []
    L.qdse_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def _strerror(code):
    try:
        return load().qdse_strerror(code).decode()
    except Exception:
        return "?"


def _last_error():
    try:
        return load().qdse_last_error().decode()
    except Exception:
        return ""


# outcomes of a solve that leave the iterate in the caller's array
_OUTCOMES = (QDSE_OK, QDSE_NOT_CONVERGED, QDSE_ENAN, QDSE_EDIVERGED, QDSE_ESPURIOUS)


def _check(code, what, allow=(QDSE_OK,)):
    if code not in allow:
        raise QdseError(code, what)
    return code


def _dev(t, shape, name):
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64
            and t.is_contiguous() and tuple(t.shape) == tuple(shape)):
        raise ValueError(f"{name} must be a contiguous float64 CUDA tensor of shape {shape}")
    return ctypes.c_void_p(t.data_ptr())


def grid_nodes(n_radial, n_angle, interp_order=3, s_min=1e-4, s_max=1e4):
    """Host-only: the grid arrays (s, u, t, W, z, wz) a context would use."""
    g = Grid(int(n_radial), int(n_angle), int(interp_order), float(s_min), float(s_max))
    out = [np.empty(n) for n in (n_radial, n_radial, n_radial + 1, n_radial + 1, n_angle,
                                 n_angle)]
    _check(load().qdse_grid_nodes(ctypes.byref(g), *[a.ctypes.data_as(_dp) for a in out]),
           "qdse_grid_nodes")
    return dict(zip(("s", "u", "t", "W", "z", "wz"), out))


class Solver:
    """One context of include/qdse.h: n_inst instances sharing one grid.

    params: sequence of (D [GeV^2], omega [GeV], m [GeV]) per instance.
    Unknowns per instance: x = [A(s_0..s_{N-1}) | B(s_0..s_{N-1})].
    zeta (GeV): the renormalised Qin-Chang setting of qdse_setup_qc
    (renormalisation at p^2 = zeta^2, m = current mass there; uv = 1 adds the
    ultraviolet term of the interaction); None: the paper's setting.
    """

    def __init__(self, n_radial, n_angle, params, interp_order=3, s_min=1e-4, s_max=1e4,
                 precision=QDSE_FP64, stream=None, zeta=None, uv=1, solver=QDSE_PICARD):
        import torch
        L = load()
        self.n, self.na, self.order = int(n_radial), int(n_angle), int(interp_order)
        self.params = [tuple(map(float, p)) for p in params]
        self.n_inst = len(self.params)
        self.device = torch.device("cuda", torch.cuda.current_device())
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        g = Grid(self.n, self.na, self.order, float(s_min), float(s_max))
        P = (Params * max(1, self.n_inst))(*[Params(*p) for p in self.params])
        h = _vp()
        if zeta is None:
            _check(L.qdse_setup(ctypes.byref(g), P, self.n_inst, int(precision), int(solver),
                                _vp(self.stream.cuda_stream), ctypes.byref(h)), "qdse_setup")
        else:
            q = Qc(int(uv), float(zeta))
            _check(L.qdse_setup_qc(ctypes.byref(g), P, self.n_inst, ctypes.byref(q),
                                   _vp(self.stream.cuda_stream), ctypes.byref(h)),
                   "qdse_setup_qc")
        self._h = h
        self.s = np.empty(self.n)
        self.t = np.empty(self.n + 1)
        _check(L.qdse_nodes(h, self.s.ctypes.data_as(_dp), self.t.ctypes.data_as(_dp)),
               "qdse_nodes")

    def close(self):
        if getattr(self, "_h", None):
            load().qdse_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def shape(self):
        return (self.n_inst, 2 * self.n)

    def initial(self, A0=1.0, B0=1.0):
        import torch
        x = torch.empty(self.shape, dtype=torch.float64, device=self.device)
        x[:, :self.n] = A0
        x[:, self.n:] = B0
        return x

    def iterate(self, x, out=None, fp32=False, matrix=False, resid=None):
        """One sweep: FP64 direct (default), FP32 MFMA (fp32=True) or FP64 MFMA
        split form (matrix=True). resid (FP64 direct only): a float64 CUDA
        tensor [n_inst] that receives the sweep's test statistic."""
        import torch
        if out is None:
            out = torch.empty_like(x)
        if fp32 or matrix:
            if resid is not None:
                raise ValueError("resid is returned by the FP64 direct sweep only")
            fn = load().qdse_iterate_fp32 if fp32 else load().qdse_iterate_fp64_matrix
            _check(fn(self._h, _dev(x, self.shape, "x"), _dev(out, self.shape, "out")),
                   "qdse_iterate")
            return out
        r = None if resid is None else _dev(resid, (self.n_inst,), "resid")
        _check(load().qdse_iterate(self._h, _dev(x, self.shape, "x"), _dev(out, self.shape, "out"),
                                   r), "qdse_iterate")
        return out

    def solve(self, x, tol=1e-10, max_iter=1000, conv_mode=QDSE_CONV_MASS):
        """In place. Returns (status, iters[n_inst], resid[n_inst]); iters
        counts evaluations (sweeps, and Newton's sweeps and Jacobian-vector
        products); solve_status() gives each instance's outcome."""
        it = np.zeros(self.n_inst, dtype=np.int32)
        rs = np.zeros(self.n_inst)
        rc = load().qdse_solve(self._h, _dev(x, self.shape, "x"), float(tol), int(max_iter),
                               int(conv_mode), it.ctypes.data_as(_ip), rs.ctypes.data_as(_dp))
        _check(rc, "qdse_solve", allow=_OUTCOMES)
        return rc, it, rs

    def solve_kernel_us(self):
        """Duration (us) of the last solve's single-launch kernel, or None if
        the last solve used the kernel-per-sweep driver."""
        v = ctypes.c_double(0.0)
        rc = load().qdse_solve_kernel_us(self._h, ctypes.byref(v))
        if rc == QDSE_ENOTSUP:
            return None
        _check(rc, "qdse_solve_kernel_us")
        return v.value

    def solve_status(self):
        """Per-instance outcome codes of the last solve."""
        st = np.zeros(self.n_inst, dtype=np.int32)
        _check(load().qdse_solve_status(self._h, st.ctypes.data_as(_ip)), "qdse_solve_status")
        return st

    def newton(self, x, tol=1e-12, max_newton=30, lin_tol=1e-10):
        """In place Newton-Krylov. Returns (status, steps[n_inst], max|F(x)-x|[n_inst])."""
        it = np.zeros(self.n_inst, dtype=np.int32)
        rs = np.zeros(self.n_inst)
        rc = load().qdse_newton(self._h, _dev(x, self.shape, "x"), float(tol), int(max_newton),
                                float(lin_tol), it.ctypes.data_as(_ip), rs.ctypes.data_as(_dp))
        _check(rc, "qdse_newton", allow=_OUTCOMES)
        return rc, it, rs

    def solve_stats(self):
        """(FP32 sweeps, FP64 sweeps) per instance of the last solve."""
        a = np.zeros(self.n_inst, dtype=np.int32)
        b = np.zeros(self.n_inst, dtype=np.int32)
        _check(load().qdse_solve_stats(self._h, a.ctypes.data_as(_ip), b.ctypes.data_as(_ip)),
               "qdse_solve_stats")
        return a, b

    def jvp(self, x, v, out=None):
        import torch
        out = torch.empty_like(x) if out is None else out
        _check(load().qdse_jvp(self._h, _dev(x, self.shape, "x"), _dev(v, self.shape, "v"),
                               _dev(out, self.shape, "out")), "qdse_jvp")
        return out

    def vjp(self, x, w, out=None):
        import torch
        out = torch.empty_like(x) if out is None else out
        _check(load().qdse_vjp(self._h, _dev(x, self.shape, "x"), _dev(w, self.shape, "w"),
                               _dev(out, self.shape, "out")), "qdse_vjp")
        return out

    def vjp_noalloc(self, x, w, out):
        """qdse_vjp_noalloc: the reverse sweep with the library's fixed
        workspace (out must be given; nothing is allocated)."""
        _check(load().qdse_vjp_noalloc(self._h, _dev(x, self.shape, "x"), _dev(w, self.shape, "w"),
                                       _dev(out, self.shape, "out")), "qdse_vjp_noalloc")
        return out

    def jacobian_band(self, x, bw, out=None):
        """Band of dF/dx at x: [n_inst][N][2 bw + 1][4] blocks (AA, AB, BA, BB)
        for l = i - bw + o."""
        import torch
        n_inst, n2 = self.shape
        shp = (n_inst, n2 // 2, 2 * int(bw) + 1, 4)
        if out is None:
            out = torch.empty(shp, dtype=torch.float64, device=x.device)
        elif not (out.is_cuda and out.dtype == torch.float64 and out.is_contiguous()
                  and tuple(out.shape) == shp):
            raise ValueError(f"out must be a contiguous float64 CUDA tensor of shape {shp}")
        _check(load().qdse_jacobian_band(self._h, _dev(x, self.shape, "x"), int(bw),
                                         ctypes.c_void_p(out.data_ptr())), "qdse_jacobian_band")
        return out

    def grad(self, xstar, g, tol=1e-12, max_iter=400):
        """theta_bar[n_inst][3] = dL/d(D, omega, m) through the fixed point."""
        tb = np.zeros((self.n_inst, 3))
        rc = load().qdse_grad(self._h, _dev(xstar, self.shape, "xstar"), _dev(g, self.shape, "g"),
                              float(tol), int(max_iter), tb.ctypes.data_as(_dp))
        _check(rc, "qdse_grad", allow=(QDSE_OK, QDSE_NOT_CONVERGED))
        return tb, rc

    def autotune(self, reps=20, cache=None):
        """qdse_autotune: times the launch shapes on this batch and keeps the
        fastest (cache: path of a JSON file of winners). Returns a dict."""
        fr, rh, hit = ctypes.c_int(0), ctypes.c_int(0), ctypes.c_int(0)
        _check(load().qdse_autotune(self._h, int(reps), None if cache is None else str(cache).encode(),
                                    ctypes.byref(fr), ctypes.byref(rh), ctypes.byref(hit)),
               "qdse_autotune")
        return {"fused_rows": fr.value, "mm_row_groups": rh.value, "from_cache": bool(hit.value)}

    def time_contraction(self, x, reps=50, which=0):
        """Average device milliseconds of one sweep-kernel launch (HIP events):
        which = 0 fused FP64 sweep, 1 FP32 matrix-core, 2 FP64 matrix-core."""
        import torch
        out = torch.empty_like(x)
        ms = ctypes.c_double()
        _check(load().qdse_time_contraction(self._h, int(which), _dev(x, self.shape, "x"),
                                            _dev(out, self.shape, "out"), int(reps),
                                            ctypes.byref(ms)), "qdse_time_contraction")
        return ms.value

    def kernel_matrices(self, inst=0):
        import torch
        K = torch.empty((3, self.n, self.n + 1), dtype=torch.float64, device=self.device)
        _check(load().qdse_kernel_matrices(self._h, int(inst), ctypes.c_void_p(K.data_ptr())),
               "qdse_kernel_matrices")
        return K


def mu_grid_nodes(n_space, n_time, n_angle, interp_order=3, r_min=1e-2, r_max=1e2, p4_max=1e2,
                  lam4=0.5, T=0.0):
    """Host-only: the finite-mu grid arrays a context would use (T > 0:
    Matsubara frequencies, loop frequencies = external ones)."""
    g = MuGrid(int(n_space), int(n_time), int(n_angle), int(interp_order), float(r_min),
               float(r_max), float(p4_max), float(lam4), float(T))
    nq4 = n_time if T > 0 else n_time + 1
    sizes = (n_space, n_time, n_space + 1, nq4, n_space + 1, nq4, n_angle, n_angle)
    out = [np.empty(k) for k in sizes]
    _check(load().qdse_mu_grid_nodes(ctypes.byref(g), *[a.ctypes.data_as(_dp) for a in out]),
           "qdse_mu_grid_nodes")
    return dict(zip(("ps", "p4", "qs", "q4", "wqs", "wq4", "z", "wz"), out))


def solve_group(solvers, xs, tol=1e-10, max_iter=1000, conv_mode=QDSE_CONV_MASS):
    """qdse_solve_group: solves several contexts together (their work overlaps
    when their streams differ). xs[q] is solvers[q]'s unknown tensor (in
    place). Returns (status, [iters per context], [resid per context])."""
    n = len(solvers)
    if n != len(xs) or n == 0:
        raise ValueError("one unknown tensor per solver is required")
    H = (_vp * n)(*[S._h for S in solvers])
    X = (_vp * n)(*[_dev(x, S.shape, "x") for S, x in zip(solvers, xs)])
    its = [np.zeros(S.n_inst, dtype=np.int32) for S in solvers]
    rss = [np.zeros(S.n_inst) for S in solvers]
    I = (_ip * n)(*[a.ctypes.data_as(_ip) for a in its])
    R = (_dp * n)(*[a.ctypes.data_as(_dp) for a in rss])
    rc = load().qdse_solve_group(H, n, X, float(tol), int(max_iter), int(conv_mode), I, R)
    _check(rc, "qdse_solve_group", allow=_OUTCOMES)
    return rc, its, rss


def mu_solve_group(solvers, xs, tol=1e-10, max_iter=500):
    """qdse_mu_solve_group: successive approximation of several finite-mu
    contexts together (their sweeps overlap when their streams differ).
    Returns (status, [iters per context], [resid per context])."""
    n = len(solvers)
    if n != len(xs) or n == 0:
        raise ValueError("one unknown tensor per solver is required")
    H = (_vp * n)(*[S._h for S in solvers])
    X = (_vp * n)(*[S._cdev(x, "x") for S, x in zip(solvers, xs)])
    its = [np.zeros(S.n_inst, dtype=np.int32) for S in solvers]
    rss = [np.zeros(S.n_inst) for S in solvers]
    I = (_ip * n)(*[a.ctypes.data_as(_ip) for a in its])
    R = (_dp * n)(*[a.ctypes.data_as(_dp) for a in rss])
    rc = load().qdse_mu_solve_group(H, n, X, float(tol), int(max_iter), I, R)
    _check(rc, "qdse_mu_solve_group", allow=(QDSE_OK, QDSE_NOT_CONVERGED, QDSE_ENAN))
    return rc, its, rss


class MuSolver:
    """Finite-mu context: unknowns complex128 [n_inst][3][n_space*n_time] (A, B, C)."""

    def __init__(self, n_space, n_time, n_angle, params, interp_order=3, r_min=1e-2, r_max=1e2,
                 p4_max=1e2, lam4=0.5, T=0.0, stream=None):
        import torch
        L = load()
        self.ns, self.n4, self.na = int(n_space), int(n_time), int(n_angle)
        self.params = [tuple(map(float, p)) for p in params]
        self.n_inst = len(self.params)
        self.device = torch.device("cuda", torch.cuda.current_device())
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        g = MuGrid(self.ns, self.n4, self.na, int(interp_order), float(r_min), float(r_max),
                   float(p4_max), float(lam4), float(T))
        P = (MuParams * self.n_inst)(*[MuParams(*p) for p in self.params])
        h = _vp()
        _check(L.qdse_mu_setup(ctypes.byref(g), P, self.n_inst, _vp(self.stream.cuda_stream),
                               ctypes.byref(h)), "qdse_mu_setup")
        self._h = h

    @property
    def shape(self):
        return (self.n_inst, 3, self.ns * self.n4)

    def close(self):
        if getattr(self, "_h", None):
            load().qdse_mu_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _cdev(self, t, name):
        import torch
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.complex128
                and t.is_contiguous() and tuple(t.shape) == self.shape):
            raise ValueError(f"{name} must be a contiguous complex128 CUDA tensor of shape {self.shape}")
        return ctypes.c_void_p(t.data_ptr())

    def iterate(self, x, out=None):
        import torch
        out = torch.empty_like(x) if out is None else out
        _check(load().qdse_mu_iterate(self._h, self._cdev(x, "x"), self._cdev(out, "out")),
               "qdse_mu_iterate")
        return out

    def solve(self, x, tol=1e-10, max_iter=500, anderson=None):
        """In place; anderson = depth m uses qdse_mu_solve_anderson."""
        it = np.zeros(self.n_inst, dtype=np.int32)
        rs = np.zeros(self.n_inst)
        if anderson is None:
            rc = load().qdse_mu_solve(self._h, self._cdev(x, "x"), float(tol), int(max_iter),
                                      it.ctypes.data_as(_ip), rs.ctypes.data_as(_dp))
        else:
            rc = load().qdse_mu_solve_anderson(self._h, self._cdev(x, "x"), float(tol),
                                               int(max_iter), int(anderson),
                                               it.ctypes.data_as(_ip), rs.ctypes.data_as(_dp))
        _check(rc, "qdse_mu_solve", allow=(QDSE_OK, QDSE_NOT_CONVERGED, QDSE_ENAN))
        return rc, it, rs


def fred_nodes(n, a, b, alpha=0.5, interp_order=3):
    """Host-only: x [n], t [n+1], w [n+1] of the general system's grid."""
    g = FredGrid(int(n), int(interp_order), float(a), float(b), float(alpha))
    x, t, w = np.empty(n), np.empty(n + 1), np.empty(n + 1)
    _check(load().qdse_fred_nodes(ctypes.byref(g), x.ctypes.data_as(_dp), t.ctypes.data_as(_dp),
                                  w.ctypes.data_as(_dp)), "qdse_fred_nodes")
    return x, t, w


class FredSolver:
    """The general system of Sec. I (qdse_fred_* in include/qdse.h).

    F: 4 x 6 coefficients (F11, F12, F21, F22 as quadratics in u, v);
    K1, K2: float64 CUDA tensors [n, n+1] (K(x_i, t_j)); f: [2n] = f1 | f2.
    The tensors are kept referenced for the solver's lifetime.
    """

    def __init__(self, n, a, b, alpha, F, K1, K2, f, interp_order=3, stream=None):
        import torch
        L = load()
        self.n = int(n)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self._keep = (K1, K2, f)
        g = FredGrid(self.n, int(interp_order), float(a), float(b), float(alpha))
        Fc = np.asarray(F, dtype=np.float64).reshape(4, 6)
        P = (FredPoly * 4)(*[FredPoly((ctypes.c_double * 6)(*row)) for row in Fc])
        h = _vp()
        _check(L.qdse_fred_setup(ctypes.byref(g), P,
                                 _dev(K1, (self.n, self.n + 1), "K1"),
                                 _dev(K2, (self.n, self.n + 1), "K2"),
                                 _dev(f, (2 * self.n,), "f"), _vp(self.stream.cuda_stream),
                                 ctypes.byref(h)), "qdse_fred_setup")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            load().qdse_fred_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def iterate(self, uv, out=None):
        import torch
        if out is None:
            out = torch.empty_like(uv)
        _check(load().qdse_fred_iterate(self._h, _dev(uv, (2 * self.n,), "uv"),
                                        _dev(out, (2 * self.n,), "out")), "qdse_fred_iterate")
        return out

    def solve(self, uv, tol=1e-12, max_iter=1000):
        """In place. Returns (status, sweeps, last change)."""
        it = ctypes.c_int(0)
        r = ctypes.c_double(0.0)
        rc = _check(load().qdse_fred_solve(self._h, _dev(uv, (2 * self.n,), "uv"), float(tol),
                                           int(max_iter), ctypes.byref(it), ctypes.byref(r)),
                    "qdse_fred_solve", allow=(QDSE_OK, QDSE_NOT_CONVERGED, QDSE_ENAN))
        return rc, it.value, r.value

    def time_sweep(self, uv, reps=50):
        import torch
        out = torch.empty_like(uv)
        ms = ctypes.c_double(0.0)
        _check(load().qdse_fred_time_sweep(self._h, _dev(uv, (2 * self.n,), "uv"),
                                           _dev(out, (2 * self.n,), "out"), int(reps),
                                           ctypes.byref(ms)), "qdse_fred_time_sweep")
        return ms.value


def measure_peaks(stream=None):
    """qdse_measure_peaks on the current device: dict of copy GB/s, read-only
    stream GB/s and the FP32 / FP64 matrix-core TFLOP/s."""
    import torch
    st = stream if stream is not None else torch.cuda.current_stream()
    c, m32, m64, rd = (ctypes.c_double(0) for _ in range(4))
    _check(load().qdse_measure_peaks(_vp(st.cuda_stream), ctypes.byref(c), ctypes.byref(m32),
                                     ctypes.byref(m64), ctypes.byref(rd)), "qdse_measure_peaks")
    return {"copy_GBs": c.value, "read_GBs": rd.value, "mfma_fp32_TFLOPs": m32.value,
            "mfma_fp64_TFLOPs": m64.value}


def measure_launch_floor(workgroups, read_bytes, stream=None):
    """qdse_measure_launch_floor: average packet-timed duration (us) of an
    empty kernel and of a one-pass streaming read of read_bytes, both on
    workgroups x 256 threads."""
    import torch
    st = stream if stream is not None else torch.cuda.current_stream()
    e, r = ctypes.c_double(0), ctypes.c_double(0)
    _check(load().qdse_measure_launch_floor(_vp(st.cuda_stream), int(workgroups), int(read_bytes),
                                            ctypes.byref(e), ctypes.byref(r)),
           "qdse_measure_launch_floor")
    return {"empty_us": e.value, "stream_read_us": r.value}

