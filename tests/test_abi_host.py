"""Host-side checks of the C ABI: the library loads, exports every function
include/qdse.h declares, and rejects bad arguments before any HIP call."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "qdse.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(qdse_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    import paper_2012_03667_amd as Q
    if not os.path.exists(Q.library_path()):
        from paper_2012_03667_amd import build
        build.build()
    return Q.load()


def test_every_declared_symbol_is_exported(L):
    names = declared_functions()
    assert "qdse_setup" in names and "qdse_solve" in names and "qdse_grad" in names
    for nm in names:
        assert hasattr(L, nm), nm


def test_setup_rejects_bad_arguments_before_hip(L):
    from paper_2012_03667_amd._lib import Grid, Params
    h = ctypes.c_void_p()
    p = (Params * 1)(Params(0.55, 0.678, 0.0))
    good = dict(n_radial=64, n_angle=32, interp_order=3, s_min=1e-4, s_max=1e4)
    bad = [dict(good, n_radial=3), dict(good, n_angle=0), dict(good, interp_order=2),
           dict(good, s_min=0.0), dict(good, s_max=1e-5)]
    for b in bad:
        g = Grid(**b)
        assert L.qdse_setup(ctypes.byref(g), p, 1, 0, 0, None, ctypes.byref(h)) == -1, b
    g = Grid(**good)
    assert L.qdse_setup(ctypes.byref(g), p, 0, 0, 0, None, ctypes.byref(h)) == -1
    assert L.qdse_setup(ctypes.byref(g), p, 1, 7, 0, None, ctypes.byref(h)) == -1
    assert L.qdse_setup(ctypes.byref(g), p, 1, 0, 3, None, ctypes.byref(h)) == -1
    assert L.qdse_setup(ctypes.byref(g), p, 1, 0, 0, None, None) == -1
    for badp in (Params(-1.0, 0.5, 0.0), Params(1.0, 0.0, 0.0), Params(1.0, 0.5, float("nan"))):
        pp = (Params * 1)(badp)
        assert L.qdse_setup(ctypes.byref(g), pp, 1, 0, 0, None, ctypes.byref(h)) == -1


def test_setup_qc_rejects_bad_arguments_before_hip(L):
    from paper_2012_03667_amd._lib import Grid, Params, Qc
    h = ctypes.c_void_p()
    p = (Params * 1)(Params(0.55, 0.678, 0.0034))
    g = Grid(n_radial=64, n_angle=32, interp_order=3, s_min=1e-4, s_max=1e4)
    assert L.qdse_setup_qc(ctypes.byref(g), p, 1, None, None, ctypes.byref(h)) == -1
    for q in (Qc(2, 19.0), Qc(1, 0.0), Qc(1, -19.0), Qc(1, 100.0), Qc(1, 1e-2),
              Qc(1, float("nan"))):
        assert L.qdse_setup_qc(ctypes.byref(g), p, 1, ctypes.byref(q), None,
                               ctypes.byref(h)) == -1, (q.uv, q.zeta)
    bad = Grid(n_radial=3, n_angle=32, interp_order=3, s_min=1e-4, s_max=1e4)
    q = Qc(1, 19.0)
    assert L.qdse_setup_qc(ctypes.byref(bad), p, 1, ctypes.byref(q), None, ctypes.byref(h)) == -1


def test_fred_entry_points_reject_bad_arguments_before_hip(L):
    import numpy as np
    from paper_2012_03667_amd._lib import FredGrid, FredPoly
    dp = ctypes.POINTER(ctypes.c_double)
    x, t, w = np.empty(70), np.empty(71), np.empty(71)
    args = [a.ctypes.data_as(dp) for a in (x, t, w)]
    good = dict(n=64, interp_order=3, a=0.0, b=1.0, alpha=0.5)
    assert L.qdse_fred_nodes(ctypes.byref(FredGrid(**good)), *args) == 0
    for bad in (dict(good, n=3), dict(good, interp_order=2), dict(good, a=1.0),
                dict(good, alpha=0.0), dict(good, alpha=1.5), dict(good, b=float("inf"))):
        assert L.qdse_fred_nodes(ctypes.byref(FredGrid(**bad)), *args) == -1, bad
    h = ctypes.c_void_p()
    F = (FredPoly * 4)()
    g = FredGrid(**good)
    assert L.qdse_fred_setup(ctypes.byref(g), F, None, None, None, None, ctypes.byref(h)) == -1
    F[1].c[2] = float("nan")
    p = ctypes.c_void_p(16)  # never dereferenced: validation fails first
    assert L.qdse_fred_setup(ctypes.byref(g), F, p, p, p, None, ctypes.byref(h)) == -1
    assert L.qdse_fred_iterate(None, None, None) == -1
    assert L.qdse_fred_solve(None, None, ctypes.c_double(1e-10), 10, None, None) == -1
    L.qdse_fred_destroy(None)


def test_entry_points_reject_null_context(L):
    assert L.qdse_iterate(None, None, None, None) == -1
    assert L.qdse_solve(None, None, ctypes.c_double(1e-10), 10, 0, None, None) == -1
    assert L.qdse_jvp(None, None, None, None) == -1
    assert L.qdse_vjp(None, None, None, None) == -1
    assert L.qdse_vjp_noalloc(None, None, None, None) == -1
    assert L.qdse_solve_status(None, None) == -1
    assert L.qdse_solve_kernel_us(None, None) == -1
    assert L.qdse_jacobian_band(None, None, 2, None) == -1
    assert L.qdse_measure_launch_floor(None, 0, 1024, None, None) == -1
    assert L.qdse_measure_launch_floor(None, 4, -1, None, None) == -1
    assert L.qdse_grad(None, None, None, ctypes.c_double(1e-10), 10, None) == -1
    assert L.qdse_dims(None, None, None, None, None) == -1
    L.qdse_destroy(None)


def test_strerror_names_every_code(L):
    for code in (0, 1, -1, -2, -3, -4, -5, -6, -7):
        assert L.qdse_strerror(code) and L.qdse_strerror(code) != b"unknown status code"
    assert L.qdse_strerror(99) == b"unknown status code"


def test_product_path_does_not_import_the_oracle():
    pkg = os.path.join(ROOT, "paper_2012_03667_amd")
    for dp, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".h")):
                src = open(os.path.join(dp, f)).read()
                assert "oracle" not in src.lower(), f


@pytest.mark.parametrize("n,na,smin,smax", [(64, 32, 1e-4, 1e4), (512, 128, 1e-4, 1e4),
                                            (37, 7, 1e-3, 1e3), (4, 1, 1e-2, 1e2)])
def test_library_grid_is_the_oracle_grid(L, n, na, smin, smax):
    """Both sides build the same discretisation independently (double-double
    Newton in C++ vs mpmath-polished numpy nodes); correctly rounded nodes and
    weights make them agree bit for bit, so parity is not limited by
    single-ulp node differences."""
    import numpy as np
    import paper_2012_03667_amd as Q
    from oracle import qdse_oracle as O
    h = Q.grid_nodes(n, na, 3, smin, smax)
    g = O.vac_grid(n, na, s_min=smin, s_max=smax)
    assert np.array_equal(h["s"], g.s) and np.array_equal(h["u"], g.u)
    assert np.array_equal(h["t"], g.t)
    assert np.array_equal(h["W"], g.W)
    assert np.array_equal(h["z"], g.z)
    assert np.allclose(h["wz"], g.wz * np.sqrt(1 - g.z ** 2), rtol=1e-12, atol=0)


@pytest.mark.parametrize("ns,n4,na,T", [(8, 8, 6, 0.0), (128, 128, 32, 0.0), (10, 7, 5, 0.0),
                                        (8, 8, 6, 0.1), (64, 40, 16, 0.02)])
def test_library_mu_grid_is_the_oracle_grid(L, ns, n4, na, T):
    import numpy as np
    import paper_2012_03667_amd as Q
    from oracle import qdse_oracle as O
    h = Q.mu_grid_nodes(ns, n4, na, 3, 1e-2, 1e2, 1e2, 0.5, T)
    g = O.mu_grid(ns, n4, na, r_min=1e-2, r_max=1e2, p4_max=1e2, lam4=0.5, T=T)
    for k in ("ps", "p4", "qs", "q4", "wqs", "wq4", "z", "wz"):
        assert np.array_equal(h[k], getattr(g, k)), k


@pytest.mark.parametrize("n,a,b", [(37, -1.0, 1.0), (64, 0.0, 1.0), (15, -0.3, 2.7), (4, 1e-3, 5.0)])
def test_library_general_system_nodes_are_the_oracle_nodes(L, n, a, b):
    """Sec. I's discretisation, built independently on both sides as correctly
    rounded x = RN(a + (b - a)(x_GL + 1)/2), w = RN((b - a)/2 w_GL): equal bit
    for bit (odd n on a symmetric interval puts a node at the exact midpoint)."""
    import numpy as np
    import paper_2012_03667_amd as Q
    from oracle import qdse_oracle_fred as OF
    x, t, w = Q.fred_nodes(n, a, b)
    xo, to, wo = OF.nodes(n, a, b)
    assert np.array_equal(x, xo) and np.array_equal(t, to) and np.array_equal(w, wo)
