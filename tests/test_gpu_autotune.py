"""The launch-shape autotuner (qdse_autotune) and the shapes it chooses
between: every shape computes the same per-row arithmetic in the same order,
so results agree bit for bit; the tuner's JSON cache is reused."""
import json
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def Q():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2012_03667_amd as Q
    Q.load()
    return Q


def test_fp64_sweep_shapes_agree_bitwise(Q):
    print("case fused rows 4/8/16", flush=True)
    params = [(0.55, 0.678, 0.005), (0.55, 0.678, 0.0), (0.6, 0.7, 0.05)]
    outs = []
    for rows in ("4", "8", "16"):
        os.environ["QDSE_FUSED_ROWS"] = rows
        try:
            S = Q.Solver(130, 24, params)
        finally:
            os.environ.pop("QDSE_FUSED_ROWS", None)
        x = S.initial(1.0, 1.0)
        rc, it, rs = S.solve(x, tol=1e-10, max_iter=400)
        torch.cuda.synchronize()
        assert rc == Q.QDSE_OK
        outs.append((x.cpu().numpy(), it.copy()))
        S.close()
    for x, it in outs[1:]:
        assert np.array_equal(x, outs[0][0]) and np.array_equal(it, outs[0][1])


def test_matrix_core_row_groups_agree_bitwise(Q):
    print("case mm row groups 1/2", flush=True)
    rng = np.random.default_rng(3)
    params = [(0.55, 0.678, float(m)) for m in rng.uniform(0, 0.2, 70)]
    outs = []
    for rh in ("1", "2"):
        os.environ["QDSE_MM_RH"] = rh
        try:
            S = Q.Solver(96, 16, params, precision=Q.QDSE_FP64_MATRIX)
        finally:
            os.environ.pop("QDSE_MM_RH", None)
        x = S.initial(1.0, 1.0)
        y = S.iterate(x, matrix=True)
        rc, it, rs = S.solve(x, tol=1e-9, max_iter=400)
        torch.cuda.synchronize()
        assert rc == Q.QDSE_OK
        outs.append((y.cpu().numpy(), x.cpu().numpy(), it.copy()))
        S.close()
    assert all(np.array_equal(a, b) for a, b in zip(outs[0], outs[1]))


def test_autotune_chooses_and_caches(Q, tmp_path):
    cache = tmp_path / "tune.json"
    params = [(0.55, 0.678, 0.005), (0.55, 0.678, 0.0)]
    S = Q.Solver(256, 32, params)
    r = S.autotune(reps=5, cache=cache)
    assert r["fused_rows"] in (4, 8, 16) and not r["from_cache"]
    x = S.initial(1.0, 1.0)
    rc, it, rs = S.solve(x, tol=1e-10, max_iter=400)
    assert rc == Q.QDSE_OK
    S.close()
    data = json.loads(cache.read_text())
    assert len(data) == 1 and list(data.values())[0] == r["fused_rows"]
    S2 = Q.Solver(256, 32, params)
    r2 = S2.autotune(reps=5, cache=cache)
    assert r2["from_cache"] and r2["fused_rows"] == r["fused_rows"]
    S2.close()
    rng = np.random.default_rng(5)
    M = Q.Solver(64, 16, [(0.55, 0.678, float(m)) for m in rng.uniform(0, 0.2, 40)],
                 precision=Q.QDSE_FP32_REFINE)
    rm = M.autotune(reps=5, cache=cache)
    assert rm["mm_row_groups"] in (1, 2) and not rm["from_cache"]
    x = M.initial(1.0, 1.0)
    rc, it, rs = M.solve(x, tol=1e-8, max_iter=400)
    assert rc == Q.QDSE_OK
    M.close()
    assert len(json.loads(cache.read_text())) == 2
