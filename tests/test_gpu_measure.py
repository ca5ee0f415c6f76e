"""The device measurements the benchmark quotes beside its rooflines
(qdse_measure_peaks, qdse_measure_launch_floor): finite, positive and
ordered as their definitions require."""
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


def test_launch_floor_is_below_a_streaming_launch(Q):
    print("case launch floor 256 workgroups, 6.36 MB", flush=True)
    f = Q.measure_launch_floor(256, 6357032)
    assert 0.0 < f["empty_us"] < 1000.0
    # streaming 6.36 MB cannot beat an empty launch of the same grid by more
    # than the timer's jitter
    assert f["stream_read_us"] > 0.9 * f["empty_us"]
    g = Q.measure_launch_floor(256, 0)
    assert g["stream_read_us"] > 0.0


def test_measured_peaks_are_positive_and_below_the_datasheet(Q):
    print("case measured peaks", flush=True)
    p = Q.measure_peaks()
    assert 0.0 < p["copy_GBs"] < 8000.0 * 1.05
    assert 0.0 < p["read_GBs"] < 8000.0 * 1.05
    assert 0.0 < p["mfma_fp32_TFLOPs"] < 157.3 * 1.05
    assert 0.0 < p["mfma_fp64_TFLOPs"] < 78.6 * 1.05
