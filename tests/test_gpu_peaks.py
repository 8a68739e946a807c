"""Roofline denominators measured on the device (hgv_device_peaks): the FP64 MFMA rate and
the copy bandwidth must be positive and within physical reach of the published MI355X
figures (78.6 TFLOP/s FP64 MFMA, 8 TB/s HBM3E); a workspace below the documented minimum
is refused with HGV_E_WORKSPACE."""
import pytest

from tests.gpu_util import require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    hgv = require_gpu()
    return hgv.Context.get("cuda:0")


def test_device_peaks_plausible(ctx):
    tflops, gbs = ctx.device_peaks(1 << 30)
    print("measured FP64 MFMA %.1f TFLOP/s, copy %.0f GB/s" % (tflops, gbs))
    assert 10.0 < tflops < 1.05 * 78.6
    assert 500.0 < gbs < 1.05 * 8000.0


def test_device_peaks_small_workspace_refused(ctx):
    import paper_1207_1773_amd as hgv
    w = ctx._work(1 << 20)
    with pytest.raises(hgv.HgvError) as e:
        hgv.hgv_device_peaks(ctx.handle, w.data_ptr(), w.numel())
    assert e.value.status == hgv.HGV_E_WORKSPACE
