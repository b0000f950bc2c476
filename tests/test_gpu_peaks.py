"""The measured FP64 FMA rate (rsai_peak_fp64) lies between a tenth of the published
MI355X FP64 vector peak and that peak plus a margin: the probe runs, is timed, and
counts its flops as the kernel performs them."""
import pytest

pytestmark = pytest.mark.gpu


def test_fp64_fma_probe_in_range():
    import paper_1503_04500_amd.rsai as rsai
    tf = rsai.peak_fp64(1 << 14)
    assert 7.86 <= tf <= 78.6 * 1.1, tf
