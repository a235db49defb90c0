"""Measured MFMA throughput (tns_mfma_peak): positive, below the published
dense peak of the instruction, and argument checks."""
import pytest

from gpu_common import say

pytestmark = pytest.mark.gpu

# published dense MFMA peaks of MI355X (TFLOP/s of the instruction's own flops)
PUBLISHED = {"f64": 78.6, "f32": 157.3, "bf16x3": 2516.6}


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16x3"])
def test_measured_peak_is_plausible(prec):
    from paper_2305_05581_amd.tns import mfma_peak
    t = mfma_peak(prec, iters=4000)
    say("measured %s MFMA peak %.1f TFLOP/s (published %.1f)" % (prec, t, PUBLISHED[prec]))
    assert 0.3 * PUBLISHED[prec] < t < 1.15 * PUBLISHED[prec]


def test_peak_rejects_bad_arguments():
    from paper_2305_05581_amd.tns import mfma_peak, TnsError
    with pytest.raises(TnsError):
        mfma_peak("f32", iters=0)
