"""GPU: the achievable-peak probes report plausible rates (below the chip's
published peaks, above a tenth of them)."""
import pytest

from paper_2307_08006_amd import labf

pytestmark = pytest.mark.gpu

VALU_PEAK = 256 * 4 * 16 * 2.4e9     # non-packed FP32 (and FP64) lane-operations/s
HBM_PEAK = 8e12                      # bytes/s


@pytest.mark.parametrize("kind, n, peak", [("fp32_fma", 1024, VALU_PEAK), ("fp64_fma", 512, VALU_PEAK),
                                           ("fp32_rsq", 512, VALU_PEAK), ("triad", 1 << 24, HBM_PEAK)])
def test_probe_rates_are_plausible(kind, n, peak):
    r = labf.probe(kind, n)
    assert 0.1 * peak < r < 1.05 * peak, (kind, r, peak)
