"""The measured ceilings of irbe_probe_rates: finite, positive and within the
published limits of the device (the VALU rate at most 256 CUs x 64 lanes x
2.4 GHz, the copy below the HBM peak of 8 TB/s), and reproducible."""
import math

import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def test_probe_rates_are_plausible():
    from paper_2204_13595_amd import irbe
    torch.cuda.set_device(0)
    r1 = irbe.probe_rates()
    r2 = irbe.probe_rates()
    for r in (r1, r2):
        assert math.isfinite(r["valu_lane_ops_per_s"]) and math.isfinite(r["copy_bytes_per_s"])
        assert 0.3 * 256 * 64 * 2.4e9 < r["valu_lane_ops_per_s"] < 1.1 * 256 * 64 * 2.4e9
        assert 0.5e12 < r["copy_bytes_per_s"] < 8.0e12
    assert abs(r1["valu_lane_ops_per_s"] / r2["valu_lane_ops_per_s"] - 1.0) < 0.2
