"""The VALU issue-rate probe behind the VALU rooflines returns plausible rates: FMA below the
published FP32 lane peak and above a quarter of it, transcendentals slower than FMA."""
import pytest

from gpu_util import announce, device_or_skip

pytestmark = pytest.mark.gpu


def test_valu_probe_rates():
    device_or_skip()
    from paper_2009_04755_amd import probe_valu
    announce("valu probe")
    r = probe_valu(0)
    peak = 157.3e12 / 2  # FP32 lane-instruction slots/s on 256 CUs at 2.4 GHz
    assert peak / 4 < r["fma_per_s"] <= peak * 1.02
    for k in ("exp2_per_s", "rcp_per_s"):
        assert peak / 64 < r[k] < r["fma_per_s"]
