"""The on-device peak probe used by the roofline report returns plausible
rates (independent FMA streams cannot beat the published MI355X peaks)."""
import pytest

pytestmark = pytest.mark.gpu


def test_peak_probe_rates():
    from paper_1011_4687_amd import envpot
    print("[probe] peak", flush=True)
    pk = envpot.peak_probe()
    print(pk, flush=True)
    assert 10.0 < pk["fp32_fma_tflops"] <= 157.3 * 1.05
    assert 5.0 < pk["fp64_fma_tflops"] <= 78.6 * 1.05
    assert pk["rsq_f32_per_s"] > 1e12
    assert all(m > 0 for m in pk["ms"])
