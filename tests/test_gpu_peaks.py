"""The device micro-benchmarks behind the roofline figures (ot_measure_peaks): every rate is
positive and finite and below what the chip's unit counts allow (256 CUs, 64 lanes of fp32 or
fp64 FMA and at most 64 lanes of exp2 per CU and clock, 2.4 GHz; 1024 float64 matrix-core
multiply-adds per 64 cycles per SIMD), the exp2 rate is below the FMA rate, the slot hops are sub-microsecond to tens of microseconds, and the same-XCD hop used
XCD-local publication on a device whose blocks are dealt round-robin to 8 XCDs."""
import math

import pytest

pytestmark = pytest.mark.gpu


def test_peaks_are_plausible(lib):
    print("[peaks] ot_measure_peaks", flush=True)
    pk = lib.ot_measure_peaks()
    print(f"[peaks] {pk}", flush=True)
    lane_ops = 256 * 64 * 2.4e9 * 1.05  # per second, 5 % clock headroom
    for key in ("fma32_per_s", "fma64_per_s", "exp2_per_s", "full_entry_mix_per_s"):
        assert math.isfinite(pk[key]) and 0 < pk[key] <= lane_ops, (key, pk[key])
    assert pk["exp2_per_s"] < pk["fma32_per_s"]
    # one entry of the full-size mix takes at least 5 issue slots
    assert pk["full_entry_mix_per_s"] < pk["fma32_per_s"] / 4
    assert 1e11 < pk["copy_bytes_per_s"] < 8.0e12 * 2
    for key in ("slot_hop_s_same_xcd", "slot_hop_s_cross_xcd"):
        assert math.isfinite(pk[key]) and 1e-8 < pk[key] < 5e-5, (key, pk[key])
    assert pk["same_xcd_local_publication"] in (0.0, 1.0)
    # float64 matrix cores: at most 1024 multiply-adds per 64 cycles per SIMD (the published
    # 78.6 TFLOP/s at 2.4 GHz), and well above the vector unit's fp64 rate
    mfma_peak = 256 * 4 * 16 * 2.4e9 * 1.05
    assert math.isfinite(pk["mfma64_madd_per_s"]) and 0 < pk["mfma64_madd_per_s"] <= mfma_peak
    assert pk["mfma64_madd_per_s"] > 0.5 * pk["fma64_per_s"]
