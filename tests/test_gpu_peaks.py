"""The machine-peak probes on the GPU: every rate positive and within a plausible band
of the datasheet figure (a probe that measured nothing, or counted its work wrongly,
falls outside it)."""
import pytest

pytestmark = pytest.mark.gpu

# (low, high) as fractions of the datasheet figure; absolute bands where there is none
BANDS = {"hbm_copy": (0.3, 1.05), "hbm_read": (0.3, 1.05), "mfma_bf16": (0.3, 1.05),
         "mfma_fp32": (0.3, 1.05), "valu_fma_fp32": (0.3, 1.05), "valu_fma_fp64": (0.3, 1.05),
         "mfma_fp64": (0.3, 1.05)}
ABS = {"valu_exp2": (2.0, 80.0), "lds_read": (10.0, 160.0)}


def test_peaks_in_band():
    from paper_1806_08593_amd import peaks as PK
    got = PK.measure()
    print("PEAKS", got)
    for name, r in got.items():
        v = r["value"]
        assert v > 0, name
        if name in BANDS:
            lo, hi = BANDS[name]
            assert lo * r["datasheet"] <= v <= hi * r["datasheet"], (name, v)
        else:
            lo, hi = ABS[name]
            assert lo <= v <= hi, (name, v)
