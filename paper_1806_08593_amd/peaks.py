"""Measured machine peaks of the GPU (lib/libtmc_peaks.so): HBM copy and read bandwidth,
the dense BF16 and FP32 MFMA rates, the FP32 FMA, exp2 and FP64 FMA rates of the vector
ALU, the LDS read bandwidth and the dense FP64 MFMA rate -- the rates the rooflines are judged against, measured
on the device instead of taken from the datasheet.

    python -m paper_1806_08593_amd.peaks      # one JSON line
"""
import ctypes
import json
import os

_LIB = os.path.join(os.path.dirname(os.path.abspath(__file__)), "lib", "libtmc_peaks.so")

# kind -> (name, unit, scale to that unit, the datasheet figure in that unit or None)
PROBES = [
    ("hbm_copy", "GB/s", 1e-9, 8000.0),        # bytes read + written
    ("hbm_read", "GB/s", 1e-9, 8000.0),
    ("mfma_bf16", "TFLOP/s", 1e-12, 2500.0),
    ("mfma_fp32", "TFLOP/s", 1e-12, 157.3),
    ("valu_fma_fp32", "TFLOP/s", 1e-12, 78.6),  # unpacked: 256 CUs x 64 lanes x 2 x 2.4 GHz
    ("valu_exp2", "T results/s", 1e-12, None),
    ("valu_fma_fp64", "TFLOP/s", 1e-12, 78.6),
    ("lds_read", "TB/s", 1e-12, None),
    ("mfma_fp64", "TFLOP/s", 1e-12, 78.6),
]


def _lib():
    if not os.path.exists(_LIB):
        raise RuntimeError(f"{_LIB} is not built (python -m paper_1806_08593_amd.build_lib)")
    lib = ctypes.CDLL(_LIB)
    lib.tmc_peaks_run.restype = ctypes.c_int
    lib.tmc_peaks_run.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_double)]
    return lib


def measure(kinds=None):
    """{name: {"value", "unit", "datasheet"}} for the probes in kinds (default all),
    on the current HIP device."""
    lib = _lib()
    out = {}
    for k, (name, unit, scale, ds) in enumerate(PROBES):
        if kinds is not None and name not in kinds:
            continue
        v = ctypes.c_double()
        rc = lib.tmc_peaks_run(k, ctypes.byref(v))
        if rc != 0:
            raise RuntimeError(f"peak probe {name} failed with HIP error {rc}")
        out[name] = dict(value=round(v.value * scale, 2), unit=unit, datasheet=ds)
    return out


if __name__ == "__main__":
    print(json.dumps(measure()))
