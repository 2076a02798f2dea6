"""Host-only checks of the C ABI (no GPU needed): the library loads, exports every
function include/tmc.h declares, the ctypes mirrors of its structs match the C
layout, and invalid problem descriptors are rejected before any device work."""
import ctypes
import os
import subprocess
import tempfile

import pytest

from paper_1806_08593_amd import tmc as T

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_exports_every_declared_function():
    names = T.header_functions()
    assert len(names) >= 15
    lib = ctypes.CDLL(T._LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
    assert T.tmc_abi_version() == 6


def test_struct_layout_matches_header():
    src = r'''
#include <stdio.h>
#include <stddef.h>
#include "tmc.h"
int main(void) {
  printf("%zu %zu %zu %zu\n", sizeof(tmc_layer), sizeof(tmc_chain), sizeof(tmc_problem), sizeof(tmc_plan_info));
  printf("%zu %zu %zu %zu %zu\n", offsetof(tmc_layer, f_off), offsetof(tmc_problem, layers),
         offsetof(tmc_problem, flags), offsetof(tmc_plan_info, waves_per_group),
         offsetof(tmc_problem, exponent));
  printf("%zu %zu %zu %d\n", sizeof(tmc_star_problem), offsetof(tmc_star_problem, D),
         offsetof(tmc_star_problem, reserved), (int)TMC_KC_COUNT);
  return 0;
}
'''
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "l.c")
        open(c, "w").write(src)
        exe = os.path.join(d, "l")
        subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), c, "-o", exe], check=True)
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split()
    got = list(map(int, out))
    want = [ctypes.sizeof(T.tmc_layer), ctypes.sizeof(T.tmc_chain), ctypes.sizeof(T.tmc_problem),
            ctypes.sizeof(T.tmc_plan_info), T.tmc_layer.f_off.offset, T.tmc_problem.layers.offset,
            T.tmc_problem.flags.offset, T.tmc_plan_info.waves_per_group.offset,
            T.tmc_problem.exponent.offset, ctypes.sizeof(T.tmc_star_problem),
            T.tmc_star_problem.D.offset, T.tmc_star_problem.reserved.offset,
            len(T.KERNEL_CLASSES)]
    assert got == want


def test_status_strings():
    assert T.tmc_status_string(T.TMC_OK) == "TMC_OK"
    assert T.tmc_status_string(T.TMC_ERR_SHAPE) == "TMC_ERR_SHAPE"
    assert T.tmc_status_string(99) == "TMC_ERR_UNKNOWN"


def _expect(problem, status, msg=None):
    with pytest.raises(T.TMCError) as ei:
        h = T.tmc_plan_create(problem)
        T.tmc_plan_destroy(h)
    assert ei.value.status == status, str(ei.value)
    if msg:
        assert msg in str(ei.value)


def test_validation_errors():
    p = T.homogeneous_problem(2, 3, 4, 5)
    p.c.precision = 7
    _expect(p, T.TMC_ERR_INVALID_ARG, "precision")
    p = T.homogeneous_problem(2, 3, 4, 5)
    p.c.reserved = 1
    _expect(p, T.TMC_ERR_INVALID_ARG, "reserved")
    _expect(T.homogeneous_problem(2, 3, 0, 5), T.TMC_ERR_SHAPE, "K=0")
    _expect(T.homogeneous_problem(2, 3, 4, 0, engine="plain"), T.TMC_ERR_SHAPE, "D=0")
    _expect(T.homogeneous_problem(1, 2, 5000, 4, precision="fp64"), T.TMC_ERR_SHAPE)
    _expect(T.homogeneous_problem(1, 2, 64, 300, precision="bf16x3"), T.TMC_ERR_SHAPE, "D=300")
    _expect(T.homogeneous_problem(1, 2, 64, 8, precision="fp64", engine="fused"), T.TMC_ERR_UNSUPPORTED)
    _expect(T.homogeneous_problem(1, 2, 8, 4, precision="bf16x3", engine="plain"),
            T.TMC_ERR_UNSUPPORTED)
    # chains sharing a layer, chain out of range
    lay = [dict(K=4, D=2, z_off=8 * i, u_off=4 * i, mu_off=8 * i, s_off=0, f_off=16 * i) for i in range(3)]
    _expect(T.Problem([(0, 2), (1, 2)], lay), T.TMC_ERR_INVALID_ARG, "belongs to chains")
    _expect(T.Problem([(2, 2)], lay), T.TMC_ERR_INVALID_ARG, "out of bounds")
    _expect(T.Problem([(0, 0)], lay), T.TMC_ERR_INVALID_ARG)
    # overlapping u blocks
    lay2 = [dict(K=4, D=2, z_off=8 * i, u_off=2 * i, mu_off=8 * i, s_off=0, f_off=16 * i) for i in range(2)]
    _expect(T.Problem([(0, 2)], lay2), T.TMC_ERR_INVALID_ARG, "u blocks")
    p = T.homogeneous_problem(2, 3, 4, 5)
    p.c.flags = 64
    _expect(p, T.TMC_ERR_INVALID_ARG, "flag")
    for bad in (-1.0, float("inf"), float("nan")):
        _expect(T.homogeneous_problem(2, 3, 4, 5, exponent=bad), T.TMC_ERR_INVALID_ARG, "exponent")


def test_valid_problem_needs_a_device():
    """With no GPU the valid descriptor passes validation and stops at the device
    query (TMC_ERR_HIP); on a GPU machine it succeeds."""
    try:
        h = T.tmc_plan_create(T.homogeneous_problem(2, 3, 4, 5, precision="fp64"))
    except T.TMCError as e:
        assert e.status == T.TMC_ERR_HIP
    else:
        T.tmc_plan_destroy(h)


def _expect_star(problem, status, msg=None):
    with pytest.raises(T.TMCError) as ei:
        h = T.tmc_star_plan_create(problem)
        T.tmc_plan_destroy(h)
    assert ei.value.status == status, str(ei.value)
    if msg:
        assert msg in str(ei.value)


def test_star_validation_errors():
    """Star descriptors are validated before any device is touched."""
    _expect_star(T.StarProblem(1, 8, 4, 4, 0), T.TMC_ERR_SHAPE, "D = 0")
    _expect_star(T.StarProblem(1, 8, 4, 4, 33), T.TMC_ERR_SHAPE, "D = 33")
    _expect_star(T.StarProblem(1, 0, 4, 4, 1), T.TMC_ERR_SHAPE, "N = 0")
    _expect_star(T.StarProblem(1, 8, 0, 4, 1), T.TMC_ERR_SHAPE, "K_theta = 0")
    _expect_star(T.StarProblem(1, 8, 4, 64 * 65535 + 1, 1), T.TMC_ERR_SHAPE, "K = ")
    _expect_star(T.StarProblem(0, 8, 4, 4, 1), T.TMC_ERR_INVALID_ARG, "n_instances")
    _expect_star(T.StarProblem(1, 8, 4, 4, 1, precision="bf16x3"), T.TMC_ERR_UNSUPPORTED)
    _expect_star(T.StarProblem(1, 8, 4, 4, 1, flags=T.TMC_FLAG_PERSISTENT), T.TMC_ERR_INVALID_ARG,
                 "flags")
    p = T.StarProblem(1, 8, 4, 4, 1)
    p.c.reserved = 3
    _expect_star(p, T.TMC_ERR_INVALID_ARG, "reserved")
    _expect_star(T.StarProblem(65536, 32768, 4, 4, 1), T.TMC_ERR_INVALID_ARG, "launch grid")
    _expect_star(T.StarProblem(1, 8, 64 * 65535, 4, 2), T.TMC_ERR_INVALID_ARG, "launch grid")


def test_peak_probe_library_loads():
    """The machine-peak probes are built beside the library and export their one entry
    point (no GPU call here)."""
    from paper_1806_08593_amd import peaks as PK
    lib = ctypes.CDLL(PK._LIB)
    assert hasattr(lib, "tmc_peaks_run")
    assert [p[0] for p in PK.PROBES] == ["hbm_copy", "hbm_read", "mfma_bf16", "mfma_fp32",
                                         "valu_fma_fp32", "valu_exp2", "valu_fma_fp64", "lds_read", "mfma_fp64"]
