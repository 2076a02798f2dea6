"""Builds libtmc.so (HIP kernels for gfx950 + the C-ABI host runtime) in-tree.

    python -m paper_1806_08593_amd.build_lib [--jobs N]

Objects go to _build/ at the repository root; the library to
paper_1806_08593_amd/lib/libtmc.so, the machine-peak probes to lib/libtmc_peaks.so.
Always recompiles every source.
"""
import argparse
import concurrent.futures as cf
import glob
import os
import re
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIBDIR = os.path.join(PKG, "lib")
BUILD = os.path.join(ROOT, "_build")
ARCH = "gfx950"

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["-O3", "-fPIC", "-std=c++17", f"--offload-arch={ARCH}",
         # keep the compiler from forming packed FP32 instructions
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-result", "-I", os.path.join(ROOT, "include")]


# Sources holding the fused kernels of one precision are compiled once per d-chunk
# bucket (the instantiations of the buckets then build in parallel).
PER_BUCKET = ("k_fused_bf16.hip", "k_fused_f32.hip")


def nkc_buckets():
    """The d-chunk buckets the fused engine instantiates (kNkcBuckets in fused.h)."""
    txt = open(os.path.join(CSRC, "fused.h")).read()
    m = re.search(r"kNkcBuckets\[\]\s*=\s*\{([^}]*)\}", txt)
    return [int(x) for x in m.group(1).split(",")]


def _units(srcs):
    """(source, extra flags, object) for every compilation unit."""
    out = []
    for src in srcs:
        base = os.path.basename(src)
        if base in PER_BUCKET:
            for n in nkc_buckets():
                out.append((src, [f"-DTMC_FUSED_NKC={n}"], os.path.join(BUILD, f"{base}.n{n}.o")))
        else:
            out.append((src, [], os.path.join(BUILD, base + ".o")))
    return out


def _compile(unit):
    src, extra, obj = unit
    cmd = [HIPCC, "-c", *FLAGS, *extra, src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    err = "\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{err}")
    return obj, err


def _stale(unit, newest_dep):
    src, _, obj = unit
    return not os.path.exists(obj) or os.path.getmtime(obj) < max(os.path.getmtime(src), newest_dep)


def build(jobs=None, verbose=False, incremental=False):
    """Compiles every unit and links lib/libtmc.so.  incremental=True (development
    only) recompiles just the units older than their source or any header."""
    os.makedirs(BUILD, exist_ok=True)
    os.makedirs(LIBDIR, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))
    jobs = jobs or min(8, os.cpu_count() or 1)
    objs = []
    # the longest units (fused kernels of the widest buckets) first
    units = sorted(_units(srcs), key=lambda u: -(int(u[1][0].split("=")[1]) if u[1] else 0))
    if incremental:
        deps = glob.glob(os.path.join(CSRC, "*.h")) + glob.glob(os.path.join(CSRC, "*.inc")) + \
            glob.glob(os.path.join(ROOT, "include", "*.h"))
        newest = max(os.path.getmtime(f) for f in deps)
        todo = [u for u in units if _stale(u, newest)]
    else:
        for f in glob.glob(os.path.join(BUILD, "*.o")):
            os.remove(f)
        todo = units
    objs = [u[2] for u in units]
    with cf.ThreadPoolExecutor(jobs) as ex:
        for obj, err in ex.map(_compile, todo):
            if verbose and err.strip():
                print(err, file=sys.stderr)
    out = os.path.join(LIBDIR, "libtmc.so")
    tmp = out + ".tmp"
    cmd = [HIPCC, "-shared", f"--offload-arch={ARCH}", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stderr}")
    os.replace(tmp, out)
    build_peaks()
    return out


def build_peaks():
    """The machine-peak probes (csrc/probe/peaks.hip) as lib/libtmc_peaks.so."""
    src = os.path.join(CSRC, "probe", "peaks.hip")
    out = os.path.join(LIBDIR, "libtmc_peaks.so")
    tmp = out + ".tmp"
    cmd = [HIPCC, "-shared", *FLAGS, src, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stderr}")
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=None)
    ap.add_argument("-v", action="store_true")
    ap.add_argument("--incremental", action="store_true",
                    help="recompile only units older than their source or a header")
    a = ap.parse_args()
    print(build(a.jobs, a.v, a.incremental))
