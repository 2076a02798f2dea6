"""ctypes binding of libtmc (include/tmc.h).

Argument marshalling only: every step of the estimator runs in the library's HIP
kernels.  Functions named tmc_* mirror the C entry points one to one and accept
torch tensors (device memory), integers (raw device addresses) or None (NULL).
Non-OK statuses raise TMCError with the library's message.

The library is loaded from paper_1806_08593_amd/lib/libtmc.so (built in-tree by
`python -m paper_1806_08593_amd.build_lib`); importing this module fails loudly if
it is missing.
"""
from __future__ import annotations

import ctypes
import os
import re
from ctypes import POINTER, c_char_p, c_double, c_int, c_int32, c_int64, c_size_t, c_void_p
from typing import Optional, Sequence

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "lib", "libtmc.so")
HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "tmc.h")

if not os.path.exists(_LIB_PATH):
    raise ImportError(f"{_LIB_PATH} is not built; run `python -m paper_1806_08593_amd.build_lib`")
# PyTorch's ROCm wheel ships its own HIP runtime under the same soname
# (libamdhip64.so.7).  Loading torch first makes libtmc bind to that runtime instead
# of loading a second HIP/HSA runtime into the process (with two, whichever
# initialises second sees no GPU, and torch's device pointers would belong to the
# other runtime).
try:
    import torch  # noqa: F401
except ImportError:  # pure C-ABI use without torch: the system HIP runtime is used
    pass
_lib = ctypes.CDLL(_LIB_PATH)

TMC_OK, TMC_ERR_INVALID_ARG, TMC_ERR_SHAPE, TMC_ERR_WORKSPACE = 0, 1, 2, 3
TMC_ERR_UNSUPPORTED, TMC_ERR_HIP, TMC_ERR_NUMERIC, TMC_ERR_STATE = 4, 5, 6, 7
TMC_FP64, TMC_FP32, TMC_BF16X3 = 0, 1, 2
TMC_ENGINE_AUTO, TMC_ENGINE_FUSED, TMC_ENGINE_PLAIN = 0, 1, 2
TMC_FLAG_FORWARD_ONLY, TMC_FLAG_PERSISTENT, TMC_FLAG_PARENT_SCALE = 1, 2, 4

PRECISIONS = {"fp64": TMC_FP64, "fp32": TMC_FP32, "bf16x3": TMC_BF16X3}
ENGINES = {"auto": TMC_ENGINE_AUTO, "fused": TMC_ENGINE_FUSED, "plain": TMC_ENGINE_PLAIN}


class tmc_layer(ctypes.Structure):
    _fields_ = [("K", c_int32), ("D", c_int32), ("z_off", c_int64), ("u_off", c_int64),
                ("mu_off", c_int64), ("s_off", c_int64), ("f_off", c_int64)]


class tmc_chain(ctypes.Structure):
    _fields_ = [("n_layers", c_int32), ("first_layer", c_int32)]


class tmc_problem(ctypes.Structure):
    _fields_ = [("n_chains", c_int32), ("n_layers", c_int32), ("chains", POINTER(tmc_chain)),
                ("layers", POINTER(tmc_layer)), ("precision", c_int32), ("engine", c_int32),
                ("flags", c_int32), ("reserved", c_int32), ("exponent", c_double)]


class tmc_plan_info(ctypes.Structure):
    _fields_ = [("factor_entries", c_int64), ("workspace_bytes", c_int64), ("engine", c_int32),
                ("precision", c_int32), ("max_depth", c_int32), ("tile_rows", c_int32),
                ("tile_cols", c_int32), ("waves_per_group", c_int32), ("persistent", c_int32),
                ("tuned", c_int32), ("wide_fwd", c_int32), ("wide_bwd", c_int32)]


class tmc_star_problem(ctypes.Structure):
    _fields_ = [("n_instances", c_int32), ("N", c_int32), ("K_theta", c_int32), ("K", c_int32),
                ("D", c_int32), ("precision", c_int32), ("flags", c_int32), ("reserved", c_int32)]


_P = c_void_p
_SIGS = {
    "tmc_abi_version": (c_int, []),
    "tmc_status_string": (c_char_p, [c_int]),
    "tmc_last_error": (c_char_p, []),
    "tmc_plan_create": (c_int, [POINTER(tmc_problem), c_int, POINTER(c_void_p)]),
    "tmc_plan_destroy": (c_int, [_P]),
    "tmc_plan_workspace_size": (c_int, [_P, POINTER(c_size_t)]),
    "tmc_plan_info_get": (c_int, [_P, POINTER(tmc_plan_info)]),
    "tmc_plan_check": (c_int, [_P, _P]),
    "tmc_gauss_fwd": (c_int, [_P, _P, _P, _P, _P, _P, _P, _P]),
    "tmc_gauss_bwd": (c_int, [_P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P]),
    "tmc_gauss_factors": (c_int, [_P, _P, _P, _P, _P, _P]),
    "tmc_gauss_fwd_noalloc": (c_int, [_P, _P, _P, _P, _P, _P, _P]),
    "tmc_logfactor_fwd": (c_int, [_P, _P, _P, _P, _P, _P]),
    "tmc_logfactor_bwd": (c_int, [_P, _P, _P, _P, _P, _P, _P, _P]),
    "tmc_plan_graph_capture_gauss": (c_int, [_P, c_int, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P,
                                             _P, _P]),
    "tmc_plan_graph_launch": (c_int, [_P, c_int, _P]),
    "tmc_plan_set_timing": (c_int, [_P, c_int]),
    "tmc_plan_timing": (c_int, [_P, c_int, POINTER(c_double), POINTER(c_int64)]),
    "tmc_plan_autotune": (c_int, [_P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, c_int, _P]),
    "tmc_logmmexp_workspace_size": (c_int, [c_int32, c_int32, c_int32, c_int32, c_int32,
                                            POINTER(c_size_t)]),
    "tmc_logmmexp": (c_int, [c_int32, c_int32, c_int32, c_int32, c_int32, _P, _P, _P, _P, _P]),
    "tmc_star_plan_create": (c_int, [POINTER(tmc_star_problem), c_int, POINTER(c_void_p)]),
    "tmc_star_gauss_fwd": (c_int, [_P, _P, _P, _P, _P, _P, _P, _P, _P]),
    "tmc_star_gauss_bwd": (c_int, [_P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P]),
}
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args


def header_functions() -> list:
    """Names of the functions include/tmc.h declares."""
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\**\s+\**(tmc_\w+)\s*\(", txt, re.M)))


class TMCError(RuntimeError):
    def __init__(self, status: int, message: str):
        self.status = status
        super().__init__(f"{tmc_status_string(status)}: {message}")


def _check(st: int):
    if st != TMC_OK:
        raise TMCError(st, tmc_last_error())


def _ptr(x) -> Optional[int]:
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


def _stream(stream) -> Optional[int]:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


# ---------------------------------------------------------------------------
# one-to-one wrappers of the C entry points
# ---------------------------------------------------------------------------

def tmc_abi_version() -> int:
    return _lib.tmc_abi_version()


def tmc_status_string(st: int) -> str:
    return _lib.tmc_status_string(st).decode()


def tmc_last_error() -> str:
    return _lib.tmc_last_error().decode()


def tmc_plan_create(problem: "Problem", device: int = 0) -> int:
    h = c_void_p()
    _check(_lib.tmc_plan_create(ctypes.byref(problem.c), device, ctypes.byref(h)))
    return h.value


def tmc_plan_destroy(plan: int):
    _check(_lib.tmc_plan_destroy(plan))


def tmc_plan_workspace_size(plan: int) -> int:
    n = c_size_t()
    _check(_lib.tmc_plan_workspace_size(plan, ctypes.byref(n)))
    return n.value


def tmc_plan_info_get(plan: int) -> dict:
    i = tmc_plan_info()
    _check(_lib.tmc_plan_info_get(plan, ctypes.byref(i)))
    return {k: getattr(i, k) for k, _ in tmc_plan_info._fields_}


def tmc_plan_check(plan: int, stream=None):
    _check(_lib.tmc_plan_check(plan, _stream(stream)))


def tmc_gauss_fwd(plan, z, mu, s, u, logp, workspace, stream=None):
    _check(_lib.tmc_gauss_fwd(plan, _ptr(z), _ptr(mu), _ptr(s), _ptr(u), _ptr(logp),
                              _ptr(workspace), _stream(stream)))


def tmc_gauss_bwd(plan, z, mu, s, u, dlogp, workspace, dz, dmu, ds, du, stream=None):
    _check(_lib.tmc_gauss_bwd(plan, _ptr(z), _ptr(mu), _ptr(s), _ptr(u), _ptr(dlogp),
                              _ptr(workspace), _ptr(dz), _ptr(dmu), _ptr(ds), _ptr(du),
                              _stream(stream)))


def tmc_gauss_fwd_noalloc(plan, z, mu, s, u, logp, stream=None):
    _check(_lib.tmc_gauss_fwd_noalloc(plan, _ptr(z), _ptr(mu), _ptr(s), _ptr(u), _ptr(logp),
                                      _stream(stream)))


TMC_NOALLOC_WORKSPACE_MAX = 64 << 20


def tmc_gauss_factors(plan, z, mu, s, f, stream=None):
    _check(_lib.tmc_gauss_factors(plan, _ptr(z), _ptr(mu), _ptr(s), _ptr(f), _stream(stream)))


def tmc_logfactor_fwd(plan, f, u, logp, workspace, stream=None):
    _check(_lib.tmc_logfactor_fwd(plan, _ptr(f), _ptr(u), _ptr(logp), _ptr(workspace),
                                  _stream(stream)))


def tmc_logfactor_bwd(plan, f, u, dlogp, workspace, df, du, stream=None):
    _check(_lib.tmc_logfactor_bwd(plan, _ptr(f), _ptr(u), _ptr(dlogp), _ptr(workspace),
                                  _ptr(df), _ptr(du), _stream(stream)))


def tmc_plan_graph_capture_gauss(plan, which, z, mu, s, u, logp, dlogp, workspace, dz, dmu, ds,
                                 du, stream):
    _check(_lib.tmc_plan_graph_capture_gauss(plan, which, _ptr(z), _ptr(mu), _ptr(s), _ptr(u),
                                             _ptr(logp), _ptr(dlogp), _ptr(workspace), _ptr(dz),
                                             _ptr(dmu), _ptr(ds), _ptr(du), _stream(stream)))


def tmc_plan_graph_launch(plan, which, stream=None):
    _check(_lib.tmc_plan_graph_launch(plan, which, _stream(stream)))


KERNEL_CLASSES = ["plain_factor", "plain_lse_fwd", "plain_lse_bwd", "plain_grad", "fused_prep",
                  "fused_fwd", "fused_bwd", "other", "star_msg", "star_bwd"]


def tmc_plan_set_timing(plan, enable: bool):
    _check(_lib.tmc_plan_set_timing(plan, int(bool(enable))))


def tmc_plan_timing(plan, kc: int):
    """(total ms, launches) of kernel class kc since timing was enabled."""
    ms, n = c_double(), c_int64()
    _check(_lib.tmc_plan_timing(plan, kc, ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


def tmc_plan_autotune(plan, z, mu, s, u, dlogp, workspace, dz=None, dmu=None, ds=None, du=None,
                      reps: int = 3, stream=None):
    _check(_lib.tmc_plan_autotune(plan, _ptr(z), _ptr(mu), _ptr(s), _ptr(u), _ptr(dlogp),
                                  _ptr(workspace), _ptr(dz), _ptr(dmu), _ptr(ds), _ptr(du), reps,
                                  _stream(stream)))


def tmc_logmmexp_workspace_size(batch, M, K, N, precision) -> int:
    prec = PRECISIONS[precision] if isinstance(precision, str) else precision
    n = c_size_t()
    _check(_lib.tmc_logmmexp_workspace_size(batch, M, K, N, prec, ctypes.byref(n)))
    return n.value


def tmc_logmmexp(batch, M, K, N, precision, X, Y, Z, workspace, stream=None):
    prec = PRECISIONS[precision] if isinstance(precision, str) else precision
    _check(_lib.tmc_logmmexp(batch, M, K, N, prec, _ptr(X), _ptr(Y), _ptr(Z), _ptr(workspace),
                             _stream(stream)))


def tmc_star_plan_create(problem: "StarProblem", device: int = 0) -> int:
    h = c_void_p()
    _check(_lib.tmc_star_plan_create(ctypes.byref(problem.c), device, ctypes.byref(h)))
    return h.value


def tmc_star_gauss_fwd(plan, mth, s, z, u, uth, logp, workspace, stream=None):
    _check(_lib.tmc_star_gauss_fwd(plan, _ptr(mth), _ptr(s), _ptr(z), _ptr(u), _ptr(uth),
                                   _ptr(logp), _ptr(workspace), _stream(stream)))


def tmc_star_gauss_bwd(plan, mth, s, z, u, dlogp, workspace, dmth, ds, dz, du, duth, stream=None):
    _check(_lib.tmc_star_gauss_bwd(plan, _ptr(mth), _ptr(s), _ptr(z), _ptr(u), _ptr(dlogp),
                                   _ptr(workspace), _ptr(dmth), _ptr(ds), _ptr(dz), _ptr(du),
                                   _ptr(duth), _stream(stream)))


# ---------------------------------------------------------------------------
# problem descriptors
# ---------------------------------------------------------------------------

class StarProblem:
    """Star-model descriptor: S instances of N local latents (K samples, width D) sharing
    one global latent (K_theta samples); buffers mth [S, Kt, D], s [S, D],
    z [S, N, K, D], u [S, N, K], uth [S, Kt]."""

    def __init__(self, S, N, Kt, K, D, precision="fp32", flags=0):
        prec = PRECISIONS[precision] if isinstance(precision, str) else precision
        self.c = tmc_star_problem(S, N, Kt, K, D, prec, flags, 0)
        self.shape = dict(S=S, N=N, Kt=Kt, K=K, D=D)


class Problem:
    """Host-side problem descriptor (keeps the ctypes arrays alive).

    layers: sequence of dicts with K, D, z_off, u_off, mu_off, s_off, f_off
    chains: sequence of (first_layer, n_layers)
    """

    def __init__(self, chains: Sequence, layers: Sequence[dict], precision="fp32",
                 engine="auto", flags=0, exponent=1.0):
        self.n_chains, self.n_layers = len(chains), len(layers)
        self._chains = (tmc_chain * max(1, len(chains)))()
        for i, (first, n) in enumerate(chains):
            self._chains[i].first_layer, self._chains[i].n_layers = first, n
        self._layers = (tmc_layer * max(1, len(layers)))()
        for i, d in enumerate(layers):
            for k in ("K", "D", "z_off", "u_off", "mu_off", "s_off", "f_off"):
                setattr(self._layers[i], k, int(d.get(k, 0)))
        prec = PRECISIONS[precision] if isinstance(precision, str) else precision
        eng = ENGINES[engine] if isinstance(engine, str) else engine
        self.c = tmc_problem(len(chains), len(layers), self._chains, self._layers, prec, eng,
                             flags, 0, float(exponent))
        self.chains = list(chains)
        self.layers = [dict(d) for d in layers]


def homogeneous_problem(B, L, K, D, precision="fp32", engine="auto", flags=0,
                        exponent=1.0) -> Problem:
    """B chains of L layers, K samples and width D each, laid out as
    z [B, L, K, D], mu [B, L-1, K, D], s [L-1, D] (shared by the batch),
    u [B, L, K] and f [B, L-1, K, K].  With TMC_FLAG_PARENT_SCALE in flags, s is
    [B, L-1, K, D] (one row per parent sample, the layout of mu)."""
    pp = bool(flags & TMC_FLAG_PARENT_SCALE)
    layers, chains = [], []
    for b in range(B):
        chains.append((b * L, L))
        for l in range(L):
            top = l == L - 1
            mo = 0 if top else ((b * (L - 1) + l) * K) * D
            layers.append(dict(K=K, D=D, z_off=((b * L + l) * K) * D, u_off=(b * L + l) * K,
                               mu_off=mo, s_off=0 if top else (mo if pp else l * D),
                               f_off=0 if top else ((b * (L - 1) + l) * K) * K))
    return Problem(chains, layers, precision, engine, flags, exponent)


def ragged_problem(shapes, precision="fp32", engine="auto", flags=0, share_s=False, exponent=1.0):
    """Chains given as a list of (K_list, D_list) (one entry per layer), packed
    back to back in flat z, mu, s, u and f buffers.  Returns (problem, sizes) with
    sizes the element counts of the flat buffers.  With TMC_FLAG_PARENT_SCALE in flags
    each s block is [K_{l+1}][D_l]."""
    pp = bool(flags & TMC_FLAG_PARENT_SCALE)
    layers, chains = [], []
    zo = uo = mo = so = fo = 0
    for Ks, Ds in shapes:
        L = len(Ks)
        chains.append((len(layers), L))
        for l in range(L):
            top = l == L - 1
            d = dict(K=Ks[l], D=Ds[l], z_off=zo, u_off=uo)
            zo += Ks[l] * Ds[l]
            uo += Ks[l]
            if not top:
                d.update(mu_off=mo, s_off=so, f_off=fo)
                mo += Ks[l + 1] * Ds[l]
                so += (Ks[l + 1] if pp else 1) * Ds[l]
                fo += Ks[l] * Ks[l + 1]
            layers.append(d)
    return (Problem(chains, layers, precision, engine, flags, exponent),
            dict(z=zo, u=uo, mu=mo, s=so, f=fo))


class Plan:
    """Owning wrapper of a tmc_plan_t (of a chain Problem or a StarProblem)."""

    def __init__(self, problem, device: int = 0):
        self.problem = problem
        self.device = device
        create = tmc_star_plan_create if isinstance(problem, StarProblem) else tmc_plan_create
        self.handle = create(problem, device)
        self.workspace_bytes = tmc_plan_workspace_size(self.handle)
        self.info = tmc_plan_info_get(self.handle)

    def new_workspace(self):
        """A 256-byte aligned uint8 device tensor of workspace_bytes bytes."""
        import torch
        n = max(self.workspace_bytes, 256)
        raw = torch.empty(n + 256, dtype=torch.uint8, device=f"cuda:{self.device}")
        off = (-raw.data_ptr()) % 256
        return raw[off:off + n]

    def close(self):
        if getattr(self, "handle", None):
            tmc_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
