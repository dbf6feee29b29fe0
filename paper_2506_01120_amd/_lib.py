"""ctypes declarations of the engine's C ABI (include/lie_closure.h).

Loading fails loudly when the HIP library is not built: there is no fallback
implementation of any step.
"""
from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "liblieclosure.so")

LIE_OK = 0
LIE_INCOMPLETE = 1

STATUS_NAMES = {
    0: "LIE_OK", 1: "LIE_INCOMPLETE", -1: "LIE_ERR_ARG", -2: "LIE_ERR_NOT_ANTIHERMITIAN", -3: "LIE_ERR_NONFINITE",
    -4: "LIE_ERR_OOM", -5: "LIE_ERR_DEVICE", -6: "LIE_ERR_STATE", -7: "LIE_ERR_CAPACITY", -8: "LIE_ERR_NUMERIC",
}

PRECISIONS = {"fp64": 0, "fp32": 1, "bf16x3": 2}
K_COUNT = 8
KERNEL_NAMES = ("comm", "dot", "sub", "reduce", "accept", "verify", "other", "growth")
DECIDES = {"fp64": 0, "strict": 1, "screen": 2}

# Every symbol include/lie_closure.h declares.
EXPORTS = (
    "lie_closure_config_default", "lie_closure_init", "lie_closure_run", "lie_closure_run_budget",
    "lie_closure_dim", "lie_closure_basis", "lie_closure_basis_device", "lie_closure_raw_basis",
    "lie_pauli_coordinates", "lie_pauli_matrix",
    "lie_closure_orthogonality", "lie_closure_orthogonality_noalloc",
    "lie_closure_init_pauli_sparse", "lie_closure_basis_pauli_sparse",
    "lie_closure_stats_get", "lie_closure_free", "lie_status_string", "lie_last_error",
    "lie_closure_batch_init", "lie_closure_batch_run", "lie_closure_batch_dim", "lie_closure_batch_basis",
    "lie_closure_batch_stats_get", "lie_closure_batch_free",
)


class Config(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32),
        ("precision", ctypes.c_int32),
        ("decide", ctypes.c_int32),
        ("block", ctypes.c_int32),
        ("early_exit", ctypes.c_int32),
        ("device", ctypes.c_int32),
        ("tau_rej", ctypes.c_double),
        ("max_dim", ctypes.c_int64),
        ("stream", ctypes.c_void_p),
        ("use_graphs", ctypes.c_int32),
        ("profile", ctypes.c_int32),
        ("autotune", ctypes.c_int32),
        ("reserved0", ctypes.c_int32),
        ("tune_cache", ctypes.c_char_p),
        ("raw_basis", ctypes.c_int32),
        ("method", ctypes.c_int32),
        ("representation", ctypes.c_int32),
        ("gemm_tile", ctypes.c_int32),
        ("reserved", ctypes.c_int32 * 2),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32),
        ("done", ctypes.c_int32),
        ("dim", ctypes.c_int64),
        ("ambient", ctypes.c_int64),
        ("candidates", ctypes.c_int64),
        ("generator_checks", ctypes.c_int64),
        ("zero_brackets", ctypes.c_int64),
        ("screen_rejected", ctypes.c_int64),
        ("fp64_decided", ctypes.c_int64),
        ("accepted", ctypes.c_int64),
        ("block_qr_accepted", ctypes.c_int64),
        ("blocks", ctypes.c_int64),
        ("host_syncs", ctypes.c_int64),
        ("min_accepted_residual", ctypes.c_double),
        ("max_rejected_residual", ctypes.c_double),
        ("max_screen_rejected", ctypes.c_double),
        ("screen_max_dependent", ctypes.c_double),
        ("screen_min_independent", ctypes.c_double),
        ("run_ms", ctypes.c_double),
        ("precision", ctypes.c_int32),
        ("decide", ctypes.c_int32),
        ("block", ctypes.c_int32),
        ("early_exit", ctypes.c_int32),
        ("tile_dot", ctypes.c_int32),
        ("tile_sub", ctypes.c_int32),
        ("autotuned", ctypes.c_int32),
        ("block_growth", ctypes.c_int32),
        ("kernel_launches", ctypes.c_int64 * K_COUNT),
        ("kernel_ms", ctypes.c_double * K_COUNT),
        ("kernel_flops", ctypes.c_double * K_COUNT),
        ("kernel_bytes", ctypes.c_double * K_COUNT),
        ("reorth_passes", ctypes.c_int64),
        ("pauli_terms", ctypes.c_int64),
    ]

    def as_dict(self) -> dict:
        out = {}
        for name, _ in self._fields_:
            if name == "struct_size":
                continue
            v = getattr(self, name)
            if name.startswith("kernel_"):
                v = {KERNEL_NAMES[i]: v[i] for i in range(len(KERNEL_NAMES))}
            out[name] = v
        return out


_lib = None


def _declare(lib: ctypes.CDLL) -> ctypes.CDLL:
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    pp = ctypes.POINTER(ctypes.c_void_p)
    st = ctypes.c_int
    i64p = ctypes.POINTER(ctypes.c_int64)
    dblp = ctypes.POINTER(ctypes.c_double)
    sigs = {
        "lie_closure_config_default": (st, [ctypes.POINTER(Config)]),
        "lie_closure_init": (st, [pp, vp, i32, i32, dbl, ctypes.POINTER(Config)]),
        "lie_closure_run": (st, [vp]),
        "lie_closure_run_budget": (st, [vp, i64]),
        "lie_closure_dim": (st, [vp, i64p]),
        "lie_closure_basis": (st, [vp, vp, i64, i64p]),
        "lie_closure_basis_device": (st, [vp, vp, i64, i64p]),
        "lie_closure_raw_basis": (st, [vp, vp, i64, i64p]),
        "lie_pauli_coordinates": (st, [ctypes.c_int32, vp, vp]),
        "lie_pauli_matrix": (st, [ctypes.c_int32, vp, vp]),
        "lie_closure_orthogonality": (st, [vp, dblp]),
        "lie_closure_orthogonality_noalloc": (st, [vp, vp]),
        "lie_closure_init_pauli_sparse": (st, [pp, i32, i32, vp, vp, vp, dbl, i64, ctypes.POINTER(Config)]),
        "lie_closure_basis_pauli_sparse": (st, [vp, vp, vp, vp, i64, i64p]),
        "lie_closure_stats_get": (st, [vp, ctypes.POINTER(Stats)]),
        "lie_closure_free": (None, [vp]),
        "lie_status_string": (ctypes.c_char_p, [st]),
        "lie_last_error": (ctypes.c_char_p, []),
        "lie_closure_batch_init": (st, [pp, i32, ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_int32),
                                        ctypes.POINTER(ctypes.c_int32), dblp, ctypes.POINTER(Config)]),
        "lie_closure_batch_run": (st, [vp]),
        "lie_closure_batch_dim": (st, [vp, i32, i64p]),
        "lie_closure_batch_basis": (st, [vp, i32, vp, i64, i64p]),
        "lie_closure_batch_stats_get": (st, [vp, i32, ctypes.POINTER(Stats)]),
        "lie_closure_batch_free": (None, [vp]),
    }
    for name, (res, args) in sigs.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


def load() -> ctypes.CDLL:
    """Load the built HIP library; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is not built; run `python -m paper_2506_01120_amd.build` (hipcc, gfx950) first")
        # One HIP runtime per process.  PyTorch-ROCm ships its own libamdhip64; if this
        # library's (from /opt/rocm) were loaded first, torch's would load beside it and torch
        # would see no device.  With torch loaded first, this library binds to its runtime.
        import torch  # noqa: F401

        _lib = _declare(ctypes.CDLL(LIB_PATH))
    return _lib


class LieError(RuntimeError):
    def __init__(self, status: int, message: str):
        self.status = status
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")


def check(status: int, allow_incomplete: bool = False) -> int:
    if status == LIE_OK or (allow_incomplete and status == LIE_INCOMPLETE):
        return status
    msg = load().lie_last_error().decode(errors="replace")
    raise LieError(status, msg)
