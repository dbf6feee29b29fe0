"""C-ABI checks that need no GPU: symbols, struct layout, argument validation.

Validation happens on the host before any HIP call, so every rejected
argument below is exercised without a device.
"""
from __future__ import annotations

import ctypes
import os
import re
import subprocess
import tempfile

import numpy as np
import pytest

from paper_2506_01120_amd import _lib, make_config, workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lie_closure.h")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2506_01120_amd import build
        build.build()
    return _lib.load()


def header_functions() -> set[str]:
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return set(re.findall(r"\b(lie_[a-z_]+)\s*\(", text))


def test_header_and_binding_agree():
    assert header_functions() == set(_lib.EXPORTS)


def test_library_exports_every_declared_symbol(lib):
    nm = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True, text=True, check=True)
    exported = {line.split()[-1] for line in nm.stdout.splitlines() if line.strip()}
    missing = header_functions() - exported
    assert not missing, missing
    for name in header_functions():
        assert hasattr(lib, name)


def test_struct_layout_matches_header():
    """sizeof/offsetof from a C compile of the header equal the ctypes mirrors."""
    fields_cfg = [f for f, _ in _lib.Config._fields_]
    fields_st = [f for f, _ in _lib.Stats._fields_]
    prog = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{HEADER}"', "int main(void){"]
    prog.append('printf("%zu %zu\\n", sizeof(lie_closure_config), sizeof(lie_closure_stats));')
    for f in fields_cfg:
        prog.append(f'printf("%zu ", offsetof(lie_closure_config, {f}));')
    prog.append('printf("\\n");')
    for f in fields_st:
        prog.append(f'printf("%zu ", offsetof(lie_closure_stats, {f}));')
    prog.append('printf("\\n"); return 0; }')
    with tempfile.TemporaryDirectory() as tmp:
        src = os.path.join(tmp, "layout.c")
        exe = os.path.join(tmp, "layout")
        open(src, "w").write("\n".join(prog))
        subprocess.run(["gcc", "-std=c99", src, "-o", exe], check=True)
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split("\n")
    sizes = list(map(int, out[0].split()))
    assert sizes == [ctypes.sizeof(_lib.Config), ctypes.sizeof(_lib.Stats)]
    assert list(map(int, out[1].split())) == [getattr(_lib.Config, f).offset for f in fields_cfg]
    assert list(map(int, out[2].split())) == [getattr(_lib.Stats, f).offset for f in fields_st]


def _init(lib, gens, n_gen, d, tol, cfg=None):
    h = ctypes.c_void_p()
    ptr = gens.ctypes.data if gens is not None else None
    st = lib.lie_closure_init(ctypes.byref(h), ptr, n_gen, d, tol, ctypes.byref(cfg) if cfg is not None else None)
    return st, h


def test_status_strings(lib):
    for code, name in _lib.STATUS_NAMES.items():
        assert lib.lie_status_string(code).decode() == name


@pytest.mark.parametrize("case", ["null_gens", "n_gen0", "d0", "d_too_big", "tol0", "tol1", "tol_nan"])
def test_init_rejects_bad_arguments(lib, case):
    g = np.ascontiguousarray(W.ising(2))
    args = {"null_gens": (None, 3, 4, 1e-10), "n_gen0": (g, 0, 4, 1e-10), "d0": (g, 3, 0, 1e-10),
            "d_too_big": (g, 3, 4096, 1e-10), "tol0": (g, 3, 4, 0.0), "tol1": (g, 3, 4, 1.0),
            "tol_nan": (g, 3, 4, float("nan"))}[case]
    st, h = _init(lib, *args)
    assert st == -1 and not h.value
    assert lib.lie_last_error().decode()


def test_init_rejects_nonfinite(lib):
    g = np.ascontiguousarray(W.ising(2))
    g[1, 0, 1] = np.nan
    st, _ = _init(lib, g, 3, 4, 1e-10)
    assert st == -3


def test_init_rejects_hermitian_input(lib):
    g = np.ascontiguousarray(-1j * W.ising(2))  # Hermitian Pauli strings
    st, _ = _init(lib, g, 3, 4, 1e-10)
    assert st == -2
    assert "anti-Hermitian" in lib.lie_last_error().decode()


def test_config_validation(lib):
    g = np.ascontiguousarray(W.ising(2))
    cfg = make_config()
    cfg.struct_size = 3
    assert _init(lib, g, 3, 4, 1e-10, cfg)[0] == -1
    for field, bad in (("precision", 7), ("decide", -1), ("block", 20000), ("max_dim", -2)):
        cfg = make_config()
        setattr(cfg, field, bad)
        assert _init(lib, g, 3, 4, 1e-10, cfg)[0] == -1, field
    cfg = make_config()
    cfg.method = 5
    assert _init(lib, g, 3, 4, 1e-10, cfg)[0] == -1
    cfg = make_config(precision="fp32")
    cfg.method = 1  # the rank-test baseline runs in FP64 only
    assert _init(lib, g, 3, 4, 1e-10, cfg)[0] == -1
    cfg = make_config()
    cfg.raw_basis = 3
    assert _init(lib, g, 3, 4, 1e-10, cfg)[0] == -1
    cfg = make_config()
    cfg.reserved0 = 1
    assert _init(lib, g, 3, 4, 1e-10, cfg)[0] == -1
    cfg = make_config()
    cfg.autotune = 2
    assert _init(lib, g, 3, 4, 1e-10, cfg)[0] == -1
    # screening GEMM tiles: 1-2 for the screened precisions, none for FP64
    for prec, tile in (("fp64", 1), ("fp32", 3), ("fp32", -1), ("bf16x3", 3)):
        cfg = make_config(precision=prec)
        cfg.gemm_tile = tile
        assert _init(lib, g, 3, 4, 1e-10, cfg)[0] == -1


def test_null_handle_calls(lib):
    n = ctypes.c_int64()
    assert lib.lie_closure_dim(None, ctypes.byref(n)) == -1
    assert lib.lie_closure_run(None) == -1
    assert lib.lie_closure_run_budget(None, 5) == -1
    lib.lie_closure_free(None)
    lib.lie_closure_batch_free(None)
    assert lib.lie_closure_batch_run(None) == -1


def test_python_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(_lib, "_lib", None)
    with pytest.raises(ImportError):
        _lib.load()


def test_binding_loads_one_hip_runtime():
    """PyTorch-ROCm ships its own HIP runtime; the binding loads torch before the library so
    the library binds to it, whatever the caller imported first (a second runtime loaded
    beside torch's leaves torch without a device).  Checked in a fresh process: the HIP runtime
    files mapped after loading the library through the binding, then torch."""
    code = (
        "from paper_2506_01120_amd import _lib\n"
        "_lib.load()\n"
        "import torch\n"
        "maps = open('/proc/self/maps').read().splitlines()\n"
        "print(len({l.split()[-1] for l in maps if 'libamdhip64' in l}))\n"
    )
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    out = subprocess.run(["python", "-c", code], cwd=root, capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr
    assert out.stdout.strip().splitlines()[-1] == "1"
