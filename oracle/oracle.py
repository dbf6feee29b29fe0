"""Python front end of the CPU reference (``lie_oracle.c``).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke entry and the benchmark's
CPU-baseline leg are the only callers.  The GPU library never imports this.

The closure follows Algorithm 4 of arXiv 2506.01120 (dimension-only
orthonormalization) with the independence test done as an explicit
least-squares residual (proof of Theorem 1); see the header of
``lie_oracle.c`` for every reading of the paper it takes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lie_oracle.c")
_LIB = os.path.join(_HERE, "liblie_oracle.so")

_lib = None


def build(src: str = _SRC, out: str = _LIB, extra_flags: tuple[str, ...] = ()) -> str:
    """Compile the reference with gcc into a shared library and return its path."""
    cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", *extra_flags, src, "-o", out + ".tmp", "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


def _declare(lib: ctypes.CDLL) -> ctypes.CDLL:
    vp, i64, i32, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_double
    dptr = ctypes.POINTER(ctypes.c_double)
    lib.lo_new.restype = vp
    lib.lo_new.argtypes = [i32, i64, dbl, i32]
    lib.lo_free.restype = None
    lib.lo_free.argtypes = [vp]
    lib.lo_generator.restype = i32
    lib.lo_generator.argtypes = [vp, dptr, dptr]
    lib.lo_brackets.restype = i64
    lib.lo_brackets.argtypes = [vp, i32, i64, i64]
    for name in ("lo_dim", "lo_candidates", "lo_zero_brackets", "lo_generator_checks",
                 "lo_cursor_row", "lo_cursor_col", "lo_log_len"):
        getattr(lib, name).restype = i64
        getattr(lib, name).argtypes = [vp]
    lib.lo_done.restype = i32
    lib.lo_done.argtypes = [vp]
    for name in ("lo_min_accepted", "lo_max_rejected"):
        getattr(lib, name).restype = dbl
        getattr(lib, name).argtypes = [vp]
    lib.lo_basis.restype = None
    lib.lo_basis.argtypes = [vp, dptr]
    lib.lo_raw_basis.restype = None
    lib.lo_raw_basis.argtypes = [vp, dptr]
    lib.lo_enable_raw.restype = i32
    lib.lo_enable_raw.argtypes = [vp]
    lib.lo_log_copy.restype = None
    lib.lo_log_copy.argtypes = [vp, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    lib.lo_residual_of.restype = dbl
    lib.lo_residual_of.argtypes = [vp, dptr]
    return lib


def load(path: str | None = None) -> ctypes.CDLL:
    """Load the compiled reference, compiling it first if it is not built."""
    global _lib
    if path is not None:
        return _declare(ctypes.CDLL(path))
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        _lib = _declare(ctypes.CDLL(_LIB))
    return _lib


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def ambient_bound(gens: np.ndarray, rel: float = 1e-12) -> int:
    """d^2 - 1 if every generator is traceless (relative to its norm), else d^2."""
    d = gens.shape[-1]
    for g in gens:
        if abs(np.trace(g)) > rel * max(1.0, np.linalg.norm(g)):
            return d * d
    return d * d - 1


@dataclass
class OracleResult:
    dim: int
    basis: np.ndarray                 # (dim, d, d) complex128, <V_i, V_j> = delta_ij
    candidates: int                   # bracket candidates evaluated
    zero_brackets: int
    generator_checks: int
    accepted_generators: list[int]    # input indices of generators that were appended
    done: bool
    min_accepted: float
    max_rejected: float
    log: dict = field(default_factory=dict)
    raw_basis: np.ndarray | None = None  # Algorithm 3: (dim, d, d) raw elements (generators, brackets)


class Oracle:
    """Stateful reference closure; supports budgeted runs that resume exactly."""

    def __init__(self, gens: np.ndarray, tol: float, *, max_dim: int | None = None, log: bool = False,
                 raw: bool = False, lib: ctypes.CDLL | None = None):
        gens = np.ascontiguousarray(np.asarray(gens, dtype=np.complex128))
        if gens.ndim != 3 or gens.shape[1] != gens.shape[2]:
            raise ValueError("generators must have shape (n_gen, d, d)")
        self.lib = lib if lib is not None else load()
        self.d = int(gens.shape[1])
        self.tol = float(tol)
        self.ambient = ambient_bound(gens)
        cap = int(max_dim) if max_dim else self.d * self.d
        self._s = self.lib.lo_new(self.d, cap, self.tol, 1 if log else 0)
        if not self._s:
            raise MemoryError("oracle allocation failed")
        self.raw = bool(raw)
        if self.raw and self.lib.lo_enable_raw(self._s) != 0:
            raise MemoryError("oracle allocation failed (raw basis)")
        self.accepted_generators = []
        for i, g in enumerate(gens):
            buf = np.ascontiguousarray(g).view(np.float64).reshape(-1)
            r = ctypes.c_double(0.0)
            rc = self.lib.lo_generator(self._s, _dptr(buf), ctypes.byref(r))
            if rc < 0:
                raise RuntimeError("oracle basis full during the generator phase")
            if rc == 1:
                self.accepted_generators.append(i)

    def __del__(self):
        s = getattr(self, "_s", None)
        if s:
            self.lib.lo_free(s)
            self._s = None

    def run(self, *, early_exit: bool = False, budget: int = -1) -> int:
        n = self.lib.lo_brackets(self._s, 1 if early_exit else 0, self.ambient, int(budget))
        if n < 0:
            raise RuntimeError("oracle basis reached its capacity")
        return int(n)

    @property
    def dim(self) -> int:
        return int(self.lib.lo_dim(self._s))

    @property
    def done(self) -> bool:
        return bool(self.lib.lo_done(self._s))

    @property
    def candidates(self) -> int:
        """Bracket candidates evaluated so far."""
        return int(self.lib.lo_candidates(self._s))

    def basis(self) -> np.ndarray:
        n = self.dim
        out = np.empty((n, self.d, self.d), dtype=np.complex128)
        if n:
            self.lib.lo_basis(self._s, _dptr(out.view(np.float64).reshape(-1)))
        return out

    def raw_basis(self) -> np.ndarray | None:
        """Algorithm 3's raw elements B (accepted generators and brackets, unnormalised)."""
        if not self.raw:
            return None
        n = self.dim
        out = np.empty((n, self.d, self.d), dtype=np.complex128)
        if n:
            self.lib.lo_raw_basis(self._s, _dptr(out.view(np.float64).reshape(-1)))
        return out

    def residual_of(self, x: np.ndarray) -> float:
        buf = np.ascontiguousarray(np.asarray(x, dtype=np.complex128)).view(np.float64).reshape(-1)
        return float(self.lib.lo_residual_of(self._s, _dptr(buf)))

    def cursor(self) -> tuple[int, int]:
        return int(self.lib.lo_cursor_row(self._s)), int(self.lib.lo_cursor_col(self._s))

    def log(self) -> dict:
        n = int(self.lib.lo_log_len(self._s))
        out = {
            "l": np.empty(n, dtype=np.int32),
            "m": np.empty(n, dtype=np.int32),
            "r": np.empty(n, dtype=np.float64),
            "acc": np.empty(n, dtype=np.int8),
        }
        if n:
            self.lib.lo_log_copy(self._s, out["l"].ctypes.data, out["m"].ctypes.data,
                                 out["r"].ctypes.data, out["acc"].ctypes.data)
        return out

    def result(self) -> OracleResult:
        return OracleResult(
            dim=self.dim,
            basis=self.basis(),
            candidates=int(self.lib.lo_candidates(self._s)),
            zero_brackets=int(self.lib.lo_zero_brackets(self._s)),
            generator_checks=int(self.lib.lo_generator_checks(self._s)),
            accepted_generators=list(self.accepted_generators),
            done=self.done,
            min_accepted=float(self.lib.lo_min_accepted(self._s)),
            max_rejected=float(self.lib.lo_max_rejected(self._s)),
            log=self.log(),
            raw_basis=self.raw_basis(),
        )


def closure(gens: np.ndarray, tol: float, *, early_exit: bool = False, max_dim: int | None = None,
            log: bool = False, raw: bool = False, lib: ctypes.CDLL | None = None) -> OracleResult:
    """Run the reference closure to completion and return its result (raw=True: Algorithm 3)."""
    o = Oracle(gens, tol, max_dim=max_dim, log=log, raw=raw, lib=lib)
    o.run(early_exit=early_exit)
    return o.result()
