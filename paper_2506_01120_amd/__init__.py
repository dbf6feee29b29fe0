"""MI355X-native Lie-closure engine (arXiv 2506.01120, dimension-only orthonormalization).

The Python layer only marshals arguments to the C ABI of ``liblieclosure.so``;
every step of the closure runs in the library's HIP kernels.  PyTorch, when
used, only supplies device memory (``basis_device``) and a HIP stream.

    >>> from paper_2506_01120_amd import LieClosure, workloads
    >>> lc = LieClosure(workloads.ising(3), tol=1e-10)
    >>> lc.run(); lc.dim
    15
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import _lib
from ._lib import LieError

__all__ = ["LieClosure", "BatchClosure", "PauliSparseClosure", "closure", "LieError", "make_config", "pauli_key"]


def make_config(*, precision: str = "fp64", decide: str = "screen", block: int = 0, early_exit: bool = False,
                tau_rej: float = 0.0, max_dim: int = 0, stream=None, device: int | None = None,
                use_graphs: bool = True, profile: bool = False, autotune: bool = False,
                tune_cache: str | None = None, raw_basis: bool = False,
                method: str = "orthonormalization", representation: str = "dense",
                gemm_tile: int = 0) -> _lib.Config:
    cfg = _lib.Config()
    _lib.check(_lib.load().lie_closure_config_default(ctypes.byref(cfg)))
    cfg.precision = _lib.PRECISIONS[precision]
    cfg.decide = _lib.DECIDES[decide]
    cfg.block = int(block)
    cfg.early_exit = 1 if early_exit else 0
    cfg.tau_rej = float(tau_rej)
    cfg.max_dim = int(max_dim)
    cfg.device = -1 if device is None else int(device)
    cfg.use_graphs = 1 if use_graphs else 0
    cfg.profile = 1 if profile else 0
    cfg.autotune = 1 if autotune else 0
    cfg.raw_basis = 1 if raw_basis else 0
    cfg.method = {"orthonormalization": 0, "rank_svd": 1, "matrix_inversion": 2}[method]
    cfg.representation = {"dense": 0, "pauli": 1}[representation]
    cfg.gemm_tile = int(gemm_tile)
    # the bytes object must outlive the init call that reads it; the Config keeps it
    cfg._tune_cache_bytes = None if tune_cache is None else os.fsencode(tune_cache)
    cfg.tune_cache = cfg._tune_cache_bytes
    if stream is not None:
        cfg.stream = int(getattr(stream, "cuda_stream", stream))
    return cfg


def _host_generators(generators) -> np.ndarray:
    if hasattr(generators, "detach"):  # a torch tensor
        generators = generators.detach().cpu().numpy()
    g = np.ascontiguousarray(np.asarray(generators, dtype=np.complex128))
    if g.ndim == 2:
        g = g[None]
    if g.ndim != 3 or g.shape[1] != g.shape[2]:
        raise ValueError("generators must have shape (n_gen, d, d)")
    return g


class LieClosure:
    """One closure problem on the GPU.  Wraps lie_closure_init/run/dim/basis/stats/free."""

    def __init__(self, generators, tol: float, **config):
        self._libh = _lib.load()
        g = _host_generators(generators)
        self.d = int(g.shape[1])
        self.n_gen = int(g.shape[0])
        self.tol = float(tol)
        self._cfg = make_config(**config)
        self._gens = g  # kept alive only for the duration of init (the library copies)
        h = ctypes.c_void_p()
        _lib.check(self._libh.lie_closure_init(ctypes.byref(h), g.ctypes.data, self.n_gen, self.d, self.tol,
                                               ctypes.byref(self._cfg)))
        self._h = h
        self._gens = None

    def close(self) -> None:
        h = getattr(self, "_h", None)
        if h:
            self._libh.lie_closure_free(h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def run(self, budget: int | None = None) -> bool:
        """Run the bracket loop; with ``budget`` at most that many candidates.  Returns True when complete."""
        if budget is None:
            _lib.check(self._libh.lie_closure_run(self._h))
            return True
        st = _lib.check(self._libh.lie_closure_run_budget(self._h, int(budget)), allow_incomplete=True)
        return st == _lib.LIE_OK

    @property
    def dim(self) -> int:
        n = ctypes.c_int64()
        _lib.check(self._libh.lie_closure_dim(self._h, ctypes.byref(n)))
        return int(n.value)

    def basis(self) -> np.ndarray:
        """V as a host complex128 array (dim, d, d), in append order, <V_i, V_j> = delta_ij."""
        n = self.dim
        out = np.empty((max(n, 1), self.d, self.d), dtype=np.complex128)
        w = ctypes.c_int64()
        _lib.check(self._libh.lie_closure_basis(self._h, out.ctypes.data, n, ctypes.byref(w)))
        return out[: w.value]

    def raw_basis(self) -> np.ndarray:
        """Algorithm 3's raw basis B (dim, d, d): accepted generators and nested brackets,
        unnormalised, in append order (handle created with raw_basis=True)."""
        n = self.dim
        out = np.empty((max(n, 1), self.d, self.d), dtype=np.complex128)
        w = ctypes.c_int64()
        _lib.check(self._libh.lie_closure_raw_basis(self._h, out.ctypes.data, n, ctypes.byref(w)))
        return out[: w.value]

    def basis_device(self):
        """V as a torch complex128 CUDA tensor (dim, d, d) written by the library."""
        import torch

        n = self.dim
        out = torch.empty((max(n, 1), self.d, self.d), dtype=torch.complex128, device="cuda")
        w = ctypes.c_int64()
        _lib.check(self._libh.lie_closure_basis_device(self._h, ctypes.c_void_p(out.data_ptr()), n, ctypes.byref(w)))
        return out[: w.value]

    def orthogonality(self) -> float:
        """||G - I||_F, G_ij = <V_i, V_j>, computed in FP64 on the GPU."""
        x = ctypes.c_double()
        _lib.check(self._libh.lie_closure_orthogonality(self._h, ctypes.byref(x)))
        return float(x.value)

    def orthogonality_noalloc(self, out) -> None:
        """Enqueue ||G - I||_F into `out` (a one-element float64 tensor on the handle's
        device) without allocating; the value is there once the handle's stream has run."""
        _lib.check(self._libh.lie_closure_orthogonality_noalloc(self._h, ctypes.c_void_p(out.data_ptr())))

    def stats(self) -> dict:
        s = _lib.Stats()
        s.struct_size = ctypes.sizeof(_lib.Stats)
        _lib.check(self._libh.lie_closure_stats_get(self._h, ctypes.byref(s)))
        return s.as_dict()


def closure(generators, tol: float, **config):
    """Run a closure to completion; return (dim, basis, stats)."""
    with LieClosure(generators, tol, **config) as lc:
        lc.run()
        return lc.dim, lc.basis(), lc.stats()


class BatchClosure:
    """Many independent closure problems advanced together (lie_closure_batch_*)."""

    def __init__(self, problems, tols, **config):
        self._libh = _lib.load()
        gens = [_host_generators(g) for g in problems]
        n = len(gens)
        if np.isscalar(tols):
            tols = [float(tols)] * n
        self.ds = [int(g.shape[1]) for g in gens]
        ptrs = (ctypes.c_void_p * n)(*[g.ctypes.data for g in gens])
        ngen = (ctypes.c_int32 * n)(*[int(g.shape[0]) for g in gens])
        dd = (ctypes.c_int32 * n)(*self.ds)
        tt = (ctypes.c_double * n)(*[float(t) for t in tols])
        self._cfg = make_config(**config)
        h = ctypes.c_void_p()
        _lib.check(self._libh.lie_closure_batch_init(ctypes.byref(h), n, ptrs, ngen, dd, tt, ctypes.byref(self._cfg)))
        self._h = h
        self.n = n

    def close(self) -> None:
        h = getattr(self, "_h", None)
        if h:
            self._libh.lie_closure_batch_free(h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def run(self) -> None:
        _lib.check(self._libh.lie_closure_batch_run(self._h))

    def dim(self, i: int) -> int:
        n = ctypes.c_int64()
        _lib.check(self._libh.lie_closure_batch_dim(self._h, i, ctypes.byref(n)))
        return int(n.value)

    def basis(self, i: int) -> np.ndarray:
        n = self.dim(i)
        d = self.ds[i]
        out = np.empty((max(n, 1), d, d), dtype=np.complex128)
        w = ctypes.c_int64()
        _lib.check(self._libh.lie_closure_batch_basis(self._h, i, out.ctypes.data, n, ctypes.byref(w)))
        return out[: w.value]

    def stats(self, i: int) -> dict:
        s = _lib.Stats()
        s.struct_size = ctypes.sizeof(_lib.Stats)
        _lib.check(self._libh.lie_closure_batch_stats_get(self._h, i, ctypes.byref(s)))
        return s.as_dict()


def pauli_key(label: str) -> int:
    """64-bit key (x << 32) | z of a Pauli-string label such as "XIZY" (qubit 0 leftmost,
    the most significant bit of the basis index): X sets x, Z sets z, Y sets both."""
    n = len(label)
    x = z = 0
    for q, c in enumerate(label):
        b = 1 << (n - 1 - q)
        if c in "XY":
            x |= b
        if c in "ZY":
            z |= b
        if c not in "IXYZ":
            raise ValueError(f"not a Pauli label: {label!r}")
    return (x << 32) | z


def pauli_label(key: int, n: int) -> str:
    """Inverse of :func:`pauli_key` for n qubits."""
    x, z = key >> 32, key & 0xFFFFFFFF
    out = []
    for q in range(n):
        b = 1 << (n - 1 - q)
        out.append("Y" if (x & b and z & b) else "X" if x & b else "Z" if z & b else "I")
    return "".join(out)


class PauliSparseClosure:
    """A closure problem in the sparse Pauli-sum representation (lie_closure_init_pauli_sparse).

    ``generators`` is a list of dicts {label: c}, the generator being sum c iP_label with
    real c.  ``basis()`` returns the basis as a list of such dicts, in Algorithm 4's order."""

    def __init__(self, n_qubits: int, generators, tol: float, max_terms: int = 0, **config):
        self._libh = _lib.load()
        self.n = int(n_qubits)
        offs, keys, coefs = [0], [], []
        for g in generators:
            for label, c in g.items():
                if len(label) != self.n:
                    raise ValueError(f"label {label!r} is not on {self.n} qubits")
                keys.append(pauli_key(label))
                coefs.append(float(c))
            offs.append(len(keys))
        self._offs = np.asarray(offs, dtype=np.int64)
        self._keys = np.asarray(keys, dtype=np.uint64)
        self._coefs = np.asarray(coefs, dtype=np.float64)
        self._cfg = make_config(**config)
        h = ctypes.c_void_p()
        _lib.check(self._libh.lie_closure_init_pauli_sparse(
            ctypes.byref(h), self.n, len(generators), self._offs.ctypes.data, self._keys.ctypes.data,
            self._coefs.ctypes.data, float(tol), int(max_terms), ctypes.byref(self._cfg)))
        self._h = h

    def close(self) -> None:
        h = getattr(self, "_h", None)
        if h:
            self._libh.lie_closure_free(h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def run(self, budget: int | None = None) -> bool:
        """Run the bracket loop (to completion, or at most `budget` candidates); True when complete."""
        if budget is None:
            _lib.check(self._libh.lie_closure_run(self._h))
            return True
        st = _lib.check(self._libh.lie_closure_run_budget(self._h, int(budget)), allow_incomplete=True)
        return st == 0

    @property
    def dim(self) -> int:
        n = ctypes.c_int64()
        _lib.check(self._libh.lie_closure_dim(self._h, ctypes.byref(n)))
        return int(n.value)

    def stats(self) -> dict:
        s = _lib.Stats()
        s.struct_size = ctypes.sizeof(_lib.Stats)
        _lib.check(self._libh.lie_closure_stats_get(self._h, ctypes.byref(s)))
        return s.as_dict()

    def basis_arrays(self):
        """(offsets, keys, coefficients) of the basis as numpy arrays."""
        dim = self.dim
        offs = np.zeros(dim + 1, dtype=np.int64)
        w = ctypes.c_int64()
        st = self._libh.lie_closure_basis_pauli_sparse(self._h, offs.ctypes.data, None, None, 0, ctypes.byref(w))
        if st not in (0, -7):
            _lib.check(st)
        keys = np.zeros(max(w.value, 1), dtype=np.uint64)
        coefs = np.zeros(max(w.value, 1), dtype=np.float64)
        _lib.check(self._libh.lie_closure_basis_pauli_sparse(self._h, offs.ctypes.data, keys.ctypes.data,
                                                             coefs.ctypes.data, int(w.value), ctypes.byref(w)))
        return offs, keys[: w.value], coefs[: w.value]

    def basis(self) -> list[dict]:
        offs, keys, coefs = self.basis_arrays()
        return [{pauli_label(int(keys[t]), self.n): float(coefs[t]) for t in range(offs[k], offs[k + 1])}
                for k in range(len(offs) - 1)]

