"""GPU: the sparse Pauli-sum representation (term lists, supports joined) against the CPU
reference and against exact closed forms.

* n <= 6: the dense CPU reference runs the same generators as d x d matrices; the sparse
  basis, expanded to matrices, must equal it element by element, with the same candidate
  count (Ising chains, XX+YY chains, Pauli-string sets, multi-term random Pauli sums).
* n = 8..10 (d = 256..1024, where the dense engine does not go): the Ising chain closes to
  so(2n), dim n(2n - 1); every element is a single Pauli string (+-1), and the set of
  strings equals the exact closure of the generator strings under anticommuting products
  (an independent symplectic computation).  Memory is one 16-byte term per element.
"""
from __future__ import annotations

import numpy as np
import pytest

import pins
from oracle import oracle as O
from paper_2506_01120_amd import LieError, PauliSparseClosure, workloads as W

pytestmark = pytest.mark.gpu


def dense_of(elem: dict, n: int) -> np.ndarray:
    return sum(c * 1j * W.pauli_string(s) for s, c in elem.items())


def run_sparse(n, gens, tol, **cfg):
    print(f"[gpu] sparse pauli n={n} gens={len(gens)} tol={tol} cfg={cfg}", flush=True)
    with PauliSparseClosure(n, gens, tol, **cfg) as pc:
        pc.run()
        return pc.dim, pc.basis(), pc.stats()


def normalised(gens, n):
    """Frobenius-normalised generators (as the dense workloads are): c / sqrt(d sum c^2)."""
    d = 2 ** n
    out = []
    for g in gens:
        s = np.sqrt(d * sum(c * c for c in g.values()))
        out.append({k: v / s for k, v in g.items()})
    return out


CASES = {
    "ising3": (3, lambda: W.ising_terms(3), lambda: W.ising(3), 1e-10),
    "ising5": (5, lambda: W.ising_terms(5), lambda: W.ising(5), 1e-10),
    "ising6": (6, lambda: W.ising_terms(6), lambda: W.ising(6), 1e-10),
    "xxyy5": (5, lambda: W.xxyy_terms(5), lambda: W.xxyy(5), 1e-10),
    "pauli4x5": (4, lambda: W.pauli_set_terms(4, 5, 7), lambda: W.pauli_set(4, 5, 7), 1e-10),
    "sums4": (4, lambda: normalised(W.pauli_sums_terms(4, 2, 3, 3), 4), lambda: W.pauli_sums(4, 2, 3, 3), 1e-10),
    "sums5": (5, lambda: normalised(W.pauli_sums_terms(5, 2, 3, 5), 5), lambda: W.pauli_sums(5, 2, 3, 5), 1e-10),
}


@pytest.mark.parametrize("name", list(CASES))
def test_sparse_matches_reference(name):
    n, sparse_gens, dense_gens, tol = CASES[name]
    g = dense_gens()
    ref = O.closure(g, tol)
    dim, basis, st = run_sparse(n, sparse_gens(), tol)
    assert dim == ref.dim
    assert st["candidates"] == ref.candidates
    v = np.stack([dense_of(e, n) for e in basis])
    assert np.max(np.abs(v - ref.basis)) <= 1e-9
    for e in basis:
        assert abs(sum(c * c for c in e.values()) - 1.0) <= 1e-12


@pytest.mark.parametrize("n", [8, 9, 10])
def test_sparse_ising_large(n):
    gens = W.ising_terms(n)
    dim, basis, st = run_sparse(n, gens, 1e-10)
    assert dim == n * (2 * n - 1)
    assert st["candidates"] == dim * (dim - 1) // 2
    assert all(len(e) == 1 for e in basis)
    assert all(abs(abs(c) - 1.0) <= 1e-12 for e in basis for c in e.values())
    labels = {s for e in basis for s in e}
    assert labels == pins.pauli_closure([next(iter(g)) for g in gens])
    assert st["pauli_terms"] == dim  # one 16-byte term per element
    print(f"ising({n}): dim {dim}, {st['pauli_terms']} terms = {16 * st['pauli_terms']} bytes "
          f"(dense packed FP64 would hold {dim * 4 ** n * 8} bytes)")


def test_sparse_early_exit_and_budget():
    gens = normalised(W.pauli_sums_terms(3, 2, 3, 11), 3)
    with PauliSparseClosure(3, gens, 1e-10) as full:
        full.run()
        want_dim, want = full.dim, full.basis_arrays()
    with PauliSparseClosure(3, gens, 1e-10) as pc:
        while not pc.run(budget=37):
            pass
        got = pc.basis_arrays()
        assert pc.dim == want_dim
    for a, b in zip(got, want):
        assert a.shape == b.shape and np.array_equal(a, b)
    if want_dim == 63:  # su(8): early exit stops at the ambient bound
        with PauliSparseClosure(3, gens, 1e-10, early_exit=True) as pc:
            pc.run()
            assert pc.dim == 63 and pc.stats()["candidates"] < want_dim * (want_dim - 1) // 2


def test_sparse_errors():
    with pytest.raises(LieError):
        PauliSparseClosure(3, [{"XIZ": float("nan")}], 1e-10)
    with pytest.raises(LieError):
        PauliSparseClosure(3, [{"XIZ": 1.0}], 1.5)
    with pytest.raises(LieError):  # the basis outgrows max_dim
        with PauliSparseClosure(3, W.ising_terms(3), 1e-10, max_dim=10) as pc:
            pc.run()
