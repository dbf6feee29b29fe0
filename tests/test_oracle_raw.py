"""Pins of the CPU reference's Algorithm 3 mode (raw basis B kept alongside V).

Algorithm 3 brackets the raw elements -- the accepted generators and accepted
brackets themselves -- and tests each bracket against the span of the accepted
candidates.  Checked against: closed-form dimensions, the hand-derived su(2)
example, the span of V, the bracket structure of B (recomputed with numpy), and
the scale invariance that the relative threshold gives.
"""
from __future__ import annotations

import numpy as np
import pytest

import pins
from oracle import oracle as O
from paper_2506_01120_amd import workloads as W

PAULI = {
    "I": np.eye(2, dtype=np.complex128),
    "X": np.array([[0, 1], [1, 0]], dtype=np.complex128),
    "Y": np.array([[0, -1j], [1j, 0]], dtype=np.complex128),
    "Z": np.array([[1, 0], [0, -1]], dtype=np.complex128),
}


def test_su2_worked_example():
    """iX, iY: the only pair is (l, m) = (1, 0), so B = (iX, iY, [iY, iX] = 2iZ) and
    V = (iX, iY, iZ); dim 3."""
    g = np.stack([1j * PAULI["X"], 1j * PAULI["Y"]])
    r = O.closure(g, 1e-10, raw=True)
    assert r.dim == 3 and r.candidates == 3
    assert np.allclose(r.raw_basis[0], 1j * PAULI["X"], atol=0)
    assert np.allclose(r.raw_basis[1], 1j * PAULI["Y"], atol=0)
    assert np.allclose(r.raw_basis[2], 2j * PAULI["Z"], atol=1e-15)
    assert np.allclose(r.basis[2], 1j * PAULI["Z"], atol=1e-15)


@pytest.mark.parametrize("make,expected", [
    (lambda: W.ising(3), 15), (lambda: W.ising(4), 28), (lambda: W.xxyy(4), 6),
    (lambda: W.rand_pair(8, seed=1), 63), (lambda: W.rand_pair(6, seed=9), 35),
])
def test_closed_form_dims_and_span(make, expected):
    g = make()
    r = O.closure(g, 1e-10, raw=True)
    r4 = O.closure(g, 1e-10)
    assert r.dim == r4.dim == expected
    # B spans the closure: its orthonormalised span equals V's, and V's equals Algorithm 4's
    assert pins.span_distance(r.raw_basis, r.basis) <= 1e-9
    assert pins.span_distance(r.basis, r4.basis) <= 1e-9
    assert pins.orthonormality_loss(r.basis) <= 1e-12


@pytest.mark.parametrize("make", [lambda: W.ising(3), lambda: W.rand_pair(6, seed=3), lambda: W.pauli_set(3, 4, 5)])
def test_raw_elements_are_generators_or_brackets(make):
    """B starts with the accepted generators verbatim; each later B_k = [B_l, B_m] for the
    accepted candidate (l, m) of the log, recomputed here with numpy products."""
    g = make()
    o = O.Oracle(g, 1e-10, raw=True, log=True)
    o.run()
    r = o.result()
    ng = len(r.accepted_generators)
    for k, i in enumerate(r.accepted_generators):
        assert np.array_equal(r.raw_basis[k], g[i])
    acc = np.flatnonzero(r.log["acc"] == 1)
    assert len(acc) == r.dim - ng
    for k, idx in enumerate(acc, start=ng):
        l, m = int(r.log["l"][idx]), int(r.log["m"][idx])
        assert m < l < k
        a, b = r.raw_basis[l], r.raw_basis[m]
        want = a @ b - b @ a
        assert np.max(np.abs(r.raw_basis[k] - want)) <= 1e-13 * max(1.0, np.max(np.abs(want)))


@pytest.mark.parametrize("scale", [1e-3, 1e3])
def test_relative_threshold_scale_invariance(scale):
    """Scaling the generators by c scales a depth-k raw bracket by c^(k+1); the relative
    threshold keeps every decision unchanged (an absolute one would not)."""
    g = W.ising(3)
    a = O.Oracle(g, 1e-10, raw=True, log=True)
    a.run()
    b = O.Oracle(g * scale, 1e-10, raw=True, log=True)
    b.run()
    assert a.dim == b.dim == 15
    assert np.array_equal(a.log()["acc"], b.log()["acc"])


def test_early_exit_and_budget_resume():
    g = W.rand_pair(6, seed=3)
    full = O.closure(g, 1e-10, raw=True, early_exit=True)
    assert full.dim == 35
    o = O.Oracle(g, 1e-10, raw=True)
    while not o.done:
        o.run(early_exit=True, budget=7)
    r = o.result()
    assert r.dim == full.dim and r.candidates == full.candidates
    assert np.array_equal(r.raw_basis, full.raw_basis)
