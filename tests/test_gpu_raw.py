"""GPU parity of Algorithm 3 (config.raw_basis): the raw basis B and V against the CPU
reference's Algorithm 3 mode, through the C ABI.

Both sides bracket raw elements [B_l, B_m] in the same order and take the same
decisions, so B agrees element by element (to rounding, relative to each element's
scale) and V as in Algorithm 4's parity.
"""
from __future__ import annotations

import numpy as np
import pytest

import pins
from oracle import oracle as O
from paper_2506_01120_amd import BatchClosure, LieClosure, LieError, workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.fail("no GPU visible to torch")


def raw_closure(gens, tol, **cfg):
    print(f"[gpu] raw d={gens.shape[-1]} n_gen={len(gens)} tol={tol} cfg={cfg}", flush=True)
    with LieClosure(gens, tol, raw_basis=True, **cfg) as lc:
        lc.run()
        return lc.dim, lc.basis(), lc.raw_basis(), lc.stats(), lc.orthogonality()


def assert_raw_parity(gens, tol, *, early_exit=False, span_tol=1e-8, elem=True, expected=None, **cfg):
    ref = O.closure(gens, tol, raw=True, early_exit=early_exit)
    dim, v, b, st, orth = raw_closure(gens, tol, early_exit=early_exit, **cfg)
    assert dim == ref.dim, (dim, ref.dim)
    if expected is not None:
        assert dim == expected
    if not early_exit:
        assert st["candidates"] == ref.candidates
    assert pins.span_distance(v, ref.basis) <= span_tol
    assert orth <= 1e-10
    # B spans the closure
    assert pins.span_distance(b, v) <= span_tol * 10
    if elem:
        for k in range(dim):
            scale = max(1e-300, float(np.max(np.abs(ref.raw_basis[k]))))
            assert np.max(np.abs(b[k] - ref.raw_basis[k])) <= 1e-8 * scale, k
        assert np.max(np.abs(v - ref.basis)) <= 1e-8
    return dim, b


@pytest.mark.parametrize("block", [0, 1, 7])
def test_raw_ising3(block):
    assert_raw_parity(W.ising(3), 1e-10, block=block, expected=15)


@pytest.mark.parametrize("case", ["pair6", "ising4", "xxyy4", "pauli4x5"])
def test_raw_small_fp64(case):
    make, expected = {
        "pair6": (lambda: W.rand_pair(6, seed=9), 35),
        "ising4": (lambda: W.ising(4), 28),
        "xxyy4": (lambda: W.xxyy(4), 6),
        "pauli4x5": (lambda: W.pauli_set(4, 5, 10), None),
    }[case]
    assert_raw_parity(make(), 1e-10, expected=expected)


def test_raw_su8_early_exit():
    assert_raw_parity(W.rand_pair(8, seed=1), 1e-10, early_exit=True, expected=63)


def test_raw_scale_invariance():
    """The relative threshold keeps decisions when all generators are scaled by 1e-3."""
    g = W.ising(3)
    d1, b1 = assert_raw_parity(g, 1e-10, expected=15)
    d2, b2 = assert_raw_parity(g * 1e-3, 1e-10, expected=15)
    assert d1 == d2


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_raw_screened(precision):
    """Screened brackets of raw elements (relative screen policy), FP64 decisions of survivors."""
    assert_raw_parity(W.rand_pair(8, seed=1), 1e-10, precision=precision, span_tol=1e-5, elem=False, expected=63)
    assert_raw_parity(W.ising(4), 1e-10, precision=precision, span_tol=1e-5, elem=False, expected=28)


def test_raw_errors():
    with LieClosure(W.ising(2), 1e-10) as lc:
        lc.run()
        with pytest.raises(LieError):
            lc.raw_basis()
    with pytest.raises(LieError):
        BatchClosure([W.ising(2), W.ising(3)], 1e-10, raw_basis=True)
