"""GPU: the standard algorithm with the SVD rank test (the comparison baseline).

It brackets raw elements in the same order as Algorithm 3, so with clean
independence gaps both take the same decisions: the dimension, the candidate
count and the raw basis B must equal the CPU reference's Algorithm 3 mode.
"""
from __future__ import annotations

import numpy as np
import pytest

from oracle import oracle as O
from paper_2506_01120_amd import LieClosure, LieError, workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.fail("no GPU visible to torch")


CASES = {
    "ising3": (lambda: W.ising(3), 15),
    "pair4": (lambda: W.rand_pair(4, seed=11), 15),
    "pair6": (lambda: W.rand_pair(6, seed=9), 35),
    "xxyy4": (lambda: W.xxyy(4), 6),
    "pauli3x4": (lambda: W.pauli_set(3, 4, 5), None),
}


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("early_exit", [False, True])
def test_rank_svd_matches_reference(case, early_exit):
    make, expected = CASES[case]
    g = make()
    ref = O.closure(g, 1e-10, raw=True, early_exit=early_exit)
    print(f"[gpu] rank_svd {case} early_exit={early_exit}", flush=True)
    with LieClosure(g, 1e-10, method="rank_svd", early_exit=early_exit) as lc:
        lc.run()
        dim, b, st = lc.dim, lc.raw_basis(), lc.stats()
    assert dim == ref.dim
    if expected is not None:
        assert dim == expected
    assert st["candidates"] == ref.candidates and st["done"] == 1
    for k in range(dim):
        scale = max(1e-300, float(np.max(np.abs(ref.raw_basis[k]))))
        assert np.max(np.abs(b[k] - ref.raw_basis[k])) <= 1e-10 * scale, k


def test_rank_svd_budget_resume():
    g = W.rand_pair(6, seed=9)
    with LieClosure(g, 1e-10, method="rank_svd") as full:
        full.run()
        want = full.raw_basis()
    with LieClosure(g, 1e-10, method="rank_svd") as lc:
        while not lc.run(budget=50):
            pass
        got = lc.raw_basis()
    assert got.shape == want.shape and np.array_equal(got, want)


def test_rank_svd_errors():
    with LieClosure(W.ising(2), 1e-10, method="rank_svd") as lc:
        lc.run()
        with pytest.raises(LieError):
            lc.basis()
        with pytest.raises(LieError):
            lc.orthogonality()
    with pytest.raises(LieError):
        LieClosure(W.rand_pair(32, seed=1), 1e-10, method="rank_svd")
