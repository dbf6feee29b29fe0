"""GPU: the allocation-free orthogonality report against the allocating one.

lie_closure_orthogonality_noalloc forms the Gram matrix of the basis in row panels inside
the library's fixed per-device workspace; lie_closure_orthogonality allocates a full n x n
Gram matrix per call.  Both sum the same FP64 squares (in a different order), so their
values agree to a few units of rounding of the sum.  Two calls in a row on one device,
the second on a smaller basis, check that the shared workspace carries nothing over, and
every value is also checked against ||Q^H Q - I||_F formed by numpy from the host basis.
"""
from __future__ import annotations

import numpy as np
import pytest

import pins
from paper_2506_01120_amd import LieClosure, workloads as W

pytestmark = pytest.mark.gpu


def _noalloc(lc):
    import torch

    out = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    lc.orthogonality_noalloc(out)
    torch.cuda.synchronize()
    return float(out.item())


def _check(lc, d):
    ref = lc.orthogonality()
    got = _noalloc(lc)
    npv = pins.orthonormality_loss(lc.basis())
    print(f"[noalloc] d={d} dim={lc.dim}: noalloc {got:.6e} alloc {ref:.6e} numpy {npv:.6e}", flush=True)
    assert np.isfinite(got)
    assert abs(got - ref) <= 1e-9 * ref + 1e-18, (got, ref)
    assert abs(got - npv) <= 0.1 * npv + 1e-13, (got, npv)
    return got


def test_noalloc_orthogonality_two_calls_second_smaller():
    print("[noalloc] su(32), then su(8)", flush=True)
    with LieClosure(W.rand_pair(32, seed=3), 1e-8, precision="bf16x3") as big:
        big.run()
        assert big.dim == 1023
        a = _check(big, 32)
    with LieClosure(W.rand_pair(8, seed=11), 1e-10) as small:
        small.run()
        assert small.dim == 63
        b = _check(small, 8)
    assert a <= 1e-10 and b <= 1e-10


def test_noalloc_orthogonality_after_generator_phase_only():
    """A handle whose bracket loop has not run: the basis holds only the generators."""
    with LieClosure(W.ising(3), 1e-10) as lc:
        assert lc.dim == 5
        _check(lc, 8)
