"""GPU closures at the full sizes of the benchmark configurations, checked by properties.

The oracle finishes su(16) in seconds (its parity tests compare element by element), but
not su(32) in full certification or su(64).  At these sizes the results are checked by
what holds at any size:

* the dimension equals the closed form d^2 - 1 of a generic traceless pair;
* in full certification every unordered pair of the final basis was decided exactly
  once, N(N-1)/2 candidates;
* the span is su(d): for dim V = d^2 - 1 elements that are anti-Hermitian by
  construction, ||P_V - P_su||_F = sqrt(2 sum_k |tr V_k / d|^2) (the traces vanish);
* the basis is orthonormal in the paper's inner product, ||V^H V - I||_F.

The runs use the launch configuration of the benchmark (adaptive blocks, graph replay;
the autotuner where the benchmark table uses it).
"""
from __future__ import annotations

import pytest

import pins
from paper_2506_01120_amd import LieClosure, workloads as W

pytestmark = pytest.mark.gpu

SPAN_TOL_FP64 = 1e-8
SPAN_TOL_MIXED = 1e-8  # screened runs keep only FP64-recomputed rows: the FP64 bar


def closure(d, seed, tol, **cfg):
    print(f"[gpu] su({d}) seed={seed} tol={tol} cfg={cfg}", flush=True)
    with LieClosure(W.rand_pair(d, seed=seed), tol, **cfg) as lc:
        lc.run()
        return lc.dim, lc.basis(), lc.stats(), lc.orthogonality()


def check(dim, v, st, orth, d, full, span_tol, orth_tol):
    assert dim == d * d - 1
    assert st["done"] == 1
    if full:
        assert st["candidates"] == dim * (dim - 1) // 2
    assert pins.su_span_distance(v) <= span_tol
    assert orth <= orth_tol


@pytest.mark.parametrize("precision,decide", [("fp64", "fp64"), ("fp32", "screen"), ("bf16x3", "screen")])
def test_su32_full_certification(precision, decide):
    """d = 32 (seed 3), tol 1e-8: 522,753 brackets, dim 1023."""
    dim, v, st, orth = closure(32, 3, 1e-8, precision=precision, decide=decide)
    check(dim, v, st, orth, 32, True, SPAN_TOL_FP64 if precision == "fp64" else SPAN_TOL_MIXED, 1e-10)


@pytest.mark.parametrize("tile", [1, 2])
def test_su32_bf16_tiles(tile):
    """d = 32 (seed 3), tol 1e-8, split-BF16 screen with each workgroup tile of the screening GEMMs."""
    dim, v, st, orth = closure(32, 3, 1e-8, precision="bf16x3", decide="screen", gemm_tile=tile)
    check(dim, v, st, orth, 32, True, SPAN_TOL_MIXED, 1e-10)
    assert st["tile_dot"] == tile and st["tile_sub"] == tile


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_su64_early_exit(precision):
    """d = 64 (seed 5), tol 1e-8, stopped at the ambient bound 4095."""
    dim, v, st, orth = closure(64, 5, 1e-8, precision=precision, decide="screen", early_exit=True)
    check(dim, v, st, orth, 64, False, SPAN_TOL_MIXED, 1e-9)


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_su64_full_certification(precision):
    """d = 64 (seed 5), tol 1e-8: 8,382,465 brackets, dim 4095, autotuned as benchmarked."""
    dim, v, st, orth = closure(64, 5, 1e-8, precision=precision, decide="screen", autotune=True)
    check(dim, v, st, orth, 64, True, SPAN_TOL_MIXED, 1e-9)
