"""GPU parity of the bracket and projection kernels at every range of d, element by element.

The bracket has four kernels by size: d <= 16, 16 < d <= 32 (consecutive candidates grouped
by their shared left operand), 32 < d <= 64 (one candidate per workgroup, operands in LDS)
and d > 64 (16 x 16 tile pairs), each in FP64 and FP32, and the projection GEMMs tile d^2
with ragged edges whenever d is odd or not a power of two.  Every range is compared here with
the CPU reference element by element (<= 1e-8) at sizes it finishes in seconds:

* d = 33: a random traceless pair with early exit (su(33), dim 1088);
* d = 48: the same (su(48), dim 2303; the reference takes about half a minute);
* d = 33, 48, 72, 100: small algebras embedded in d x d and conjugated by a random unitary,
  so every operand is a dense d x d matrix, in full certification.

The screened kernels are checked on the same inputs in the audit mode (decide = "fp64",
fixed blocks, the screen computed on every block): the returned basis must equal the
reference's, and every snapshot-dependent candidate must screen below the precision's
threshold while every independent one screens above it -- a wrong screened bracket or
projection shows up in one of the two.
"""
from __future__ import annotations

import numpy as np
import pytest

import pins
from oracle import oracle as O
from paper_2506_01120_amd import LieClosure, workloads as W

pytestmark = pytest.mark.gpu

ELEM_TOL = 1e-8
TAU = {"fp32": 1e-4, "bf16x3": 1e-2}

_REF = {}


def reference(key, gens, tol, early_exit):
    if key not in _REF:
        print(f"[ref] {key}", flush=True)
        _REF[key] = O.closure(gens, tol, early_exit=early_exit)
    return _REF[key]


def gpu_run(gens, tol, **cfg):
    print(f"[gpu] d={gens.shape[-1]} n_gen={len(gens)} tol={tol} cfg={cfg}", flush=True)
    with LieClosure(gens, tol, **cfg) as lc:
        lc.run()
        return lc.dim, lc.basis(), lc.stats(), lc.orthogonality()


CASES = {
    "pair33_early": (lambda: W.rand_pair(33, seed=103), 1e-8, True, 1088),
    "pair48_early": (lambda: W.rand_pair(48, seed=118), 1e-8, True, 2303),
    "ising3_at_33": (lambda: W.embed(W.ising(3), 33, seed=33), 1e-10, False, 15),
    "pair6_at_48": (lambda: W.embed(W.rand_pair(6, seed=16), 48, seed=48), 1e-10, False, 35),
    "ising3_at_72": (lambda: W.embed(W.ising(3), 72, seed=72), 1e-10, False, 15),
    "pair6_at_100": (lambda: W.embed(W.rand_pair(6, seed=16), 100, seed=100), 1e-10, False, 35),
}

_GENS = {}


def case(name):
    make, tol, early, dim = CASES[name]
    if name not in _GENS:
        _GENS[name] = make()
    gens = _GENS[name]
    return gens, tol, early, dim, reference(name, gens, tol, early)


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("block", [0, 97])
def test_fp64_ranges(name, block):
    gens, tol, early, want, ref = case(name)
    dim, v, st, orth = gpu_run(gens, tol, early_exit=early, block=block)
    assert dim == ref.dim == want
    if not early:
        assert st["candidates"] == ref.candidates
    assert np.max(np.abs(v - ref.basis)) <= ELEM_TOL
    assert orth <= 1e-10


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_screened_ranges_audit(name, precision):
    gens, tol, early, want, ref = case(name)
    dim, v, st, orth = gpu_run(gens, tol, early_exit=early, precision=precision, decide="fp64", block=256)
    assert dim == ref.dim == want
    assert np.max(np.abs(v - ref.basis)) <= ELEM_TOL
    assert orth <= 1e-10
    print("screen margin:", name, precision, st["screen_max_dependent"], st["screen_min_independent"])
    assert st["screen_max_dependent"] < TAU[precision] < st["screen_min_independent"]


@pytest.mark.parametrize("name", ["pair33_early", "pair6_at_48", "pair6_at_100"])
@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_screened_ranges_certified(name, precision):
    """The default (certified) screen, adaptive blocks: the reference's basis."""
    gens, tol, early, want, ref = case(name)
    dim, v, st, orth = gpu_run(gens, tol, early_exit=early, precision=precision, decide="screen")
    assert dim == ref.dim == want
    assert np.max(np.abs(v - ref.basis)) <= ELEM_TOL


def test_embedded_spans_closed_form():
    """The embedded Ising chain spans the conjugated so(6): a check that needs no reference."""
    gens = W.embed(W.ising(3), 72, seed=72)
    dim, v, _, _ = gpu_run(gens, 1e-10)
    assert dim == 15
    u_small = W.ising(3)
    _, v8, _, _ = gpu_run(u_small, 1e-10)
    # conjugate the d = 8 basis into the d = 72 frame and compare spans
    big = W.embed(v8, 72, seed=72)
    big = big * np.sqrt(72 / 8)  # unit norm in the d = 72 inner product
    assert pins.span_distance(v, big) <= 1e-8
