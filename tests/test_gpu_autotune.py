"""GPU: the autotuner's choices are admissible, cached, and leave the results unchanged.

The tuner times the saturated block step's projection GEMMs at init; whatever it
picks, the closure must still match the CPU reference (dims exact, spans within
the FP64 / mixed bars).
"""
from __future__ import annotations

import pytest

import pins
from oracle import oracle as O
from paper_2506_01120_amd import LieClosure, workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.fail("no GPU visible to torch")


@pytest.mark.parametrize("precision,span_tol", [("fp64", 1e-8), ("fp32", 1e-5), ("bf16x3", 1e-5)])
def test_autotuned_su16_matches_reference(tmp_path, precision, span_tol):
    gens = W.rand_pair(16, seed=2)
    ref = O.closure(gens, 1e-10)
    cache = tmp_path / "tune.txt"
    print(f"[gpu] autotune su16 {precision}", flush=True)
    with LieClosure(gens, 1e-10, precision=precision, autotune=True, tune_cache=str(cache)) as lc:
        lc.run()
        st = lc.stats()
        dim, v = lc.dim, lc.basis()
    assert dim == ref.dim == 255 and st["candidates"] == ref.candidates
    assert pins.span_distance(v, ref.basis) <= span_tol
    assert st["autotuned"] in (1, 2)
    assert -st["block"] in (1024, 2048, 4096, 8192, 16384)
    if precision == "fp64":
        assert st["tile_dot"] == st["tile_sub"] == 0
    else:
        assert st["tile_dot"] in (1, 2) and st["tile_sub"] in (1, 2)
    # a second handle of the same shape reuses the choice without timing
    with LieClosure(gens, 1e-10, precision=precision, autotune=True, tune_cache=str(cache)) as lc2:
        st2 = lc2.stats()
    assert st2["autotuned"] == 2
    assert (st2["block"], st2["tile_dot"], st2["tile_sub"]) == (st["block"], st["tile_dot"], st["tile_sub"])


def test_tune_cache_file_format(tmp_path):
    cache = tmp_path / "tune.txt"
    gens = W.rand_pair(8, seed=21)
    print("[gpu] autotune cache file d=8", flush=True)
    with LieClosure(gens, 1e-10, precision="fp32", autotune=True, tune_cache=str(cache)) as lc:
        st = lc.stats()
    if st["autotuned"] == 1:  # timed in this process: the line was appended
        lines = cache.read_text().splitlines()
        assert len(lines) == 1 and lines[0].startswith("lie-tune v2 arch=")
        assert " precision=1 d=8 ambient=63 " in lines[0]
        assert f"block_sat={-st['block']} tile_dot={st['tile_dot']} tile_sub={st['tile_sub']}" in lines[0]


def test_autotuned_su32_early_exit_screened():
    gens = W.rand_pair(32, seed=3)
    ref = O.closure(gens, 1e-8, early_exit=True)
    print("[gpu] autotune su32 early exit fp32", flush=True)
    with LieClosure(gens, 1e-8, precision="fp32", early_exit=True, autotune=True) as lc:
        lc.run()
        dim, v = lc.dim, lc.basis()
    assert dim == ref.dim == 1023
    assert pins.su_span_distance(v) <= 1e-5
