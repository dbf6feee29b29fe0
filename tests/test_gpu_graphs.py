"""Graph replay of the steady-state block step equals eager execution, bit for bit.

Within one closure the captured step is replayed many times, interleaved with
eager block steps and host synchronisations; every replayed block's decisions
feed the next, so any replay that differed from eager execution would change
the basis or the counters.
"""
from __future__ import annotations

import numpy as np
import pytest

from paper_2506_01120_amd import LieClosure, workloads as W

pytestmark = pytest.mark.gpu


def run(gens, tol, **cfg):
    print(f"[gpu] d={gens.shape[-1]} cfg={cfg}", flush=True)
    with LieClosure(gens, tol, **cfg) as lc:
        lc.run()
        return lc.basis(), lc.stats()


@pytest.mark.parametrize("case,precision,block", [
    ("su16", "fp64", 0), ("su16", "fp32", 0), ("su16", "bf16x3", 0),
    ("su16", "fp64", 300), ("ising5", "fp32", 64), ("pauli4x6", "fp64", 40), ("su8", "fp32", 100),
])
def test_graph_replay_matches_eager(case, precision, block):
    gens, tol = {
        "su16": (W.rand_pair(16, seed=2), 1e-10),
        "ising5": (W.ising(5), 1e-10),
        "pauli4x6": (W.pauli_set(4, 6, 11), 1e-10),
        "su8": (W.rand_pair(8, seed=31), 1e-10),
    }[case]
    v_eager, s_eager = run(gens, tol, precision=precision, block=block, use_graphs=False)
    v_graph, s_graph = run(gens, tol, precision=precision, block=block, use_graphs=True)
    assert s_graph["dim"] == s_eager["dim"]
    for k in ("candidates", "accepted", "zero_brackets", "screen_rejected", "fp64_decided"):
        assert s_graph[k] == s_eager[k], k
    np.testing.assert_array_equal(v_graph, v_eager)
