"""GPU parity of the dense bracket beyond d = 64 (the tile-pair matrix-core kernel).

At d = 128 (seven qubits) the Ising chain's closure is spanned by the closure of its
generators' Pauli strings under anticommuting products (91 strings, so(14)), so its GPU
basis must span exactly those strings; the XX+YY chain's 21-dimensional closure lies
inside the 42-string closure of the strings of its generators.  Each basis element is
checked through its explicit residual against the strings, and the dimensions against
the closed forms 91 and n(n-1)/2 = 21.  FP64 and the FP32 screen both run the dense
operators.
"""
from __future__ import annotations

import pytest

import pins
from paper_2506_01120_amd import LieClosure, workloads as W

pytestmark = pytest.mark.gpu


def chain_strings(kind: str, n: int) -> list[str]:
    one = lambda q0, c: "".join(c if q == q0 else "I" for q in range(n))
    two = lambda q0, c: "".join(c if q in (q0, q0 + 1) else "I" for q in range(n))
    if kind == "ising":
        return [one(j, "X") for j in range(n)] + [two(j, "Z") for j in range(n - 1)]
    return [two(j, "X") for j in range(n - 1)] + [two(j, "Y") for j in range(n - 1)]


@pytest.mark.parametrize("kind,dim", [("ising", 91), ("xxyy", 21)])
@pytest.mark.parametrize("precision,decide", [("fp64", "fp64"), ("fp32", "screen")])
def test_dense_d128(kind, dim, precision, decide):
    gens = W.ising(7) if kind == "ising" else W.xxyy(7)
    print(f"[gpu] dense d=128 {kind} precision={precision} decide={decide}", flush=True)
    with LieClosure(gens, 1e-10 if precision == "fp64" else 1e-8, precision=precision, decide=decide) as lc:
        lc.run()
        got, v, st = lc.dim, lc.basis(), lc.stats()
    assert got == dim
    assert st["candidates"] == dim * (dim - 1) // 2
    closed = pins.pauli_closure(chain_strings(kind, 7))
    assert len(closed) == (dim if kind == "ising" else 2 * dim)
    # span equality for the Ising chain, containment for XX+YY (the residual outside the strings)
    assert pins.pauli_subset_span_distance(v, closed) <= (1e-8 if precision == "fp64" else 1e-5)
