"""The pins are strong enough to catch plausible mistakes in the reference.

Each case copies ``oracle/lie_oracle.c``, plants one mistake (a flipped sign,
a dropped conjugate, a transposed operand, a wrong loop bound, a missing
scale), compiles the copy into a temporary library and runs the same quick
pins the reference passes.  At least one pin must fail for every mutant.
Everything runs on the CPU; the real reference is never modified.
"""
from __future__ import annotations

import os
import tempfile

import numpy as np
import pytest

import pins
from oracle import oracle as O
from paper_2506_01120_amd import workloads as W

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "lie_oracle.c")

MUTANTS = {
    "anticommutator": ("s->x[k] = s->t1[k] - s->t2[k];", "s->x[k] = s->t1[k] + s->t2[k];"),
    "one_product_twice": ("matmul(d, b, a, s->t2);", "matmul(d, a, b, s->t2);"),
    "transposed_operand": ("acc += a[(int64_t)i * d + k] * b[(int64_t)k * d + j];",
                           "acc += a[(int64_t)i * d + k] * b[(int64_t)j * d + k];"),
    "dropped_conjugate": ("dot += conj(u[k]) * v[k];", "dot += u[k] * v[k];"),
    "reflector_factor": ("    dot *= 2.0;\n", "\n"),
    "skip_first_reflector": ("for (int64_t j = N - 1; j >= 0; --j)", "for (int64_t j = N - 1; j > 0; --j)"),
    "euclidean_residual": ("return vec_norm2(s->y + s->N, s->n - s->N) / sqrt((double)s->d);",
                           "return vec_norm2(s->y + s->N, s->n - s->N);"),
    "unit_euclidean_basis": ("const double scale = sqrt((double)s->d) / ynorm;",
                             "const double scale = 1.0 / ynorm;"),
    "diagonal_pairs": ("if (++s->m == s->l) {", "if (++s->m > s->l) {"),
    "row_skips_first_column": ("            s->l++;\n            s->m = 0;", "            s->l++;\n            s->m = 1;"),
    "early_exit_off_by_one": ("if (early_exit && s->N >= ambient)", "if (early_exit && s->N + 1 >= ambient)"),
}


def _battery(lib) -> list[str]:
    """Run the quick pins against a (possibly mutated) reference; return the names that fail."""
    failed = []

    def check(name, fn):
        try:
            ok = fn()
        except Exception:  # a crash in the mutant counts as a caught mistake
            ok = False
        if not ok:
            failed.append(name)

    def worked():
        o = O.Oracle(W.ising(2), 1e-10, log=True, lib=lib)
        o.run()
        v = o.basis()
        want = [1j * W.pauli_string(s) * c for s, c in
                (("XI", 1), ("IX", 1), ("ZZ", 1), ("YZ", -1), ("ZY", -1), ("YY", 1))]
        if len(v) != 6:
            return False
        log = o.log()
        return (np.allclose(v, np.stack(want), atol=1e-13)
                and np.allclose(log["r"][[1, 2, 4]], 2.0, atol=1e-13))

    def ising3():
        r = O.closure(W.ising(3), 1e-10, lib=lib)
        closed = pins.pauli_closure(["XII", "IXI", "IIX", "ZZI", "IZZ"])
        return r.dim == 15 and pins.pauli_span_distance(r.basis, closed) < 1e-12

    def pair4():
        r = O.closure(W.rand_pair(4, seed=104), 1e-10, lib=lib)
        return (r.dim == 15 and pins.su_span_distance(r.basis) < 1e-12
                and pins.orthonormality_loss(r.basis) < 1e-12)

    def xxyy4():
        return O.closure(W.xxyy(4), 1e-10, lib=lib).dim == 6

    def counts():
        r = O.closure(W.ising(3), 1e-10, lib=lib)
        return r.candidates == r.dim * (r.dim - 1) // 2

    def lstsq():
        rng = np.random.default_rng(0)
        ws = rng.standard_normal((3, 3, 3)) + 1j * rng.standard_normal((3, 3, 3))
        o = O.Oracle(ws, 1e-12, lib=lib)
        x = rng.standard_normal((3, 3)) + 1j * rng.standard_normal((3, 3))
        a = ws.reshape(3, 9).T
        c, *_ = np.linalg.lstsq(a, x.reshape(-1), rcond=None)
        want = np.linalg.norm(a @ c - x.reshape(-1)) / np.sqrt(3)
        return abs(o.residual_of(x) - want) < 1e-12

    def early():
        return O.closure(W.rand_pair(4, seed=104), 1e-10, early_exit=True, lib=lib).dim == 15

    for name, fn in (("worked", worked), ("ising3", ising3), ("pair4", pair4), ("xxyy4", xxyy4),
                     ("counts", counts), ("lstsq", lstsq), ("early_exit", early)):
        check(name, fn)
    return failed


def test_unmutated_reference_passes_battery():
    assert _battery(O.load()) == []


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site for {name} not found exactly once"
    with tempfile.TemporaryDirectory() as tmp:
        path = os.path.join(tmp, "mutant.c")
        with open(path, "w") as f:
            f.write(src.replace(old, new))
        lib = O.load(O.build(src=path, out=os.path.join(tmp, f"libmutant_{name}.so")))
        failed = _battery(lib)
    assert failed, f"mutant {name} passed every pin"
