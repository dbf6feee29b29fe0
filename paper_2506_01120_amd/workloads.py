"""Seeded synthetic generator sets for the Lie-closure engine.

This module builds *inputs* only: dense complex128 anti-Hermitian generator
matrices of the families the closure tests and benchmarks use.  It contains
none of the closure method's arithmetic (no brackets, no projections, no
independence tests), so both the GPU path and the CPU reference may draw
their inputs from here.

Conventions
-----------
* Pauli matrices X = [[0,1],[1,0]], Y = [[0,-i],[i,0]], Z = diag(1,-1).
* Qubit 0 is the leftmost Kronecker factor.
* A generator set is a complex128 array of shape (n_gen, d, d), C order.
* Hermitian physics operators H enter as iH, so every generator is
  anti-Hermitian (the paper studies closures inside su(d), Section 2.1).
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "pauli_string",
    "ising",
    "xxyy",
    "pauli_set",
    "pauli_set_strings",
    "rand_pair",
    "batch_problems",
    "Problem",
    "weak_coupling",
    "embed",
]

_P1 = {
    "I": np.array([[1, 0], [0, 1]], dtype=np.complex128),
    "X": np.array([[0, 1], [1, 0]], dtype=np.complex128),
    "Y": np.array([[0, -1j], [1j, 0]], dtype=np.complex128),
    "Z": np.array([[1, 0], [0, -1]], dtype=np.complex128),
}


def pauli_string(s: str) -> np.ndarray:
    """Dense 2^n x 2^n matrix of the Pauli string ``s`` (e.g. "XIZ")."""
    m = np.ones((1, 1), dtype=np.complex128)
    for c in s:
        m = np.kron(m, _P1[c])
    return m


def _site(n: int, ops: dict[int, str]) -> str:
    return "".join(ops.get(q, "I") for q in range(n))


def ising(n: int) -> np.ndarray:
    """Open transverse-field Ising chain: [iX_0..iX_{n-1}, iZ_0Z_1..iZ_{n-2}Z_{n-1}]."""
    if n < 1:
        raise ValueError("n must be >= 1")
    gens = [1j * pauli_string(_site(n, {j: "X"})) for j in range(n)]
    gens += [1j * pauli_string(_site(n, {j: "Z", j + 1: "Z"})) for j in range(n - 1)]
    return np.ascontiguousarray(np.stack(gens))


def xxyy(n: int) -> np.ndarray:
    """Open XX+YY chain: one generator i(X_jX_{j+1} + Y_jY_{j+1}) per bond."""
    if n < 2:
        raise ValueError("n must be >= 2")
    gens = [
        1j * (pauli_string(_site(n, {j: "X", j + 1: "X"})) + pauli_string(_site(n, {j: "Y", j + 1: "Y"})))
        for j in range(n - 1)
    ]
    return np.ascontiguousarray(np.stack(gens))


def pauli_set_strings(n: int, k: int, seed: int) -> tuple[list[str], list[complex]]:
    """k distinct non-identity Pauli strings on n qubits, each with coefficient +i or -i.

    Strings are drawn uniformly without replacement from {I,X,Y,Z}^n minus I^n
    with numpy's PCG64 ``default_rng(seed)``; signs are fair coin flips.
    """
    if k > 4 ** n - 1:
        raise ValueError("more strings requested than exist")
    rng = np.random.default_rng(seed)
    idx = rng.choice(4 ** n - 1, size=k, replace=False) + 1
    letters = "IXYZ"
    strings = []
    for v in idx:
        s = []
        for _ in range(n):
            s.append(letters[int(v) % 4])
            v //= 4
        strings.append("".join(reversed(s)))
    signs = rng.integers(0, 2, size=k)
    coeffs = [1j if b == 0 else -1j for b in signs]
    return strings, coeffs


def pauli_set(n: int, k: int, seed: int) -> np.ndarray:
    """Generators c_j * P_j for the strings and signs of :func:`pauli_set_strings`."""
    strings, coeffs = pauli_set_strings(n, k, seed)
    return np.ascontiguousarray(np.stack([c * pauli_string(s) for s, c in zip(strings, coeffs)]))


def pauli_sums_terms(n: int, k: int, terms: int, seed: int) -> list[dict[str, float]]:
    """The generators of :func:`pauli_sums` as {label: weight} dicts, before normalisation:
    k sums of `terms` distinct random non-identity strings with standard-normal weights
    (numpy PCG64 ``default_rng(seed)``)."""
    rng = np.random.default_rng(seed)
    letters = "IXYZ"
    out = []
    for _ in range(k):
        picked = set()
        while len(picked) < terms:
            s = "".join(letters[i] for i in rng.integers(0, 4, size=n))
            if s != "I" * n:
                picked.add(s)
        out.append(dict(zip(sorted(picked), (float(w) for w in rng.standard_normal(terms)))))
    return out


def pauli_sums(n: int, k: int, terms: int, seed: int) -> np.ndarray:
    """k generators, each i * sum of `terms` distinct random non-identity Pauli strings on n
    qubits with standard-normal real weights (numpy PCG64 ``default_rng(seed)``),
    Frobenius-normalised: sparse sums of Pauli strings, the operators of the sparse
    representation."""
    out = []
    for g in pauli_sums_terms(n, k, terms, seed):
        m = 1j * sum(w * pauli_string(s) for s, w in g.items())
        out.append(m / np.linalg.norm(m))
    return np.ascontiguousarray(np.stack(out))


def ising_terms(n: int) -> list[dict[str, float]]:
    """:func:`ising` as sparse generators {label: c} (generator = sum c iP_label)."""
    gens = [{_site(n, {j: "X"}): 1.0} for j in range(n)]
    gens += [{_site(n, {j: "Z", j + 1: "Z"}): 1.0} for j in range(n - 1)]
    return gens


def xxyy_terms(n: int) -> list[dict[str, float]]:
    """:func:`xxyy` as sparse generators."""
    return [{_site(n, {j: "X", j + 1: "X"}): 1.0, _site(n, {j: "Y", j + 1: "Y"}): 1.0} for j in range(n - 1)]


def pauli_set_terms(n: int, k: int, seed: int) -> list[dict[str, float]]:
    """:func:`pauli_set` as sparse generators (c P = Im(c) iP for c = +-i)."""
    strings, coeffs = pauli_set_strings(n, k, seed)
    return [{s: float(c.imag)} for s, c in zip(strings, coeffs)]


def rand_pair(d: int, seed: int) -> np.ndarray:
    """Two random traceless anti-Hermitian d x d matrices, Frobenius-normalised.

    For each of the two: G has i.i.d. standard complex Gaussian entries
    (real part then imaginary part drawn from ``default_rng(seed)``),
    A = (G - G^H)/2, the trace part (tr A / d) I is removed, and A /= ||A||_F.
    """
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(2):
        g = rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))
        a = (g - g.conj().T) / 2
        a = a - (np.trace(a) / d) * np.eye(d)
        a = a / np.linalg.norm(a)
        out.append(a)
    return np.ascontiguousarray(np.stack(out))


class Problem:
    """One closure problem of a batch: generators, tolerance and the closed-form dimension."""

    def __init__(self, name: str, gens: np.ndarray, tol: float, expected_dim: int | None):
        self.name = name
        self.gens = gens
        self.tol = tol
        self.expected_dim = expected_dim

    @property
    def d(self) -> int:
        return int(self.gens.shape[-1])

    def __repr__(self) -> str:  # pragma: no cover - debugging aid
        return f"Problem({self.name}, d={self.d}, n_gen={len(self.gens)}, expected={self.expected_dim})"


def batch_problems(tol: float = 1e-8, count: int = 64) -> list[Problem]:
    """The 64-problem mixed batch: Ising n=3..7, XX+YY n=3..6, random Pauli sets, random pairs.

    Problem i uses seed 1000+i.  Index ranges:
      0-4   ising(3..7)                       expected n(2n-1)
      5-8   xxyy(3..6)                        expected n(n-1)/2
      9-37  pauli_set(n=4+(i-9)%3, k=3+((i-9)//3)%4)   expected from the Pauli closure (None here)
      38-63 rand_pair(d=8+(i-38)%17)          expected d^2-1
    The closed forms are stated for reference; the Pauli-set value has no
    closed form and is left as None.
    """
    probs: list[Problem] = []
    for i in range(count):
        seed = 1000 + i
        if i <= 4:
            n = 3 + i
            probs.append(Problem(f"ising{n}", ising(n), tol, n * (2 * n - 1)))
        elif i <= 8:
            n = 3 + (i - 5)
            probs.append(Problem(f"xxyy{n}", xxyy(n), tol, n * (n - 1) // 2))
        elif i <= 37:
            n = 4 + (i - 9) % 3
            k = 3 + ((i - 9) // 3) % 4
            probs.append(Problem(f"pauli{n}x{k}s{seed}", pauli_set(n, k, seed), tol, None))
        else:
            d = 8 + (i - 38) % 17
            probs.append(Problem(f"pair{d}s{seed}", rand_pair(d, seed), tol, d * d - 1))
    return probs


def weak_coupling(eps: float, seed: int = 7) -> np.ndarray:
    """Two d = 16 generators A (+) 0 and B (+) eps*C, with A, B = rand_pair(8, seed) in the upper
    block and C = i diag(1, -1, 0, ..., 0) in the lower one.  The closure is su(8) (+) span(0 (+) C),
    dim 64; the direction 0 (+) C enters only through the small eps, so the candidate that adds it
    has a residual of a few eps -- a closure whose last direction couples weakly."""
    a, b = rand_pair(8, seed)
    c = np.zeros((8, 8), dtype=np.complex128)
    c[0, 0], c[1, 1] = 1j, -1j
    g = np.zeros((2, 16, 16), dtype=np.complex128)
    g[0, :8, :8] = a
    g[1, :8, :8] = b
    g[1, 8:, 8:] = eps * c
    return g


def embed(gens: np.ndarray, d: int, seed: int | None = None) -> np.ndarray:
    """Generators of size k placed in the upper-left k x k block of d x d zero matrices (d >= k),
    then, with a seed, conjugated by one seeded random unitary U (QR of a complex Gaussian matrix):
    g -> U g U^H.  Conjugation keeps anti-Hermiticity, traces and the closure's dimension and
    spreads every element over the whole d x d matrix, so a closure of a small algebra exercises
    kernels at any d with dense operands."""
    gens = np.asarray(gens, dtype=np.complex128)
    k = gens.shape[-1]
    if d < k:
        raise ValueError("d must be at least the generators' size")
    out = np.zeros((gens.shape[0], d, d), dtype=np.complex128)
    out[:, :k, :k] = gens
    if seed is not None:
        rng = np.random.default_rng(seed)
        z = rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))
        q, r = np.linalg.qr(z)
        u = q * (np.diag(r) / np.abs(np.diag(r)))  # a unitary with a fixed phase convention
        out = u[None] @ out @ u.conj().T[None]
        out = 0.5 * (out - np.conj(np.swapaxes(out, 1, 2)))  # exactly anti-Hermitian after rounding
    return out
