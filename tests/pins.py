"""Independent checks that pin the reference closure (and the GPU path) to
facts fixed by mathematics rather than by either implementation.

Nothing here imports the reference or the GPU library.  Each function states
the fact it computes:

* ``pauli_closure``      -- closure of a set of Pauli strings under the bracket.
  For strings P, Q: [P, Q] = 0 if they commute and 2PQ (a phase times one
  string) if they anticommute; distinct strings are orthonormal under
  <a,b> = tr(a^H b)/d (the membership idea the paper credits to Wiersema et
  al., Section 3).  So the closure's dimension is the size of the string set
  closed under "anticommuting P, Q  =>  PQ".
* ``modular_closure_dim`` -- brute-force dimension of the span of all
  right-normed brackets [g1,[g2,[...,gk]]] of the generators, grown by depth
  until one more depth adds nothing (then the span is closed under ad_g for
  every generator g, hence it is the Lie closure).  Arithmetic is exact: the
  entries (Gaussian integers, or dyadic rationals for float inputs) are mapped
  into F_p with i -> sqrt(-1) mod p for primes p = 1 (mod 4).
* ``span_distance``      -- ||P1 - P2||_F for the orthogonal projectors onto two
  spans given by orthonormal bases, computed without cancellation.
* ``su_span_distance``   -- distance of span(V) from the traceless matrices.
* ``pauli_span_distance``-- distance of span(V) from the span of a string set.
"""
from __future__ import annotations

import itertools

import numpy as np

# Two primes p = 1 (mod 4) below 2^25 (so d * p^2 fits in int64 for d <= 128),
# each with a square root of -1 modulo p.
PRIMES = ((33554393, 33479089), (33554341, 6840426))

# ------------------------------------------------------------------ Pauli strings

_LETTER_BITS = {"I": (0, 0), "X": (1, 0), "Y": (1, 1), "Z": (0, 1)}


def string_bits(s: str) -> tuple[int, int]:
    """Symplectic (x, z) bit masks of a Pauli string (qubit 0 is the most significant bit)."""
    x = z = 0
    for c in s:
        bx, bz = _LETTER_BITS[c]
        x = (x << 1) | bx
        z = (z << 1) | bz
    return x, z


def bits_string(x: int, z: int, n: int) -> str:
    out = []
    for q in range(n):
        bit = n - 1 - q
        bx, bz = (x >> bit) & 1, (z >> bit) & 1
        out.append({(0, 0): "I", (1, 0): "X", (1, 1): "Y", (0, 1): "Z"}[(bx, bz)])
    return "".join(out)


def anticommute(a: tuple[int, int], b: tuple[int, int]) -> bool:
    return (bin(a[0] & b[1]).count("1") + bin(a[1] & b[0]).count("1")) % 2 == 1


def pauli_closure(strings: list[str]) -> set[str]:
    """Smallest set containing ``strings`` and closed under anticommuting products."""
    n = len(strings[0])
    cur = {string_bits(s) for s in strings}
    frontier = list(cur)
    while frontier:
        new = []
        for a in frontier:
            for b in list(cur):
                if anticommute(a, b):
                    c = (a[0] ^ b[0], a[1] ^ b[1])
                    if c not in cur:
                        cur.add(c)
                        new.append(c)
        frontier = new
    return {bits_string(x, z, n) for x, z in cur}


# ------------------------------------------------------------------ exact modular brute force

def _to_mod(v: float, p: int) -> int:
    num, den = float(v).as_integer_ratio()
    return (num % p) * pow(den, -1, p) % p


def to_modp(m: np.ndarray, p: int, iota: int) -> np.ndarray:
    """Map a complex matrix with dyadic-rational parts exactly into F_p (i -> iota)."""
    re = np.vectorize(lambda v: _to_mod(v, p), otypes=[np.int64])(m.real)
    im = np.vectorize(lambda v: _to_mod(v, p), otypes=[np.int64])(m.imag)
    return (re + im * iota) % p


def _bracket_modp(a: np.ndarray, b: np.ndarray, p: int) -> np.ndarray:
    return ((a @ b) % p - (b @ a) % p) % p


class _EchelonModP:
    """Incremental row echelon form over F_p (vectors as int64 arrays)."""

    def __init__(self, p: int):
        self.p = p
        self.rows: list[np.ndarray] = []
        self.pivots: list[int] = []

    def add(self, v: np.ndarray) -> bool:
        p = self.p
        v = v.copy() % p
        for row, piv in zip(self.rows, self.pivots):
            c = int(v[piv])
            if c:
                v = (v - c * row) % p
        nz = np.flatnonzero(v)
        if nz.size == 0:
            return False
        piv = int(nz[0])
        v = (v * pow(int(v[piv]), -1, p)) % p
        # keep rows fully reduced at existing pivots so later reductions stay one pass
        for k, (row, pv) in enumerate(zip(self.rows, self.pivots)):
            c = int(row[piv])
            if c:
                self.rows[k] = (row - c * v) % p
        self.rows.append(v)
        self.pivots.append(piv)
        return True

    @property
    def rank(self) -> int:
        return len(self.rows)


def modular_closure_dim(gens: np.ndarray, max_depth: int = 64, prime_index: int = 0,
                        return_depths: bool = False, traceless: bool = False):
    """Dimension of the Lie closure by brute force over right-normed brackets, exact mod p.

    Depth D holds the span L_D of right-normed brackets of <= D generators;
    L_{D+1} = L_D + [G, L_D].  Stops when a depth adds nothing.  Returns the
    rank (and, optionally, the cumulative rank per depth).

    ``traceless`` removes the trace exactly in F_p (a -= tr(a)/d * I) -- for
    float inputs whose trace was removed in floating point, leaving only a
    rounding residue that exact arithmetic would otherwise see.
    """
    p, iota = PRIMES[prime_index]
    g_mod = [to_modp(g, p, iota) for g in gens]
    if traceless:
        d = gens.shape[-1]
        inv_d = pow(d, -1, p)
        for g in g_mod:
            t = int(np.trace(g) % p) * inv_d % p
            g[np.diag_indices(d)] = (g[np.diag_indices(d)] - t) % p
    ech = _EchelonModP(p)
    frontier = []
    for g in g_mod:
        if ech.add(g.reshape(-1)):
            frontier.append(g)
    depths = [ech.rank]
    for _ in range(max_depth):
        new = []
        for g in g_mod:
            for x in frontier:
                y = _bracket_modp(g, x, p)
                if ech.add(y.reshape(-1)):
                    new.append(y)
        if not new:
            break
        depths.append(ech.rank)
        frontier = new
    else:
        raise RuntimeError("closure did not stabilise within max_depth")
    return (ech.rank, depths) if return_depths else ech.rank


# ------------------------------------------------------------------ spans

def _orthonormal_columns(v: np.ndarray) -> np.ndarray:
    """Columns vec(V_k)/sqrt(d): Euclidean-orthonormal iff <V_i, V_j> = delta_ij."""
    n, d, _ = v.shape
    return v.reshape(n, d * d).T / np.sqrt(d)


def span_distance(v1: np.ndarray, v2: np.ndarray) -> float:
    """||P1 - P2||_F for two orthonormal bases of equal size, as sqrt(2)*||Q1 - Q2 Q2^H Q1||_F."""
    if v1.shape[0] != v2.shape[0]:
        return float("inf")
    q1 = _orthonormal_columns(v1)
    q2 = _orthonormal_columns(v2)
    r = q1 - q2 @ (q2.conj().T @ q1)
    return float(np.sqrt(2.0) * np.linalg.norm(r))


def su_span_distance(v: np.ndarray) -> float:
    """||P_V - P_su||_F when dim V = d^2 - 1: sqrt(2 * sum_k |tr(V_k)/d|^2)."""
    d = v.shape[-1]
    tr = np.trace(v, axis1=1, axis2=2) / d
    return float(np.sqrt(2.0 * np.sum(np.abs(tr) ** 2)))


def pauli_coefficients(v: np.ndarray) -> tuple[list[str], np.ndarray]:
    """<P, V_k> = tr(P V_k)/d for every Pauli string P (brute force; small d only)."""
    from paper_2506_01120_amd.workloads import pauli_string

    d = v.shape[-1]
    n = d.bit_length() - 1
    names = ["".join(t) for t in itertools.product("IXYZ", repeat=n)]
    mats = np.stack([pauli_string(s) for s in names])  # Hermitian
    coef = np.einsum("pij,kji->kp", mats, v) / d
    return names, coef


def pauli_span_distance(v: np.ndarray, strings: set[str]) -> float:
    """||P_V - P_S||_F for dim V = |S|: sqrt(2 * sum_k sum_{P not in S} |<P, V_k>|^2)."""
    names, coef = pauli_coefficients(v)
    outside = np.array([s not in strings for s in names])
    return float(np.sqrt(2.0 * np.sum(np.abs(coef[:, outside]) ** 2)))


def orthonormality_loss(v: np.ndarray) -> float:
    """||G - I||_F with G_ij = <V_i, V_j>."""
    q = _orthonormal_columns(v)
    g = q.conj().T @ q
    return float(np.linalg.norm(g - np.eye(g.shape[0])))


def pauli_subset_span_distance(v: np.ndarray, strings) -> float:
    """||P_V - P_S||_F for dim V = |S|, from the explicit residual V_k - sum_{P in S} <P,V_k> P.

    Only the strings of S are formed, so this scales to large d when |S| is small.
    """
    from paper_2506_01120_amd.workloads import pauli_string

    d = v.shape[-1]
    mats = np.stack([pauli_string(s) for s in sorted(strings)])  # Hermitian, <P,Q> = delta
    coef = np.einsum("pij,kji->kp", mats, v) / d
    resid = v - np.einsum("kp,pij->kij", coef, mats)
    return float(np.sqrt(2.0 * np.sum(np.abs(resid) ** 2) / d))
