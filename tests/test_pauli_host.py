"""CPU checks of the Pauli-coordinate transforms of the C ABI (host code, no GPU).

coords[x * 2^n + z] = -i tr(P_s M) / d with P_s the Kronecker product of I, X, Y, Z
selected by the bit masks (qubit q <-> bit n-1-q of the basis index).  Pinned
against brute-force traces with explicit Kronecker products, the round trip, the
orthonormality of the strings, and the commutator rule of two strings.
"""
from __future__ import annotations

import ctypes
import itertools

import numpy as np
import pytest

from paper_2506_01120_amd import _lib, workloads as W

SIG = {
    (0, 0): np.eye(2, dtype=np.complex128),
    (1, 0): np.array([[0, 1], [1, 0]], dtype=np.complex128),
    (1, 1): np.array([[0, -1j], [1j, 0]], dtype=np.complex128),
    (0, 1): np.array([[1, 0], [0, -1]], dtype=np.complex128),
}


def string_matrix(x: int, z: int, n: int) -> np.ndarray:
    m = np.ones((1, 1), dtype=np.complex128)
    for q in range(n):
        b = n - 1 - q
        m = np.kron(m, SIG[((x >> b) & 1, (z >> b) & 1)])
    return m


@pytest.fixture(scope="module")
def lib():
    try:
        return _lib.load()
    except ImportError:
        pytest.skip("library not built")


def coords(lib, m):
    d = m.shape[0]
    buf = np.ascontiguousarray(m, dtype=np.complex128)
    out = np.empty(d * d)
    assert lib.lie_pauli_coordinates(d, buf.ctypes.data, out.ctypes.data) == 0
    return out


def matrix(lib, c):
    d = int(round(np.sqrt(c.size)))
    out = np.empty((d, d), dtype=np.complex128)
    assert lib.lie_pauli_matrix(d, np.ascontiguousarray(c).ctypes.data, out.ctypes.data) == 0
    return out


@pytest.mark.parametrize("n", [1, 2, 3])
def test_coordinates_against_brute_force(lib, n):
    d = 1 << n
    g = W.rand_pair(d, seed=40 + n)[0]
    c = coords(lib, g)
    for x, z in itertools.product(range(d), range(d)):
        want = (-1j * np.trace(string_matrix(x, z, n) @ g) / d)
        assert abs(want.imag) < 1e-14
        assert abs(c[(x << n) | z] - want.real) < 1e-14


@pytest.mark.parametrize("n", [1, 3, 5, 7])
def test_round_trip(lib, n):
    d = 1 << n
    g = W.rand_pair(d, seed=50 + n)[1]
    c = coords(lib, g)
    assert abs(np.dot(c, c) - np.real(np.trace(g.conj().T @ g)) / d) < 1e-12  # orthonormal coordinates
    assert np.max(np.abs(matrix(lib, c) - g)) < 1e-13


def test_strings_and_bracket_rule(lib):
    """Each iP_s maps to the unit vector e_s; [iP_a, iP_b] is 0 or +-2 iP_{a xor b}."""
    n = 2
    d = 1 << n
    for a in range(d * d):
        pa = 1j * string_matrix(a >> n, a & (d - 1), n)
        ca = coords(lib, pa)
        assert ca[a] == pytest.approx(1.0) and np.sum(np.abs(ca)) == pytest.approx(1.0)
        for b in range(d * d):
            pb = 1j * string_matrix(b >> n, b & (d - 1), n)
            cb = coords(lib, pa @ pb - pb @ pa)
            nz = np.flatnonzero(np.abs(cb) > 1e-12)
            xa, za, xb, zb = a >> n, a & (d - 1), b >> n, b & (d - 1)
            anti = (bin(xa & zb).count("1") + bin(za & xb).count("1")) & 1
            if not anti:
                assert nz.size == 0
            else:
                assert list(nz) == [a ^ b] and abs(abs(cb[a ^ b]) - 2.0) < 1e-12
                # sign: P_a P_b = i^e P_c, e = |xa&za| + |xb&zb| - |xc&zc| + 2|za&xb|, bracket 2 i^(e+1)
                xc, zc = xa ^ xb, za ^ zb
                pc = lambda v: bin(v).count("1")
                e = pc(xa & za) + pc(xb & zb) - pc(xc & zc) + 2 * pc(za & xb)
                assert cb[a ^ b] == pytest.approx(2.0 if (e + 1) % 4 == 0 else -2.0)


def test_bad_arguments(lib):
    out = np.empty(36)
    m = np.zeros((6, 6), dtype=np.complex128)
    assert lib.lie_pauli_coordinates(6, m.ctypes.data, out.ctypes.data) == -1
    assert lib.lie_pauli_coordinates(4, None, out.ctypes.data) == -1
