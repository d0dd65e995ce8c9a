"""Dense Pauli-basis brute force for n <= 6 qubits (test infrastructure only).

Builds O = sum_I O_I sigma_I as a 2^n x 2^n matrix, conjugates it by every
gate G = exp(-i theta sigma_J / 2) as O <- G^dag O G (the left-hand side of
Eq. update_rule), and reads every coefficient back as
O_I = Tr[sigma_I O] / 2^n.  No ORQA algebra is used.
"""

from __future__ import annotations

import math

import numpy as np


def pauli_matrix(n: int, w) -> np.ndarray:
    x = int(w[0]) | (int(w[1]) << 64)
    z = int(w[2]) | (int(w[3]) << 64)
    dim = 1 << n
    b = np.arange(dim, dtype=np.int64)
    ny = bin(x & z).count("1")
    sign = 1.0 - 2.0 * (np.bitwise_count(b & z) & 1)
    M = np.zeros((dim, dim), dtype=np.complex128)
    M[b ^ x, b] = (1j ** ny) * sign
    return M


def all_strings(n: int):
    """Every Pauli string on n qubits as (x0,x1,z0,z1) words."""
    for x in range(1 << n):
        for z in range(1 << n):
            yield (x & ((1 << 64) - 1), x >> 64, z & ((1 << 64) - 1), z >> 64)


def heisenberg(n: int, terms, coeffs, gens, thetas) -> dict:
    """Propagate sum_t coeffs[t] sigma_{terms[t]} through the gates (Heisenberg
    order) and return {words: coefficient} for every nonzero coefficient."""
    dim = 1 << n
    O = np.zeros((dim, dim), dtype=np.complex128)
    for w, c in zip(terms, coeffs):
        O += float(c) * pauli_matrix(n, w)
    eye = np.eye(dim)
    for w, th in zip(gens, thetas):
        th = float(th)
        G = math.cos(th / 2) * eye - 1j * math.sin(th / 2) * pauli_matrix(n, w)
        O = G.conj().T @ O @ G
    out = {}
    for w in all_strings(n):
        P = pauli_matrix(n, w)
        v = np.trace(P @ O) / dim
        assert abs(v.imag) < 1e-12, "Hermitian operator must have real Pauli coefficients"
        if abs(v.real) > 1e-13:
            out[tuple(int(t) for t in w)] = float(v.real)
    return out


def letters_product(a: str, b: str) -> tuple[complex, str]:
    """Single-qubit product table sigma_a sigma_b = phase * sigma_c from matrices."""
    mats = {"I": np.eye(2), "X": np.array([[0, 1], [1, 0]]), "Y": np.array([[0, -1j], [1j, 0]]),
            "Z": np.array([[1, 0], [0, -1]])}
    prod = mats[a] @ mats[b]
    for c, m in mats.items():
        for ph in (1, 1j, -1, -1j):
            if np.allclose(prod, ph * m):
                return ph, c
    raise AssertionError
