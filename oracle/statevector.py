"""Schrodinger-picture statevector brute force (test infrastructure only).

Computes <psi_t| P |psi_t> for |psi_t> = U^t |0...0> directly, with no Pauli
propagation at all, so it pins the Heisenberg-picture propagation from the
outside (Appendix E compares the method against exactly this).

Basis index bit q is qubit q.  A Pauli string P with x/z masks acts as
P|b> = i^{#Y} (-1)^{popcount(b & z)} |b xor x>  (Y = i X Z per site).
"""

from __future__ import annotations

import math

import numpy as np


def _masks(n: int, w) -> tuple[int, int]:
    x = int(w[0]) | (int(w[1]) << 64)
    z = int(w[2]) | (int(w[3]) << 64)
    assert x >> n == 0 and z >> n == 0, "generator acts outside the register"
    return x, z


def apply_pauli(psi: np.ndarray, n: int, x: int, z: int) -> np.ndarray:
    idx = np.arange(psi.size, dtype=np.int64)
    ny = bin(x & z).count("1")
    sign = 1.0 - 2.0 * (np.bitwise_count(idx & z) & 1)
    out = np.empty_like(psi)
    out[idx ^ x] = (1j ** ny) * sign * psi
    return out


def apply_rotation(psi: np.ndarray, n: int, x: int, z: int, theta: float) -> np.ndarray:
    """exp(-i theta P / 2) |psi> = cos(theta/2)|psi> - i sin(theta/2) P|psi>."""
    return math.cos(theta / 2) * psi - 1j * math.sin(theta / 2) * apply_pauli(psi, n, x, z)


def expectation(psi: np.ndarray, n: int, x: int, z: int) -> float:
    v = np.vdot(psi, apply_pauli(psi, n, x, z))
    return float(v.real)


def zero_state(n: int) -> np.ndarray:
    psi = np.zeros(1 << n, dtype=np.complex128)
    psi[0] = 1.0
    return psi


def run_circuit(n: int, gates_schrodinger) -> np.ndarray:
    """Apply gates (generator words, angle) to |0> in the order given."""
    psi = zero_state(n)
    for w, th in gates_schrodinger:
        x, z = _masks(n, w)
        psi = apply_rotation(psi, n, x, z, float(th))
    return psi


def kicked_ising_magnetization(n: int, edges, q: int, theta_x: float, steps: int,
                               theta_zz: float = -math.pi / 2, observable=None) -> list[float]:
    """<M_t> = <0|(U^dag)^t O U^t|0>, U = U_zz U_x (U_x acts first on the state),
    for t = 1..steps (Eq. (u), Eq. (magnetization)).  O defaults to Z_q;
    `observable` may be a dict {qubit: letter}."""
    idx = np.arange(1 << n, dtype=np.int64)
    # U_zz is diagonal: exp(-i theta_zz/2 * (-1)^{b_a xor b_b}) per edge.
    phase = np.zeros(1 << n)
    for a, b in edges:
        par = ((idx >> a) ^ (idx >> b)) & 1
        phase += -0.5 * theta_zz * (1.0 - 2.0 * par)
    uzz = np.exp(1j * phase)
    if observable is None:
        observable = {q: "Z"}
    ox = sum(1 << k for k, v in observable.items() if v in "XY")
    oz = sum(1 << k for k, v in observable.items() if v in "YZ")
    c, s = math.cos(theta_x / 2), math.sin(theta_x / 2)
    psi = zero_state(n)
    out = []
    for _ in range(steps):
        for j in range(n):  # U_x: exp(-i theta_x X_j / 2) on every qubit
            psi = c * psi - 1j * s * psi[idx ^ (1 << j)]
        psi = uzz * psi
        out.append(expectation(psi, n, ox, oz))
    return out
