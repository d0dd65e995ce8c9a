"""Gate lists for Heisenberg-picture propagation.

A gate is the pair (J, theta) standing for the unitary exp(-i theta sigma_J / 2)
(Appendix A, gate tuple).  Gate lists here are already in Heisenberg order: the
observable is conjugated by the first gate first.  For the kicked Ising Trotter
step U = U_zz U_x (Eq. (u)) conjugation O -> U^dag O U applies the U_zz factors
first and the U_x factors second, so one step is "RZZ on every edge, then RX on
every qubit" (RX in ascending qubit order).
"""

from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from .lattice import Lattice

_LETTERS = {"I": (0, 0), "X": (1, 0), "Y": (1, 1), "Z": (0, 1)}


def pauli_words(n: int, ops: dict[int, str]) -> np.ndarray:
    """(x0, x1, z0, z1) uint64 words of the Pauli string with letters `ops`."""
    w = [0, 0, 0, 0]
    for q, letter in ops.items():
        assert 0 <= q < n, (q, n)
        xb, zb = _LETTERS[letter.upper()]
        if xb:
            w[q >> 6] |= 1 << (q & 63)
        if zb:
            w[2 + (q >> 6)] |= 1 << (q & 63)
    return np.array(w, dtype=np.uint64)


def words_to_letters(n: int, w) -> str:
    names = {(0, 0): "I", (1, 0): "X", (1, 1): "Y", (0, 1): "Z"}
    out = []
    for q in range(n):
        xb = (int(w[q >> 6]) >> (q & 63)) & 1
        zb = (int(w[2 + (q >> 6)]) >> (q & 63)) & 1
        out.append(names[(xb, zb)])
    return "".join(out)


@dataclass
class GateList:
    """gens: (G, 4) uint64 generator words; thetas: (G, L) float64 angles."""
    gens: np.ndarray
    thetas: np.ndarray

    def __len__(self) -> int:
        return int(self.gens.shape[0])

    @staticmethod
    def concat(parts: list["GateList"]) -> "GateList":
        return GateList(np.concatenate([p.gens for p in parts]).astype(np.uint64),
                        np.concatenate([p.thetas for p in parts]).astype(np.float64))


def _as_lane_thetas(theta, lanes: int | None) -> np.ndarray:
    t = np.atleast_1d(np.asarray(theta, dtype=np.float64))
    if lanes is not None and t.size == 1 and lanes > 1:
        t = np.repeat(t, lanes)
    return t


def rzz_layer(lat: Lattice, theta_zz: float = -math.pi / 2, lanes: int = 1) -> GateList:
    g = np.stack([pauli_words(lat.n, {a: "Z", b: "Z"}) for a, b in lat.edges])
    th = np.tile(_as_lane_thetas(theta_zz, lanes), (len(lat.edges), 1))
    return GateList(g.astype(np.uint64), th)


def rx_layer(lat: Lattice, theta_x, lanes: int | None = None) -> GateList:
    t = _as_lane_thetas(theta_x, lanes)
    g = np.stack([pauli_words(lat.n, {q: "X"}) for q in range(lat.n)])
    th = np.tile(t, (lat.n, 1))
    return GateList(g.astype(np.uint64), th)


def kicked_ising_step(lat: Lattice, theta_x, theta_zz: float = -math.pi / 2,
                      lanes: int | None = None) -> tuple[GateList, GateList]:
    """One Trotter step in Heisenberg order: (RZZ layer, RX layer)."""
    t = _as_lane_thetas(theta_x, lanes)
    L = t.size
    return rzz_layer(lat, theta_zz, lanes=L), rx_layer(lat, t)


def kicked_ising_circuit(lat: Lattice, theta_x, steps: int, theta_zz: float = -math.pi / 2,
                         lanes: int | None = None) -> GateList:
    zz, rx = kicked_ising_step(lat, theta_x, theta_zz, lanes)
    return GateList.concat([zz, rx] * steps)


def single_pauli_term(n: int, ops: dict[int, str], coeff: float = 1.0, lanes: int = 1):
    """Initial operator holding one Pauli string: (terms (1,4) uint64, coeffs (1,L))."""
    return pauli_words(n, ops)[None, :], np.full((1, lanes), coeff, dtype=np.float64)
