"""Seeded synthetic inputs (splitmix64 stream, fully reproducible).

splitmix64 (Steele, Lea, Flood 2014): state += 0x9E3779B97F4A7C15, then the
output z is mixed by z = (z ^ z>>30) * 0xBF58476D1CE4E5B9,
z = (z ^ z>>27) * 0x94D049BB133111EB, z ^ z>>31.
"""

from __future__ import annotations

import math

import numpy as np

from .circuit import GateList, pauli_words

_M64 = (1 << 64) - 1


def splitmix64(seed: int, count: int) -> np.ndarray:
    """`count` consecutive splitmix64 outputs starting from state `seed`."""
    out = np.empty(count, dtype=np.uint64)
    s = seed & _M64
    for i in range(count):
        s = (s + 0x9E3779B97F4A7C15) & _M64
        z = s
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
        out[i] = z ^ (z >> 31)
    return out


def _splitmix64_np(seed: int, count: int) -> np.ndarray:
    """Vectorised splitmix64 (same stream as `splitmix64`)."""
    with np.errstate(over="ignore"):
        idx = np.arange(1, count + 1, dtype=np.uint64)
        z = np.uint64(seed & _M64) + idx * np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def _uniform01(u64: np.ndarray) -> np.ndarray:
    return (u64 >> np.uint64(11)).astype(np.float64) * (1.0 / (1 << 53))


def random_pauli_set(n_qubits: int, count: int, seed: int, support: list[int] | None = None,
                     eps0: float = 1e-4, lanes: int = 1) -> tuple[np.ndarray, np.ndarray]:
    """`count` distinct random Pauli strings with random I/X/Y/Z letters on
    `support` (default: all qubits), and coefficients with random sign and
    log-uniform magnitude in [eps0, 1] (the coefficient density with a sharp
    cutoff at the truncation threshold, Appendix D).  Returns (terms (m,4)
    uint64, coeffs (m, lanes) float64); m <= count after de-duplication."""
    if support is None:
        support = list(range(n_qubits))
    support = np.asarray(support, dtype=np.int64)
    k = support.size
    r = _splitmix64_np(seed, count * (k + 1 + lanes))
    letters = (r[: count * k] & np.uint64(3)).reshape(count, k)
    x = (letters == 1) | (letters == 2)
    z = (letters == 2) | (letters == 3)
    words = np.zeros((count, 4), dtype=np.uint64)
    for col, q in enumerate(support):
        bit = np.uint64(1) << np.uint64(int(q) & 63)
        w = int(q) >> 6
        words[:, w] |= np.where(x[:, col], bit, np.uint64(0))
        words[:, 2 + w] |= np.where(z[:, col], bit, np.uint64(0))
    words, first = np.unique(words, axis=0, return_index=True)
    rest = r[count * k:].reshape(count, 1 + lanes)[first]
    sign = np.where((rest[:, :1] & np.uint64(1)) == 1, -1.0, 1.0)
    mag = np.exp(math.log(eps0) * (1.0 - _uniform01(rest[:, 1:])))
    return words, sign * mag


def random_observables(n_qubits: int, count: int, seed: int) -> list[dict[int, str]]:
    """`count` distinct Z observables of weight 1 or 2 (uniform), their qubits
    distinct and uniform over the register, from one splitmix64 stream."""
    r = splitmix64(seed, 64 * count + 64)
    out: list[dict[int, str]] = []
    i = 0
    while len(out) < count:
        w = 1 + int(r[i] & np.uint64(1))
        i += 1
        qs: list[int] = []
        while len(qs) < w:
            q = int(r[i] % np.uint64(n_qubits))
            i += 1
            if q not in qs:
                qs.append(q)
        ops = {q: "Z" for q in sorted(qs)}
        if ops not in out:
            out.append(ops)
    return out


def random_gates(n_qubits: int, count: int, seed: int, max_weight: int | None = None,
                 clifford_fraction: float = 0.2, lanes: int = 1) -> GateList:
    """Random Pauli rotations: generator letters uniform over {X,Y,Z} on a
    random subset of qubits, angles uniform in (-pi, pi) with a fraction at
    exact multiples of pi/2."""
    if max_weight is None:
        max_weight = n_qubits
    r = _splitmix64_np(seed, count * (2 + 2 * n_qubits + lanes))
    r = r.reshape(count, -1)
    gens = []
    thetas = np.empty((count, lanes), dtype=np.float64)
    for g in range(count):
        row = r[g]
        w = 1 + int(row[0] % np.uint64(max_weight))
        perm = np.argsort(row[2:2 + n_qubits])[:w]
        ops = {int(q): "XYZ"[int(row[2 + n_qubits + int(q)] % np.uint64(3))] for q in perm}
        gens.append(pauli_words(n_qubits, ops))
        u = _uniform01(row[2 + 2 * n_qubits: 2 + 2 * n_qubits + lanes])
        if _uniform01(row[1:2])[0] < clifford_fraction:
            k = (row[2 + 2 * n_qubits: 2 + 2 * n_qubits + lanes] % np.uint64(8)).astype(np.int64) - 4
            thetas[g] = k * (math.pi / 2)
        else:
            thetas[g] = (2.0 * u - 1.0) * math.pi
    return GateList(np.stack(gens).astype(np.uint64), thetas)
