"""Learned truncation scorer: feature table, parameter layout and training driver.

The scorer estimates, from a Pauli string's key alone, log10 of the weight
|g_I| with which the string still reaches <Z> after the rest of the circuit.
The paper truncates by coefficient magnitude only (Eq. truncation1) and leaves
truncation tailored to the problem as future work (Conclusion, Appendix D);
learned truncation keeps a string iff |O_I| * min(1, g_I) > eps * max|O|, so
the magnitude rule is the special case g = 1.

Feature f of a string counts the qubits of the region qmask[f] that carry the
letter letters[f] (0 X, 1 Y, 2 Z, 3 any non-identity), times scales[f]:
  0..47    rings of equal graph distance d = 0..15 from the observable qubit
           (ring 15 holds every d >= 15), letters X, Y, Z, scale 1/4;
  48..86   13 bands of consecutive qubit indices, letters X, Y, Z, scale 1/8;
  87..90   all qubits, letters any, X, Y, Z (the weight and its split), 1/32;
  91..159  the 23 qubits nearest the observable (by distance, then index),
           each with letters X, Y, Z, scale 1.
All counts times these scales are exact in bf16.
"""

from __future__ import annotations

from collections import deque

import numpy as np

N_FEATURES, N_HIDDEN = 160, 128
N_RINGS, N_BANDS, N_NEAR = 16, 13, 23
SHAPES = (("W1", (N_HIDDEN, N_FEATURES)), ("b1", (N_HIDDEN,)), ("W2", (N_HIDDEN, N_HIDDEN)),
          ("b2", (N_HIDDEN,)), ("W3", (1, N_HIDDEN)), ("b3", (1,)))
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)  # 37249


def graph_distances(n_qubits: int, edges, source: int) -> np.ndarray:
    """Breadth-first distances from `source` (unreachable qubits get n_qubits)."""
    adj = [[] for _ in range(n_qubits)]
    for a, b in edges:
        adj[int(a)].append(int(b))
        adj[int(b)].append(int(a))
    dist = np.full(n_qubits, n_qubits, dtype=np.int64)
    dist[source] = 0
    q = deque([source])
    while q:
        u = q.popleft()
        for v in adj[u]:
            if dist[v] > dist[u] + 1:
                dist[v] = dist[u] + 1
                q.append(v)
    return dist


def _mask(qubits) -> tuple[int, int]:
    m = 0
    for q in qubits:
        m |= 1 << int(q)
    return m & 0xFFFFFFFFFFFFFFFF, m >> 64


def feature_table(n_qubits: int, edges, obs_qubit: int):
    """(qmask (160,2) uint64, letters (160,) uint8, scales (160,) float32)."""
    if not 1 <= n_qubits <= 128:
        raise ValueError("n_qubits must be in 1..128")
    dist = graph_distances(n_qubits, edges, obs_qubit)
    regions, letters, scales = [], [], []
    for d in range(N_RINGS):
        ring = [q for q in range(n_qubits) if (dist[q] == d if d < N_RINGS - 1 else dist[q] >= d)]
        for letter in range(3):
            regions.append(ring), letters.append(letter), scales.append(0.25)
    for b in range(N_BANDS):
        band = [q for q in range(n_qubits) if q * N_BANDS // n_qubits == b]
        for letter in range(3):
            regions.append(band), letters.append(letter), scales.append(0.125)
    for letter in (3, 0, 1, 2):
        regions.append(list(range(n_qubits))), letters.append(letter), scales.append(1.0 / 32)
    near = sorted(range(n_qubits), key=lambda q: (dist[q], q))[:N_NEAR]
    for j in range(N_NEAR):
        reg = [near[j]] if j < len(near) else []
        for letter in range(3):
            regions.append(reg), letters.append(letter), scales.append(1.0)
    assert len(regions) == N_FEATURES
    qmask = np.array([_mask(r) for r in regions], dtype=np.uint64)
    return qmask, np.array(letters, dtype=np.uint8), np.array(scales, dtype=np.float32)


def pack_params(p: dict) -> np.ndarray:
    """Flat fp32 parameter vector in the library's layout (W1 b1 W2 b2 W3 b3)."""
    return np.concatenate([np.asarray(p[k], dtype=np.float64).reshape(-1) for k, _ in SHAPES]).astype(np.float32)


def unpack_params(flat) -> dict:
    flat = np.asarray(flat)
    if flat.size != N_PARAMS:
        raise ValueError(f"expected {N_PARAMS} parameters")
    out, o = {}, 0
    for k, shape in SHAPES:
        m = int(np.prod(shape))
        out[k] = flat[o:o + m].reshape(shape).astype(np.float64)
        o += m
    return out


def init_params(seed: int = 0) -> np.ndarray:
    """He-style normal initialisation, zero biases (flat fp32)."""
    rng = np.random.default_rng(seed)
    p = {
        "W1": rng.normal(0, 1 / np.sqrt(N_FEATURES), (N_HIDDEN, N_FEATURES)),
        "b1": np.zeros(N_HIDDEN),
        "W2": rng.normal(0, 1 / np.sqrt(N_HIDDEN), (N_HIDDEN, N_HIDDEN)),
        "b2": np.zeros(N_HIDDEN),
        "W3": rng.normal(0, 1 / np.sqrt(N_HIDDEN), (1, N_HIDDEN)),
        "b3": np.zeros(1),
    }
    return pack_params(p)


def constant_params(y: float) -> np.ndarray:
    """A network whose output is y for every string (all weights zero)."""
    flat = np.zeros(N_PARAMS, dtype=np.float32)
    flat[-1] = y
    return flat


def save_params(path: str, flat, meta: dict):
    """Parameters and their provenance as a plain .npz (no pickled objects)."""
    np.savez(path, params=np.asarray(flat, dtype=np.float32),
             meta=np.array([f"{k}={v}" for k, v in sorted(meta.items())]))


def load_params(path: str):
    with np.load(path, allow_pickle=False) as z:
        meta = dict(s.split("=", 1) for s in z["meta"].tolist())
        return z["params"].astype(np.float32), meta
