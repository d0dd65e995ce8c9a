"""The benchmark workload at its full size (needs a GPU): 127 q, theta_h = 0.8,
eps0 = 1e-4, FP64, the operator after 19 Trotter steps (~1.5e7 strings), in
the launch configuration bench.py times.  The oracle cannot propagate that
far in seconds, so the next gates are checked on sampled outputs, each one
recomputed by the oracle from the input strings that feed it, and through
properties that hold at any size (key sets, bijection, sortedness)."""

import sys

import numpy as np
import pytest

import workload as w
from oracle import OracleSum
from gpu_common import gpu_sum

pytestmark = pytest.mark.gpu

SAMPLES = 1500


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def _void(keys):
    return np.ascontiguousarray(keys, dtype=np.uint64).view(np.dtype((np.void, 32))).ravel()


class KeyIndex:
    """Exact membership and coefficient lookup in an exported operator."""

    def __init__(self, keys, coeffs):
        self.v = _void(keys)
        self.order = np.argsort(self.v, kind="stable")
        self.sorted = self.v[self.order]
        self.coeffs = coeffs

    def find(self, keys):
        q = _void(keys)
        pos = np.searchsorted(self.sorted, q)
        pos = np.minimum(pos, len(self.sorted) - 1)
        hit = self.sorted[pos] == q
        return hit, self.order[pos]


def _x_major_sorted(keys):
    """Export order: (x1, x0, z1, z0) ascending, every key once."""
    k = keys.astype(np.uint64)
    a, b = k[:-1], k[1:]
    lt = np.zeros(len(a), dtype=bool)
    eq = np.ones(len(a), dtype=bool)
    for col in (1, 0, 3, 2):
        lt |= eq & (a[:, col] < b[:, col])
        eq &= a[:, col] == b[:, col]
    return bool(np.all(lt))


def test_benchmark_workload_full_size_sampled():
    lat = w.eagle_127()
    zz, rx = w.kicked_ising_step(lat, 0.8)
    terms, coef = w.single_pauli_term(lat.n, {lat.center: "Z"})
    g = gpu_sum(lat.n, terms, coef)
    for _ in range(19):
        g.apply_rotation_layer(zz, 1e-4).apply_rotation_layer(rx, 1e-4)
    k0, c0 = g.export()
    say(f"full size: {len(k0)} strings after 19 steps")
    assert len(k0) > 10_000_000 and _x_major_sorted(k0)
    rng = np.random.default_rng(2025)

    # ---- the Clifford RZZ layer (fused pass + re-sort), untruncated: a signed
    # permutation, so every sampled input string lands on exactly one output
    g.apply_rotation_layer(zz)
    k1, c1 = g.export()
    assert len(k1) == len(k0) and _x_major_sorted(k1)
    idx1 = KeyIndex(k1, c1)
    pick = rng.choice(len(k0), SAMPLES, replace=False)
    for j in pick:
        o = OracleSum(lat.n, k0[j:j + 1], c0[j:j + 1]).apply(zz)
        ok, oc = o.export()
        assert len(ok) == 1
        hit, where = idx1.find(ok)
        assert hit[0] and c1[where[0], 0] == oc[0, 0]
    say(f"Clifford layer: {SAMPLES} sampled strings bit-identical")

    # ---- the streaming RX merge on qubit 0, untruncated: every output key is
    # an input key or the child of an anticommuting one (z_0 = 1), and each
    # sampled output equals the oracle's gate applied to the strings feeding it
    gate = w.GateList(w.pauli_words(lat.n, {0: "X"})[None, :], np.array([[0.8]]))
    g.apply_rotation_layer(gate)
    k2, c2 = g.export()
    assert _x_major_sorted(k2)
    anti = (k1[:, 2] & np.uint64(1)) != 0
    child = k1[anti].copy()
    child[:, 0] ^= np.uint64(1)
    want = np.unique(_void(np.concatenate([k1, child])))
    assert len(want) == len(k2) and np.array_equal(np.sort(_void(k2)), want)
    say(f"RX(q0): {len(k1)} -> {len(k2)} strings, key set exact")
    partner = k2.copy()
    partner[:, 0] ^= np.uint64(1)
    for j in rng.choice(len(k2), SAMPLES, replace=False):
        src = np.stack([k2[j], partner[j]])
        hit, where = idx1.find(src)
        sub_k, sub_c = src[hit], c1[where[hit]]
        o = OracleSum(lat.n, sub_k, sub_c).apply(gate)
        ok, oc = o.export()
        m = np.flatnonzero((ok == k2[j]).all(axis=1))
        assert len(m) == 1 and oc[m[0], 0] == c2[j, 0], (j, oc[m[0], 0] if len(m) else None, c2[j, 0])
    say(f"RX(q0): {SAMPLES} sampled outputs bit-identical")
