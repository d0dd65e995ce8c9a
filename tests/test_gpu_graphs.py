"""RX layers replayed from HIP graphs (needs a GPU).

Every replay is compared with the eager path on the same input, bit for bit,
with eager Clifford layers and host synchronisations between the replays."""

import sys

import numpy as np
import pytest

import workload as w
from gpu_common import gpu_sum

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def _pair(n, terms, coeffs, dtype=0, capacity=0):
    eager = gpu_sum(n, terms, coeffs, dtype=dtype, capacity=capacity)
    graph = gpu_sum(n, terms, coeffs, dtype=dtype, capacity=capacity).set_graphs(True)
    return eager, graph


def _same(a, b):
    ka, ca = a.export()
    kb, cb = b.export()
    assert np.array_equal(ka, kb)
    assert np.array_equal(ca, cb)


def test_graph_replays_equal_eager_127q():
    lat = w.eagle_127()
    zz, rx = w.kicked_ising_step(lat, 0.8)
    terms, coef = w.single_pauli_term(lat.n, {62: "Z"})
    e, g = _pair(lat.n, terms, coef)
    for t in range(9):
        e.apply_rotation_layer(zz, 1e-4).apply_rotation_layer(rx, 1e-4)
        g.apply_rotation_layer(zz, 1e-4).apply_rotation_layer(rx, 1e-4)
        _same(e, g)
        assert g.expectation_z()[0] == e.expectation_z()[0]
    st = g.stats()
    say(f"graphs: {st['graph_captures']} captures, {st['graph_replays']} replays")
    assert st["graph_captures"] + st["graph_replays"] >= 9
    assert st["graph_replays"] >= 1


def test_graph_replays_with_growth_and_lanes_fp32():
    """16 observable lanes in binary32 from a small capacity: the capacity grows
    between and inside replays (graphs are dropped and captured again)."""
    lat = w.eagle_127()
    obs = w.random_observables(lat.n, 16, 20250616)
    words = np.stack([w.pauli_words(lat.n, ob) for ob in obs])
    zz, rx = w.kicked_ising_step(lat, 0.8, lanes=16)
    e, g = _pair(lat.n, words, np.eye(16), dtype=1, capacity=1024)
    for t in range(5):
        e.apply_rotation_layer(zz, 1e-4).apply_rotation_layer(rx, 1e-4)
        g.apply_rotation_layer(zz, 1e-4).apply_rotation_layer(rx, 1e-4)
        _same(e, g)
    st = g.stats()
    say(f"lanes: {st['graph_captures']} captures, {st['graph_replays']} replays, |O| = {g.size()}")
    assert st["graph_captures"] >= 2


def test_graphs_off_again_and_timing_bypass():
    lat = w.heavy_hex_21()
    zz, rx = w.kicked_ising_step(lat, 0.6)
    terms, coef = w.single_pauli_term(lat.n, {10: "Z"})
    e, g = _pair(lat.n, terms, coef)
    for t in range(4):
        if t == 2:
            g.set_graphs(False)
        if t == 3:
            g.set_graphs(True).set_timing(True)  # timing on: eager launches
        e.apply_rotation_layer(zz, 1e-6).apply_rotation_layer(rx, 1e-6)
        g.apply_rotation_layer(zz, 1e-6).apply_rotation_layer(rx, 1e-6)
        _same(e, g)
    st = g.stats()
    assert st["graph_captures"] + st["graph_replays"] >= 2


def test_graph_replays_equal_oracle_127q():
    """The benchmark workload (127 q, theta_h = 0.8, eps0 = 1e-4, binary64)
    with every RX run replayed from a graph once captured: keys and
    coefficients equal the oracle's bit for bit after every step (Eq.
    update_rule, Eq. truncation1), with at least one replay among the steps."""
    from oracle import OracleSum
    from gpu_common import assert_same_operator

    lat = w.eagle_127()
    zz, rx = w.kicked_ising_step(lat, 0.8)
    terms, coef = w.single_pauli_term(lat.n, {62: "Z"})
    # capacity for the whole run: no growth, so the buffers (part of a
    # graph's key) stay put and later steps replay
    g = gpu_sum(lat.n, terms, coef, capacity=1 << 22).set_graphs(True)
    o = OracleSum(lat.n, terms, coef)
    for t in range(5):
        g.apply_rotation_layer(zz, 1e-4).apply_rotation_layer(rx, 1e-4)
        o.apply(zz, 1e-4).apply(rx, 1e-4)
        assert_same_operator(g, o, coeff_exact=True)
        assert abs(g.expectation_z()[0] - o.expectation_z()[0]) <= 1e-12
        say(f"graph vs oracle step {t + 1}: |O| = {g.size()}")
    st = g.stats()
    say(f"graphs: {st['graph_captures']} captures, {st['graph_replays']} replays")
    assert st["graph_replays"] >= 1
