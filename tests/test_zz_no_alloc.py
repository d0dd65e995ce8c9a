"""The allocation-free histogram entry point (pauli_sum_histogram_noalloc),
called through the C ABI, against pauli_sum_histogram on the same operators
and against the oracle's bin rule: two calls in a row, the second with a
smaller operator and fewer bins, so counters left by the first call would
show."""

import sys

import numpy as np
import pytest

import workload as w
from oracle import OracleSum
from oracle.diag import density_counts
from gpu_common import gpu_sum, run_both

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def test_noalloc_histogram_matches_allocating_call_twice():
    import paper_2506_13241_amd as P
    lat = w.eagle_127()
    say("noalloc: 127q theta 0.8 eps 1e-4, 3 steps, 4096 signed bins")
    g, o, _ = run_both(lat, lat.center, 0.8, 3, 1e-4, check_each=False)
    _, oc = o.export()
    big = np.linspace(-1.0, 1.0, 4097)  # the maximum bin count
    want = density_counts(oc[:, 0], big, True)
    a1 = g.histogram(big, True, noalloc=False)
    b1 = g.histogram(big, True, noalloc=True)
    assert np.array_equal(a1, want)
    assert np.array_equal(b1, want)
    assert int(b1.sum()) == g.size()

    say("noalloc: second call, 21q patch, 2 steps, 3 lanes, 33 unsigned bins")
    small = w.heavy_hex_21()
    terms, coef = w.single_pauli_term(small.n, {10: "Z"})
    coef3 = np.repeat(coef.reshape(-1, 1), 3, axis=1) * np.array([1.0, -0.5, 2.0])
    g2 = gpu_sum(small.n, terms, coef3)
    o2 = OracleSum(small.n, terms, coef3)
    zz, rx = w.kicked_ising_step(small, 0.6)
    for _ in range(2):
        g2.apply_rotation_layer(zz, 1e-3).apply_rotation_layer(rx, 1e-3)
        o2.apply(zz, 1e-3).apply(rx, 1e-3)
    _, oc2 = o2.export()
    edges = np.logspace(-4, 0, 34)
    for lane in range(3):
        want2 = density_counts(oc2[:, lane], edges, False)
        b2 = g2.histogram(edges, False, lane, noalloc=True)
        a2 = g2.histogram(edges, False, lane, noalloc=False)
        assert b2.size == 35
        assert np.array_equal(b2, want2), (lane, b2, want2)
        assert np.array_equal(a2, b2)

    # beyond the fixed array: refused before any device work
    with pytest.raises(P.PsError) as ei:
        g2.histogram(np.linspace(-1.0, 1.0, 4098), True, noalloc=True)
    assert ei.value.code == P.PS_ERR_INVALID
    # the handle still answers afterwards
    assert np.array_equal(g2.histogram(edges, False, 0, noalloc=True), density_counts(oc2[:, 0], edges, False))


def test_noalloc_histogram_empty_operator():
    n = 6
    terms, coeffs = w.single_pauli_term(n, {2: "Z"})
    g = gpu_sum(n, terms, coeffs)
    g.truncate(2.0)  # removes the only string
    assert g.size() == 0
    assert g.histogram(np.linspace(-1, 1, 9), noalloc=True).sum() == 0
