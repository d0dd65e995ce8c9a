"""Pauli-string density D_t(x) (Appendix D) on the HIP path (needs a GPU),
against the oracle's bin rule applied to the oracle's own coefficients (the
binary64 propagations are bit-identical, so the counts must be equal)."""

import sys

import numpy as np
import pytest

import workload as w
from oracle import OracleSum
from oracle.diag import density, density_counts
from gpu_common import gpu_sum, run_both

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def test_density_127q_kicked_ising_counts_equal_oracle():
    """127-q kicked Ising, theta = 0.8, eps0 = 1e-4, 4 steps: signed and
    unsigned counts on uniform and log-spaced grids, with a pending truncation
    applied before counting."""
    lat = w.eagle_127()
    g, o, _ = run_both(lat, lat.center, 0.8, 4, 1e-4, check_each=False)
    _, oc = o.export()
    c = oc[:, 0]
    grids = [(np.linspace(-1, 1, 201), True), (np.linspace(0, 1, 4097), False),
             (np.concatenate([[0.0], np.logspace(-6, 0, 61)]), False),
             (np.linspace(-0.5, 0.5, 7), True)]
    for edges, signed in grids:
        got = g.histogram(edges, signed)
        want = density_counts(c, edges, signed)
        say(f"n = {len(c)}, bins {len(edges) - 1} signed={signed}: below/above {got[-2:]}")
        assert np.array_equal(got, want)
    from paper_2506_13241_amd.diagnostics import density as gpu_density
    xg, dg = gpu_density(g, 100)
    xo, do = density(c, 100)
    assert np.array_equal(xg, xo) and np.array_equal(dg, do)


def test_density_lanes_and_ragged_sizes():
    """Three lanes with different maxima; sizes from 1 string to a ragged
    tail of a few tiles."""
    n = 10
    for m in (1, 37, 5000):
        terms, coeffs = w.random_pauli_set(n, m, seed=60 + m, lanes=3)
        coeffs[:, 1] *= 1e-3
        g, o = gpu_sum(n, terms, coeffs), OracleSum(n, terms, coeffs)
        gates = w.random_gates(n, 6, seed=61, max_weight=2, lanes=3)
        g.apply_rotation_layer(gates, 1e-3)
        o.apply(gates, 1e-3)
        _, oc = o.export()
        edges = np.linspace(-1, 1, 33)
        for lane in range(3):
            assert np.array_equal(g.histogram(edges, True, lane), density_counts(oc[:, lane], edges, True))


def test_density_empty_and_argument_errors():
    import paper_2506_13241_amd as P
    n = 6
    terms, coeffs = w.single_pauli_term(n, {2: "Z"})
    g = gpu_sum(n, terms, coeffs)
    g.truncate(2.0)  # removes the only string
    assert g.size() == 0
    assert g.histogram(np.linspace(-1, 1, 9)).sum() == 0
    g2 = gpu_sum(n, terms, coeffs)
    assert g2.histogram(np.array([0.0, 0.5, 1.0])).tolist() == [0, 1, 0, 0]
    for edges, lane in ((np.array([0.0, 0.0]), 0), (np.array([1.0]), 0), (np.linspace(0, 1, 4098), 0),
                        (np.array([0.0, np.inf]), 0), (np.array([0.0, 1.0]), 1)):
        with pytest.raises(P.PsError):
            g2.histogram(edges, True, lane)
