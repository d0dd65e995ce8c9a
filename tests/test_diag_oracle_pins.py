"""Pins of the Pauli-string density reference (Appendix D) on the CPU."""

import numpy as np

import workload as w
from oracle import OracleSum
from oracle.diag import density, density_counts


def test_hand_counted_example():
    """Coefficients -1, -0.5, 0.2, 0.5, 1 over the signed bins of width 0.5:
    [-1,-0.5) holds -1, [-0.5,0) holds -0.5, [0,0.5) holds 0.2, and the
    closed last bin [0.5,1] holds 0.5 and 1."""
    c = np.array([0.2, -1.0, 0.5, -0.5, 1.0])
    got = density_counts(c, np.array([-1.0, -0.5, 0.0, 0.5, 1.0]))
    assert got.tolist() == [1, 1, 1, 2, 0, 0]


def test_unsigned_and_out_of_range():
    """|c| / M over the bins [0.25, 0.5) and [0.5, 0.75]: 0.1 below, 0.9 and
    1 above, 0.25 in the first bin, 0.5 and 0.75 in the closed last one."""
    c = np.array([0.1, -0.9, 1.0, -0.25, 0.5, 0.75]) * 8.0
    got = density_counts(c, np.array([0.25, 0.5, 0.75]), signed=False)
    assert got.tolist() == [1, 2, 1, 2]


def test_brute_force_against_a_python_loop():
    """Random coefficients on a random grid, every value placed by scanning
    the bins one by one."""
    rng = np.random.default_rng(3)
    c = rng.normal(size=400) * rng.choice([1e-6, 1e-3, 1.0], size=400)
    edges = np.sort(rng.uniform(-1.1, 1.1, 17))
    M = np.abs(c).max()
    want = np.zeros(18, dtype=np.uint64)
    for x in c:
        placed = False
        for k in range(16):
            lo, hi = M * edges[k], M * edges[k + 1]
            if lo <= x < hi or (k == 15 and x == hi):
                want[k] += 1
                placed = True
                break
        if not placed:
            want[16 if x < M * edges[0] else 17] += 1
    assert np.array_equal(density_counts(c, edges), want)


def test_density_normalised_and_symmetric_under_sign_flip():
    """D integrates to 1, the maximum lands in an end bin, and flipping every
    sign mirrors the signed density (up to values on a bin edge)."""
    lat = w.heavy_hex_21()
    zz, rx = w.kicked_ising_step(lat, 0.6)
    o = OracleSum(lat.n, *w.single_pauli_term(lat.n, {10: "Z"}))
    for _ in range(4):
        o.apply(zz).apply(rx)
    _, c = o.export()
    x, d = density(c[:, 0], 64)
    assert abs(d.sum() * (x[1] - x[0]) - 1.0) < 1e-12
    cnt = density_counts(c[:, 0], np.linspace(-1, 1, 65))
    assert cnt[0] + cnt[63] >= 1
    edges = np.linspace(-1, 1, 65)
    a = density_counts(c[:, 0], edges)[:64]
    b = density_counts(-c[:, 0], edges)[:64][::-1]
    on_edge = np.isin(c[:, 0] / np.abs(c[:, 0]).max(), edges).sum()
    assert np.abs(a.astype(np.int64) - b.astype(np.int64)).sum() <= 2 * on_edge
