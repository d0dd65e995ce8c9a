"""Batched coefficient lanes and binary32 storage on the HIP path (needs a GPU).

Lanes in binary64 must equal the oracle's multi-lane run bit for bit (same
operations).  Binary32 runs are stated against binary64: identical key sets
when nothing is truncated, coefficients within a few binary32 ulps of the
largest coefficient, and |<Z>| differences far below the 1e-3 bar.
"""

import math
import sys

import numpy as np
import pytest

import workload as w
from oracle import OracleSum
from gpu_common import assert_same_operator, gpu_sum

pytestmark = pytest.mark.gpu
PI = math.pi


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def lib():
    import paper_2506_13241_amd as P
    P.load_library()
    return P


def theta_sweep(lanes):
    return np.linspace(0.0, PI / 2, lanes)


@pytest.mark.parametrize("lanes", [2, 3, 8, 32])
def test_theta_sweep_lanes_fp64_equal_oracle(lanes):
    """theta_h sweep carried as lanes (one key pass for all angles), 21-q patch,
    3 steps, truncation on the max over lanes: keys and every lane's
    coefficients equal the oracle's."""
    lat = w.heavy_hex_21()
    th = theta_sweep(lanes)
    zz, rx = w.kicked_ising_step(lat, th, lanes=lanes)
    terms, coef = w.single_pauli_term(lat.n, {10: "Z"}, lanes=lanes)
    g = gpu_sum(lat.n, terms, coef)
    o = OracleSum(lat.n, terms, coef)
    for _ in range(3):
        g.apply_rotation_layer(zz, 1e-4).apply_rotation_layer(rx, 1e-4)
        o.apply(zz, 1e-4).apply(rx, 1e-4)
    assert_same_operator(g, o, coeff_exact=True)
    assert np.allclose(g.expectation_z(), o.expectation_z(), atol=1e-12, rtol=0)


def test_lanes_untruncated_equal_solo_runs():
    """Each untruncated lane equals its solo run (the key set of the batch is
    the union; missing keys of a lane read as zero)."""
    lat = w.heavy_hex_21()
    th = np.array([0.3, 0.8, 1.2])
    zz, rx = w.kicked_ising_step(lat, th, lanes=3)
    terms, coef = w.single_pauli_term(lat.n, {10: "Z"}, lanes=3)
    g = gpu_sum(lat.n, terms, coef)
    for _ in range(3):
        g.apply_rotation_layer(zz).apply_rotation_layer(rx)
    batch = g.as_dict()
    for a, t in enumerate(th):
        z1, r1 = w.kicked_ising_step(lat, float(t))
        t1, c1 = w.single_pauli_term(lat.n, {10: "Z"})
        s = gpu_sum(lat.n, t1, c1)
        for _ in range(3):
            s.apply_rotation_layer(z1).apply_rotation_layer(r1)
        solo = s.as_dict()
        for k, v in batch.items():
            assert v[a] == solo.get(k, np.zeros(1))[0]
        for k in solo:
            assert k in batch


def test_observable_batch_lanes_127q():
    """16 weight-1/2 Z observables (seed 20250616) as lanes on the 127-q
    lattice, theta_h = 0.8, eps0 = 1e-4: equal to the oracle's batched run."""
    lat = w.eagle_127()
    obs = w.random_observables(lat.n, 16, 20250616)
    words = np.stack([w.pauli_words(lat.n, ob) for ob in obs])
    coeffs = np.eye(16)
    zz, rx = w.kicked_ising_step(lat, 0.8, lanes=16)
    g = gpu_sum(lat.n, words, coeffs)
    o = OracleSum(lat.n, words, coeffs)
    for t in range(3):
        say(f"observable batch step {t + 1}")
        g.apply_rotation_layer(zz, 1e-4).apply_rotation_layer(rx, 1e-4)
        o.apply(zz, 1e-4).apply(rx, 1e-4)
    assert_same_operator(g, o, coeff_exact=True)


def test_fp32_untruncated_patch_against_fp64():
    """Binary32 storage, no truncation: same keys as binary64; coefficients
    within 1e-5 of the largest; <Z> within 1e-6."""
    lat = w.heavy_hex_21()
    zz, rx = w.kicked_ising_step(lat, 0.6)
    terms, coef = w.single_pauli_term(lat.n, {10: "Z"})
    g64 = gpu_sum(lat.n, terms, coef, dtype=0)
    g32 = gpu_sum(lat.n, terms, coef, dtype=1)
    for _ in range(4):
        g64.apply_rotation_layer(zz).apply_rotation_layer(rx)
        g32.apply_rotation_layer(zz).apply_rotation_layer(rx)
    k64, c64 = g64.export()
    k32, c32 = g32.export()
    assert np.array_equal(k64, k32)
    assert np.abs(c32.astype(np.float64) - c64).max() <= 1e-5 * np.abs(c64).max()
    assert abs(g32.expectation_z()[0] - g64.expectation_z()[0]) <= 1e-6
    assert abs(g32.norm2()[0] - 1.0) <= 1e-5


def test_fp32_compensated_products_are_correctly_rounded_singletons():
    """A single RX gate on a random set: every binary32 output that comes from
    one product equals the binary64 value rounded to binary32 (error-free
    product of the split cos/sin, one rounding)."""
    n = 20
    terms, coeffs = w.random_pauli_set(n, 3000, seed=3, support=list(range(10)))
    coeffs32 = coeffs.astype(np.float32).astype(np.float64)  # exactly representable inputs
    gate = w.GateList(w.pauli_words(n, {0: "X"})[None, :], np.array([[0.7]]))
    g32 = gpu_sum(n, terms, coeffs32, dtype=1).apply_rotation_layer(gate)
    o = OracleSum(n, terms, coeffs32).apply(gate)
    k32, c32 = g32.export()
    ok, oc = o.export()
    assert np.array_equal(k32, ok)
    ref = oc[:, 0].astype(np.float32)
    # pairs round twice in binary64 then once more; singletons are exact
    diff = np.abs(c32[:, 0].astype(np.float64) - ref.astype(np.float64))
    ulp = np.spacing(np.abs(ref)).astype(np.float64)
    assert np.all(diff <= ulp)
    assert np.mean(diff == 0) > 0.9


def test_fp32_127q_theta08_delta_z_against_fp64():
    """The precision form of the benchmark workload: binary32 + two-sum against
    binary64 on the same GPU, eps0 = 1e-4, 12 Trotter steps: |delta <Z62>| per
    step stays below the 1e-3 bar."""
    lat = w.eagle_127()
    zz, rx = w.kicked_ising_step(lat, 0.8)
    terms, coef = w.single_pauli_term(lat.n, {62: "Z"})
    g64 = gpu_sum(lat.n, terms, coef, dtype=0)
    g32 = gpu_sum(lat.n, terms, coef, dtype=1)
    worst = 0.0
    for t in range(12):
        g64.apply_rotation_layer(zz, 1e-4).apply_rotation_layer(rx, 1e-4)
        g32.apply_rotation_layer(zz, 1e-4).apply_rotation_layer(rx, 1e-4)
        d = abs(g32.expectation_z()[0] - g64.expectation_z()[0])
        worst = max(worst, d)
        say(f"fp32 step {t + 1}: |dZ62| = {d:.3e}  |O| = {g64.size()} / {g32.size()}")
    assert worst <= 1e-3


def _sweep_127q(lanes=32):
    lat = w.eagle_127()
    th = theta_sweep(lanes)
    zz, rx = w.kicked_ising_step(lat, th, lanes=lanes)
    terms, coef = w.single_pauli_term(lat.n, {62: "Z"}, lanes=lanes)
    return lat, th, zz, rx, terms, coef


def test_fp32_theta_lanes_single_gate_within_one_ulp_of_oracle():
    """32 theta lanes (linspace(0, pi/2, 32)) in binary32 on the 127-q
    operator after 4 untruncated steps (2774 strings): one RX gate from that
    state (exactly representable in binary32) gives every lane's coefficient
    within one binary32 ulp of the oracle's binary64 value rounded to binary32
    (error-free products of the split cos/sin, two-sum, one rounding); keys
    equal."""
    lat, th, zz, rx, terms, coef = _sweep_127q()
    g = gpu_sum(lat.n, terms, coef, dtype=1)
    for _ in range(4):
        g.apply_rotation_layer(zz).apply_rotation_layer(rx)
    k0, c0 = g.export()
    c0 = c0.astype(np.float64)  # binary32 values, exact in binary64
    gate = w.GateList(w.pauli_words(lat.n, {0: "X"})[None, :], th[None, :].copy())
    g1 = gpu_sum(lat.n, k0, c0, dtype=1).apply_rotation_layer(gate)
    o1 = OracleSum(lat.n, k0, c0).apply(gate)
    k32, c32 = g1.export()
    ok, oc = o1.export()
    assert np.array_equal(k32, ok)
    ref = oc.astype(np.float32)
    diff = np.abs(c32.astype(np.float64) - ref.astype(np.float64))
    ulp = np.spacing(np.abs(ref)).astype(np.float64)
    say(f"single gate, 32 lanes: {k32.shape[0]} strings, exact {np.mean(diff == 0):.4f}")
    assert np.all(diff <= ulp)


def test_fp32_theta_lanes_untruncated_equal_oracle_within_rounding_bound():
    """The same 32 binary32 lanes for 5 untruncated steps (2.1e6 strings)
    against the oracle's binary64 lanes: identical key sets; per lane the
    2-norm of the coefficient error stays within G * 2^-22, G the number of
    RX gates.  Why: each gate is an orthogonal map on the pairs {I, I xor J}
    (Eq. update_rule), so it carries the incoming error vector without growth,
    and adds a rounding error of at most one ulp (2^-23 relative) per output
    plus the residue of the split cos/sin (below 2^-47); the lanes start with
    norm 1 and keep it."""
    lat, th, zz, rx, terms, coef = _sweep_127q()
    g = gpu_sum(lat.n, terms, coef, dtype=1)
    o = OracleSum(lat.n, terms, coef)
    steps = 5
    for t in range(steps):
        g.apply_rotation_layer(zz).apply_rotation_layer(rx)
        o.apply(zz).apply(rx)
        say(f"untruncated 32-lane step {t + 1}: |O| = {g.size()} / {o.size()}")
    gk, gc = g.export()
    ok, oc = o.export()
    assert np.array_equal(gk, ok)
    err = gc.astype(np.float64) - oc
    G = steps * len(rx.gens)
    per_lane = np.sqrt((err * err).sum(axis=0))
    say(f"per-lane error 2-norm max {per_lane.max():.3e}, elementwise max {np.abs(err).max():.3e}, "
        f"bound {G * 2.0 ** -22:.3e}")
    assert np.all(per_lane <= G * 2.0 ** -22)
    assert np.allclose(g.expectation_z(), o.expectation_z(), atol=G * 2.0 ** -22, rtol=0)


def test_fp32_theta_lanes_truncated_expectation_against_oracle():
    """32 binary32 theta lanes, eps0 = 1e-4 (keep a string when any lane is
    above its own threshold), 5 steps: <Z62> per lane within 1e-6 of the
    oracle's binary64 lanes at every step."""
    lat, th, zz, rx, terms, coef = _sweep_127q()
    g = gpu_sum(lat.n, terms, coef, dtype=1)
    o = OracleSum(lat.n, terms, coef)
    for t in range(5):
        g.apply_rotation_layer(zz, 1e-4).apply_rotation_layer(rx, 1e-4)
        o.apply(zz, 1e-4).apply(rx, 1e-4)
        d = np.abs(g.expectation_z() - o.expectation_z())
        say(f"eps 1e-4 32-lane step {t + 1}: |O| = {g.size()} / {o.size()}, max |dZ| = {d.max():.3e}")
        assert d.max() <= 1e-6


def test_fp32_two_sum_127q_eps1e5_against_fp64_per_step():
    """The precision form at its stated threshold: binary32 + two-sum against
    binary64 on the same GPU, 127 q, theta_h = 0.8, eps0 = 1e-5, Trotter steps
    1..20 while each run stays within a time budget of 55 s (the binary64
    run first, then the binary32 run, one at a time in device memory):
    |delta <Z62>| <= 1e-3 at every step, each step's value printed."""
    import time
    lat = w.eagle_127()
    zz, rx = w.kicked_ising_step(lat, 0.8)
    terms, coef = w.single_pauli_term(lat.n, {62: "Z"})
    budget, steps = 55.0, 20
    ez = {}
    for dt in (0, 1):
        g = gpu_sum(lat.n, terms, coef, dtype=dt)
        t0 = time.perf_counter()
        ez[dt] = []
        for t in range(steps if dt == 0 else len(ez[0])):
            g.apply_rotation_layer(zz, 1e-5).apply_rotation_layer(rx, 1e-5)
            ez[dt].append(float(g.expectation_z()[0]))
            say(f"{'f64' if dt == 0 else 'f32'} eps 1e-5 step {t + 1}: |O| = {g.size()}, "
                f"<Z62> = {ez[dt][-1]:.12f}, {time.perf_counter() - t0:.1f} s")
            if time.perf_counter() - t0 > budget:
                break
        g.close()
    k = min(len(ez[0]), len(ez[1]))
    d = [abs(a - b) for a, b in zip(ez[0][:k], ez[1][:k])]
    for t in range(k):
        say(f"step {t + 1}: |dZ62| = {d[t]:.3e}")
    assert k >= 12
    assert max(d) <= 1e-3
