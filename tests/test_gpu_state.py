"""State handling of a handle on the HIP path (needs an MI355X): resume from
an export, the readout of an operator with a pending truncation, and the
guard of the look-back epoch, each against the FP64 oracle or the same run
without the feature, bit for bit."""

import sys

import numpy as np
import pytest

import workload as w
from oracle import OracleSum
from gpu_common import assert_same_operator, gpu_sum

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.mark.parametrize("dtype,lanes", [(0, 1), (1, 1), (0, 4)])
def test_resume_from_export_is_bit_identical(dtype, lanes):
    """10 Trotter steps == 5 steps, export, create a new handle from the
    export, 5 more steps (127 q, theta 0.8, eps0 1e-4)."""
    import paper_2506_13241_amd as P
    say(f"resume dtype={dtype} lanes={lanes}")
    lat = w.eagle_127()
    terms, coef = w.single_pauli_term(lat.n, {62: "Z"}, lanes=lanes)
    if lanes > 1:
        coef = coef * np.linspace(1.0, -0.5, lanes)
    zz, rx = w.kicked_ising_step(lat, 0.8)
    full = P.PauliSum(lat.n, terms, coef, dtype=dtype)
    first = P.PauliSum(lat.n, terms, coef, dtype=dtype)
    for _ in range(5):
        full.apply_rotation_layer(zz, 1e-4).apply_rotation_layer(rx, 1e-4)
        first.apply_rotation_layer(zz, 1e-4).apply_rotation_layer(rx, 1e-4)
    k5, c5 = first.export()
    first.close()
    resumed = P.PauliSum(lat.n, k5, c5.astype(np.float64), dtype=dtype)
    for t in range(5):
        full.apply_rotation_layer(zz, 1e-4).apply_rotation_layer(rx, 1e-4)
        resumed.apply_rotation_layer(zz, 1e-4).apply_rotation_layer(rx, 1e-4)
        ea, eb = full.expectation_z(), resumed.expectation_z()
        assert np.array_equal(ea, eb), (t, ea, eb)
    ka, ca = full.export()
    kb, cb = resumed.export()
    say(f"  {ka.shape[0]} strings after 10 steps")
    assert np.array_equal(ka, kb)
    assert np.array_equal(ca, cb)


def test_readout_with_pending_truncation_equals_materialized():
    """<Z> read while the last gate's truncation is still pending (only the
    x = 0 prefix is read) equals <Z> after the truncation has been applied
    to the whole operator, bit for bit, and the oracle's to 1e-12; the norm
    read with a pending truncation equals the norm after it to 1e-12."""
    lat = w.eagle_127()
    terms, coef = w.single_pauli_term(lat.n, {62: "Z"})
    zz, rx = w.kicked_ising_step(lat, 0.8)
    g = gpu_sum(lat.n, terms, coef)
    o = OracleSum(lat.n, terms, coef)
    for t in range(4):
        g.apply_rotation_layer(zz, 1e-4).apply_rotation_layer(rx, 1e-4)
        o.apply(zz, 1e-4).apply(rx, 1e-4)
        ez_pending = g.expectation_z()
        nrm_pending = g.norm2()
        n = g.size()  # applies the pending truncation to the whole operator
        ez_done = g.expectation_z()
        nrm_done = g.norm2()
        say(f"step {t + 1}: |O|={n} <Z62>={ez_pending[0]:.15f}")
        assert np.array_equal(ez_pending, ez_done)
        assert abs(ez_pending[0] - o.expectation_z()[0]) <= 1e-12
        assert abs(nrm_pending[0] - nrm_done[0]) <= 1e-12 * nrm_done[0]
        assert abs(nrm_done[0] - o.norm2()[0]) <= 1e-12 * nrm_done[0]
    assert_same_operator(g, o, coeff_exact=True)


def test_readout_pending_truncation_lanes_and_empty_prefix():
    """Three lanes and a pending truncation that removes every x = 0 string."""
    n = 12
    terms, coeffs = w.random_pauli_set(n, 4000, seed=5, lanes=3, eps0=1e-3)
    gates = w.random_gates(n, 8, seed=6, max_weight=2, lanes=3)
    g, o = gpu_sum(n, terms, coeffs), OracleSum(n, terms, coeffs)
    g.apply_rotation_layer(gates, 1e-2)
    o.apply(gates, 1e-2)
    assert np.abs(g.expectation_z() - o.expectation_z()).max() <= 1e-12
    assert_same_operator(g, o, coeff_exact=True)
    # only X strings: the prefix is empty; RX(0) on qubit 0 leaves them as
    # they are and leaves a truncation at 0.4 pending
    terms2 = np.zeros((3, 4), dtype=np.uint64)
    terms2[:, 0] = [1, 2, 3]
    g2 = gpu_sum(n, terms2, np.array([1.0, 0.5, 0.25]))
    g2.apply_rotation_layer(w.GateList(w.pauli_words(n, {0: "X"})[None, :], np.array([[0.0]])), 0.4)
    assert g2.expectation_z()[0] == 0.0
    assert g2.size() == 2


def test_lookback_epoch_guard_across_the_tag_wrap():
    """The epoch starts just below the 24-bit wrap; the library clears the
    status words and restarts it, and the run stays bit-identical to the
    oracle (21-q patch untruncated, then 127 q with truncation)."""
    import paper_2506_13241_amd as P
    limit = (1 << 24) - 3  # largest epoch the setter accepts
    for lat, theta, eps, steps in ((w.heavy_hex_21(), 0.6, 0.0, 4), (w.eagle_127(), 0.8, 1e-4, 4)):
        terms, coef = w.single_pauli_term(lat.n, {lat.center: "Z"})
        zz, rx = w.kicked_ising_step(lat, theta)
        g = gpu_sum(lat.n, terms, coef)
        o = OracleSum(lat.n, terms, coef)
        g.set_lookback_epoch(limit - 30)
        assert g.lookback_epoch() == limit - 30
        wrapped = False
        for t in range(steps):
            before = g.lookback_epoch()
            g.apply_rotation_layer(zz, eps).apply_rotation_layer(rx, eps)
            o.apply(zz, eps).apply(rx, eps)
            after = g.lookback_epoch()
            say(f"{lat.name} step {t + 1}: epoch {before} -> {after}")
            assert after < (1 << 24)
            wrapped |= after < before
            assert_same_operator(g, o, coeff_exact=True)
            assert abs(g.expectation_z()[0] - o.expectation_z()[0]) <= 1e-12
        assert wrapped
    with pytest.raises(P.PsError):
        g.set_lookback_epoch(0)
    with pytest.raises(P.PsError):
        g.set_lookback_epoch(limit + 1)
