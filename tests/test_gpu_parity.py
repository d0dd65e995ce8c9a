"""HIP path against the FP64 oracle, element by element (needs an MI355X).

Bar: untruncated and truncated FP64 runs give the oracle's key set exactly and
its coefficients to 1e-12 of the largest one (the arithmetic is the same, so
in practice they are bit-identical); FP32 and batched forms are stated against
FP64.
"""

import math
import sys

import numpy as np
import pytest

import workload as w
from workload.lattice import chain
from oracle import OracleSum
from oracle import statevector as sv
from gpu_common import assert_same_operator, gpu_sum, run_both

pytestmark = pytest.mark.gpu
PI = math.pi


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def lib():
    import paper_2506_13241_amd as P
    P.load_library()
    return P


# ---------------------------------------------------------------- single gates

def rx_prefix(n, upto):
    """RX(0) on qubits 0..upto-1: identity that moves the stored rotation to `upto`."""
    gens = np.stack([w.pauli_words(n, {q: "X"}) for q in range(upto)]) if upto else np.zeros((0, 4), np.uint64)
    return w.GateList(gens.astype(np.uint64), np.zeros((upto, 1)))


@pytest.mark.parametrize("n", [1, 5, 64, 65, 127, 128])
@pytest.mark.parametrize("theta", [0.37, -2.1, 0.0, PI / 2, PI, -PI / 2])
def test_single_rx_gate_random_sets(n, theta):
    say(f"single rx n={n} theta={theta}")
    size = 3000 if n > 5 else 400
    support = list(range(min(n, 9)))
    terms, coeffs = w.random_pauli_set(n, size, seed=n * 7 + 1, support=support)
    j = min(n - 1, 3)
    pre = rx_prefix(n, j)
    gate = w.GateList(w.pauli_words(n, {j: "X"})[None, :], np.array([[theta]]))
    g = gpu_sum(n, terms, coeffs)
    o = OracleSum(n, terms, coeffs)
    g.apply_rotation_layer(pre).apply_rotation_layer(gate)
    o.apply(pre).apply(gate)
    assert_same_operator(g, o, coeff_exact=True)


@pytest.mark.parametrize("eps0", [1e-3, 1e-1])
def test_rx_chain_with_truncation_many_tiles(eps0):
    """A run of RX gates over qubits 0..k on ~60k strings (many tiles, large
    and small pairing blocks) with truncation after every gate."""
    n = 20
    say(f"rx chain eps0={eps0}")
    terms, coeffs = w.random_pauli_set(n, 60000, seed=11, support=list(range(14)), eps0=1e-3)
    gates = w.GateList(np.stack([w.pauli_words(n, {q: "X"}) for q in range(n)]),
                       np.array([[0.3 + 0.1 * q] for q in range(n)]))
    g = gpu_sum(n, terms, coeffs)
    o = OracleSum(n, terms, coeffs)
    g.apply_rotation_layer(gates, eps0)
    o.apply(gates, eps0)
    assert_same_operator(g, o, coeff_exact=True)
    # a second full layer starts again at qubit 0
    g.apply_rotation_layer(gates, eps0)
    o.apply(gates, eps0)
    assert_same_operator(g, o, coeff_exact=True)


def test_clifford_zz_layer_and_resort():
    n = 127
    lat = w.eagle_127()
    say("clifford zz layer")
    terms, coeffs = w.random_pauli_set(n, 20000, seed=5, support=w.ball(lat, 62, 4))
    zz = w.kicked_ising_step(lat, 0.8)[0]
    g = gpu_sum(n, terms, coeffs)
    o = OracleSum(n, terms, coeffs)
    g.apply_rotation_layer(zz)
    o.apply(zz)
    assert_same_operator(g, o, coeff_exact=True)


def test_clifford_run_of_mixed_z_generators():
    """A run of Z-only Clifford rotations through every branch of the pass's
    composite form: weight-2 generators at 40 distinct qubit offsets (more
    than the pass groups, so some are applied one by one), repeated pairs,
    weights 1, 3 and 4, angles pi/2, -pi/2 and pi in random order; against the
    oracle, bit for bit, on 20000 random strings over all 127 qubits."""
    from workload.circuit import GateList, pauli_words
    n = 127
    rng = np.random.default_rng(77)
    gens = []
    for d in rng.choice(np.arange(1, n), 40, replace=False):
        for _ in range(3):
            a = int(rng.integers(0, n - int(d)))
            gens.append(pauli_words(n, {a: "Z", a + int(d): "Z"}))
    gens += [gens[i] for i in range(0, 30, 3)]  # repeated pairs
    for wgt in (1, 1, 3, 3, 4, 4):
        gens.append(pauli_words(n, {int(q): "Z" for q in rng.choice(n, wgt, replace=False)}))
    angles = rng.choice([PI / 2, -PI / 2, PI], len(gens))
    perm = rng.permutation(len(gens))
    layer = GateList(np.stack(gens)[perm].astype(np.uint64), angles[perm][:, None].astype(np.float64))
    terms, coeffs = w.random_pauli_set(n, 20000, seed=31)
    say(f"clifford run of {len(layer)} mixed Z generators")
    g = gpu_sum(n, terms, coeffs)
    o = OracleSum(n, terms, coeffs)
    g.apply_rotation_layer(layer)
    o.apply(layer)
    assert_same_operator(g, o, coeff_exact=True)
    assert g.size() == len(terms)


def test_empty_and_single_string():
    lat = w.heavy_hex_21()
    zz, rx = w.kicked_ising_step(lat, 0.6)
    g = gpu_sum(lat.n, np.zeros((0, 4), np.uint64), np.zeros((0, 1)))
    g.apply_rotation_layer(zz).apply_rotation_layer(rx)
    assert g.size() == 0 and g.expectation_z()[0] == 0.0
    terms, coef = w.single_pauli_term(lat.n, {10: "X"})
    g = gpu_sum(lat.n, terms, coef)
    o = OracleSum(lat.n, terms, coef)
    g.apply_rotation_layer(zz, 1e-3).apply_rotation_layer(rx, 1e-3)
    o.apply(zz, 1e-3).apply(rx, 1e-3)
    assert_same_operator(g, o, coeff_exact=True)
    # eps0 >= 1 removes everything, the max included
    g.truncate(1.0)
    assert g.size() == 0


def test_invalid_inputs_rejected():
    import paper_2506_13241_amd as P
    with pytest.raises(P.PsError) as e:
        gpu_sum(5, w.pauli_words(6, {5: "Z"})[None, :], np.ones((1, 1)))
    assert e.value.code == P.PS_ERR_INVALID
    with pytest.raises(P.PsError) as e:
        gpu_sum(5, w.pauli_words(5, {1: "Z"})[None, :], np.array([[np.nan]]))
    assert e.value.code == P.PS_ERR_NONFINITE


# ---------------------------------------------------------------- kicked Ising

def test_patch21_untruncated_against_oracle_and_statevector():
    """21-qubit patch, theta_h = 0.6, 5 steps, no truncation, FP64: key sets
    and coefficients equal the oracle's for steps 1-4; step 5 (beyond the
    oracle's memory) against the statevector <Z> and norm conservation."""
    lat = w.heavy_hex_21()
    say("patch21 steps 1-4")
    g, o, out = run_both(lat, 10, 0.6, 4, 0.0, coeff_exact=True)
    ref = sv.kicked_ising_magnetization(lat.n, lat.edges, 10, 0.6, 5)
    for t, (ez_g, ez_o, ng, no) in enumerate(out):
        assert ng == no
        assert abs(ez_g - ref[t]) <= 1e-12
    zz, rx = w.kicked_ising_step(lat, 0.6)
    say("patch21 step 5")
    g.apply_rotation_layer(zz).apply_rotation_layer(rx)
    assert abs(g.expectation_z()[0] - ref[4]) <= 1e-12
    assert abs(g.norm2()[0] - 1.0) <= 1e-11
    say(f"patch21 step5 size {g.size()}")


@pytest.mark.parametrize("eps0", [0.0, 1e-5])
def test_table1_127q(eps0):
    """Appendix E, Table 1 at 127 qubits: keys and coefficients equal the
    oracle's, and <M_t> matches the printed values."""
    from conftest import load_table1
    lat = w.eagle_127()
    steps = 4 if eps0 == 0.0 else 5
    say(f"table1 eps0={eps0}")
    _, _, out = run_both(lat, 62, 0.9 * PI, steps, eps0, coeff_exact=True)
    for (t, svv, e0, e5), (ez_g, ez_o, ng, no) in zip(load_table1(), out):
        target = svv if eps0 == 0.0 else e5
        assert abs(ez_g - target) <= 1e-13, (t, ez_g, target)


def test_theta08_eps1e4_127q_against_oracle():
    """The benchmark workload (127 q, theta_h = 0.8, eps0 = 1e-4, FP64) for the
    first steps the oracle reaches quickly."""
    lat = w.eagle_127()
    say("127q theta 0.8 eps 1e-4")
    _, _, out = run_both(lat, 62, 0.8, 5, 1e-4, coeff_exact=True)
    say(str(out))


def test_clifford_points_gpu():
    lat = w.eagle_127()
    terms, coef = w.single_pauli_term(lat.n, {62: "Z"})
    for th in (0.0, PI / 2):
        g = gpu_sum(lat.n, terms, coef)
        zz, rx = w.kicked_ising_step(lat, th)
        for _ in range(5):
            g.apply_rotation_layer(zz).apply_rotation_layer(rx)
            assert g.size() == 1
        if th == 0.0:
            assert g.expectation_z()[0] == 1.0


def test_sign_probe_y_observable_gpu():
    lat = chain(7)
    ref = sv.kicked_ising_magnetization(lat.n, lat.edges, 3, 0.7, 4, observable={3: "Y"})
    terms, coef = w.single_pauli_term(lat.n, {3: "Y"})
    g = gpu_sum(lat.n, terms, coef)
    zz, rx = w.kicked_ising_step(lat, 0.7)
    for t in range(4):
        g.apply_rotation_layer(zz).apply_rotation_layer(rx)
        assert abs(g.expectation_z()[0] - ref[t]) <= 1e-13


# ---------------------------------------------------------------- capacity, determinism

def test_capacity_growth_transparent():
    lat = w.eagle_127()
    say("capacity growth")
    terms, coef = w.single_pauli_term(lat.n, {62: "Z"})
    g = gpu_sum(lat.n, terms, coef, capacity=1)  # library minimum, grows on demand
    o = OracleSum(lat.n, terms, coef)
    zz, rx = w.kicked_ising_step(lat, 0.8)
    for _ in range(5):
        g.apply_rotation_layer(zz, 1e-4).apply_rotation_layer(rx, 1e-4)
        o.apply(zz, 1e-4).apply(rx, 1e-4)
    assert_same_operator(g, o, coeff_exact=True)


def test_determinism_bit_identical():
    lat = w.eagle_127()
    terms, coef = w.single_pauli_term(lat.n, {62: "Z"})
    res = []
    for _ in range(2):
        g = gpu_sum(lat.n, terms, coef)
        zz, rx = w.kicked_ising_step(lat, 0.8)
        for _ in range(5):
            g.apply_rotation_layer(zz, 1e-4).apply_rotation_layer(rx, 1e-4)
        k, c = g.export()
        res.append((k, c, g.expectation_z()[0]))
    assert np.array_equal(res[0][0], res[1][0]) and np.array_equal(res[0][1], res[1][1])
    assert res[0][2] == res[1][2]


def test_clifford_resort_group_sort_and_radix_fallback():
    """The re-sort after a Clifford layer sorts each x-group inside one
    workgroup when no group exceeds 2048 strings, and falls back to the radix
    sort otherwise.  Both cases against the oracle, bit for bit: a set of many
    small groups, and the same set plus one x-group of 6000 strings."""
    import paper_2506_13241_amd as P
    n = 127
    lat = w.eagle_127()
    zz = w.kicked_ising_step(lat, 0.8)[0]
    terms, coeffs = w.random_pauli_set(n, 30000, seed=21, support=w.ball(lat, 62, 4))
    # one big x-group: 6000 strings sharing the x mask of terms[0], random z on the ball
    zs, _ = w.random_pauli_set(n, 8000, seed=22, support=w.ball(lat, 62, 4))
    big = np.repeat(terms[:1], len(zs), axis=0)
    big[:, 2:] = zs[:, 2:]
    big = np.unique(big, axis=0)[:6000]
    bc = np.linspace(0.1, 1.0, len(big))[:, None]
    for label, tt, cc in (("small groups", terms, coeffs),
                          ("one group of 6000", np.concatenate([terms, big]), np.concatenate([coeffs, bc]))):
        tt, idx = np.unique(tt, axis=0, return_index=True)
        cc = cc[idx]
        say(f"resort: {label}, {len(tt)} strings")
        g = gpu_sum(n, tt, cc)
        o = OracleSum(n, tt, cc)
        g.stats(reset=True)
        g.apply_rotation_layer(zz)
        o.apply(zz)
        assert_same_operator(g, o, coeff_exact=True)
        passes = g.stats()["sort_passes"]
        if label == "small groups":
            assert passes == 1
        else:
            assert passes > 1


def test_rx_tiles_finding_their_own_boundaries_equal_oracle():
    """With the grid's boundary step switched off, every RX tile finds its
    two boundaries itself (the path a tile takes when they do not arrive in
    time): the benchmark workload still equals the oracle bit for bit
    (127 q, theta_h = 0.8, eps0 = 1e-4, 5 steps)."""
    lat = w.eagle_127()
    zz, rx = w.kicked_ising_step(lat, 0.8)
    terms, coef = w.single_pauli_term(lat.n, {62: "Z"})
    g = gpu_sum(lat.n, terms, coef).set_rx_boundary_prologue(False)
    o = OracleSum(lat.n, terms, coef)
    for t in range(5):
        g.apply_rotation_layer(zz, 1e-4).apply_rotation_layer(rx, 1e-4)
        o.apply(zz, 1e-4).apply(rx, 1e-4)
        assert_same_operator(g, o, coeff_exact=True)
