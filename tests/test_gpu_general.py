"""General Pauli rotations on the HIP path (needs a GPU): any generator
sigma_J, any angle, in any order, against the oracle (whose update rule and
signs are pinned by the dense brute force).  Binary64 runs must be
bit-identical: every key receives at most a parent part and a child part, and
both sides form the same two rounded products and one sum."""

import math
import sys

import numpy as np
import pytest

import workload as w
from oracle import OracleSum
from oracle.statevector import kicked_ising_magnetization
from gpu_common import assert_same_operator, gpu_sum

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def _both(n, terms, coeffs, dtype=0):
    return gpu_sum(n, terms, coeffs, dtype=dtype), OracleSum(n, terms, coeffs)


@pytest.mark.parametrize("eps0", [0.0, 1e-3])
def test_random_rotations_small_register(eps0):
    """40 random rotations (weights 1-4, X/Y/Z letters, 20% at Clifford
    angles) on a random 8-qubit set."""
    n = 8
    terms, coeffs = w.random_pauli_set(n, 300, seed=41)
    gates = w.random_gates(n, 40, seed=42, max_weight=4)
    g, o = _both(n, terms, coeffs)
    for k in range(0, 40, 8):  # several layers, so state carries across calls
        sub = w.GateList(gates.gens[k:k + 8], gates.thetas[k:k + 8])
        g.apply_rotation_layer(sub, eps0)
        o.apply(sub, eps0)
        assert_same_operator(g, o, coeff_exact=True)
    say(f"small register eps0={eps0}: |O| = {g.size()}")


def test_random_rotations_127_qubits_many_tiles():
    """Rotations of weight <= 3 on the 127-q register on ~50k strings
    (many tiles of the branch and merge passes), eps0 = 1e-4."""
    n = 127
    lat = w.eagle_127()
    terms, coeffs = w.random_pauli_set(n, 50000, seed=43, support=w.ball(lat, 62, 4))
    sup = w.ball(lat, 62, 3)
    gates = w.random_gates(len(sup), 12, seed=44, max_weight=3)
    # map the generators from the compact register onto the ball's qubits
    gens = []
    for row in gates.gens:
        ops = {}
        for j, q in enumerate(sup):
            xb = (int(row[j >> 6]) >> (j & 63)) & 1
            zb = (int(row[2 + (j >> 6)]) >> (j & 63)) & 1
            if xb or zb:
                ops[q] = "X" if (xb and not zb) else ("Y" if xb else "Z")
        gens.append(w.pauli_words(n, ops))
    gl = w.GateList(np.stack(gens), gates.thetas)
    g, o = _both(n, terms, coeffs)
    g.apply_rotation_layer(gl, 1e-4)
    o.apply(gl, 1e-4)
    say(f"127q random rotations: |O| = {g.size()}")
    assert_same_operator(g, o, coeff_exact=True)


def test_rx_out_of_order_and_general_gate_inside_an_rx_run():
    """RX on qubits 0, 1, 2 (streaming path), then RY on qubit 7 while the
    stored x is rotated, then RX on 0 again and RX in descending order."""
    n = 12
    terms, coeffs = w.random_pauli_set(n, 2000, seed=45)
    def rot(ops, th):
        return w.pauli_words(n, ops), th
    seq = [rot({0: "X"}, 0.3), rot({1: "X"}, 0.4), rot({2: "X"}, 0.5), rot({7: "Y"}, 0.6),
           rot({0: "X"}, 0.7), rot({5: "X"}, 0.2), rot({4: "X"}, 0.1), rot({3: "Z", 9: "Z"}, 0.9)]
    gl = w.GateList(np.stack([s[0] for s in seq]), np.array([[s[1]] for s in seq]))
    g, o = _both(n, terms, coeffs)
    g.apply_rotation_layer(gl, 1e-5)
    o.apply(gl, 1e-5)
    assert_same_operator(g, o, coeff_exact=True)
    # the streaming path resumes at qubit 0 after a general gate
    rx = w.GateList(np.stack([w.pauli_words(n, {q: "X"}) for q in range(n)]), np.full((n, 1), 0.35))
    g.apply_rotation_layer(rx, 1e-5)
    o.apply(rx, 1e-5)
    assert_same_operator(g, o, coeff_exact=True)


def test_non_clifford_zz_kicked_ising_patch():
    """Kicked Ising on the 21-q patch with theta_zz = -1.0 (not Clifford, so
    every RZZ takes the general path): equal to the oracle for 3 steps and to
    the statevector for 4."""
    lat = w.heavy_hex_21()
    zz, rx = w.kicked_ising_step(lat, 0.6, theta_zz=-1.0)
    terms, coef = w.single_pauli_term(lat.n, {10: "Z"})
    g, o = _both(lat.n, terms, coef)
    exact = kicked_ising_magnetization(lat.n, lat.edges, 10, 0.6, 4, theta_zz=-1.0)
    for t in range(4):
        g.apply_rotation_layer(zz).apply_rotation_layer(rx)
        if t < 3:
            o.apply(zz).apply(rx)
            assert_same_operator(g, o, coeff_exact=True)
        say(f"theta_zz=-1 step {t + 1}: |O| = {g.size()} <Z> = {g.expectation_z()[0]:.12f} exact {exact[t]:.12f}")
        assert abs(g.expectation_z()[0] - exact[t]) <= 1e-11


def test_general_gates_with_lanes_and_binary32():
    n = 9
    terms, coeffs = w.random_pauli_set(n, 500, seed=47, lanes=3)
    gates = w.random_gates(n, 10, seed=48, max_weight=3, lanes=3)
    g, o = _both(n, terms, coeffs)
    g.apply_rotation_layer(gates, 1e-4)
    o.apply(gates, 1e-4)
    assert_same_operator(g, o, coeff_exact=True)
    g32 = gpu_sum(n, terms, coeffs, dtype=1)
    g64 = gpu_sum(n, terms, coeffs, dtype=0)
    g32.apply_rotation_layer(gates)
    g64.apply_rotation_layer(gates)
    k32, c32 = g32.export()
    k64, c64 = g64.export()
    assert np.array_equal(k32, k64)
    assert np.abs(c32.astype(np.float64) - c64).max() <= 1e-5 * np.abs(c64).max()


def test_general_gate_capacity_growth():
    """A weight-6 rotation doubles ~40k anticommuting strings from a small
    capacity: the branch runs out of room, the handle grows and re-runs it."""
    n = 16
    terms, coeffs = w.random_pauli_set(n, 40000, seed=49)
    gate = w.GateList(w.pauli_words(n, {0: "Y", 3: "X", 5: "Z", 8: "Y", 11: "X", 14: "Z"})[None, :],
                      np.array([[0.77]]))
    g = gpu_sum(n, terms, coeffs, capacity=45000)
    o = OracleSum(n, terms, coeffs)
    g.apply_rotation_layer(gate)
    o.apply(gate)
    assert_same_operator(g, o, coeff_exact=True)


def test_z_only_rotation_inside_an_rx_run_keeps_the_stream():
    """A non-Clifford RZZ between RX gates: the general path keeps the stored x
    rotation (children stay in their x-group), sorts inside the groups, and
    the RX run continues on its streaming path; against the oracle, and a
    large x-group forces the fallback of the same stage (gathering the runs
    and merging them)."""
    n = 14
    terms, coeffs = w.random_pauli_set(n, 3000, seed=51)
    def rot(ops, th):
        return w.pauli_words(n, ops), th
    seq = [rot({0: "X"}, 0.3), rot({1: "X"}, 0.4), rot({2: "Z", 5: "Z"}, 0.7), rot({2: "X"}, 0.5),
           rot({3: "X"}, 0.6), rot({6: "Z"}, 1.1), rot({4: "X"}, 0.2)]
    gl = w.GateList(np.stack([s[0] for s in seq]), np.array([[s[1]] for s in seq]))
    for label, tt, cc in (("random set", terms, coeffs),
                          ("Z-only set (one x-group of 4000+)",
                           *w.random_pauli_set(n, 6000, seed=52))):
        if label.startswith("Z-only"):
            tt = tt.copy()
            tt[:, :2] = 0  # x = 0 for every string: a single x-group
            tt, idx = np.unique(tt, axis=0, return_index=True)
            cc = cc[idx]
        g, o = _both(n, tt, cc)
        g.apply_rotation_layer(gl, 1e-6)
        o.apply(gl, 1e-6)
        say(f"{label}: |O| = {g.size()}")
        assert_same_operator(g, o, coeff_exact=True)


def test_run_merge_sorts_general_gates_with_few_flipped_bits():
    """Generators flipping b <= 4 key bits (X and Z letters count one, Y two)
    sort their branch output by gathering 1 + 2^b sorted runs and merging them
    pairwise (odd run counts, several merge tiles); b = 5 takes the radix
    sort.  Bit for bit against the oracle after every gate."""
    n = 14
    terms, coeffs = w.random_pauli_set(n, 80000, seed=81)
    specs = [({3: "Z", 6: "X"}, 0.7, 2), ({1: "Y", 7: "Y"}, 0.45, 4), ({2: "X", 9: "Z", 11: "Z"}, 1.1, 3),
             ({5: "Y"}, 0.3, 2), ({0: "X", 4: "X", 8: "X", 12: "Z"}, 0.6, 4), ({1: "Y", 2: "Y", 3: "Z"}, 0.8, 5)]
    g, o = _both(n, terms, coeffs)
    for ops, th, b in specs:
        gate = w.GateList(w.pauli_words(n, ops)[None, :], np.array([[th]]))
        before = g.stats()
        g.apply_rotation_layer(gate, 1e-7)
        o.apply(gate, 1e-7)
        after = g.stats()
        merged = after["run_merges"] - before["run_merges"]
        radix = after["radix_sorts"] - before["radix_sorts"]
        say(f"{ops} (b = {b}): |O| = {g.size()}, run merges {merged:.0f}, radix sorts {radix:.0f}")
        assert (merged, radix) == ((1, 0) if b <= 4 else (0, 1))
        assert_same_operator(g, o, coeff_exact=True)


def test_run_merge_after_capacity_growth_and_with_lanes():
    """The tagged branch re-run after the handle grows (the run tags live in
    per-capacity arrays that move with the growth), and run merges with
    several lanes in binary64 and binary32."""
    n = 16
    terms, coeffs = w.random_pauli_set(n, 40000, seed=91)
    gate = w.GateList(w.pauli_words(n, {0: "Y", 5: "X", 9: "Z"})[None, :], np.array([[0.77]]))
    g = gpu_sum(n, terms, coeffs, capacity=45000)
    o = OracleSum(n, terms, coeffs)
    g.apply_rotation_layer(gate)
    o.apply(gate)
    assert g.stats()["run_merges"] == 1
    assert_same_operator(g, o, coeff_exact=True)
    terms, coeffs = w.random_pauli_set(n, 30000, seed=92, lanes=5)
    gens = [{1: "Z", 2: "X"}, {3: "Y", 7: "Z"}, {4: "X", 6: "X", 8: "Z"}]
    gl = w.GateList(np.stack([w.pauli_words(n, ops) for ops in gens]),
                    np.random.default_rng(93).uniform(-1.5, 1.5, (3, 5)))
    g64, o = gpu_sum(n, terms, coeffs), OracleSum(n, terms, coeffs)
    g64.apply_rotation_layer(gl, 1e-6)
    o.apply(gl, 1e-6)
    assert g64.stats()["run_merges"] == 3
    assert_same_operator(g64, o, coeff_exact=True)
    g32 = gpu_sum(n, terms, coeffs, dtype=1)
    g32.apply_rotation_layer(gl)
    g64 = gpu_sum(n, terms, coeffs)
    g64.apply_rotation_layer(gl)
    k32, c32 = g32.export()
    k64, c64 = g64.export()
    assert np.array_equal(k32, k64)
    assert np.abs(c32.astype(np.float64) - c64).max() <= 1e-5 * np.abs(c64).max()


def test_run_merge_up_to_65_runs_on_127_qubits():
    """On the 127-q register the radix sort needs 32 byte passes, so
    generators flipping five or six key bits (33 and 65 runs, 7 and 8
    passes) also take the run merge; seven bits take the radix sort."""
    n = 127
    lat = w.eagle_127()
    terms, coeffs = w.random_pauli_set(n, 50000, seed=95, support=w.ball(lat, 62, 4))
    specs = [({60: "Y", 61: "Y", 62: "X"}, 0.4, 5), ({55: "Y", 62: "Y", 70: "Y"}, 0.9, 6),
             ({60: "Y", 61: "Y", 62: "Y", 63: "X"}, 0.6, 7)]
    g, o = _both(n, terms, coeffs)
    for ops, th, b in specs:
        gate = w.GateList(w.pauli_words(n, ops)[None, :], np.array([[th]]))
        before = g.stats()
        g.apply_rotation_layer(gate, 1e-6)
        o.apply(gate, 1e-6)
        after = g.stats()
        merged = after["run_merges"] - before["run_merges"]
        radix = after["radix_sorts"] - before["radix_sorts"]
        say(f"{ops} (b = {b}): |O| = {g.size()}, run merges {merged:.0f}, radix sorts {radix:.0f}")
        assert (merged, radix) == ((1, 0) if b <= 6 else (0, 1))
        assert_same_operator(g, o, coeff_exact=True)


def test_general_gates_on_word_boundaries_of_a_128_qubit_register():
    """Generators on qubits 0, 63, 64 and 127 (the edges of the two mask
    words) on a full 128-qubit register, through the run merge (b <= 6) and
    the radix sort (b = 8), bit for bit against the oracle."""
    n = 128
    edge = [0, 1, 62, 63, 64, 65, 126, 127]
    terms, coeffs = w.random_pauli_set(n, 20000, seed=97, support=edge)
    specs = [({63: "Y", 64: "X"}, 0.5), ({0: "Z", 127: "Y"}, 1.2), ({63: "X", 64: "Z", 127: "X"}, 0.35),
             ({0: "Y", 63: "Y", 64: "Y", 127: "Y"}, 0.8)]
    g, o = _both(n, terms, coeffs)
    for ops, th in specs:
        gate = w.GateList(w.pauli_words(n, ops)[None, :], np.array([[th]]))
        g.apply_rotation_layer(gate, 1e-7)
        o.apply(gate, 1e-7)
        assert_same_operator(g, o, coeff_exact=True)
    st = g.stats()
    say(f"128-q word edges: |O| = {g.size()}, run merges {st['run_merges']:.0f}, radix sorts {st['radix_sorts']:.0f}")
    assert st["run_merges"] == 3 and st["radix_sorts"] == 1


def test_general_gate_with_x_letters_inside_an_rx_run_keeps_the_stream():
    """A general gate with X and Y letters between RX gates writes its
    outputs in the stored (rotated) x frame, so the RX run resumes on its
    streaming path: four RX gates stream, the general gate takes the run
    merge, bit for bit against the oracle."""
    n = 12
    terms, coeffs = w.random_pauli_set(n, 5000, seed=99)
    seq = [({0: "X"}, 0.3), ({1: "X"}, 0.4), ({4: "Y", 6: "X"}, 0.7), ({2: "X"}, 0.5), ({3: "X"}, 0.6)]
    gl = w.GateList(np.stack([w.pauli_words(n, ops) for ops, _ in seq]), np.array([[th] for _, th in seq]))
    g, o = _both(n, terms, coeffs)
    g.apply_rotation_layer(gl, 1e-6)
    o.apply(gl, 1e-6)
    st = g.stats()
    say(f"stream across a general gate: rx launches {st['rx_launches']:.0f}, run merges {st['run_merges']:.0f}")
    assert st["rx_launches"] == 4 and st["run_merges"] == 1
    assert_same_operator(g, o, coeff_exact=True)


@pytest.mark.parametrize("which", ["xy_weight2", "rx_out_of_order", "z_only_non_clifford", "weight3_lanes4"])
def test_fp32_general_gate_within_one_ulp_of_oracle(which):
    """Binary32 general gates are compensated like the RX merge: the branch
    keeps each product exact as a rounded head plus a low word, and the
    equal-key pass sums the (at most two) pairs of a key with two-sum and
    rounds once.  One gate on a random set whose coefficients are binary32
    values: every output is within one binary32 ulp of the oracle's binary64
    value rounded to binary32 (Eq. update_rule), for the in-group sort
    (Z-only generator), the run merge (few flipped bits) and the radix sort
    (weight 3 with lanes)."""
    n = 20
    lanes = 4 if which == "weight3_lanes4" else 1
    terms, coeffs = w.random_pauli_set(n, 4000, seed=7, support=list(range(10)), lanes=lanes)
    coeffs = coeffs.astype(np.float32).astype(np.float64)
    letters = {"xy_weight2": {1: "X", 4: "Y"}, "rx_out_of_order": {3: "X"},
               "z_only_non_clifford": {2: "Z", 5: "Z"}, "weight3_lanes4": {0: "Y", 2: "Y", 7: "X"}}[which]
    th = np.array([[0.7, -1.1, 2.3, 0.4][:lanes]])
    gate = w.GateList(w.pauli_words(n, letters)[None, :], th)
    g32 = gpu_sum(n, terms, coeffs, dtype=1).apply_rotation_layer(gate)
    o = OracleSum(n, terms, coeffs).apply(gate)
    k32, c32 = g32.export()
    ok, oc = o.export()
    assert np.array_equal(k32, ok)
    ref = oc.astype(np.float32)
    diff = np.abs(c32.astype(np.float64) - ref.astype(np.float64))
    ulp = np.spacing(np.abs(ref)).astype(np.float64)
    say(f"{which}: {k32.shape[0]} strings, exact {np.mean(diff == 0):.4f}, max diff / ulp "
        f"{np.max(diff / np.maximum(ulp, 1e-300)):.3f}")
    assert np.all(diff <= ulp)
