"""Radix-sort digit width and tile size (needs a GPU): every configuration
gives the oracle's operator bit for bit, forced one by one on the two sorts
that use it (the re-sort after a Clifford layer when an x-group is too large
for the in-group sort, and the (x, z) sort of general gates), and the online
tuner tries each once per size class before settling on one."""

import sys

import numpy as np
import pytest

import workload as w
from oracle import OracleSum
from gpu_common import assert_same_operator, gpu_sum

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def _resort_case():
    """~36k strings near qubit 62 plus one x-group of 6000 (too large for the
    in-group sort), as in the Clifford re-sort parity test."""
    n = 127
    lat = w.eagle_127()
    zz = w.kicked_ising_step(lat, 0.8)[0]
    terms, coeffs = w.random_pauli_set(n, 30000, seed=21, support=w.ball(lat, 62, 4))
    zs, _ = w.random_pauli_set(n, 8000, seed=22, support=w.ball(lat, 62, 4))
    big = np.repeat(terms[:1], len(zs), axis=0)
    big[:, 2:] = zs[:, 2:]
    big = np.unique(big, axis=0)[:6000]
    tt = np.concatenate([terms, big])
    cc = np.concatenate([coeffs, np.linspace(0.1, 1.0, len(big))[:, None]])
    tt, idx = np.unique(tt, axis=0, return_index=True)
    return n, zz, tt, cc[idx]


def _general_case():
    """Four rotations on a 14-qubit register, 80k strings, each generator
    flipping five or more key bits (a Y letter flips two), so every gate takes
    the (x, z) radix sort rather than the merge of its runs."""
    n = 14
    terms, coeffs = w.random_pauli_set(n, 80000, seed=71)
    gens = [{1: "Y", 4: "Y", 9: "X"}, {0: "Y", 2: "X", 5: "Y"}, {3: "Y", 7: "Y", 8: "Y"}, {2: "Z", 6: "Y", 10: "Y"}]
    gates = w.GateList(np.stack([w.pauli_words(n, ops) for ops in gens]), np.array([[0.3], [0.7], [1.1], [0.5]]))
    return n, gates, terms, coeffs


@pytest.mark.parametrize("bits,ipt", [(8, 8), (8, 16), (7, 16), (6, 16), (7, 8), (6, 8)])
def test_every_configuration_matches_the_oracle(bits, ipt):
    import paper_2506_13241_amd as P
    assert (bits, ipt) in P.SORT_CONFIGS
    n, zz, tt, cc = _resort_case()
    g = gpu_sum(n, tt, cc).set_sort_config(bits, ipt)
    o = OracleSum(n, tt, cc)
    g.apply_rotation_layer(zz)
    o.apply(zz)
    st = g.stats()
    assert st["radix_sorts"] == 1 and st["sort_digit_bits"] == bits and st["sort_items_per_thread"] == ipt
    assert_same_operator(g, o, coeff_exact=True)
    n, gates, tt, cc = _general_case()
    g = gpu_sum(n, tt, cc).set_sort_config(bits, ipt)
    o = OracleSum(n, tt, cc)
    g.apply_rotation_layer(gates, 1e-6)
    o.apply(gates, 1e-6)
    say(f"({bits}, {ipt}): |O| = {g.size()}, sorts {g.stats()['radix_sorts']}")
    assert g.stats()["radix_sorts"] == 4
    assert_same_operator(g, o, coeff_exact=True)


def test_online_tuning_tries_each_candidate_then_keeps_one():
    import paper_2506_13241_amd as P
    n, gates, tt, cc = _general_case()
    gl = w.GateList(np.concatenate([gates.gens] * 3), np.concatenate([gates.thetas] * 3))
    g = gpu_sum(n, tt, cc)
    o = OracleSum(n, tt, cc)
    seen = []
    for k in range(len(gl.gens)):
        one = w.GateList(gl.gens[k:k + 1], gl.thetas[k:k + 1])
        g.apply_rotation_layer(one, 1e-6)
        o.apply(one, 1e-6)
        st = g.stats()
        seen.append((int(st["sort_digit_bits"]), int(st["sort_items_per_thread"])))
    say(f"configurations used: {seen}, |O| = {g.size()}")
    assert_same_operator(g, o, coeff_exact=True)
    assert all(c in P.SORT_CONFIGS for c in seen)
    with pytest.raises(P.PsError):
        g.set_sort_config(5, 8)
    with pytest.raises(P.PsError):
        g.set_sort_config(8, 0)
    g.set_sort_config(0, 0)


def test_tuner_explores_all_candidates():
    """Twelve applications of one general gate to ~1.5e5 strings: after the
    first, the operator is closed under the gate (each string and its
    product with the generator are both present), so the sorts span at most
    two size classes and one of them sees at least six sorts, one per
    configuration."""
    import paper_2506_13241_amd as P
    n = 16
    terms, coeffs = w.random_pauli_set(n, 150000, seed=73)
    gate = w.GateList(w.pauli_words(n, {3: "Y", 9: "X", 12: "Y"})[None, :], np.array([[0.4]]))
    g = gpu_sum(n, terms, coeffs)
    o = OracleSum(n, terms, coeffs)
    used, sizes = [], []
    for _ in range(12):
        g.apply_rotation_layer(gate)
        o.apply(gate)
        st = g.stats()
        used.append((int(st["sort_digit_bits"]), int(st["sort_items_per_thread"])))
        sizes.append(g.size())
    say(f"sizes {sizes}, used {used}")
    assert len(set(sizes[1:])) == 1
    assert set(used) == set(P.SORT_CONFIGS)
    assert_same_operator(g, o, coeff_exact=True)
