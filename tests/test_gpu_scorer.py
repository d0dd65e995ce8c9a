"""Learned truncation scorer on the HIP path (needs a GPU).

Features are exact small integers times powers of two, so they must equal the
host reference bit for bit.  The bf16 MFMA forward is compared with the FP64
network of oracle/mlp.py evaluated with the same bf16 roundings (weights,
features and hidden activations); the fp32 backward with the oracle's
gradients (relative Frobenius error per parameter block); Adam with the
oracle's update applied to the GPU's own gradient.  Learned truncation inside
the propagation handle is checked against the same keep rule evaluated on the
host from exported keys, and a constant network against the oracle.
"""

import math
import sys

import numpy as np
import pytest

import workload as w
from oracle import OracleSum, mlp
from gpu_common import assert_same_operator, gpu_sum

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def P():
    import paper_2506_13241_amd as P
    P.load_library()
    return P


@pytest.fixture(scope="module")
def eagle():
    return w.eagle_127()


def make_scorer(P, lat, q=62):
    from paper_2506_13241_amd import scorer as S
    qm, let, sc = S.feature_table(lat.n, lat.edges, q)
    return P.PsScorer(lat.n, qm, let, sc), (qm, let, sc)


def host_features(keys, table):
    """Feature matrix of (m,4) uint64 keys (x0,x1,z0,z1), in float64."""
    qm, let, sc = table
    x = [int(a) | (int(b) << 64) for a, b in zip(keys[:, 0], keys[:, 1])]
    z = [int(a) | (int(b) << 64) for a, b in zip(keys[:, 2], keys[:, 3])]
    F = np.zeros((len(x), 160))
    region = [int(a) | (int(b) << 64) for a, b in qm]
    for i, (xi, zi) in enumerate(zip(x, z)):
        masks = (xi & ~zi, xi & zi, zi & ~xi, xi | zi)
        for f in range(160):
            F[i, f] = sc[f] * bin(masks[let[f]] & region[f]).count("1")
    return F


def random_keys(n, m, seed):
    terms, _ = w.random_pauli_set(n, m, seed=seed, support=list(range(n)))
    return np.ascontiguousarray(terms, dtype=np.uint64)


def bf16_forward(p, F):
    """oracle network with the kernel's bf16 roundings (fp32 biases)."""
    W1, W2, W3 = (mlp.to_bf16(p[k]) for k in ("W1", "W2", "W3"))
    b1, b2, b3 = (p[k].astype(np.float32).astype(np.float64) for k in ("b1", "b2", "b3"))
    h1 = mlp.to_bf16(mlp.gelu(F @ W1.T + b1))
    h2 = mlp.to_bf16(mlp.gelu(h1 @ W2.T + b2))
    return (h2 @ W3.T + b3)[:, 0]


def rounded_params(flat):
    from paper_2506_13241_amd import scorer as S
    p = S.unpack_params(flat)
    for k in ("W1", "W2", "W3"):
        p[k] = mlp.to_bf16(p[k])
    return p


def test_features_exact(P, eagle):
    s, table = make_scorer(P, eagle)
    keys = random_keys(eagle.n, 3000, 11)
    keys[0] = 0  # identity string
    s.set_data(keys, np.zeros(len(keys)))
    _, f = s.forward(features=True)
    got = (f.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    assert np.array_equal(got, host_features(keys, table))


@pytest.mark.parametrize("m", [1, 63, 64, 65, 5000])
def test_forward_matches_bf16_oracle_network(P, eagle, m):
    from paper_2506_13241_amd import scorer as S
    s, table = make_scorer(P, eagle)
    flat = S.init_params(5)
    flat[S.N_PARAMS - 1] = -0.7
    rng = np.random.default_rng(m)
    flat[:-1] += 0.02 * rng.normal(size=S.N_PARAMS - 1).astype(np.float32)  # non-zero biases too
    s.set_params(flat)
    keys = random_keys(eagle.n, m, 100 + m)
    s.set_data(keys, np.zeros(m))
    y = s.forward().astype(np.float64)
    ref = bf16_forward(S.unpack_params(flat), host_features(keys, table))
    err = np.abs(y - ref)
    say(f"forward m={m}: max err {err.max():.2e}, median {np.median(err):.2e}, |y| max {np.abs(ref).max():.2f}")
    assert err.max() <= 5e-3 * (1 + np.abs(ref).max())
    assert np.median(err) <= 2e-4 * (1 + np.abs(ref).max())


def test_gradients_match_oracle(P, eagle):
    from paper_2506_13241_amd import scorer as S
    s, table = make_scorer(P, eagle)
    flat = S.init_params(9)
    s.set_params(flat)
    m = 3000
    keys = random_keys(eagle.n, m, 77)
    F = host_features(keys, table)
    rng = np.random.default_rng(4)
    t = rng.normal(-2.0, 1.0, size=m).astype(np.float32)
    s.set_data(keys, t)
    loss, g = s.loss_grad()
    y = s.forward().astype(np.float64)
    assert abs(loss - np.mean((y - t.astype(np.float64)) ** 2)) <= 1e-6 * loss
    ref_loss, ref_g = mlp.loss_and_grads(rounded_params(flat), F, t.astype(np.float64))
    assert abs(loss - ref_loss) <= 1e-2 * ref_loss
    gg = S.unpack_params(g)
    for k in ref_g:
        rel = np.linalg.norm(gg[k] - ref_g[k]) / max(np.linalg.norm(ref_g[k]), 1e-30)
        say(f"grad {k}: rel err {rel:.2e}")
        assert rel <= 1e-2, k


def test_adam_steps_match_oracle_update(P, eagle):
    from paper_2506_13241_amd import scorer as S
    s, _ = make_scorer(P, eagle)
    flat = S.init_params(2)
    s.set_params(flat)
    keys = random_keys(eagle.n, 1000, 8)
    s.set_data(keys, np.full(1000, -1.5, dtype=np.float32))
    p = S.unpack_params(flat)
    m = {k: np.zeros_like(v) for k, v in p.items()}
    v = {k: np.zeros_like(val) for k, val in p.items()}
    for step in (1, 2, 3):
        _, g = s.loss_grad()
        s.adam_step(1e-3)
        mlp.adam_step(p, S.unpack_params(g), m, v, step, lr=1e-3)
        got = S.unpack_params(s.get_params())
        for k in p:
            assert np.abs(got[k] - p[k]).max() <= 2e-6 * (1 + np.abs(p[k]).max()), (step, k)
        p = got  # continue from the GPU's fp32 parameters


def test_training_reduces_loss(P, eagle):
    """A learnable synthetic target (weight-dependent) is fitted by the GPU's
    own forward/backward/Adam kernels."""
    from paper_2506_13241_amd import scorer as S
    s, table = make_scorer(P, eagle)
    s.set_params(S.init_params(1))
    keys = random_keys(eagle.n, 4096, 21)
    F = host_features(keys, table)
    target = (-0.15 * F[:, 87] * 32 - 0.5 * F[:, 91:94].sum(axis=1)).astype(np.float32)
    s.set_data(keys, target)
    first = s.loss_grad(grad=False)
    for _ in range(300):
        s.loss_grad(grad=False)
        s.adam_step(3e-3)
    last = s.loss_grad(grad=False)
    say(f"training: loss {first:.4f} -> {last:.5f}")
    assert last <= 0.05 * first


def test_learned_without_scorer_is_rejected(P):
    lat = w.heavy_hex_21()
    zz, _ = w.kicked_ising_step(lat, 0.6)
    terms, coef = w.single_pauli_term(lat.n, {10: "Z"})
    g = gpu_sum(lat.n, terms, coef)
    with pytest.raises(P.PsError) as e:
        g.apply_rotation_layer(zz, 1e-4, P.PS_TRUNC_LEARNED)
    assert e.value.code == P.PS_ERR_INVALID


def test_constant_scorer_equals_oracle_with_tighter_threshold(P):
    """Output y = -1 for every string (g = 0.1): the learned rule at eps is the
    magnitude rule at 10 eps, applied once per Trotter step at the Clifford
    layer, on top of the per-gate rule at eps."""
    from paper_2506_13241_amd import scorer as S
    lat = w.heavy_hex_21()
    s, _ = make_scorer(P, lat, q=10)
    s.set_params(S.constant_params(-1.0))
    zz, rx = w.kicked_ising_step(lat, 0.6)
    terms, coef = w.single_pauli_term(lat.n, {10: "Z"})
    g = gpu_sum(lat.n, terms, coef).load_scorer(s)
    o = OracleSum(lat.n, terms, coef)
    eps = 1e-5
    for t in range(4):
        g.apply_rotation_layer(zz, eps, P.PS_TRUNC_LEARNED).apply_rotation_layer(rx, eps, P.PS_TRUNC_LEARNED)
        o.truncate(10 * eps)
        o.apply(zz, eps).apply(rx, eps)
        say(f"constant scorer step {t + 1}: |O| = {g.size()}")
        assert_same_operator(g, o, coeff_exact=True)


def test_learned_keep_rule_on_rotated_layout(P, eagle):
    """Random network: after an RX layer (keys stored rotated, front and back
    runs), learned truncation keeps exactly the strings with
    |c| * min(1, 10^y) > eps * max|c|, y being the network output for the key
    (taken from the scorer's own forward on the exported keys)."""
    from paper_2506_13241_amd import scorer as S
    s, _ = make_scorer(P, eagle)
    flat = S.init_params(13)
    flat[-1] = -1.0
    s.set_params(flat)
    n = eagle.n
    terms, coeffs = w.random_pauli_set(n, 3000, seed=5, support=list(range(55, 70)))
    _, rx = w.kicked_ising_step(eagle, 0.8)
    g = gpu_sum(n, terms, coeffs).load_scorer(s)
    g.apply_rotation_layer(rx)
    k0, c0 = g.export()
    s.set_data(k0, np.zeros(len(k0)))
    y = s.forward().astype(np.float64)
    eps = 3e-2
    M = np.abs(c0[:, 0]).max()
    keep = np.abs(c0[:, 0]) * np.minimum(1.0, 10.0 ** y) > eps * M
    g.truncate(eps, P.PS_TRUNC_LEARNED)
    k1, c1 = g.export()
    say(f"learned keep rule: {len(k0)} -> {len(k1)} (expected {keep.sum()})")
    assert 0 < keep.sum() < len(k0)
    assert np.array_equal(k1, k0[keep])
    assert np.array_equal(c1, c0[keep])


def test_learned_clifford_stage_scores_rotated_input(P, eagle):
    """The scorer runs on the Clifford stage's input as stored by the RX merge
    (rotated keys, front/back runs): a learned ZZ layer equals the host keep
    rule on the exported state followed by the oracle's ZZ layer."""
    from paper_2506_13241_amd import scorer as S
    s, _ = make_scorer(P, eagle)
    flat = S.init_params(17)
    flat[-1] = -0.5
    s.set_params(flat)
    n = eagle.n
    terms, coeffs = w.random_pauli_set(n, 3000, seed=6, support=list(range(55, 70)))
    zz, rx = w.kicked_ising_step(eagle, 0.8)
    g = gpu_sum(n, terms, coeffs).load_scorer(s)
    g.apply_rotation_layer(rx)
    k0, c0 = g.export()
    s.set_data(k0, np.zeros(len(k0)))
    y = s.forward().astype(np.float64)
    eps = 1e-2
    keep = np.abs(c0[:, 0]) * np.minimum(1.0, 10.0 ** y) > eps * np.abs(c0[:, 0]).max()
    g.apply_rotation_layer(zz, eps, P.PS_TRUNC_LEARNED)
    # per-gate magnitude rule at eps, relative to the max of the kept strings
    o = OracleSum(n, k0[keep], c0[keep]).apply(zz, eps)
    assert_same_operator(g, o, coeff_exact=True)


def test_scorer_api_rejects_bad_input(P, eagle):
    from paper_2506_13241_amd import scorer as S
    s, _ = make_scorer(P, eagle)
    with pytest.raises(P.PsError) as e:
        s.set_params(np.zeros(10, dtype=np.float32))
    assert e.value.code == P.PS_ERR_INVALID
    bad = S.init_params(0)
    bad[5] = np.nan
    with pytest.raises(P.PsError) as e:
        s.set_params(bad)
    assert e.value.code == P.PS_ERR_NONFINITE
    with pytest.raises(P.PsError) as e:  # no training set yet
        s.loss_grad()
    assert e.value.code == P.PS_ERR_INVALID
    with pytest.raises(ValueError):
        s.set_data(random_keys(eagle.n, 10, 1), np.zeros(9))
    # an empty training set is accepted; forward returns nothing
    s.set_data(np.zeros((0, 4), dtype=np.uint64), np.zeros(0))
    assert s.forward().shape == (0,)


def test_learned_truncate_needs_scorer_and_handles_empty_operator(P):
    from paper_2506_13241_amd import scorer as S
    lat = w.heavy_hex_21()
    terms, coef = w.single_pauli_term(lat.n, {10: "Z"})
    g = gpu_sum(lat.n, terms, coef)
    with pytest.raises(P.PsError) as e:
        g.truncate(1e-3, P.PS_TRUNC_LEARNED)
    assert e.value.code == P.PS_ERR_INVALID
    s, _ = make_scorer(P, lat, q=10)
    s.set_params(S.constant_params(-1.0))
    empty = gpu_sum(lat.n, np.zeros((0, 4), dtype=np.uint64), np.zeros((0, 1))).load_scorer(s)
    zz, rx = w.kicked_ising_step(lat, 0.6)
    empty.apply_rotation_layer(zz, 1e-3, P.PS_TRUNC_LEARNED).apply_rotation_layer(rx, 1e-3, P.PS_TRUNC_LEARNED)
    empty.truncate(1e-3, P.PS_TRUNC_LEARNED)
    assert empty.size() == 0 and empty.expectation_z()[0] == 0.0
