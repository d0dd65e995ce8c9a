"""Host logic of the learned scorer: feature table, parameter layout and the
committed weights (no GPU)."""

import os

import numpy as np

import workload as w
from paper_2506_13241_amd import scorer as S


def _bits(qm_row):
    m = int(qm_row[0]) | (int(qm_row[1]) << 64)
    return {q for q in range(128) if (m >> q) & 1}


def test_feature_table_regions_eagle():
    lat = w.eagle_127()
    qm, let, sc = S.feature_table(lat.n, lat.edges, 62)
    assert qm.shape == (160, 2) and let.shape == (160,) and sc.shape == (160,)
    dist = S.graph_distances(lat.n, lat.edges, 62)
    # rings partition the qubits (per letter); ring 0 is the observable qubit
    rings = [_bits(qm[3 * d]) for d in range(16)]
    assert rings[0] == {62}
    assert rings[1] == {61, 63, 72}
    assert set().union(*rings) == set(range(lat.n))
    assert sum(len(r) for r in rings) == lat.n
    for d in range(15):
        assert all(dist[q] == d for q in rings[d])
    # bands partition the qubits too
    bands = [_bits(qm[48 + 3 * b]) for b in range(13)]
    assert set().union(*bands) == set(range(lat.n)) and sum(len(b) for b in bands) == lat.n
    # totals, then the nearest qubits (observable first)
    assert [int(x) for x in let[87:91]] == [3, 0, 1, 2] and _bits(qm[87]) == set(range(lat.n))
    assert _bits(qm[91]) == {62} and list(let[91:94]) == [0, 1, 2]
    near = [min(_bits(qm[91 + 3 * j])) for j in range(23)]
    assert [dist[q] for q in near] == sorted(dist[q] for q in near)
    # counts times scales are exact in bf16 (8 significant bits)
    for f in range(160):
        for cnt in range(len(_bits(qm[f])) + 1):
            v = np.float32(sc[f] * cnt)
            assert (v.view(np.uint32) & 0xFFFF) == 0


def test_param_layout_roundtrip():
    flat = S.init_params(4)
    assert flat.shape == (S.N_PARAMS,) and S.N_PARAMS == 37249
    p = S.unpack_params(flat)
    assert p["W1"].shape == (128, 160) and p["W3"].shape == (1, 128) and p["b3"].shape == (1,)
    assert np.array_equal(S.pack_params(p), flat)
    c = S.constant_params(-1.5)
    assert np.count_nonzero(c) == 1 and c[-1] == np.float32(-1.5)


def test_committed_weights_load():
    path = os.path.join(os.path.dirname(__file__), "..", "paper_2506_13241_amd", "data",
                        "scorer_eagle127_z62_theta0.8.npz")
    params, meta = S.load_params(path)
    assert params.shape == (S.N_PARAMS,) and np.all(np.isfinite(params))
    assert meta["lattice"] == "eagle127" and meta["obs"] == "62" and float(meta["theta"]) == 0.8
    assert float(meta["loss_last"]) < 0.25 * float(meta["target_sd"]) ** 2


def test_stratified_sample_spreads_over_log_magnitude_bins():
    """The training sampler takes up to count/bins strings from each of the
    log10(|c|/max|c|) bins between log10(eps) and 0, without repeats, and
    nothing from an all-zero operator."""
    from paper_2506_13241_amd.train_scorer import stratified_sample
    rng = np.random.default_rng(5)
    c = np.concatenate([np.full(1000, 1e-5), np.full(10, 0.5), np.full(3000, 2e-2), [1.0]])
    idx = stratified_sample(c, 120, 1e-6, rng, bins=6)
    assert len(np.unique(idx)) == len(idx) and np.all(np.diff(idx) > 0)
    r = np.log10(np.abs(c[idx]))
    counts = np.histogram(r, bins=np.linspace(-6, 0, 7))[0]
    # bins holding enough strings give count / bins = 20 each; the 0.5 and
    # 1.0 strings share the top bin (11 strings)
    assert counts.tolist() == [0, 20, 0, 0, 20, 11]
    assert len(stratified_sample(np.zeros(10), 5, 1e-3, rng)) == 0


def test_log_density_edges():
    from paper_2506_13241_amd.diagnostics import log_density_edges
    e = log_density_edges(1e-6, 70)
    assert len(e) == 71 and abs(e[0] - 1e-7) < 1e-20 and e[-1] == 1.0
    assert np.allclose(np.diff(np.log10(e)), 0.1)
