"""What the trained scorer gains over plain magnitude truncation (needs a GPU).

127-qubit kicked Ising, theta_h = 0.8, observable Z62, 10 Trotter steps.  The
error reference is the magnitude run at eps0 = 1e-5 (the exact value is out
of reach at this size).  The committed network
(paper_2506_13241_amd/data, trained by paper_2506_13241_amd.train_scorer on
strings from 8-step runs, horizon-3 labels) is compared at matched operating
points: learned truncation at eps must keep fewer strings summed over the
steps than magnitude truncation at 10 eps, with a smaller worst and mean
|<Z62> - reference|.  The reference is itself a magnitude run, which favours
the magnitude side of the comparison."""

import os
import sys

import numpy as np
import pytest

import workload as w

pytestmark = pytest.mark.gpu
WEIGHTS = os.path.join(os.path.dirname(__file__), "..", "paper_2506_13241_amd", "data",
                       "scorer_eagle127_z62_theta0.8.npz")


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def test_learned_truncation_keeps_fewer_strings_at_lower_error():
    import paper_2506_13241_amd as P
    from paper_2506_13241_amd import scorer as S
    P.load_library()
    lat = w.eagle_127()
    zz, rx = w.kicked_ising_step(lat, 0.8)
    params, meta = S.load_params(WEIGHTS)
    sc = P.PsScorer(lat.n, *S.feature_table(lat.n, lat.edges, 62)).set_params(params)

    def run(eps, mode):
        terms, coef = w.single_pauli_term(lat.n, {62: "Z"})
        op = P.PauliSum(lat.n, terms, coef)
        if mode == P.PS_TRUNC_LEARNED:
            op.load_scorer(sc)
        ez, sz = [], []
        for _ in range(10):
            op.apply_rotation_layer(zz, eps, mode).apply_rotation_layer(rx, eps, mode)
            ez.append(op.expectation_z()[0])
            sz.append(op.size())
        op.close()
        return np.array(ez), int(np.sum(sz))

    ref, ref_size = run(1e-5, P.PS_TRUNC_MAGNITUDE)
    say(f"reference eps 1e-5: sum|O| = {ref_size:.3e}")
    for eps in (1e-5, 5e-6):
        ez_m, n_m = run(10 * eps, P.PS_TRUNC_MAGNITUDE)
        ez_l, n_l = run(eps, P.PS_TRUNC_LEARNED)
        em, el = np.abs(ez_m - ref), np.abs(ez_l - ref)
        say(f"magnitude {10 * eps:g}: sum|O| {n_m:.3e} max {em.max():.2e} mean {em.mean():.2e} | "
            f"learned {eps:g}: sum|O| {n_l:.3e} max {el.max():.2e} mean {el.mean():.2e}")
        assert n_l < 0.75 * n_m
        assert el.max() < em.max()
        assert el.mean() < em.mean()
