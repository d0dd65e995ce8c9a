"""What the trained scorer gains over plain magnitude truncation, and its
fallback to magnitude truncation (needs a GPU).

127-qubit kicked Ising, theta_h = 0.8, observable Z62.  The gain is measured
against a reference magnitude run at eps0 = 2.5e-6, a quarter of the smallest threshold
compared and independent of both arms, over the 6 Trotter steps that run
fits on one GPU.  The committed network (paper_2506_13241_amd/data, trained
by paper_2506_13241_amd.train_scorer on strings from 8-step runs,
horizon-3 labels) at eps0 = 5e-6 must keep fewer strings summed over the
steps than magnitude truncation at 1e-5, with a smaller worst |<Z62> -
reference|, both below 1e-3 (the gain at matched error)."""

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


def _setup():
    import paper_2506_13241_amd as P
    from paper_2506_13241_amd import scorer as S
    P.load_library()
    lat = w.eagle_127()
    zz, rx = w.kicked_ising_step(lat, 0.8)
    params, meta = S.load_params(WEIGHTS)
    sc = P.PsScorer(lat.n, *S.feature_table(lat.n, lat.edges, 62)).set_params(params)

    def run(eps, mode, steps, ratio=1.0, tol=0.0):
        terms, coef = w.single_pauli_term(lat.n, {62: "Z"})
        op = P.PauliSum(lat.n, terms, coef)
        if mode == P.PS_TRUNC_LEARNED:
            op.load_scorer(sc).set_learned(ratio, tol)
        ez, sz = [], []
        for _ in range(steps):
            op.apply_rotation_layer(zz, eps, mode).apply_rotation_layer(rx, eps, mode)
            ez.append(op.expectation_z()[0])
            sz.append(op.size())
        st = op.stats()
        op.close()
        return np.array(ez), int(np.sum(sz)), st

    return P, run


def test_learned_truncation_keeps_fewer_strings_at_lower_error():
    P, run = _setup()
    ref, n_j, _ = run(2.5e-6, P.PS_TRUNC_MAGNITUDE, 6)
    say(f"reference eps 2.5e-6: sum|O| = {n_j:.3e}")
    ez_m, n_m, _ = run(1e-5, P.PS_TRUNC_MAGNITUDE, 6)
    ez_l, n_l, _ = run(5e-6, P.PS_TRUNC_LEARNED, 6)
    em, el = np.abs(ez_m - ref), np.abs(ez_l - ref)
    say(f"magnitude 1e-5: sum|O| {n_m:.3e} max {em.max():.2e} | learned 5e-6: sum|O| {n_l:.3e} max {el.max():.2e}")
    assert n_l < 0.5 * n_m
    assert el.max() < em.max() <= 1e-3


def test_learned_fallback_meets_the_magnitude_run():
    """With a fallback tolerance (pauli_sum_set_learned), passes whose
    estimated learned error exceeds it apply the magnitude rule alone: over
    12 steps the learned run at eps0 = 1e-5 stays within 1e-3 of the binary64
    magnitude run at the same eps0 (the learned rule alone leaves it by
    several 1e-3 from step 7 on)."""
    P, run = _setup()
    ref, n_r, _ = run(1e-5, P.PS_TRUNC_MAGNITUDE, 12)
    ez_f, n_f, st = run(1e-5, P.PS_TRUNC_LEARNED, 12, 1.0, 1e-4)
    d = np.abs(ez_f - ref)
    say(f"fallback run: {st['learned_fallbacks']:.0f} of {st['learned_passes']:.0f} passes fell back, "
        f"sum|O| {n_f:.3e} vs {n_r:.3e}, max |dZ62| {d.max():.2e}")
    assert st["learned_fallbacks"] >= 1
    assert d.max() <= 1e-3
