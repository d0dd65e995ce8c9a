"""Helpers shared by the GPU tests (comparison of the HIP path with the oracle)."""

import numpy as np

import workload as w
from oracle import OracleSum


def gpu_sum(n, terms, coeffs, dtype=0, capacity=0):
    import paper_2506_13241_amd as P
    return P.PauliSum(n, terms, coeffs, dtype=dtype, capacity=capacity)


def assert_same_operator(gpu, orc, rtol=1e-12, exact_keys=True, coeff_exact=False):
    """Key sets identical; coefficients equal within rtol of the largest one."""
    gk, gc = gpu.export()
    ok, oc = orc.export()
    assert gk.shape == ok.shape, (gk.shape, ok.shape)
    if exact_keys:
        assert np.array_equal(gk, ok)
    gc = gc.astype(np.float64)
    scale = max(np.abs(oc).max(initial=0.0), 1e-300)
    if coeff_exact:
        assert np.array_equal(gc, oc), np.abs(gc - oc).max()
    else:
        err = np.abs(gc - oc).max(initial=0.0)
        assert err <= rtol * scale, (err, scale)


def run_both(lat, q, theta, steps, eps0, dtype=0, capacity=0, check_each=True, rtol=1e-12, coeff_exact=False):
    terms, coef = w.single_pauli_term(lat.n, {q: "Z"})
    g = gpu_sum(lat.n, terms, coef, dtype=dtype, capacity=capacity)
    o = OracleSum(lat.n, terms, coef)
    zz, rx = w.kicked_ising_step(lat, theta)
    out = []
    for t in range(steps):
        g.apply_rotation_layer(zz, eps0).apply_rotation_layer(rx, eps0)
        o.apply(zz, eps0).apply(rx, eps0)
        ez_g, ez_o = g.expectation_z()[0], o.expectation_z()[0]
        out.append((ez_g, ez_o, g.size(), o.size()))
        if check_each:
            assert_same_operator(g, o, rtol=rtol, coeff_exact=coeff_exact)
    return g, o, out
