"""The curve and sweep drivers of the diagnostics module (needs a GPU), on the
21-qubit patch without truncation, against the statevector."""

import json
import math

import numpy as np
import pytest

import workload as w
from oracle.statevector import kicked_ising_magnetization

pytestmark = pytest.mark.gpu


def test_curves_match_statevector_and_density_counts_every_string():
    from paper_2506_13241_amd import diagnostics as D
    lat = w.heavy_hex_21()
    th = 0.1 * math.pi
    exact = kicked_ising_magnetization(lat.n, lat.edges, 10, th, 5)
    rows = D.run_curves(lat, 10, th, 0.0, 5, emit=lambda s: None)
    assert [r["t"] for r in rows] == [1, 2, 3, 4, 5]
    for r, e in zip(rows, exact):
        assert abs(r["M"] - e) <= 1e-11
    out = []
    rows = D.run_curves(lat, 10, th, 1e-6, 5, density_bins=40, emit=out.append)
    for r, line in zip(rows, out):
        assert json.loads(line)["t"] == r["t"]
        assert sum(r["counts"]) + r["below"] + r["above"] == r["size"]
        assert r["above"] == 0 and r["counts"][-1] >= 1  # the largest string sits in the top bin
        assert r["below"] == 0  # nothing survives below eps * max
        assert abs(r["M"] - exact[r["t"] - 1]) <= 1e-4


@pytest.mark.parametrize("dtype,tol", [(0, 1e-11), (1, 1e-5)])
def test_sweep_lanes_match_statevector_per_angle(dtype, tol):
    from paper_2506_13241_amd import diagnostics as D
    lat = w.heavy_hex_21()
    row = D.run_sweep(lat, 10, 8, 0.0, 4, dtype=dtype, emit=lambda s: None)
    assert row["t"] == 4
    for th, m in zip(row["theta_x"], row["M"]):
        e = kicked_ising_magnetization(lat.n, lat.edges, 10, th, 4)[-1]
        assert abs(m - e) <= tol, (th, m, e)
    per = D.run_sweep(lat, 10, 8, 0.0, 4, per_angle=True, dtype=0, emit=lambda s: None)
    for a, b in zip(per, row["M"]):
        assert abs(a["M"] - b) <= tol
    assert max(p["size"] for p in per) <= row["size"]
