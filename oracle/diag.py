"""Diagnostics reference (test infrastructure only): the Pauli-string density
of Appendix D.

D_t(x) is the normalized histogram of x = O_I / max_I |O_I| over the strings
kept after t layers.  `density_counts` states the bin rule used by the library
call it checks: with M = max |O_I| and thresholds t_k = M * edges[k] (binary64
products), a value v (O_I, or |O_I| when unsigned) falls in bin k when
t_k <= v < t_(k+1), the last bin being closed at t_nb; values below t_0 and
above t_nb are counted apart.
"""

from __future__ import annotations

import numpy as np


def density_counts(coeffs, edges, signed: bool = True) -> np.ndarray:
    """Counts per bin, then below the range, then above it (length nb + 2)."""
    c = np.asarray(coeffs, dtype=np.float64)
    e = np.asarray(edges, dtype=np.float64)
    nb = e.size - 1
    M = float(np.abs(c).max(initial=0.0))
    t = M * e
    v = c if signed else np.abs(c)
    out = np.zeros(nb + 2, dtype=np.uint64)
    for x in v.tolist():
        if x < t[0]:
            out[nb] += 1
        elif x > t[nb]:
            out[nb + 1] += 1
        else:
            k = int(np.searchsorted(t, x, side="right")) - 1
            out[min(k, nb - 1)] += 1
    return out


def density(coeffs, n_bins: int = 200, signed: bool = True):
    """(bin centres, D(x)) on [-1, 1] (signed) or [0, 1], integrating to 1."""
    edges = np.linspace(-1.0 if signed else 0.0, 1.0, n_bins + 1)
    cnt = density_counts(coeffs, edges, signed)[:n_bins].astype(np.float64)
    width = edges[1] - edges[0]
    total = cnt.sum()
    return 0.5 * (edges[1:] + edges[:-1]), (cnt / (total * width) if total else cnt)
