"""The property behind the run merge of general gates (CPU): in a key set
sorted by (x, z), the strings that agree on the key bits a generator J flips
keep their relative order when J is xor-ed into them, so the children of one
class, taken in input order, form a sorted run; stored x may be any fixed
rotation of the true x."""

import numpy as np


def _sorted_keys(rng, m, nq):
    x = rng.integers(0, 1 << nq, m, dtype=np.int64)
    z = rng.integers(0, 1 << nq, m, dtype=np.int64)
    keys = np.unique(np.stack([x, z], axis=1), axis=0)  # lexicographic (x, z)
    return keys[:, 0], keys[:, 1]


def _rotr(v, r, nq):
    return ((v >> r) | (v << (nq - r))) & ((1 << nq) - 1)


def test_children_of_one_class_form_sorted_runs():
    rng = np.random.default_rng(11)
    nq = 10
    for trial in range(200):
        x, z = _sorted_keys(rng, 400, nq)
        xj = int(rng.integers(0, 1 << nq)) & int(rng.integers(0, 1 << nq))
        zj = int(rng.integers(0, 1 << nq)) & int(rng.integers(0, 1 << nq))
        pos_x = [q for q in range(nq) if xj >> q & 1]
        pos_z = [q for q in range(nq) if zj >> q & 1]
        cls = np.zeros(len(x), dtype=np.int64)
        for k, q in enumerate(pos_x):
            cls |= ((x >> q) & 1) << k
        for k, q in enumerate(pos_z):
            cls |= ((z >> q) & 1) << (len(pos_x) + k)
        cx, cz = x ^ xj, z ^ zj
        for c in np.unique(cls):
            sel = cls == c
            run = cx[sel] * (1 << nq) + cz[sel]
            assert np.all(np.diff(run) > 0), (trial, c)


def test_runs_hold_in_a_rotated_frame():
    """Stored x = true x rotated right by r: sorting and flipping in the
    stored frame (generator rotated the same way) keeps the property."""
    rng = np.random.default_rng(12)
    nq = 9
    for trial in range(100):
        r = int(rng.integers(0, nq))
        xt, z = _sorted_keys(rng, 300, nq)
        xs = _rotr(xt, r, nq)
        order = np.lexsort((z, xs))
        xs, z = xs[order], z[order]
        xj_true = int(rng.integers(0, 1 << nq)) & int(rng.integers(0, 1 << nq))
        xjs = int(_rotr(np.int64(xj_true), r, nq))
        pos = [q for q in range(nq) if xjs >> q & 1]
        cls = np.zeros(len(xs), dtype=np.int64)
        for k, q in enumerate(pos):
            cls |= ((xs >> q) & 1) << k
        cx = xs ^ xjs
        for c in np.unique(cls):
            sel = cls == c
            run = cx[sel] * (1 << nq) + z[sel]
            assert np.all(np.diff(run) > 0)
