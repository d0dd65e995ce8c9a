"""Train the learned truncation scorer on propagation data the method generates.

    python -m paper_2506_13241_amd.train_scorer --out weights.npz

1. Sample runs: propagate the observable Z_q through `sample_steps` kicked
   Ising steps with magnitude truncation at `sample_eps`; after step k keep a
   sample of the live strings, stratified by log10(|c| / max|c|) so that the
   band where truncation decisions are taken is well covered.
2. Labels: the weight of a sampled string I is max over h = 1..horizon of
   |g_I,h|, g_I,h = <0| (h further steps applied to sigma_I) |0> being the
   factor with which its coefficient reaches <Z> h steps later (Heisenberg
   picture, Eq. expectation; <Z> is linear in the strings), so a string that
   matters to any of the next `horizon` readouts scores high.  32 sampled
   strings are propagated at once as 32 binary32 coefficient lanes (lane a
   starts as the a-th string with coefficient 1), dropping paths whose weight
   falls below `label_eps` (absolute).  Target: log10(|g_I| + floor).
3. Fit: full-batch Adam on the mean squared error, with the library's own
   forward, backward and Adam kernels.

Every step runs through the library (PauliSum, PsScorer); nothing here does
propagation arithmetic itself.  Lattices and gate lists come from the seeded
input module `workload`.
"""

from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np

import workload as w

from . import PauliSum, PsScorer, load_library
from . import scorer as S


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def stratified_sample(coeffs: np.ndarray, count: int, eps: float, rng, bins: int = 12) -> np.ndarray:
    """Indices of up to `count` strings, spread evenly over log10(|c|/max|c|)
    bins between log10(eps) and 0."""
    mag = np.abs(coeffs)
    M = mag.max(initial=0.0)
    if M == 0.0 or len(mag) == 0:
        return np.zeros(0, dtype=np.int64)
    r = np.log10(np.maximum(mag / M, 1e-300))
    edges = np.linspace(math.log10(eps), 0.0, bins + 1)
    which = np.clip(np.digitize(r, edges) - 1, 0, bins - 1)
    per = max(1, count // bins)
    out = []
    for b in range(bins):
        idx = np.flatnonzero(which == b)
        if len(idx):
            out.append(rng.choice(idx, size=min(per, len(idx)), replace=False))
    return np.sort(np.concatenate(out)) if out else np.zeros(0, dtype=np.int64)


def sample_strings(n_qubits, edges, obs_qubit, theta, sample_steps, sample_eps, per_step, seed):
    """Keys sampled after each step k = 1..sample_steps-1, with k."""
    rng = np.random.default_rng(seed)
    lat = w.Lattice(n_qubits, [tuple(e) for e in edges])
    zz, rx = w.kicked_ising_step(lat, theta)
    op = PauliSum(n_qubits, *w.single_pauli_term(n_qubits, {obs_qubit: "Z"}))
    keys, step = [], []
    for k in range(1, sample_steps):
        t0 = time.time()
        op.apply_rotation_layer(zz, sample_eps).apply_rotation_layer(rx, sample_eps)
        kk, cc = op.export()
        idx = stratified_sample(cc[:, 0], per_step, sample_eps, rng)
        keys.append(kk[idx])
        step.append(np.full(len(idx), k))
        _say(f"  sample run step {k}: |O| = {len(kk)}, sampled {len(idx)} ({time.time() - t0:.1f} s)")
    op.close()
    return np.concatenate(keys), np.concatenate(step)


def _label_batch(n_qubits, zz, rx, keys, horizon, label_eps, lanes, reduce="max"):
    """max over h = 1..horizon of |g_h| for up to `lanes` keys, one lane each.
    An identity string with coefficient 1 in every lane anchors the lane
    maximum at 1, so the lane-wise relative threshold acts as an absolute one:
    paths whose weight falls below label_eps are dropped (without the anchor, a
    string with many Y/Z letters spawns ~2^w children of nearly equal size that
    a relative threshold never removes).  The anchor commutes with every gate
    and adds exactly 1 to <Z>."""
    m = len(keys)
    words = np.concatenate([np.zeros((1, 4), dtype=np.uint64), keys])
    coeffs = np.zeros((m + 1, lanes))
    coeffs[0, :] = 1.0
    coeffs[1 + np.arange(m), np.arange(m)] = 1.0
    op = PauliSum(n_qubits, words, coeffs, dtype=1)
    best = np.zeros(m)
    try:
        for h in range(horizon):
            op.apply_rotation_layer(zz, label_eps).apply_rotation_layer(rx, label_eps)
            if reduce == "max" or h == horizon - 1:
                best = np.maximum(best, np.abs(op.expectation_z()[:m] - 1.0))
        return best
    finally:
        op.close()


def label_strings(n_qubits, edges, theta, keys, horizon, label_eps, lanes=32, log=None, reduce="max"):
    """max over h = 1..horizon of |g_I,h| (reduce="max") or |g_I,horizon|
    (reduce="last"), g_I,h being <Z> after h further steps from sigma_I, with
    paths below label_eps dropped.  Returns (g, ok);
    ok is False for keys whose batch exceeded device memory even alone (their g
    is 0)."""
    from . import PsError
    zz, rx = w.kicked_ising_step(w.Lattice(n_qubits, [tuple(e) for e in edges]), theta, lanes=lanes)
    g = np.zeros(len(keys))
    ok = np.ones(len(keys), dtype=bool)
    t0 = time.time()
    todo = [np.arange(b, min(b + lanes, len(keys))) for b in range(0, len(keys), lanes)]
    done = 0
    while todo:
        sel = todo.pop(0)
        try:
            g[sel] = _label_batch(n_qubits, zz, rx, keys[sel], horizon, label_eps, lanes, reduce)
            done += len(sel)
        except PsError:
            if len(sel) == 1:
                ok[sel] = False
                done += 1
            else:  # split the batch and retry the halves
                todo[:0] = [sel[: len(sel) // 2], sel[len(sel) // 2:]]
        if log and done and (done // lanes) % log == 0 and len(sel):
            _say(f"  labels {done}/{len(keys)} ({time.time() - t0:.1f} s)")
    return g, ok


def fit(n_qubits, table, keys, targets, iters, lr, seed, log=100):
    sc = PsScorer(n_qubits, *table)
    sc.set_params(S.init_params(seed))
    sc.set_data(keys, targets)
    first = sc.loss_grad(grad=False)
    loss = first
    for it in range(iters):
        loss = sc.loss_grad(grad=False)
        sc.adam_step(lr if it < iters * 3 // 4 else lr / 10)
        if log and it % log == 0:
            _say(f"  fit iter {it}: loss {loss:.4f}")
    return sc, first, sc.loss_grad(grad=False)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--lattice", default="eagle127", choices=["eagle127", "patch21"])
    ap.add_argument("--obs", type=int, default=None)
    ap.add_argument("--theta", type=float, default=0.8)
    ap.add_argument("--sample-steps", type=int, default=8)
    ap.add_argument("--sample-eps", type=float, default=1e-4)
    ap.add_argument("--per-step", type=int, default=8192)
    ap.add_argument("--horizon", type=int, default=3)
    ap.add_argument("--label-eps", type=float, default=1e-3)
    ap.add_argument("--label", default="max", choices=["max", "last"])
    ap.add_argument("--floor", type=float, default=1e-3)
    ap.add_argument("--iters", type=int, default=3000)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--seed", type=int, default=20250616)
    ap.add_argument("--out", required=True)
    a = ap.parse_args(argv)
    load_library()
    lat = w.eagle_127() if a.lattice == "eagle127" else w.heavy_hex_21()
    n, edges = lat.n, lat.edges
    obs = lat.center if a.obs is None else a.obs
    table = S.feature_table(n, edges, obs)
    t0 = time.time()
    keys, step = sample_strings(n, edges, obs, a.theta, a.sample_steps, a.sample_eps, a.per_step, a.seed)
    _say(f"sampled {len(keys)} strings in {time.time() - t0:.1f} s")
    t1 = time.time()
    g, ok = label_strings(n, edges, a.theta, keys, a.horizon, a.label_eps, log=20, reduce=a.label)
    keys, g = keys[ok], g[ok]
    targets = np.log10(np.abs(g) + a.floor).astype(np.float32)
    _say(f"labelled in {time.time() - t1:.1f} s; target mean {targets.mean():.3f} sd {targets.std():.3f}")
    sc, first, last = fit(n, table, keys, targets, a.iters, a.lr, a.seed)
    meta = dict(lattice=a.lattice, obs=obs, theta=a.theta, sample_steps=a.sample_steps, sample_eps=a.sample_eps,
                per_step=a.per_step, horizon=a.horizon, label=a.label, label_eps=a.label_eps, floor=a.floor,
                iters=a.iters,
                lr=a.lr, seed=a.seed, n_samples=len(keys), loss_first=first, loss_last=last,
                target_sd=float(targets.std()))
    S.save_params(a.out, sc.get_params(), meta)
    print(json.dumps(meta))
    return 0


if __name__ == "__main__":
    sys.exit(main())
