"""Train the learned truncation scorer on propagation data the method generates.

    python -m paper_2506_13241_amd.train_scorer --out weights.npz

1. Sample runs: propagate the observable Z_q through `sample_steps` kicked
   Ising steps with magnitude truncation at `sample_eps`; after step k keep a
   sample of the live strings, stratified by log10(|c| / max|c|) so that the
   band where truncation decisions are taken is well covered.
2. Labels: the weight of string I sampled after k steps is
   g_I = <0| (remaining steps applied to sigma_I) |0>, the factor with which
   its coefficient reaches <Z> (Heisenberg picture, Eq. expectation; the sum
   is linear in the strings).  The remaining steps are capped at
   `horizon`; 32 sampled strings are propagated at once as 32 coefficient
   lanes (lane a starts as the a-th string with coefficient 1), with lane-wise
   magnitude truncation at `label_eps`.  Target: log10(|g_I| + floor).
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


def label_strings(n_qubits, edges, theta, keys, remaining, label_eps, lanes=32, log=None):
    """g_I for each key: <Z> after `remaining[i]` further steps from sigma_I."""
    zz, rx = w.kicked_ising_step(w.Lattice(n_qubits, [tuple(e) for e in edges]), theta, lanes=lanes)
    g = np.zeros(len(keys))
    order = np.argsort(remaining, kind="stable")
    t0 = time.time()
    for b in range(0, len(keys), lanes):
        sel = order[b:b + lanes]
        r = int(remaining[sel[0]])
        sel = sel[remaining[sel] == r]  # one horizon per batch
        coeffs = np.zeros((len(sel), lanes))
        coeffs[np.arange(len(sel)), np.arange(len(sel))] = 1.0
        op = PauliSum(n_qubits, keys[sel], coeffs)
        for _ in range(r):
            op.apply_rotation_layer(zz, label_eps).apply_rotation_layer(rx, label_eps)
        g[sel] = op.expectation_z()[: len(sel)]
        op.close()
        if log and (b // lanes) % log == 0:
            _say(f"  labels {b + len(sel)}/{len(keys)} (horizon {r}, {time.time() - t0:.1f} s)")
    return g


def label_strings_all(n_qubits, edges, theta, keys, remaining, label_eps, lanes=32, log=20):
    """Batches never mix horizons: keys are grouped by horizon first."""
    g = np.zeros(len(keys))
    for r in np.unique(remaining):
        idx = np.flatnonzero(remaining == r)
        g[idx] = label_strings(n_qubits, edges, theta, keys[idx], remaining[idx], label_eps, lanes, log)
    return g


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
    ap.add_argument("--sample-eps", type=float, default=1e-6)
    ap.add_argument("--per-step", type=int, default=4096)
    ap.add_argument("--horizon", type=int, default=3)
    ap.add_argument("--label-eps", type=float, default=1e-4)
    ap.add_argument("--floor", type=float, default=1e-5)
    ap.add_argument("--iters", type=int, default=2000)
    ap.add_argument("--lr", type=float, default=2e-3)
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
    remaining = np.minimum(a.sample_steps - step, a.horizon)
    _say(f"sampled {len(keys)} strings in {time.time() - t0:.1f} s")
    t1 = time.time()
    g = label_strings_all(n, edges, a.theta, keys, remaining, a.label_eps)
    targets = np.log10(np.abs(g) + a.floor).astype(np.float32)
    _say(f"labelled in {time.time() - t1:.1f} s; target mean {targets.mean():.3f} sd {targets.std():.3f}")
    sc, first, last = fit(n, table, keys, targets, a.iters, a.lr, a.seed)
    meta = dict(lattice=a.lattice, obs=obs, theta=a.theta, sample_steps=a.sample_steps, sample_eps=a.sample_eps,
                per_step=a.per_step, horizon=a.horizon, label_eps=a.label_eps, floor=a.floor, iters=a.iters,
                lr=a.lr, seed=a.seed, n_samples=len(keys), loss_first=first, loss_last=last,
                target_sd=float(targets.std()))
    S.save_params(a.out, sc.get_params(), meta)
    print(json.dumps(meta))
    return 0


if __name__ == "__main__":
    sys.exit(main())
