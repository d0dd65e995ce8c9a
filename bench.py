#!/usr/bin/env python
"""Benchmark of the Heisenberg Pauli-propagation hot path on one MI355X.

Workload: the 127-qubit heavy-hex kicked Ising circuit (Eq. (u)), observable
sigma_z^62, theta_h = 0.8, theta_zz = -pi/2, relative truncation eps0 = 1e-4
after every gate, binary64 coefficients.  One step = one Trotter step: the
fused RZZ(-pi/2) layer with its re-sort, the 127 RX gates (each one streaming
merge pass) and the <Z62> readout.  --warmup W Trotter steps run untimed (they
also build the operator the timed steps start from), then --steps K steps are
timed: Trotter steps W+1 .. W+K of the circuit.

Metric: Pauli-string updates per second = sum over the 271 gates of every
timed step of the number of strings the gate acts on, divided by the wall time
(Results: the paper's per-gate cost is linear in |O|).  The roofline entry is
for the dominant kernel, the RX merge pass: algorithmic bytes per launch =
(strings read + strings written) x 40 B, divided by its mean launch time from
HIP events on the library's stream.

--lanes theta32 | obs16 times the batched forms instead: 32 values of theta_h
in [0, pi/2] carried as binary32 coefficient lanes of one operator, or 16
random weight-1/2 Z observables (seed 20250616) at theta_h = 0.8; their line
also reports string x lane updates per second, and the roofline bytes per
string are 32 + 4 x 32 (key words + padded lanes).
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, vendor figure
# (eps0, warmup steps, timed steps, dtype) of the batched forms at one GPU
# (measured: theta32 holds 4.8e7 strings at step 15 at 3e-3; obs16 5.4e8 at 2e-4, while 1e-4
# outgrows 288 GB at step 6 for both)
LANES_ONE_GPU = {"theta32": (3e-3, 13, 2, "f32"), "obs16": (2e-4, 13, 2, "f32")}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


KERNEL_SOURCES = ("orqa_kernels.hip", "orqa_device.h", "orqa_internal.h")


def kernel_source_sha():
    """sha256 (16 hex digits) over the sources the RX merge kernel is built from."""
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_2506_13241_amd", "csrc", name), "rb").read())
    return h.hexdigest()[:16]


def workload_key(args) -> str:
    """The configuration a committed counter figure belongs to."""
    return (f"lanes={args.lanes} dtype={args.dtype} eps={args.eps:g} theta={args.theta:g} "
            f"theta_zz={args.theta_zz:.6f} trunc={args.trunc} steps={args.warmup + 1}-{args.warmup + args.steps}")


def read_profile_fields(path):
    fields = {}
    for line in open(path):
        if ":" in line and not line.startswith(("#", " ", "|", "-")):
            k, v = line.split(":", 1)
            fields[k.strip()] = v.strip()
    return fields


def measured_traffic(key):
    """HBM bytes per RX merge launch from a committed rocprofv3 summary taken
    on this workload key (configuration and step window) with the current
    kernel sources, as (bytes, algorithmic bytes of those launches, file);
    (None, None, None) when no summary matches."""
    import glob
    sha = kernel_source_sha()
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "k_rx_merge__*.md"))):
        f = read_profile_fields(path)
        if f.get("kernel_source_sha256_16") == sha and f.get("workload_key") == key and \
                "traffic_bytes_per_launch" in f and "algorithmic_bytes_per_launch" in f:
            return float(f["traffic_bytes_per_launch"]), float(f["algorithmic_bytes_per_launch"]), \
                os.path.basename(path)
    return None, None, None


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(theta, eps0, budget_s, theta_zz=-math.pi / 2):
    """The FP64 std::map oracle, single-threaded, on a bounded sample of the
    same workload: Trotter steps 1.. from the start, gate by gate, until the
    time budget is spent.  Same metric (string-updates/s)."""
    import numpy as np
    import workload as w
    from oracle import OracleSum, build

    build(force=False)
    lat = w.eagle_127()
    terms, coef = w.single_pauli_term(lat.n, {62: "Z"})
    o = OracleSum(lat.n, terms, coef)
    zz, rx = w.kicked_ising_step(lat, theta, theta_zz=theta_zz)
    gates = w.GateList.concat([zz, rx])
    t0 = time.perf_counter()
    n_gates = 0
    steps_done = 0
    ez = []
    while time.perf_counter() - t0 < budget_s:
        for g in range(len(gates)):
            o.apply(w.GateList(gates.gens[g:g + 1], gates.thetas[g:g + 1]), eps0)
            n_gates += 1
            if time.perf_counter() - t0 >= budget_s:
                break
        else:
            steps_done += 1
            ez.append(float(o.expectation_z()[0]))
    dt = time.perf_counter() - t0
    part = n_gates - steps_done * len(gates)
    return {
        "value": o.updates() / dt,
        "unit": "string-updates/s",
        "cores": 1,
        "cpu_model": cpu_model(),
        "kind": "oracle",
        "sample": f"Trotter steps 1-{steps_done} of the same workload plus {part} gates of step "
                  f"{steps_done + 1} ({n_gates} gates, {dt:.1f} s, {o.updates():.3g} string-updates)",
    }, ez


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed Trotter steps (default 2)")
    ap.add_argument("--warmup", type=int, default=None,
                    help="untimed Trotter steps before them (default 18; with --lanes, the one-GPU form's)")
    ap.add_argument("--lanes", choices=["none", "theta32", "obs16"], default="none",
                    help="batched forms: 32 theta_h lanes, or 16 observable lanes (binary32 by default)")
    ap.add_argument("--theta", type=float, default=0.8)
    ap.add_argument("--theta-zz", type=float, default=-math.pi / 2,
                    help="RZZ angle; away from multiples of pi/2 every RZZ takes the general-rotation path")
    ap.add_argument("--eps", type=float, default=None, help="eps0 (default 1e-4; with --lanes, the one-GPU form's)")
    ap.add_argument("--dtype", choices=["f64", "f32"], default=None, help="default f64; f32 with --lanes")
    ap.add_argument("--reference-f64", action="store_true",
                    help="after the run, repeat it untimed in binary64 (magnitude rule) and report |delta <Z62>| per step")
    ap.add_argument("--trunc", choices=["magnitude", "learned"], default="magnitude",
                    help="learned: the committed trained scorer (127q, Z62, theta 0.8) on top of the magnitude rule")
    ap.add_argument("--learned-ratio", type=float, default=1.0,
                    help="learned threshold = ratio x eps (pauli_sum_set_learned)")
    ap.add_argument("--learned-tol", type=float, default=0.0,
                    help="fall back to the magnitude rule when the estimated learned error exceeds this (0: never)")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--verbose", action="store_true")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="only run a plain device-to-device copy of BYTES (calibrates rocprofv3 byte counters)")
    args = ap.parse_args()
    # the largest batched forms that fit one GPU (measured: the 15-step runs at
    # eps0 = 1e-4 outgrow 288 GB at step 6)
    one_gpu = {"none": (1e-4, 18, 2, "f64"), "theta32": LANES_ONE_GPU["theta32"],
               "obs16": LANES_ONE_GPU["obs16"]}[args.lanes]
    if args.eps is None:
        args.eps = one_gpu[0]
    if args.warmup is None:
        args.warmup = one_gpu[1]
    if args.steps is None:
        args.steps = one_gpu[2]
    if args.dtype is None:
        args.dtype = one_gpu[3]
    if args.copy_probe:
        import torch
        x = torch.empty(args.copy_probe // 4, dtype=torch.float32, device="cuda").fill_(1.0)
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(6)]
        for i in range(5):
            ev[i].record()
            y.copy_(x)
        ev[5].record()
        torch.cuda.synchronize()
        ms = [ev[i].elapsed_time(ev[i + 1]) for i in range(1, 5)]  # first copy is a warm-up
        gbs = 2 * x.numel() * 4 / (sum(ms) / len(ms) * 1e-3) / 1e9
        print(json.dumps({"copy_probe_bytes": x.numel() * 4, "launches": 5, "mean_ms": sum(ms) / len(ms),
                          "read_plus_write_GBps": round(gbs, 1)}))
        return

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (each MI355X "
              "would hold the strings of one hash class of the z mask).", file=sys.stderr)
        sys.exit(2)

    import torch
    import numpy as np
    import paper_2506_13241_amd as P
    import workload as w

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    lat = w.eagle_127()
    lanes = {"none": 1, "theta32": 32, "obs16": 16}[args.lanes]
    if args.lanes == "theta32":
        thetas = np.linspace(0.0, math.pi / 2, 32)
        zz, rx = w.kicked_ising_step(lat, thetas, theta_zz=args.theta_zz, lanes=32)
        terms, coef = w.single_pauli_term(lat.n, {62: "Z"}, lanes=32)
        what = "theta_h = 32 values in [0, pi/2] as binary32 lanes, O0=Z62"
    elif args.lanes == "obs16":
        obs = w.random_observables(lat.n, 16, 20250616)
        terms = np.stack([w.pauli_words(lat.n, ob) for ob in obs])
        coef = np.eye(16)
        zz, rx = w.kicked_ising_step(lat, args.theta, theta_zz=args.theta_zz, lanes=16)
        what = f"16 weight-1/2 Z observables (seed 20250616) as lanes, theta_h={args.theta}"
    else:
        zz, rx = w.kicked_ising_step(lat, args.theta, theta_zz=args.theta_zz)
        terms, coef = w.single_pauli_term(lat.n, {62: "Z"})
        what = f"O0=Z62, theta_h={args.theta}"
    dtype = P.PS_F64 if args.dtype == "f64" else P.PS_F32
    ps = P.PauliSum(lat.n, terms, coef, dtype=dtype, capacity=1 << 22)
    mode = P.PS_TRUNC_MAGNITUDE
    if args.trunc == "learned":
        from paper_2506_13241_amd import scorer as S
        params, _ = S.load_params(os.path.join(ROOT, "paper_2506_13241_amd", "data",
                                               "scorer_eagle127_z62_theta0.8.npz"))
        sc = P.PsScorer(lat.n, *S.feature_table(lat.n, lat.edges, 62)).set_params(params)
        ps.load_scorer(sc).set_learned(args.learned_ratio, args.learned_tol)
        mode = P.PS_TRUNC_LEARNED

    ez_all = []
    t_start = time.perf_counter()
    for s in range(args.warmup):
        ps.apply_rotation_layer(zz, args.eps, mode).apply_rotation_layer(rx, args.eps, mode)
        ez_all.append([float(v) for v in ps.expectation_z()])
        if args.verbose:
            log(f"warmup step {s + 1}: |O|={ps.size()} <Z>={ez_all[-1][0]:.12f} t={time.perf_counter() - t_start:.2f}s")
    n_before = ps.size()
    ps.stats(reset=True)
    ps.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        ps.apply_rotation_layer(zz, args.eps, mode).apply_rotation_layer(rx, args.eps, mode)
        ez_all.append([float(v) for v in ps.expectation_z()])
        if args.verbose:
            log(f"timed step {args.warmup + s + 1}: <Z>={ez_all[-1][0]:.12f} t={time.perf_counter() - t0:.2f}s")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    st = ps.stats()
    ps.set_timing(False)
    n_after = ps.size()

    updates = st["updates"]
    bps = st["bytes_per_string"]
    rx_bytes = (st["rx_in"] + st["rx_out"]) * bps
    rx_ms_mean = st["rx_ms"] / max(st["rx_launches"], 1)
    achieved = rx_bytes / (st["rx_ms"] * 1e-3) / 1e9 if st["rx_ms"] > 0 else 0.0
    alg_per_launch = rx_bytes / max(st["rx_launches"], 1)
    roofline = {
        "bound": "hbm",
        "kernel": "k_rx_merge",
        "achieved": round(achieved, 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": None,
        "traffic_source": None,
        "launches": int(st["rx_launches"]),
        "mean_launch_ms": round(rx_ms_mean, 4),
        "algorithmic_bytes_per_launch": round(alg_per_launch),
        "bytes_per_string": bps,
    }
    key = workload_key(args)
    traffic, traffic_alg, tsrc = measured_traffic(key)
    if traffic is not None:
        # the counters were taken on this workload key (same launches): their
        # ratio to the algorithmic bytes is carried over to this run's launches
        roofline["traffic"] = round(traffic / traffic_alg * alg_per_launch)
        roofline["traffic_source"] = f"{tsrc}: {traffic:.0f} B per launch against {traffic_alg:.0f} algorithmic"
    roofline["workload_key"] = key
    rx_updates = st["rx_in"]
    extra = {
        "strings_before": n_before,
        "strings_after": n_after,
        "rx_updates_per_s": rx_updates / dt,
        "rx_updates_note": "string-updates of the 127 RX gates of each step only (value also counts the 144 "
                           "RZZ gates, which one fused pass applies)",
        "ez_per_step": ez_all if lanes > 1 else [e[0] for e in ez_all],
        "ms_rx_merge_total": round(st["rx_ms"], 3),
        "ms_clifford_total": round(st["cliff_ms"], 3),
        "ms_sort_total": round(st["sort_ms"], 3),
        "sort_passes": int(st["sort_passes"]),
        "radix_sorts": int(st["radix_sorts"]),
        "run_merges": int(st["run_merges"]),
        "paper_time_per_gate_ms": round(dt / args.steps / 271 * 1e3, 4),
    }
    if st["radix_sorts"] == 0 and st["sort_passes"] == st["cliff_launches"] and st["cliff_ms"] > 0 \
            and st["sort_ms"] > 0:
        # one Clifford pass (reads cliff_in strings, writes its survivors with
        # their 4-byte group rank) and one in-group re-sort (reads and writes
        # the survivors) per step
        n_cl_out = st["sort_elems"]
        cl_bytes = st["cliff_in"] * bps + n_cl_out * (bps + 4)
        gs_bytes = 2 * n_cl_out * bps
        for name, kern, b, ms, launches in (("clifford", "k_compact", cl_bytes, st["cliff_ms"], st["cliff_launches"]),
                                            ("group_sort", "k_group_sort_xor", gs_bytes, st["sort_ms"],
                                             st["sort_passes"])):
            gbs = b / (ms * 1e-3) / 1e9
            extra[name] = {"kernel": kern, "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": round(gbs / HBM_PEAK_GBS, 4), "launches": int(launches),
                           "mean_launch_ms": round(ms / max(launches, 1), 4),
                           "algorithmic_bytes_per_launch": round(b / max(launches, 1))}
    if lanes > 1:
        extra["lanes"] = lanes
        extra["string_lane_updates_per_s"] = updates * lanes / dt
        extra["bytes_per_string_lane"] = bps / lanes
    if args.trunc == "learned":
        extra["learned"] = {"ratio": args.learned_ratio, "tol": args.learned_tol,
                            "passes": int(st["learned_passes"]), "fallbacks": int(st["learned_fallbacks"]),
                            "last_estimate": st["learned_est"]}
    if st["score_launches"] > 0:
        flop = 2 * (160 * 128 + 128 * 128 + 128) * st["score_in"]
        extra["scorer"] = {
            "kernel": "k_scorer_forward", "launches": int(st["score_launches"]), "strings": int(st["score_in"]),
            "ms_total": round(st["score_ms"], 3),
            "tflops": round(flop / (st["score_ms"] * 1e-3) / 1e12, 2) if st["score_ms"] > 0 else None,
            "frac_of_bf16_peak": round(flop / (st["score_ms"] * 1e-3) / 2.5e15, 4) if st["score_ms"] > 0 else None,
        }
    if args.reference_f64:
        ps.close()
        ref = P.PauliSum(lat.n, terms, coef, dtype=P.PS_F64)
        ez_ref = []
        for s in range(args.warmup + args.steps):
            ref.apply_rotation_layer(zz, args.eps).apply_rotation_layer(rx, args.eps)
            ez_ref.append([float(v) for v in ref.expectation_z()])
        ref.close()
        d = [max(abs(a - b) for a, b in zip(x, y)) for x, y in zip(ez_all, ez_ref)]
        extra["ez_f64_magnitude"] = ez_ref if lanes > 1 else [e[0] for e in ez_ref]
        extra["dz_vs_f64_per_step"] = d
        extra["dz_vs_f64_max"] = max(d)
    cpu = None
    if not args.no_cpu_baseline and args.trunc == "magnitude" and lanes == 1:
        cpu, ez_cpu = cpu_baseline(args.theta, args.eps, args.cpu_budget, args.theta_zz)
        k = min(len(ez_cpu), len(ez_all))
        if k:
            extra["dz_vs_oracle_max"] = max(abs(a[0] - b) for a, b in zip(ez_all[:k], ez_cpu[:k]))
            extra["dz_vs_oracle_steps"] = k
    line = {
        "metric": "Pauli-string updates/s (and s per Trotter step) at 127q",
        "value": updates / dt,
        "unit": "string-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic: deterministic kicked-Ising circuit, no dataset",
        "config": {
            "workload": f"kicked Ising 127q heavy-hex, {what}, "
                        + ("theta_zz=-pi/2, " if abs(args.theta_zz + math.pi / 2) < 1e-15 else f"theta_zz={args.theta_zz}, ")
                        + f"eps0={args.eps} per gate"
                        + (f" + learned truncation once per step (ratio {args.learned_ratio:g}, fallback tol "
                           f"{args.learned_tol:g})" if args.trunc == "learned" else "")
                        + f", Trotter steps {args.warmup + 1}-{args.warmup + args.steps}",
            "qubits": 127,
            "gates_per_step": 271,
            "lanes": lanes,
        },
        "roofline": roofline,
        "cpu_baseline": cpu,
        "extra": extra,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
