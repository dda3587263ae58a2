#!/usr/bin/env python3
"""Throughput of the whole MD step (Tasks 1-5: kick-drift, skin test + list rebuild when
due, EAM density, EAM + Morse forces with the fused final kick, energies every 10 steps)
on one MI355X, in atom-steps/s.

Default workload: the 216,000-atom Cr film (60x60x30 BCC cells) with a 2 nm carbon
hemisphere indenter moving -0.001 A/fs, FP64, 2000 steps of 1 fs (inputs resident in
HBM before the timed region).  Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c1] [--precision fp64]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "atom-steps/s EAM+Morse MD step, FP32-mixed & batched vs FP64 at ≤1e-5 force err"
HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    "c0": (0, "bcc_bulk_2k_periodic"),
    "c1": (1, "cr_film_60x60x30_216k_indenter_r20"),
    "c2": (2, "cr_film_100x100x50_1m_indenter_r30"),
    "c3": (3, "ensemble_64_replicas_1.6k-36k"),
    "c4": (4, "cr_film_200x200x100_8m_indenter_r50_preindented"),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def force_bytes_per_atom(mean_list: float) -> float:
    """Algorithmic HBM bytes of the force pass per atom: x_i (24) + F'(rho_i) (8) + list count
    (4) + list entries (4 each) + force write (24) + velocity read/write for the fused kick
    (48).  Neighbour positions are gathered from cache (atoms are cell-sorted)."""
    return 24 + 8 + 4 + 4 * mean_list + 24 + 48


def cpu_baseline(system, steps_per_build: float) -> dict:
    """The FP64 oracle as it stands, on a bounded sample of the same workload: one list
    build (brute force, O(N^2)) plus about one rebuild interval of list-mode steps."""
    import oracle as O
    k = int(max(1, min(round(steps_per_build), 50)))
    t0 = time.perf_counter()
    out = O.md_run(system, k, use_lists=True, cap=64)
    t = time.perf_counter() - t0
    builds = int(out["obs"][-1, 14])
    return {"value": system.n * k / t, "unit": "atom-steps/s", "cores": O.num_threads(),
            "kind": "oracle",
            "sample": f"{system.name}: {k} steps of the FP64 oracle from t=0 in list mode, "
                      f"{builds} O(N^2) list build(s) included (one rebuild interval of the GPU run), "
                      f"{t:.1f} s wall"}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="c1", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default=None, choices=["fp64", "mixed"])
    ap.add_argument("--energy-every", type=int, default=10)
    ap.add_argument("--tpa", type=int, default=2, choices=[1, 2, 4, 8],
                    help="lanes per atom in the density / force passes")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args(argv)

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from paper_1507_07068_amd import inputs as I
    from paper_1507_07068_amd import md

    idx, wname = WORKLOADS[args.workload]
    cfg = I.config(idx)
    systems = cfg if isinstance(cfg, list) else [cfg]
    precision = args.precision or systems[0].precision
    steps = args.steps if args.steps is not None else systems[0].steps
    ee = args.energy_every
    n_atoms = sum(s.n for s in systems)
    log(f"[bench] workload {args.workload} ({wname}): {len(systems)} system(s), {n_atoms} Cr, "
        f"{sum(s.n_c for s in systems)} C, precision {precision}, steps {steps}, warmup {args.warmup}")

    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        sim = md.Simulation(systems, precision=precision, xcap=160, tpa=args.tpa)
        sim.initial_forces()
        if args.warmup:
            sim.md_run(args.warmup)
        flags = sim.md_check()
        if flags["overflow"] or flags["xoverflow"] or flags["sync_timeout"]:
            raise SystemExit(f"list capacity / sync problem after warm-up: {flags}")
        nobs = steps // ee if ee > 0 else 0
        obs = torch.zeros((max(nobs, 1), sim.nrep, md.MD_NOBS), dtype=torch.float64, device="cuda")
        events = [torch.cuda.Event(enable_timing=True) for _ in range(2 * steps)]
        for e in events:          # torch creates the HIP event at its first record
            e.record(stream)
        builds0 = flags["nbuilds"]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.md_run(steps, energy_every=ee, obs=obs, events=events)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        flags = sim.md_check()
        if flags["overflow"] or flags["xoverflow"] or flags["nonfinite"] or flags["sync_timeout"]:
            raise SystemExit(f"invalid run: {flags}")
        k_ms = np.array([events[2 * k].elapsed_time(events[2 * k + 1]) for k in range(steps)])
        cnt = sim.list_counts()
        live = np.concatenate([np.arange(o, o + s.n) for o, s in zip(sim.offsets, systems)])
        mean_list = float(cnt[live].mean()) if live.size else 0.0
        o = obs.cpu().numpy()
    builds = flags["nbuilds"] - builds0
    rate = n_atoms * steps / wall
    bytes_launch = n_atoms * force_bytes_per_atom(mean_list)
    k_avg = float(k_ms.mean()) * 1e-3
    achieved = bytes_launch / k_avg / 1e9
    e_tot = o[:, :, 0:4].sum(-1).sum(-1) if nobs else np.zeros(1)
    log(f"[bench] {rate:.4e} atom-steps/s, {wall / steps * 1e3:.4f} ms/step, force kernel "
        f"{k_avg * 1e6:.2f} us avg ({achieved:.0f} GB/s algorithmic), mean list {mean_list:.2f}, "
        f"{builds} list builds, E_tot first/last {e_tot[0]:.6f} / {e_tot[-1]:.6f} eV")

    result = {
        "metric": METRIC,
        "value": rate,
        "unit": "atom-steps/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": wall / steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if precision == "fp64" else "f32-mixed",
        "data": "synthetic",
        "config": {"workload": wname, "cr_atoms": n_atoms, "c_atoms": sum(s.n_c for s in systems),
                   "replicas": len(systems), "precision": precision, "energy_every": ee,
                   "list_builds": builds, "mean_list_len": round(mean_list, 3),
                   "lanes_per_atom": args.tpa},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "k_force (EAM Eq. 1 + Morse + final kick)",
                     "avg_us": k_avg * 1e6, "bytes_per_launch": bytes_launch},
        "cpu_baseline": None,
    }
    if not args.no_cpu_baseline and len(systems) == 1:
        spb = steps / max(builds, 1)
        log(f"[bench] CPU baseline: oracle on {systems[0].name}, ~{spb:.0f} steps ...")
        result["cpu_baseline"] = cpu_baseline(I.config(idx), spb)
        log(f"[bench] CPU baseline {result['cpu_baseline']['value']:.4e} atom-steps/s")
    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
