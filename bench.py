#!/usr/bin/env python3
"""Throughput of the whole MD step (Tasks 1-5: kick-drift, skin test + list rebuild when
due, EAM density, EAM + Morse forces with the fused final kick, energies every 10 steps)
on one MI355X, in atom-steps/s.

Default workload: the 216,000-atom Cr film (60x60x30 BCC cells) with a 2 nm carbon
hemisphere indenter moving -0.001 A/fs, FP64, 2000 steps of 1 fs, inputs resident in HBM
before the timed region.  Beside it (in "variants"): the same film with FP32-mixed
forces and their error against the FP64 path, the 64-replica ensemble in FP32-mixed run
as captured HIP graphs with an autotuned launch shape, and the NVE energy drift of the
periodic 2,000-atom bulk.  Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c1] [--precision fp64]
    python bench.py --copy-probe 512      # plain copy of 512 MiB (counter calibration)
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "atom-steps/s EAM+Morse MD step, FP32-mixed & batched vs FP64 at ≤1e-5 force err"
HBM_PEAK_GBS = 8000.0
TIME_EVERY = 8   # kernel timing events on one step in TIME_EVERY (--time-every)
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "c1_fp64_hbm_traffic.txt")
SOURCES = {k: [os.path.join(ROOT, "paper_1507_07068_amd", "csrc", f) for f in v]
           for k, v in (("force", ("md_forces.hip", "md_device.hpp")),
                        ("list", ("md_rebuild.hip", "md_device.hpp")))}

WORKLOADS = {
    "c0": (0, "bcc_bulk_10x10x10_2k_periodic"),
    "c1": (1, "cr_film_60x60x30_216k_indenter_r20"),
    "c2": (2, "cr_film_100x100x50_1m_indenter_r30"),
    "c3": (3, "ensemble_64_replicas_1.6k-36k"),
    "c4": (4, "cr_film_200x200x100_8m_indenter_r50_preindented"),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def force_bytes_per_atom(mean_list: float, drift: bool = False) -> float:
    """Algorithmic HBM bytes of one EAM force launch per atom: q_i = (x, y, z, F') 32,
    list count 4, list entries 4 each, Cr-C count 4 (the few atoms with carbons in range
    also read their 32-byte Cr-C record), fixed flag 1, velocity read + write for the fused
    kick 48, force write 24; with the next step's drift in the same launch (FP64 steps
    whose velocities are not observed: all but the energy steps and the last) also the new
    position 32 and the reference position 24.  Neighbour positions are gathered from
    cache (atoms are cell-sorted, so each one is fetched from HBM once per pass)."""
    return 32 + 4 + 4 * mean_list + 4 + 1 + 48 + 24 + (56 if drift else 0)


def list_bytes_per_atom(mean_list: float) -> float:
    """Algorithmic HBM bytes of one Cr-Cr list-build launch per rebuilt atom: read the
    cell-sorted state (q 32, FP32 copy 16, v 24, f 24, fixed 1, id 4) = 101; write it back
    (q 32, reference position 24, v 24, f 24, fixed 1, id 4) plus the list count 4 and list
    entries 4 each = 113 + 4 L.  Candidate positions come from cache (each cell row is
    staged once per block).  The Cr-C lists that the launch's leading blocks build for the
    atoms near the indenter are not counted (a few thousand atoms of the 216,000)."""
    return 101 + 113 + 4 * mean_list


def source_hash(kind: str) -> str:
    """Hash of a kernel's sources with // comments and trailing blanks removed (the sources
    hold no string literal with //), so that a comment edit keeps recorded counters valid."""
    h = hashlib.sha256()
    for f in SOURCES[kind]:
        with open(f, encoding="utf-8") as fh:
            for line in fh:
                code = line.split("//", 1)[0].rstrip()
                if code:
                    h.update(code.encode() + b"\n")
    return h.hexdigest()[:16]


def measured_traffic(kind: str, n_launch_atoms: int):
    """HBM bytes per launch of the force ("force") or list-build ("list") kernel from the
    committed counter summary (FETCH_SIZE and WRITE_SIZE per dispatch, each scaled by the
    same counter's reading for a plain copy of known size), or None when there is no
    summary for this workload or the kernel's sources changed since the counters were
    taken."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    kv = {}
    with open(TRAFFIC_FILE) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    try:
        if kv[kind + "_source_sha256"] != source_hash(kind) or int(kv["atoms"]) != n_launch_atoms:
            return None
        copy_b = float(kv["copy_bytes"])
        f_scale = copy_b / (float(kv["copy_fetch_kib"]) * 1024.0)
        w_scale = copy_b / (float(kv["copy_write_kib"]) * 1024.0)
        return (float(kv[kind + "_fetch_kib"]) * 1024.0 * f_scale
                + float(kv[kind + "_write_kib"]) * 1024.0 * w_scale)
    except (KeyError, ValueError, ZeroDivisionError):
        return None


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


class TimingEvent:
    """A HIP event for kernel timing, created with hipEventDisableSystemFence: recording it
    skips the system-scope cache write-back and invalidation that a default event does,
    which would otherwise slow the kernel that follows it.  Uses the HIP runtime that torch
    has already loaded."""
    _hip = None

    def __init__(self):
        import ctypes as C
        if TimingEvent._hip is None:
            hip = C.CDLL("libamdhip64.so.7", mode=os.RTLD_NOLOAD | C.RTLD_GLOBAL)
            hip.hipEventCreateWithFlags.argtypes = [C.POINTER(C.c_void_p), C.c_uint]
            hip.hipEventElapsedTime.argtypes = [C.POINTER(C.c_float), C.c_void_p, C.c_void_p]
            hip.hipEventDestroy.argtypes = [C.c_void_p]
            TimingEvent._hip = hip
        h = C.c_void_p()
        if TimingEvent._hip.hipEventCreateWithFlags(C.byref(h), 0x20000000) != 0:
            raise RuntimeError("hipEventCreateWithFlags failed")
        self.cuda_event = h.value

    def elapsed_time(self, end) -> float:
        import ctypes as C
        ms = C.c_float()
        if TimingEvent._hip.hipEventElapsedTime(C.byref(ms), self.cuda_event, end.cuda_event) != 0:
            raise RuntimeError("hipEventElapsedTime failed")
        return ms.value

    def __del__(self):
        if self.cuda_event and TimingEvent._hip is not None:
            TimingEvent._hip.hipEventDestroy(self.cuda_event)


def timed_run(systems, precision, steps, warmup, ee, tpa, events=True, time_every=TIME_EVERY):
    """Build, warm up, then time `steps` whole steps with md_run.  Returns a dict."""
    import numpy as np
    import torch

    from paper_1507_07068_amd import md

    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        sim = md.Simulation(systems, precision=precision, xcap=160, tpa=tpa)
        sim.initial_forces()
        if warmup:
            sim.md_run(warmup)
        flags = sim.md_check()
        if flags["overflow"] or flags["xoverflow"] or flags["sync_timeout"]:
            raise SystemExit(f"list capacity / sync problem after warm-up: {flags}")
        nobs = steps // ee if ee > 0 else 0
        obs = torch.zeros((max(nobs, 1), sim.nrep, md.MD_NOBS), dtype=torch.float64, device="cuda")
        ev = None
        timed = []
        if events:   # a seeded random sample of the steps (a stride could alias with the
                     # rebuild pattern, which is nearly periodic)
            rng = np.random.default_rng(12345)
            timed = sorted(rng.choice(steps, size=max(1, steps // max(time_every, 1)), replace=False).tolist())
        if events:
            # events around the force and list kernels of the sampled steps (on every step
            # they would add several per cent to the step time)
            ev = [None] * (4 * steps)
            for k in timed:
                for u in range(4):
                    ev[4 * k + u] = TimingEvent()
        builds0 = flags["nbuilds"]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.md_run(steps, energy_every=ee, obs=obs, events=ev)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        flags = sim.md_check()
        if flags["overflow"] or flags["xoverflow"] or flags["nonfinite"] or flags["sync_timeout"]:
            raise SystemExit(f"invalid run: {flags}")
        k_ms = (np.array([ev[4 * k].elapsed_time(ev[4 * k + 1]) for k in timed])
                if events else np.zeros(1))
        l_ms = (np.array([ev[4 * k + 2].elapsed_time(ev[4 * k + 3]) for k in timed])
                if events else np.zeros(1))
        cnt = sim.list_counts()
        live = np.concatenate([np.arange(o, o + s.n) for o, s in zip(sim.offsets, systems)])
        mean_list = float(cnt[live].mean()) if live.size else 0.0
        o = obs.cpu().numpy()
    n_atoms = sum(s.n for s in systems)
    builds = flags["nbuilds"] - builds0
    # sampled list-kernel launches: those that rebuilt are far longer than those that return
    # at once, so they are told apart by the geometric mean of the extremes (when the two
    # kinds differ); the sample is random, so the run's list-kernel time is its mean x steps
    l_avg = 0.0
    if events and builds:
        lo, hi = max(float(l_ms.min()), 1e-6), float(l_ms.max())
        reb = l_ms[l_ms > np.sqrt(lo * hi)] if hi > 4 * lo else l_ms
        l_avg = float(reb.mean()) * 1e-3
    l_total = float(l_ms.mean()) * 1e-3 * steps if events else 0.0
    return dict(sim=sim, rate=n_atoms * steps / wall, wall=wall, ms_per_step=wall / steps * 1e3,
                k_avg=float(k_ms.mean()) * 1e-3, l_avg=l_avg, l_total=l_total,
                k_total=float(k_ms.mean()) * 1e-3 * steps, mean_list=mean_list,
                builds=builds, obs=o[:nobs], n_atoms=n_atoms)


def force_error_vs_fp64(systems, tpa):
    """Relative RMS difference of the FP32-mixed and FP64 GPU forces on the start state
    (the FP64 path itself matches the oracle to 1e-10, see the parity tests)."""
    import numpy as np

    from paper_1507_07068_amd import md
    f = {}
    for prec in ("fp64", "mixed"):
        sim = md.Simulation(systems, precision=prec, xcap=160, tpa=tpa)
        sim.initial_forces()
        f[prec] = np.concatenate([st["f"] for st in sim.state()])
        sim.close()
    d = f["mixed"] - f["fp64"]
    return float(np.sqrt((d * d).sum() / (f["fp64"] ** 2).sum()))


def drift_per_ns(obs, n_atoms, dt_fs, ee):
    """Least-squares slope of E_total / N over time, in eV/atom/ns (obs rows every ee steps)."""
    import numpy as np
    e = obs[:, :, 0:4].sum(-1).sum(-1) / n_atoms
    t_ns = (np.arange(1, e.size + 1) * ee * dt_fs) * 1e-6
    return float(np.polyfit(t_ns, e, 1)[0])


def batched_graph_run(systems, steps, tpa, chunk=100):
    """The ensemble as captured HIP graphs of `chunk` whole steps each."""
    import torch

    from paper_1507_07068_amd import md
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        # small replicas can hold an indenter wider than their periodic box, whose
        # overlapping images crowd the Cr-C lists: give those lists more room
        sim = md.Simulation(systems, precision="mixed", xcap=256, tpa=tpa)
        sim.initial_forces()
        g = sim.md_graph_create(chunk)
        sim.md_graph_launch(g)                    # warm-up chunk
        torch.cuda.synchronize()
        n = max(1, steps // chunk)
        t0 = time.perf_counter()
        for _ in range(n):
            sim.md_graph_launch(g)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        flags = sim.md_check()
        sim.close()
    if flags["overflow"] or flags["xoverflow"] or flags["nonfinite"] or flags["sync_timeout"]:
        raise SystemExit(f"invalid batched run: {flags}")
    n_atoms = sum(s.n for s in systems)
    return dict(rate=n_atoms * n * chunk / wall, steps=n * chunk, ms_per_step=wall / (n * chunk) * 1e3)


def variants(tpa_main):
    from paper_1507_07068_amd import inputs as I
    from paper_1507_07068_amd import tune

    out = {}
    c1 = I.config(1)
    r = timed_run([c1], "mixed", c1.steps, 20, 10, tpa_main, events=False)
    r["sim"].close()
    out["mixed_c1"] = {"value": r["rate"], "unit": "atom-steps/s", "ms_per_step": r["ms_per_step"],
                       "steps": c1.steps, "dtype": "f32 pair math, f64 state",
                       "force_rel_rms_vs_fp64": force_error_vs_fp64([c1], tpa_main),
                       "list_builds": r["builds"]}
    log(f"[bench] mixed c1: {r['rate']:.4e} atom-steps/s, force rel-RMS vs FP64 "
        f"{out['mixed_c1']['force_rel_rms_vs_fp64']:.2e}")
    ens = I.config(3)
    best, times = tune.choose_tpa(ens, "mixed")
    b = batched_graph_run(ens, ens[0].steps, best)
    out["batched_c3"] = {"value": b["rate"], "unit": "atom-steps/s", "ms_per_step": b["ms_per_step"],
                         "steps": b["steps"], "replicas": len(ens), "cr_atoms": sum(s.n for s in ens),
                         "precision": "mixed", "launch": "hipGraph of 100 whole steps",
                         "tpa_autotuned": best,
                         "tpa_ms_per_step": {str(k): round(v * 1e3, 4) for k, v in times.items()}}
    log(f"[bench] batched c3: {b['rate']:.4e} atom-steps/s (tpa {best})")
    c0 = I.config(0)
    nve = {}
    for prec in ("fp64", "mixed"):
        r = timed_run([c0], prec, 10000, 0, 10, 1, events=False)
        r["sim"].close()
        nve[prec] = drift_per_ns(r["obs"], c0.n, c0.dt, 10)
    out["nve_c0"] = {"steps": 10000, "dt_fs": c0.dt, "drift_ev_per_atom_per_ns_fp64": nve["fp64"],
                     "drift_ev_per_atom_per_ns_mixed": nve["mixed"]}
    log(f"[bench] NVE c0 drift: fp64 {nve['fp64']:.3e}, mixed {nve['mixed']:.3e} eV/atom/ns")
    return out


def copy_probe(mib: int) -> int:
    import torch
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"probe": "copy", "bytes_per_copy": n * 4, "copies": 5}), flush=True)
    return 0


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
    ap.add_argument("--time-every", type=int, default=TIME_EVERY, metavar="K",
                    help="record the kernel timing events on a random one in K steps")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MiB")
    args = ap.parse_args(argv)

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        return 2
    if args.copy_probe:
        return copy_probe(args.copy_probe)

    from paper_1507_07068_amd import inputs as I

    idx, wname = WORKLOADS[args.workload]
    cfg = I.config(idx)
    systems = cfg if isinstance(cfg, list) else [cfg]
    precision = args.precision or systems[0].precision
    steps = args.steps if args.steps is not None else systems[0].steps
    ee = args.energy_every
    log(f"[bench] workload {args.workload} ({wname}): {len(systems)} system(s), "
        f"{sum(s.n for s in systems)} Cr, {sum(s.n_c for s in systems)} C, precision {precision}, "
        f"steps {steps}, warmup {args.warmup}")
    r = timed_run(systems, precision, steps, args.warmup, ee, args.tpa, time_every=args.time_every)
    r["sim"].close()
    n_atoms, rate, k_avg, mean_list = r["n_atoms"], r["rate"], r["k_avg"], r["mean_list"]
    # FP64 runs (no shadow) drift the atoms in the force pass of most steps
    bytes_launch = n_atoms * force_bytes_per_atom(mean_list, drift=precision == "fp64")
    achieved = bytes_launch / k_avg / 1e9
    e_tot = r["obs"][:, :, 0:4].sum(-1).sum(-1) if r["obs"].size else [0.0]
    log(f"[bench] {rate:.4e} atom-steps/s, {r['ms_per_step']:.4f} ms/step, EAM force kernel "
        f"{k_avg * 1e6:.2f} us avg ({achieved:.0f} GB/s algorithmic), mean list {mean_list:.2f}, "
        f"{r['builds']} list builds, E_tot first/last {e_tot[0]:.6f} / {e_tot[-1]:.6f} eV")
    # (+24 B per atom for the fixed-point shadow and build cell written in mixed runs)
    lbytes = (n_atoms * (list_bytes_per_atom(mean_list) + (24 if precision == "mixed" else 0))
              if len(systems) == 1 else None)
    l_achieved = lbytes / r["l_avg"] / 1e9 if (lbytes and r["l_avg"] > 0) else None
    traffic = ltraffic = None   # measured HBM bytes per launch (compare with bytes_per_launch)
    if args.workload == "c1" and precision == "fp64" and args.tpa == 2:
        traffic = measured_traffic("force", n_atoms)
        ltraffic = measured_traffic("list", n_atoms)
    log(f"[bench] list kernel {r['l_avg'] * 1e6:.2f} us per rebuild launch"
        + (f" ({l_achieved:.0f} GB/s algorithmic)" if l_achieved else "")
        + f"; GPU time in list / force kernels {r['l_total'] * 1e3:.1f} / {r['k_total'] * 1e3:.1f} ms")
    result = {
        "metric": METRIC,
        "value": rate,
        "unit": "atom-steps/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if precision == "fp64" else "f32-mixed",
        "data": "synthetic",
        "config": {"workload": wname, "cr_atoms": n_atoms, "c_atoms": sum(s.n_c for s in systems),
                   "replicas": len(systems), "precision": precision, "energy_every": ee,
                   "list_builds": r["builds"], "mean_list_len": round(mean_list, 3),
                   "lanes_per_atom": args.tpa},
        "roofline": None,
        "roofline_force": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                           "kernel": ("k_force (EAM Eq. 1 with the Cr-C forces, fused kicks"
                                      + (" and next drift)" if precision == "fp64" else ")")),
                           "avg_us": k_avg * 1e6, "bytes_per_launch": bytes_launch,
                           "gpu_ms_total": r["k_total"] * 1e3},
        "cpu_baseline": None,
    }
    if l_achieved:
        result["roofline_list"] = {"bound": "hbm", "achieved": l_achieved, "peak": HBM_PEAK_GBS,
                                   "unit": "GB/s", "frac": l_achieved / HBM_PEAK_GBS, "traffic": ltraffic,
                                   "kernel": "k_list_tiles (Cr-Cr Verlet list build with the Cr-C lists in leading blocks, rebuild launches)",
                                   "avg_us": r["l_avg"] * 1e6, "bytes_per_launch": lbytes,
                                   "gpu_ms_total": r["l_total"] * 1e3}
    # the dominant kernel: the one with the most GPU time over the timed steps
    dom = ("roofline_list" if ("roofline_list" in result
                               and r["l_total"] > r["k_total"]) else "roofline_force")
    result["roofline"] = dict(result[dom], dominant_of=["k_force", "k_list_tiles"])
    if not args.no_variants and args.workload == "c1" and args.steps is None:
        result["variants"] = variants(args.tpa)
    if not args.no_cpu_baseline and len(systems) == 1 and systems[0].n <= 300_000:
        spb = steps / max(r["builds"], 1)
        log(f"[bench] CPU baseline: oracle on {systems[0].name}, ~{spb:.0f} steps ...")
        result["cpu_baseline"] = cpu_baseline(I.config(idx), spb)
        log(f"[bench] CPU baseline {result['cpu_baseline']['value']:.4e} atom-steps/s")
    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
