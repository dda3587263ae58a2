#!/usr/bin/env python3
"""Throughput of the whole MD step (Tasks 1-5: kick-drift, skin test + list rebuild when
due, EAM density with the Cr-C Morse pass, EAM + Morse forces with the fused final kick,
energies every 10 steps) on one MI355X, in Cr atom-steps/s.

Headline (`value`): the largest single-GPU workload, the 8M-atom Cr film (200x200x100 BCC
cells, 5 nm carbon hemisphere pre-indented 2 nm, moving -0.001 A/fs) in FP64, inputs
resident in HBM before the timed region, K timed steps after W warm-up steps.

Beside it, in the same JSON line, whatever --steps says:
  kernels      per-kernel times from a separate pass of K steps with events around the force,
               density and list kernels of every step (outside the timed region), the list
               kernel split by whether the step rebuilt (read from the device);
  roofline     for the kernel with the most GPU time in that pass;
  variants     the same film in FP32-mixed (force error against the FP64 path on all atoms
               and against the oracle on sampled atoms), the 64-replica ensemble in
               FP32-mixed as captured HIP graphs with the autotuned launch shape, NVE drift of
               the periodic 2,000-atom bulk (mean over seeds), and the drift of E_tot + W on the
               216k-atom film with its moving indenter (W: work of the indenter's load);
  full_runs    each workload over its full step count (8M film 500, 216k film 2000, ensemble
               1000), with its list-build count;
  cpu_baseline the FP64 oracle (cell-grid lists) on the same 8M-atom film, all host threads,
               a bounded number of steps; cpu_baseline_1thread the same with one thread (two steps).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c4] [--precision fp64]
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
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_c4_film_8m.txt")
SOURCES = {k: [os.path.join(ROOT, "paper_1507_07068_amd", "csrc", f) for f in v]
           for k, v in (("force", ("md_forces.hip", "md_device.hpp")),
                        ("density", ("md_forces.hip", "md_device.hpp")),
                        ("list", ("md_rebuild.hip", "md_device.hpp")))}

WORKLOADS = {
    "c0": (0, "bcc_bulk_10x10x10_2k_periodic"),
    "c1": (1, "cr_film_60x60x30_216k_indenter_r20"),
    "c2": (2, "cr_film_100x100x50_1m_indenter_r30"),
    "c3": (3, "ensemble_64_replicas_1.6k-36k"),
    "c4": (4, "cr_film_200x200x100_8m_indenter_r50_preindented"),
}
KERNEL_NAMES = {
    "force": "k_force (EAM Eq. 1 with the Cr-C forces and the fused kicks; on steps whose "
             "velocities are not observed the full kick without the force store, and the drift)",
    "density": "k_density (rho and F'(rho), with the Cr-C Morse pass in its leading blocks)",
    "list": "k_list_tiles (Cr-Cr Verlet list build with the Cr-C lists in leading blocks), "
            "launches of steps that rebuilt",
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# ------------------------------------------------------------------------------------------
# Algorithmic bytes (HBM, per atom, per launch)
# ------------------------------------------------------------------------------------------
def force_bytes_per_atom(mean_list: float, mixed: bool, full: bool) -> float:
    """One EAM force launch: the atom's own record (FP64 q = x, y, z, F' 32 B; mixed: the
    16-byte fixed-point shadow), list count 4, list entries 4 each, Cr-C count 4, fixed flag
    1, velocity read + write for the fused kick 48.  A launch that also gives the next step's
    first half kick (full: every step of md_run but the last) does not store the force; the
    last writes it (24, the FP64 force array in both paths).  A full launch also drifts the
    atoms: the new position 32 and the reference position 24 (mixed: also the FP64 position
    32, the new shadow 16 and the build cell 8).
    Neighbour records are gathered from cache (atoms are cell-sorted, so each one comes from
    HBM about once per pass): they are not counted."""
    own = 16 if mixed else 32
    drift = (56 + (56 if mixed else 0)) if full else 0
    return own + 4 + 4 * mean_list + 4 + 1 + 48 + (0 if full else 24) + drift


def density_bytes_per_atom(mean_list: float, mixed: bool) -> float:
    """One density launch: own record (32 FP64 / 16 shadow), list count 4, entries 4 each,
    F'(rho) written into the record (8; mixed also its FP32 copy in the shadow, 4).  The Cr-C
    pass of its leading blocks touches the few atoms near the indenter only (not counted)."""
    return (16 + 4 + 4 * mean_list + 8 + 4) if mixed else (32 + 4 + 4 * mean_list + 8)


def list_bytes_per_atom(mean_list: float, mixed: bool) -> float:
    """One Cr-Cr list-build launch of md_run that rebuilds, per atom: read the cell-sorted
    state (q 32, FP32 copy 16, v 24, fixed 1, id 4) = 77; write it back (q 32, reference
    position 24, v 24, fixed 1, id 4) plus the list count 4 and the entries 4 each = 89 + 4 L
    (inside md_run the forces are not permuted: no kick reads them before the next force
    pass stores them); mixed runs also write the fixed-point shadow 16 and the build cell 8.
    Candidates come from cache (each staged cell row once per block); the Cr-C lists of the
    leading blocks (a few thousand atoms near the indenter) are not counted."""
    return 77 + 89 + 4 * mean_list + (24 if mixed else 0)


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


def measured_traffic(kind: str, n_atoms: int, precision: str):
    """HBM bytes per launch of a kernel from the committed counter summary (FETCH_SIZE and
    WRITE_SIZE per dispatch, each scaled by the same counter's reading for a plain copy of
    known size), with the mean list length of the run the counters were taken on, or None
    when the summary is for another workload or the kernel's sources changed since."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    kv = {}
    with open(TRAFFIC_FILE) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    try:
        if (kv[kind + "_source_sha256"] != source_hash(kind) or int(kv["atoms"]) != n_atoms
                or kv["precision"] != precision):
            return None
        copy_b = float(kv["copy_bytes"])
        f_scale = copy_b / (float(kv["copy_fetch_kib"]) * 1024.0)
        w_scale = copy_b / (float(kv["copy_write_kib"]) * 1024.0)
        return {"bytes": float(kv[kind + "_fetch_kib"]) * 1024.0 * f_scale
                + float(kv[kind + "_write_kib"]) * 1024.0 * w_scale,
                "mean_list": float(kv["mean_list"])}
    except (KeyError, ValueError, ZeroDivisionError):
        return None


# ------------------------------------------------------------------------------------------
# Timing helpers
# ------------------------------------------------------------------------------------------
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


def check_flags(flags, what):
    if flags["overflow"] or flags["xoverflow"] or flags["nonfinite"] or flags["sync_timeout"]:
        raise SystemExit(f"{what}: invalid run: {flags}")


def mean_list_len(sim, systems) -> float:
    import numpy as np
    cnt = sim.list_counts()
    live = np.concatenate([np.arange(o, o + s.n) for o, s in zip(sim.offsets, systems)])
    return float(cnt[live].mean()) if live.size else 0.0


def make_sim(systems, precision, tpa, xcap=160, cap=None, icap=0, list_tgt=0):
    from paper_1507_07068_amd import md
    return md.Simulation(systems, precision=precision, xcap=xcap, tpa=tpa, cap=cap, icap=icap, list_tgt=list_tgt)


def free_sim(sim):
    """Destroy the handle and drop the device arrays now (not when the name goes away)."""
    import torch
    torch.cuda.synchronize()
    sim.close()
    sim.__dict__.clear()
    torch.cuda.empty_cache()


def timed_run(sim, systems, steps, warmup, ee, what):
    """Warm up, then time `steps` whole steps with md_run (no events in the timed region)."""
    import torch

    from paper_1507_07068_amd import md
    if warmup:
        sim.md_run(warmup)
    flags = sim.md_check()
    check_flags(flags, what + " (warm-up)")
    nobs = steps // ee if ee > 0 else 0
    obs = torch.zeros((max(nobs, 1), sim.nrep, md.MD_NOBS), dtype=torch.float64, device="cuda")
    builds0 = flags["nbuilds"]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.md_run(steps, energy_every=ee, obs=obs)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    flags = sim.md_check()
    check_flags(flags, what)
    n_atoms = sum(s.n for s in systems)
    return dict(rate=n_atoms * steps / wall, wall=wall, ms_per_step=wall / steps * 1e3, steps=steps,
                builds=flags["nbuilds"] - builds0, obs=obs.cpu().numpy()[:nobs], n_atoms=n_atoms,
                mean_list=mean_list_len(sim, systems))


def kernel_pass(sim, systems, steps, ee, precision):
    """`steps` more whole steps with events around the force, list and density kernels of
    every step and the build counts recorded after every step; per-kernel times."""
    import numpy as np
    import torch

    from paper_1507_07068_amd import md
    L0 = mean_list_len(sim, systems)
    ev = [TimingEvent() for _ in range(md.MD_TRACE_EVENTS * steps)]
    builds = torch.zeros((steps, sim.nrep), dtype=torch.int32, device="cuda")
    nobs = steps // ee if ee > 0 else 0
    obs = torch.zeros((max(nobs, 1), sim.nrep, md.MD_NOBS), dtype=torch.float64, device="cuda")
    b0 = sim.md_check()["nbuilds"]
    torch.cuda.synchronize()
    sim.md_run(steps, energy_every=ee, obs=obs, events=ev, builds=builds)
    torch.cuda.synchronize()
    check_flags(sim.md_check(), "kernel timing pass")
    L1 = mean_list_len(sim, systems)
    E = md.MD_TRACE_EVENTS
    t = {name: np.array([ev[E * k + a].elapsed_time(ev[E * k + a + 1]) for k in range(steps)]) * 1e-3
         for name, a in (("force", 0), ("list", 2), ("density", 4), ("inner", 6))}
    b = builds.cpu().numpy().sum(axis=1).astype(np.int64)
    rebuilt = np.diff(np.concatenate([[b0], b])) > 0
    n_atoms = sum(s.n for s in systems)
    L = 0.5 * (L0 + L1)
    mixed = precision == "mixed"
    # every step but the last gives the next step's first half kick and drift inside the force
    # launch: steps whose velocities are not observed as one full kick, observed ones as two
    # half kicks around the energies
    full = np.array([(k + 1) < steps for k in range(steps)])
    fbytes = n_atoms * np.array([force_bytes_per_atom(L, mixed, u) for u in full])
    out = {"steps": steps, "mean_list": L, "rebuilt_steps": int(rebuilt.sum())}
    out["force"] = dict(avg_us=float(t["force"].mean() * 1e6), total_ms=float(t["force"].sum() * 1e3),
                        bytes_per_launch=float(fbytes.mean()),
                        achieved=float(fbytes.sum() / t["force"].sum() / 1e9))
    dbytes = n_atoms * density_bytes_per_atom(L, mixed)
    out["density"] = dict(avg_us=float(t["density"].mean() * 1e6), total_ms=float(t["density"].sum() * 1e3),
                          bytes_per_launch=dbytes, achieved=float(dbytes / t["density"].mean() / 1e9))
    lst = dict(total_ms=float(t["list"].sum() * 1e3), rebuild_launches=int(rebuilt.sum()),
               avg_us_no_rebuild=float(t["list"][~rebuilt].mean() * 1e6) if (~rebuilt).any() else None)
    if rebuilt.any() and len(systems) == 1:
        lb = n_atoms * list_bytes_per_atom(L, mixed)
        lst.update(avg_us=float(t["list"][rebuilt].mean() * 1e6), bytes_per_launch=lb,
                   achieved=float(lb / t["list"][rebuilt].mean() / 1e9))
    out["list"] = lst
    if sim.icap:
        out["inner"] = dict(avg_us=float(t["inner"].mean() * 1e6), total_ms=float(t["inner"].sum() * 1e3))
    out["step_ms"] = float(np.mean([ev[E * k].elapsed_time(ev[E * (k + 1)]) for k in range(steps - 1)])) \
        if steps > 1 else None
    return out


def roofline_of(kern, kind, n_atoms, precision):
    k = kern[kind]
    if "achieved" not in k:
        return None
    r = {"bound": "hbm", "achieved": k["achieved"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
         "frac": k["achieved"] / HBM_PEAK_GBS, "traffic": None, "kernel": KERNEL_NAMES[kind],
         "avg_us": k["avg_us"], "bytes_per_launch": k["bytes_per_launch"],
         "mean_list": kern["mean_list"], "gpu_ms_total": k["total_ms"]}
    if r["frac"] > 1.0:   # algorithmic bytes over event time cannot beat the peak: a timing fault
        r["invalid"] = "achieved above the HBM peak"
    tr = measured_traffic(kind, n_atoms, precision)
    if tr is not None:
        # counter bytes per launch, and the algorithmic bytes at the list length of the run the
        # counters were taken on (the same state), for the ratio
        alg = {"force": lambda L: force_bytes_per_atom(L, precision == "mixed", True),
               "density": lambda L: density_bytes_per_atom(L, precision == "mixed"),
               "list": lambda L: list_bytes_per_atom(L, precision == "mixed")}[kind]
        r["traffic"] = tr["bytes"]
        r["traffic_state"] = {"mean_list": tr["mean_list"], "algorithmic_bytes": n_atoms * alg(tr["mean_list"]),
                              "ratio": tr["bytes"] / (n_atoms * alg(tr["mean_list"]))}
    return r


# ------------------------------------------------------------------------------------------
# Variants
# ------------------------------------------------------------------------------------------
def force_errors(f, ref):
    import numpy as np
    diff = np.sqrt(np.sum((f - ref) ** 2, axis=1))
    rms = np.sqrt(np.mean(np.sum(ref ** 2, axis=1)))
    return float(np.sqrt(np.sum(diff ** 2) / np.sum(ref ** 2))), float(diff.max() / rms)


def mixed_force_errors(system, tpa, n_sample=24, seed=11):
    """FP32-mixed forces at the start state against the FP64 GPU path on every atom, and
    against the FP64 oracle (one atom at a time, all-atom loops) on sampled atoms: a seeded
    draw plus the atoms nearest the indenter tip."""
    import numpy as np

    import oracle as O
    f = {}
    for prec in ("fp64", "mixed"):
        sim = make_sim([system], prec, tpa)
        sim.initial_forces()
        st = sim.state()[0]
        f[prec] = st["f"]
        free_sim(sim)
    rel_all, max_all = force_errors(f["mixed"], f["fp64"])
    rng = np.random.default_rng(seed)
    rows = set(rng.choice(system.n, size=n_sample, replace=False).tolist())
    if system.n_c:
        tip = system.xc[np.argmin(system.xc[:, 2])]
        d = system.x - tip
        rows |= set(np.argsort(np.einsum("ij,ij->i", d, d))[:8].tolist())
    rows = np.array(sorted(rows), dtype=np.int64)
    fo, _, _, _ = O.sample_forces(system, rows, x=O.wrap(system))
    rel_o, max_o = force_errors(f["mixed"][rows], fo)
    rel_o64, _ = force_errors(f["fp64"][rows], fo)
    return {"rel_rms_vs_fp64_gpu_all_atoms": rel_all, "max_over_rms_vs_fp64_gpu": max_all,
            "rel_rms_vs_oracle_sampled": rel_o, "max_over_rms_vs_oracle_sampled": max_o,
            "fp64_gpu_rel_rms_vs_oracle_sampled": rel_o64, "sampled_atoms": int(rows.size)}


def drift_per_ns(e_per_atom, t_fs):
    """Least-squares slope of an energy per atom over time, in eV/atom/ns."""
    import numpy as np
    return float(np.polyfit(t_fs * 1e-6, e_per_atom, 1)[0])


def nve_drift(seeds=(0, 1, 2, 3), steps=10000, ee=10):
    """NVE drift of the periodic 2,000-atom bulk (no indenter) over `steps`, per seed."""
    import numpy as np

    from paper_1507_07068_amd import inputs as I
    out = {}
    for prec in ("fp64", "mixed"):
        d = []
        for seed in seeds:
            s = I.bulk(10, seed=seed, noise=0.02, steps=steps, name=f"c0_seed{seed}")
            sim = make_sim([s], prec, 1)
            sim.initial_forces()
            r = timed_run(sim, [s], steps, 0, ee, "NVE drift")
            free_sim(sim)
            e = r["obs"][:, 0, 0:4].sum(-1) / s.n
            d.append(drift_per_ns(e, np.arange(1, e.size + 1) * ee * s.dt))
        out[prec] = {"mean": float(np.mean(d)), "std": float(np.std(d, ddof=1)), "per_seed": d}
    return {"steps": steps, "dt_fs": 1.0, "seeds": list(seeds),
            "drift_ev_per_atom_per_ns": out}


def indenter_work_drift(system, tpa):
    """E_tot + W on a film with its moving indenter (W = sum over steps of the trapezoid
    (F_ind,z(t) + F_ind,z(t + dt)) / 2 * dz_ind, the work of the load on the indenter): its
    drift, next to that of E_tot alone, energies every step."""
    import numpy as np
    sim = make_sim([system], "fp64", tpa)
    sim.initial_forces()
    o0 = sim.md_energy()[0]
    r = timed_run(sim, [system], system.steps, 0, 1, "indenter work drift")
    free_sim(sim)
    o = np.concatenate([o0[None], r["obs"][:, 0]], axis=0)
    e = o[:, 0:4].sum(-1)
    fz, z = o[:, 12], o[:, 13]
    w = np.concatenate([[0.0], np.cumsum(0.5 * (fz[1:] + fz[:-1]) * np.diff(z))])
    t = np.arange(o.shape[0]) * system.dt
    return {"steps": system.steps, "workload": system.name,
            "drift_e_tot_ev_per_atom_per_ns": drift_per_ns(e / system.n, t),
            "drift_e_tot_plus_w_ev_per_atom_per_ns": drift_per_ns((e + w) / system.n, t),
            "w_total_ev": float(w[-1])}


def batched_graph_run(systems, steps, tpa, chunk=100, list_tgt=0):
    """The ensemble as captured HIP graphs of `chunk` whole steps each."""
    import torch
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        # small replicas can hold an indenter wider than their periodic box, whose
        # overlapping images crowd the Cr-C lists: give those lists more room
        sim = make_sim(systems, "mixed", tpa, xcap=256, list_tgt=list_tgt)
        sim.initial_forces()
        g = sim.md_graph_create(chunk)
        sim.md_graph_launch(g)                    # warm-up chunk
        torch.cuda.synchronize()
        b0 = sim.md_check()["nbuilds"]
        n = max(1, steps // chunk)
        t0 = time.perf_counter()
        for _ in range(n):
            sim.md_graph_launch(g)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        flags = sim.md_check()
        free_sim(sim)
    check_flags(flags, "batched run")
    n_atoms = sum(s.n for s in systems)
    return dict(rate=n_atoms * n * chunk / wall, steps=n * chunk, ms_per_step=wall / (n * chunk) * 1e3,
                builds=flags["nbuilds"] - b0)


def paper_form_run(system, tpa, two_tier, steps=300, warmup=20, ee=10, kern_steps=20):
    """The paper's own EAM form on `system` with the indenter at rest (the set-up of the
    paper's timing runs, Section 4.1: 300 steps), over one list (cutoff r* + 0.3 A) or over
    Section 2.6's two-tier lists (outer 1.7 r*, inner r* refilled every step)."""
    from paper_1507_07068_amd import inputs as I
    s = system.copy()
    s.v_ind = 0.0
    s.potential = "paper"
    if two_tier:
        I.two_tier(s)
        sim = make_sim([s], "fp64", tpa, xcap=320, cap=1152, icap=256)
    else:
        sim = make_sim([s], "fp64", tpa, cap=256)
    sim.initial_forces()
    what = f"paper form {s.name} {'two-tier' if two_tier else 'one list'}"
    r = timed_run(sim, [s], steps, warmup, ee, what)
    kern = kernel_pass(sim, [s], kern_steps, ee, "fp64")
    inner_mean = None
    if two_tier:
        import numpy as np
        inner_mean = float(np.mean(sim.icnt.cpu().numpy()[:s.n]))
    free_sim(sim)
    out = {"value": r["rate"], "unit": "atom-steps/s", "steps": steps, "warmup": warmup,
           "ms_per_step": r["ms_per_step"], "precision": "fp64", "list_builds": r["builds"],
           "mean_list_len": round(r["mean_list"], 3), "list_radius": round(s.r_list, 4),
           "kernels_us": {k: round(kern[k]["avg_us"], 2) for k in ("force", "density", "inner") if k in kern}}
    out["kernels_us"]["list_per_rebuild"] = kern["list"].get("avg_us")
    if two_tier:
        out["inner_mean_len"] = round(inner_mean, 3)
    log(f"[bench] {what}: {r['rate']:.4e} atom-steps/s, {r['ms_per_step']:.4f} ms/step, "
        f"{r['builds']} builds, kernels {out['kernels_us']}")
    return out


def protocol_run(tpa, relax_steps=10000):
    """Section 4.3's complete nano-indentation at the paper's scale: the 19 x 19 x 14-cell film
    (periodic laterally here) at 10 K with the paper's form, an R = 9.78 A indenter 0.5 A above
    it, relaxed for 10,000 steps, loaded at 1e-4 A/fs to 3.08 A below the initial surface and
    unloaded; the recorded load-depth curve analysed as Section 4.3 does."""
    import numpy as np

    from paper_1507_07068_amd import inputs as I
    from paper_1507_07068_amd import protocol as P
    s = I.film(19, 19, 14, radius=9.78, gap=0.5, seed=5, temperature=10.0, v_ind=0.0,
               name="paper_indentation_19x19x14")
    s.potential = "paper"
    pr = P.Protocol(relax_steps=relax_steps)
    sim = make_sim([s], "fp64", tpa, xcap=160, cap=256)
    sim.initial_forces()
    steps = sum(n for _, n, _ in pr.phases(s))
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rec = P.run(sim, s, pr)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    check_flags(sim.md_check(), "indentation protocol")
    free_sim(sim)
    ana = P.analyse(rec, radius=9.78)
    load_rec = rec["phase"] > 0
    out = {"cr_atoms": s.n, "c_atoms": s.n_c, "steps": steps, "wall_s": round(wall, 3),
           "value": s.n * steps / wall, "unit": "atom-steps/s", "potential": "paper (synthetic parameters)",
           "temperature_K": 10.0, "speed_A_per_fs": pr.speed, "target_depth_A": pr.depth,
           "analysis": {k: (round(float(v), 4) if isinstance(v, (float, np.floating)) else v) for k, v in ana.items()},
           "curve_every_100_steps": {"depth_A": [round(float(x), 4) for x in rec["depth"][load_rec][::20]],
                                     "load_eV_per_A": [round(float(x), 4) for x in rec["load"][load_rec][::20]]}}
    log(f"[bench] indentation protocol ({s.n} Cr, {s.n_c} C, {steps} steps): {out['value']:.3e} atom-steps/s, "
        f"P_max {ana.get('p_max', 0):.3f} eV/A at {ana.get('h_max', 0):.3f} A, S {ana.get('unloading_slope', 0):.3f}, "
        f"E* {ana.get('e_star_gpa', float('nan')):.1f} GPa, H {ana.get('hardness_gpa', float('nan')):.1f} GPa")
    return out


def full_run(systems, precision, tpa, warmup=20, ee=10):
    sim = make_sim(systems, precision, tpa)
    sim.initial_forces()
    r = timed_run(sim, systems, systems[0].steps, warmup, ee, f"full run {systems[0].name}")
    free_sim(sim)
    return {"value": r["rate"], "unit": "atom-steps/s", "steps": r["steps"], "warmup": warmup,
            "ms_per_step": r["ms_per_step"], "precision": precision, "list_builds": r["builds"],
            "mean_list_len": round(r["mean_list"], 3)}


# ------------------------------------------------------------------------------------------
# CPU baseline
# ------------------------------------------------------------------------------------------
def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(system, threads=None, budget_s=20.0, max_steps=40) -> dict:
    """The FP64 oracle as it stands (lists through its cell grid), on the same workload: the
    set-up at t = 0 (list build, first forces) is timed on its own and taken out, so the rate
    is of whole steps (drift, skin test, rebuilds when due, forces, kicks).  The step count is
    chosen from a 2-step probe to fit `budget_s`."""
    import oracle as O
    if threads:
        O.set_num_threads(threads)
    try:
        def run(k):
            t0 = time.perf_counter()
            out = O.md_run(system, k, use_lists="cells", cap=64)
            return time.perf_counter() - t0, int(out["obs"][-1, 14])
        t_setup, _ = run(0)
        t2, _ = run(2)
        per_step = max((t2 - t_setup) / 2, 1e-6)
        k = int(max(2, min(max_steps, budget_s // per_step)))
        tk, builds = (t2, None) if k == 2 else run(k)
        if builds is None:
            builds = run(0)[1]
        cores = O.num_threads()
    finally:
        if threads:
            O.set_num_threads(os.cpu_count() or 1)
    return {"value": system.n * k / max(tk - t_setup, 1e-9), "unit": "atom-steps/s", "cores": cores,
            "kind": "oracle",
            "sample": f"{system.name} ({system.n} Cr): {k} whole steps of the FP64 oracle (cell-grid "
                      f"Verlet lists, {builds} list builds incl. the one at t=0) in {tk:.1f} s, less "
                      f"the {t_setup:.1f} s set-up at t=0 (first build + forces) timed alone",
            "host": {"cpu_model": cpu_model(), "nproc": os.cpu_count(),
                     "affinity": len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None}}


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


# ------------------------------------------------------------------------------------------
def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed steps (default: the workload's own)")
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="c4", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--energy-every", type=int, default=10)
    ap.add_argument("--tpa", type=int, default=2, choices=[1, 2, 4, 8],
                    help="lanes per atom in the density / force passes")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true", help="headline and kernel pass only")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MiB")
    args = ap.parse_args(argv)

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        return 2
    if args.copy_probe:
        return copy_probe(args.copy_probe)

    import torch

    from paper_1507_07068_amd import inputs as I
    from paper_1507_07068_amd import tune

    idx, wname = WORKLOADS[args.workload]
    cfg = I.config(idx)
    systems = cfg if isinstance(cfg, list) else [cfg]
    precision = args.precision
    steps = args.steps if args.steps is not None else systems[0].steps
    ee = args.energy_every
    n_atoms = sum(s.n for s in systems)
    log(f"[bench] workload {args.workload} ({wname}): {len(systems)} system(s), {n_atoms} Cr, "
        f"{sum(s.n_c for s in systems)} C, precision {precision}, steps {steps}, warmup {args.warmup}")
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        sim = make_sim(systems, precision, args.tpa)
        sim.initial_forces()
        r = timed_run(sim, systems, steps, args.warmup, ee, "headline")
        log(f"[bench] {r['rate']:.4e} atom-steps/s, {r['ms_per_step']:.4f} ms/step, {r['builds']} list "
            f"builds, mean list {r['mean_list']:.2f}")
        kern = kernel_pass(sim, systems, steps, ee, precision)
        free_sim(sim)
    log(f"[bench] kernel pass ({steps} steps, events on every step): force {kern['force']['avg_us']:.1f} us "
        f"({kern['force']['achieved']:.0f} GB/s), density {kern['density']['avg_us']:.1f} us "
        f"({kern['density']['achieved']:.0f} GB/s), list {kern['list'].get('avg_us', 0):.1f} us per rebuild "
        f"over {kern['list']['rebuild_launches']} rebuilds, {kern['list']['avg_us_no_rebuild'] or 0:.1f} us "
        f"otherwise")
    totals = {k: kern[k]["total_ms"] for k in ("force", "density", "list")}
    rl = {k: roofline_of(kern, k, n_atoms, precision) for k in totals}
    dom = max((k for k in totals if rl[k] is not None), key=lambda k: totals[k])
    result = {
        "metric": METRIC,
        "value": r["rate"],
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
                   "list_builds": r["builds"], "mean_list_len": round(r["mean_list"], 3),
                   "lanes_per_atom": args.tpa},
        "roofline": dict(rl[dom], dominant_of={k: round(v, 3) for k, v in totals.items()}),
        "roofline_kernels": {k: v for k, v in rl.items() if v is not None},
        "kernels": kern,
        "cpu_baseline": None,
    }
    if not args.no_variants:
        var, full = {}, {}
        if len(systems) == 1:
            other = "mixed" if precision == "fp64" else "fp64"
            s0 = systems[0]
            rr = full_run([s0], other, args.tpa, warmup=args.warmup, ee=ee)
            rr["force_errors"] = mixed_force_errors(s0, args.tpa)
            var[f"{other}_{args.workload}"] = rr
            log(f"[bench] {other} {args.workload}: {rr['value']:.4e} atom-steps/s, force rel-RMS vs FP64 "
                f"{rr['force_errors']['rel_rms_vs_fp64_gpu_all_atoms']:.2e} (all atoms), vs oracle "
                f"{rr['force_errors']['rel_rms_vs_oracle_sampled']:.2e} (sampled)")
            if steps == s0.steps:   # the headline run is the full run
                full[f"{args.workload}_{precision}"] = {
                    "value": r["rate"], "unit": "atom-steps/s", "steps": steps, "warmup": args.warmup,
                    "ms_per_step": r["ms_per_step"], "precision": precision, "list_builds": r["builds"],
                    "mean_list_len": round(r["mean_list"], 3)}
            else:
                full[f"{args.workload}_{precision}"] = full_run([s0], precision, args.tpa, warmup=args.warmup,
                                                                ee=ee)
            full[f"{args.workload}_{other}"] = {k: rr[k] for k in rr if k != "force_errors"}
        ens = I.config(3)
        tuned = tune.choose(ens, "mixed")
        b = batched_graph_run(ens, ens[0].steps, tuned["tpa"], list_tgt=tuned["list_tgt"])
        var["batched_c3"] = {"value": b["rate"], "unit": "atom-steps/s", "ms_per_step": b["ms_per_step"],
                             "steps": b["steps"], "list_builds": b["builds"], "replicas": len(ens),
                             "cr_atoms": sum(s.n for s in ens), "precision": "mixed",
                             "launch": "hipGraph of 100 whole steps",
                             "autotuned": {"tpa": tuned["tpa"], "list_tgt": tuned["list_tgt"],
                                           "key": tuned["key"], "from_cache": tuned["from_cache"],
                                           "ms_per_step": tuned["ms_per_step"]}}
        full["c3_mixed_graph"] = var["batched_c3"]
        log(f"[bench] batched c3: {b['rate']:.4e} atom-steps/s (tpa {tuned['tpa']}, list_tgt {tuned['list_tgt']})")
        c1 = I.config(1)
        full["c1_fp64"] = full_run([c1], "fp64", args.tpa)
        log(f"[bench] c1 fp64 full: {full['c1_fp64']['value']:.4e} atom-steps/s")
        var["paper_form_c1"] = paper_form_run(c1, args.tpa, two_tier=False)
        var["paper_form_two_tier_c1"] = paper_form_run(c1, args.tpa, two_tier=True)
        var["indentation_protocol"] = protocol_run(args.tpa)
        var["nve_c0"] = nve_drift()
        var["indenter_work_c1"] = indenter_work_drift(c1, args.tpa)
        log(f"[bench] NVE c0 drift (mean of seeds): fp64 "
            f"{var['nve_c0']['drift_ev_per_atom_per_ns']['fp64']['mean']:.3e}, mixed "
            f"{var['nve_c0']['drift_ev_per_atom_per_ns']['mixed']['mean']:.3e} eV/atom/ns; c1 E_tot+W "
            f"{var['indenter_work_c1']['drift_e_tot_plus_w_ev_per_atom_per_ns']:.3e}")
        result["variants"] = var
        result["full_runs"] = full
    if not args.no_cpu_baseline and len(systems) == 1:
        log(f"[bench] CPU baseline: oracle on {systems[0].name} ...")
        result["cpu_baseline"] = cpu_baseline(systems[0])
        log(f"[bench] CPU baseline {result['cpu_baseline']['value']:.4e} atom-steps/s "
            f"({result['cpu_baseline']['cores']} threads)")
        # one thread on the same workload: two whole steps (a step of the 8M-atom film takes a
        # single core several seconds)
        result["cpu_baseline_1thread"] = cpu_baseline(systems[0], threads=1, budget_s=1.0, max_steps=2)
        log(f"[bench] CPU baseline 1 thread ({systems[0].name}) {result['cpu_baseline_1thread']['value']:.4e}")
    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
