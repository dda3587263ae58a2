"""Autotuner for the launch shape of the MD step.

Two shape parameters change speed but not results:

* ``tpa``: the lanes that share one atom in the density and force passes (1, 2, 4 or 8; the
  list is interleaved to match).  Few lanes per atom leave long serial gathers; many lanes
  spend more on the cross-lane reduction and on idle lanes of short lists.
* ``list_tgt``: the atoms a work item of the list build aims at.  Smaller items spread a
  rebuild over more blocks (good for many small replicas); larger ones stage each cell row for
  more centres.

The best choice depends on the list lengths, on the atoms a launch has to fill the chip with,
and on how often lists are rebuilt, so it is measured.  Each candidate runs a short stretch of
whole steps on the workload itself: ``tpa`` first at the default ``list_tgt``, then
``list_tgt`` at the best ``tpa``.  Results are kept per (GPU architecture, kernel sources,
precision, potential, size class) in memory and in a JSON file: ``$MD_TUNE_CACHE``, else
``~/.cache/paper_1507_07068_amd/tune.json``.
"""
from __future__ import annotations

import hashlib
import json
import math
import os
import time

_CACHE: dict = {}
TPA = (1, 2, 4, 8)
LIST_TGT = (128, 160, 224)
DEFAULT_LIST_TGT = 224


def cache_path() -> str:
    return os.environ.get("MD_TUNE_CACHE") or os.path.join(os.path.expanduser("~"), ".cache",
                                                            "paper_1507_07068_amd", "tune.json")


def sources_hash() -> str:
    """Hash of the kernel sources and the public header (a kernel change invalidates the cache)."""
    here = os.path.dirname(os.path.abspath(__file__))
    files = sorted(os.path.join(here, "csrc", f) for f in os.listdir(os.path.join(here, "csrc")))
    files.append(os.path.join(os.path.dirname(here), "include", "md.h"))
    h = hashlib.sha256()
    for f in files:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:12]


def size_class(systems) -> str:
    """Replicas (log2 bucket), total Cr atoms (log2 bucket), periodic patterns, carbons or not."""
    n = sum(s.n for s in systems)
    per = sorted({"".join("p" if p else "o" for p in s.periodic) for s in systems})
    return (f"r{int(math.log2(len(systems)))}-n{int(math.log2(max(n, 1)))}-{'+'.join(per)}-"
            f"{'c' if any(s.n_c for s in systems) else 'noc'}")


def key(systems, precision: str, arch: str) -> str:
    pot = getattr(systems[0], "potential", "fs")
    return f"{arch}|{sources_hash()}|{precision}|{pot}|{size_class(systems)}"


def _load() -> dict:
    try:
        with open(cache_path()) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def _store(k: str, v: dict):
    try:
        path = cache_path()
        os.makedirs(os.path.dirname(path), exist_ok=True)
        data = _load()
        data[k] = v
        tmp = path + f".{os.getpid()}.tmp"
        with open(tmp, "w") as fh:
            json.dump(data, fh, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass   # a read-only home: the in-memory cache still serves this process


def _time_shape(systems, precision, tpa, list_tgt, steps, warmup) -> float:
    import torch

    from . import md
    sim = md.Simulation(systems, precision=precision, xcap=256, tpa=tpa, list_tgt=list_tgt)
    try:
        sim.initial_forces(energy=False)
        sim.md_run(warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.md_run(steps)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        flags = sim.md_check()
    finally:
        sim.close()
    if flags["overflow"] or flags["xoverflow"] or flags["nonfinite"]:
        return float("inf")   # a shape whose lists do not fit is not a choice
    return dt


def choose(systems, precision: str, steps: int = 40, warmup: int = 10, stream=None,
           use_file: bool = True) -> dict:
    """Tuned shape for these systems: {"tpa", "list_tgt", "ms_per_step": {...}, "key",
    "from_cache"}."""
    import torch
    arch = torch.cuda.get_device_properties(torch.cuda.current_device()).gcnArchName.split(":")[0]
    k = key(systems, precision, arch)
    if k in _CACHE:
        return dict(_CACHE[k], from_cache="memory")
    if use_file:
        hit = _load().get(k)
        if hit:
            _CACHE[k] = hit
            return dict(hit, from_cache="file")
    st = stream or torch.cuda.current_stream()
    times = {}
    with torch.cuda.stream(st):
        for t in TPA:
            times[f"tpa{t}/tgt{DEFAULT_LIST_TGT}"] = _time_shape(systems, precision, t, DEFAULT_LIST_TGT,
                                                                 steps, warmup)
        best_t = min(TPA, key=lambda t: times[f"tpa{t}/tgt{DEFAULT_LIST_TGT}"])
        for g in LIST_TGT:
            if g != DEFAULT_LIST_TGT:
                times[f"tpa{best_t}/tgt{g}"] = _time_shape(systems, precision, best_t, g, steps, warmup)
    best = min(times, key=times.get)
    tpa, tgt = best.split("/")
    res = {"tpa": int(tpa[3:]), "list_tgt": int(tgt[3:]), "key": k,
           "ms_per_step": {s: round(v * 1e3, 4) for s, v in times.items()}}
    _CACHE[k] = res
    if use_file:
        _store(k, res)
    return dict(res, from_cache=None)


def choose_tpa(systems, precision: str, steps: int = 40, warmup: int = 10, stream=None) -> tuple[int, dict]:
    """(best tpa, {tpa: seconds per step}) at the default list_tgt (the first stage of choose)."""
    r = choose(systems, precision, steps, warmup, stream)
    per = {int(s.split("/")[0][3:]): v / 1e3 for s, v in r["ms_per_step"].items()
           if s.endswith(f"/tgt{DEFAULT_LIST_TGT}")}
    return r["tpa"], per
