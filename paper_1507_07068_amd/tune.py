"""Autotuner for the launch shape of the MD step.

The one shape parameter of the force path is ``tpa``: the number of lanes that share one
atom in the density and force passes (1, 2, 4 or 8; the list is interleaved to match).
Few lanes per atom leave long serial gathers; many lanes spend more on the cross-lane
reduction and idle lanes of short lists.  The best value depends on the list lengths and
on how many atoms a launch has to fill the chip with, so it is measured: each candidate
runs a short stretch of whole steps on the workload itself and the fastest is kept.
Results are cached per workload signature for the life of the process.
"""
from __future__ import annotations

import time

_CACHE: dict = {}


def signature(systems, precision: str) -> tuple:
    return (precision, len(systems), sum(s.n for s in systems), sum(s.n_c for s in systems),
            tuple(sorted({tuple(s.periodic.tolist()) for s in systems})))


def choose_tpa(systems, precision: str, candidates=(1, 2, 4, 8), steps: int = 40,
               warmup: int = 10, stream=None) -> tuple[int, dict]:
    """Return (best tpa, {tpa: seconds per step}) for these systems and precision."""
    import torch

    from . import md

    key = signature(systems, precision)
    if key in _CACHE:
        return _CACHE[key]
    times = {}
    st = stream or torch.cuda.current_stream()
    with torch.cuda.stream(st):
        for t in candidates:
            sim = md.Simulation(systems, precision=precision, xcap=256, tpa=t)
            sim.initial_forces(energy=False)
            sim.md_run(warmup)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sim.md_run(steps)
            torch.cuda.synchronize()
            times[t] = (time.perf_counter() - t0) / steps
            flags = sim.md_check()
            sim.close()
            if flags["overflow"] or flags["xoverflow"] or flags["nonfinite"]:
                times[t] = float("inf")   # a shape whose lists do not fit is not a choice
    best = min(times, key=times.get)
    _CACHE[key] = (best, times)
    return best, times
