"""md_workspace_bind_static: the library's static device scratch as the workspace, for callers
that cannot allocate.  Through the C ABI, its results must equal those of the same system on
a caller-owned workspace (md_workspace_bind), bitwise (the kernels are the same), on two
bindings in a row, the second with a smaller system."""
import ctypes as C

import numpy as np
import pytest

from paper_1507_07068_amd import inputs as I
from paper_1507_07068_amd import md

pytestmark = pytest.mark.gpu


def _run(s, precision, static, steps=30):
    import torch
    print(f"[case] {s.name} n={s.n} n_c={s.n_c} {precision} static={static}", flush=True)
    sim = md.Simulation(s, precision=precision, xcap=160, tpa=2, static_workspace=static)
    sim.initial_forces()
    obs = torch.zeros((steps // 10, 1, md.MD_NOBS), dtype=torch.float64, device="cuda")
    sim.md_run(steps, energy_every=10, obs=obs)
    flags = sim.md_check()
    assert not (flags["overflow"] or flags["xoverflow"] or flags["nonfinite"] or flags["sync_timeout"]), flags
    return sim, sim.state()[0], obs.cpu().numpy(), flags


def _same(a, b):
    for k in ("x", "v", "f", "dF", "ids"):
        assert np.array_equal(a[1][k], b[1][k]), k
    assert np.array_equal(a[2], b[2])
    assert a[3] == b[3]


def test_static_workspace_equals_caller_workspace_twice():
    big = I.small_film(nx=10, ny=10, nz=6, radius=8.0, gap=0.2, seed=61, noise=0.03)
    small = I.small_film(nx=6, ny=6, nz=4, radius=6.0, gap=-0.5, seed=62, noise=0.04)
    assert small.n < big.n
    for s, prec in ((big, "fp64"), (small, "mixed")):
        ref = _run(s, prec, static=False)
        got = _run(s, prec, static=True)
        _same(got, ref)
        ref[0].close()
        got[0].close()


def test_static_workspace_takeover_and_size_limit():
    a_sys = I.small_film(nx=8, ny=8, nz=5, radius=6.0, gap=0.3, seed=63, noise=0.03)
    a = md.Simulation(a_sys, static_workspace=True)
    a.initial_forces()
    b = md.Simulation(I.small_film(nx=6, ny=6, nz=4, radius=5.0, gap=0.3, seed=64), static_workspace=True)
    with pytest.raises(md.MDError, match="no workspace bound"):   # b took the scratch over
        a.md_build_neighbors(force=True)
    a.bind()
    a.initial_forces()
    assert a.md_check()["nbuilds"] == 1
    with pytest.raises(md.MDError, match="no workspace bound"):
        b.md_build_neighbors()
    b.close()
    a.close()
    big = I.film(48, 48, 20, 0.0, 0.0, 1)   # 92,160 atoms: ~24 MB of workspace
    descs = (md.ReplicaDesc * 1)(md.make_replica_desc(big))
    p = md.make_params(big, 64, 64, 1)
    h = C.c_void_p()
    lib = md.load_library()
    assert lib.md_system_create(C.cast(descs, C.c_void_p), 1, C.byref(p), C.byref(h)) == md.MD_OK
    assert lib.md_workspace_bytes(h) > md.MD_SCRATCH_BYTES
    assert lib.md_workspace_bind_static(h, None) == md.MD_ERR_ARG
    lib.md_system_destroy(h)
