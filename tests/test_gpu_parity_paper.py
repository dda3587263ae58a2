"""Parity of the HIP path with the oracle for the paper's own EAM form (Appendix, Eqs. A1-A4:
logarithmic embedding, the M(P) term with P_i = sum_j f^2, power-law density cut at r*,
Pasianot pair), through the C ABI.  Bars as for the synthetic potential: neighbour sets
bit-exact, FP64 forces within 1e-10 (rel-RMS and max/RMS), energies within 1e-12, FP32-mixed
forces within 1e-5."""
import numpy as np
import pytest

import oracle as O
from paper_1507_07068_amd import inputs as I
from paper_1507_07068_amd import md
from tests.test_gpu_parity import (FP64_TOL, MIXED_TOL, _assert_obs, assert_forces, check_lists, force_errors,
                                   min_image_diff)

pytestmark = pytest.mark.gpu

CAP = 256   # about 220 pairs within r* + skin


def paper(s):
    s.potential = "paper"
    return s


def psim(s, precision="fp64", tpa=1, shadow=None):
    print(f"[case] paper {s.name} n={s.n} n_c={s.n_c} precision={precision} tpa={tpa} shadow={shadow}",
          flush=True)
    return md.Simulation(s, precision=precision, cap=CAP, xcap=160, tpa=tpa, shadow=shadow)


def initial(sim):
    sim.md_build_neighbors(force=True)
    sim.md_eam_forces(md.MD_F_DENSITY | md.MD_F_FORCE | md.MD_F_MORSE | md.MD_F_ENERGY, rho=True)
    st = sim.md_check()
    assert st["overflow"] == 0 and st["xoverflow"] == 0 and st["nonfinite"] == 0, st
    return sim.md_energy()[0], sim.state()[0]


def ref_obs(s, ref):
    o = ref["obs"].copy()
    mob = s.fixed == 0
    o[3] = 0.5 * s.mass * np.sum(s.v[mob] ** 2) / I.EV_PER_U_TO_A2_FS2
    return o


@pytest.mark.parametrize("n_cells", [7, 9])
def test_paper_bulk_lists_density_forces(n_cells):
    """A periodic bulk of 7 cells (fewer than three list cells per axis: the per-atom list
    kernel) and of 9 (the staged list kernel)."""
    s = paper(I.bulk(n_cells, seed=40 + n_cells, noise=0.06, name=f"paper_bulk{n_cells}"))
    sim = psim(s)
    obs, st = initial(sim)
    assert check_lists(sim, s, cap=CAP) > 150 * s.n
    ref = O.evaluate(s, O.wrap(s))
    assert np.allclose(st["rho"], ref["rho"], rtol=1e-12, atol=0)
    assert np.allclose(st["dF"], ref["dF"], rtol=1e-10, atol=1e-13)
    assert_forces(st["f"], ref["f"], FP64_TOL)
    _assert_obs(obs, ref_obs(s, ref), 1e-12)


@pytest.mark.parametrize("tpa", [1, 2, 4, 8])
def test_paper_film_with_indenter(tpa):
    s = paper(I.small_film(nx=10, ny=10, nz=5, radius=7.0, gap=-1.0, seed=44, noise=0.05))
    sim = psim(s, tpa=tpa)
    obs, st = initial(sim)
    ref = O.evaluate(s, O.wrap(s))
    assert_forces(st["f"], ref["f"], FP64_TOL)
    _assert_obs(obs, ref_obs(s, ref), 1e-12)
    check_lists(sim, s, cross=True)


@pytest.mark.parametrize("shadow", [True, False])
def test_paper_mixed_precision(shadow):
    for s in (paper(I.bulk(9, seed=45, noise=0.06, name="paper_bulk9")),
              paper(I.small_film(nx=10, ny=10, nz=5, radius=7.0, gap=-1.0, seed=46, noise=0.05))):
        sim = psim(s, precision="mixed", tpa=2, shadow=shadow)
        obs, st = initial(sim)
        ref = O.evaluate(s, O.wrap(s))
        rel, mx = force_errors(st["f"], ref["f"])
        print(f"  paper mixed: force rel-RMS {rel:.3e} max/RMS {mx:.3e}", flush=True)
        assert rel <= MIXED_TOL
        e, er = obs[0] + obs[1], ref["obs"][0] + ref["obs"][1]
        assert abs(e - er) <= 1e-6 * abs(er)


@pytest.mark.parametrize("energy_every", [1, 10])
def test_paper_run_against_oracle_trajectory(energy_every):
    """md_run (kicks of unobserved steps merged, FP64 drift in the force pass) against the
    oracle's trajectory, with the list rebuild schedule."""
    import torch
    s = paper(I.small_film(nx=10, ny=10, nz=5, radius=7.0, gap=0.2, seed=47, noise=0.03, steps=30))
    sim = psim(s, tpa=2)
    sim.initial_forces()
    nobs = 30 // energy_every
    obs = torch.zeros((nobs, 1, md.MD_NOBS), dtype=torch.float64, device="cuda")
    sim.md_run(30, energy_every=energy_every, obs=obs)
    o = obs.cpu().numpy()[:, 0]
    ref = O.md_run(s, 30)
    st = sim.state()[0]
    dx = np.abs(min_image_diff(st["x"], ref["x"], s)).max()
    print(f"  paper md_run: max|dx| {dx:.2e}", flush=True)
    assert dx < 1e-9 and np.abs(st["v"] - ref["v"]).max() < 1e-11
    assert_forces(st["f"], ref["f"], 1e-9)
    steps = np.arange(1, nobs + 1) * energy_every
    ro = ref["obs"][steps]
    assert np.array_equal(o[:, 14], ro[:, 14])
    etot, rtot = o[:, 0:4].sum(1), ro[:, 0:4].sum(1)
    assert np.abs(etot - rtot).max() < 1e-9 * np.abs(rtot).max()
    flags = sim.md_check()
    assert not (flags["overflow"] or flags["xoverflow"] or flags["nonfinite"] or flags["sync_timeout"]), flags


def test_paper_batched_equals_single():
    reps = [paper(I.small_film(nx=9 + r, ny=9, nz=4 + r, radius=6.0, gap=0.3, seed=50 + r, noise=0.03))
            for r in range(3)]
    b = md.Simulation(reps, precision="fp64", cap=CAP, xcap=160, tpa=2)
    b.initial_forces()
    b.run(15)
    stb = b.state()
    for r, s in enumerate(reps):
        a = psim(s, tpa=2)
        a.initial_forces()
        a.run(15)
        sta = a.state()[0]
        for k in ("x", "v", "f", "dF"):
            assert np.array_equal(sta[k], stb[r][k]), (r, k)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_paper_film_216k_sampled(precision):
    """The 216,000-atom film with the paper's form at full size: sampled atoms (a seeded draw,
    the atoms nearest the indenter tip) against the oracle's one-atom-at-a-time evaluation,
    then a stretch of whole steps with clean status words."""
    s = paper(I.config(1))
    rng = np.random.default_rng(17)
    rows = set(rng.choice(s.n, size=24, replace=False).tolist())
    tip = s.xc[np.argmin(s.xc[:, 2])]
    d = s.x - tip
    rows |= set(np.argsort(np.einsum("ij,ij->i", d, d))[:8].tolist())
    rows = np.array(sorted(rows), dtype=np.int64)
    sim = psim(s, precision=precision, tpa=2)
    sim.initial_forces()
    st = sim.state()[0]
    xw = O.wrap(s)
    assert np.array_equal(st["x"], xw)
    f, rho, dF = O.sample_forces_paper(s, rows, x=xw)
    rel, mx = force_errors(st["f"][rows], f)
    print(f"  sampled force rel-RMS {rel:.3e} max/RMS {mx:.3e}", flush=True)
    tol = FP64_TOL if precision == "fp64" else MIXED_TOL
    assert rel <= tol and mx <= tol * (10 if tol > FP64_TOL else 1)
    if precision == "fp64":
        got = sim.neighbor_sets(0, only=rows)
        cnt, idx = O.neighbors(s, s.r_list, x=xw, rows=rows, cap=CAP)
        for t, i in enumerate(rows):
            assert got[i] == idx[t, :cnt[t]].tolist(), i
    sim.md_run(10)
    flags = sim.md_check()
    assert not (flags["overflow"] or flags["xoverflow"] or flags["nonfinite"] or flags["sync_timeout"]), flags
