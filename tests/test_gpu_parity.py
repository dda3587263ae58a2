"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Bars: neighbour lists bit-exact as sorted id sets (and wrapped positions bit-exact);
FP64 forces rel-RMS <= 1e-10 and max |dF_i| <= 1e-10 * RMS|F|; energies <= 1e-12
relative; mixed precision rel-RMS <= 1e-5.  Inputs come from the seeded generator only.
"""
import numpy as np
import pytest

import oracle as O
from paper_1507_07068_amd import inputs as I
from paper_1507_07068_amd import md

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-10
MIXED_TOL = 1e-5


def sim_of(s, precision="fp64", cap=None, xcap=128, tpa=1):
    print(f"[case] {s.name} n={s.n} n_c={s.n_c} precision={precision} tpa={tpa}", flush=True)
    return md.Simulation(s, precision=precision, cap=cap, xcap=xcap, tpa=tpa)


def min_image_diff(a, b, s):
    d = a - b
    per = np.asarray(s.periodic, bool)
    d[:, per] -= s.box_len[per] * np.round(d[:, per] / s.box_len[per])
    return d


def force_errors(f, ref):
    rms = np.sqrt(np.mean(np.sum(ref ** 2, axis=1)))
    diff = np.sqrt(np.sum((f - ref) ** 2, axis=1))
    rel_rms = np.sqrt(np.sum(diff ** 2) / max(np.sum(ref ** 2), 1e-300))
    return rel_rms, diff.max() / max(rms, 1e-300)


def assert_forces(f, ref, tol):
    rel, mx = force_errors(f, ref)
    print(f"  force rel-RMS {rel:.3e}  max/RMS {mx:.3e}", flush=True)
    assert rel <= tol and mx <= tol * (10 if tol > FP64_TOL else 1), (rel, mx)


def check_lists(sim, s, cross=False, ind_z=0.0, rows=None, cap=256):
    """GPU neighbour sets (id space) vs the oracle's brute force on its own wrap."""
    xw = O.wrap(s)
    st = sim.state()[0]
    assert np.array_equal(st["x"], xw), "wrapped positions differ"
    got = sim.neighbor_sets(0, cross=cross)
    if cross:
        cnt, idx = O.cross_neighbors(s, s.r_list_cross, x=xw, ind_z=ind_z, rows=rows, cap=256)
    else:
        cnt, idx = O.neighbors(s, s.r_list, x=xw, rows=rows, cap=cap)
    ref = O.neighbor_sets(cnt, idx)
    ids = range(s.n) if rows is None else rows
    for t, i in enumerate(ids):
        assert got[i] == ref[t], (i, got[i], ref[t])
    return sum(len(r) for r in ref)


# ------------------------------------------------------------------------------------------
# Lists
# ------------------------------------------------------------------------------------------
def test_lists_bulk_c0():
    s = I.config(0)
    sim = sim_of(s)
    sim.md_build_neighbors(force=True)
    st = sim.md_check()
    assert st["overflow"] == 0 and st["nbuilds"] == 1 and st["sync_timeout"] == 0
    assert check_lists(sim, s) > 0


@pytest.mark.parametrize("n,per", [(1, (1, 1, 1)), (2, (1, 1, 0)), (255, (1, 1, 1)),
                                   (257, (1, 1, 0)), (1000, (1, 1, 1)), (2999, (0, 0, 0)),
                                   (4097, (1, 1, 0))])
def test_lists_random_gas_ragged(n, per):
    """Irregular counts (one partial tile, several tiles + a ragged tail), atoms outside the
    box on periodic axes (wrapped at the build), open axes, close pairs."""
    box = max((n / 0.08) ** (1 / 3), 9.0)
    s = I.random_gas(n, box, seed=100 + n, periodic=per)
    sim = sim_of(s, cap=96)
    sim.md_build_neighbors(force=True)
    assert sim.md_check()["overflow"] == 0
    check_lists(sim, s)


@pytest.mark.parametrize("n,density,per", [(4000, 0.08, (1, 1, 1)), (3000, 0.08, (0, 1, 0)),
                                           (15000, 0.3, (1, 1, 1))])
def test_lists_long_crowded_rows(n, density, per):
    """Cell rows longer than one list-build run (more than 42 cells along x) and holding
    more atoms than one block pass: each row is cut into several runs of cells; at the
    highest density the runs per row are capped, so a run's atoms take several passes of
    the block's threads.  The runs at either end of a periodic row stage the wrapped cell."""
    ly = lz = 13.0
    lx = n / (density * ly * lz)
    s = I.random_gas(n, lx, seed=500 + n, periodic=per, lengths=(lx, ly, lz))
    sim = sim_of(s, cap=384)   # up to ~270 neighbours where wrapped margins overlap at 0.3/A^3
    sim.md_build_neighbors(force=True)
    st = sim.md_check()
    assert st["overflow"] == 0 and st["sync_timeout"] == 0
    assert check_lists(sim, s, cap=384) > 0


def test_lists_small_periodic_box_fewer_than_three_cells():
    """A 3x3x3-cell box (8.655 A): fewer than 3 list cells per periodic axis."""
    s = I.bulk(3, seed=4, noise=0.05)
    sim = sim_of(s)
    sim.md_build_neighbors(force=True)
    check_lists(sim, s)


def test_lists_pairs_at_the_list_radius():
    """Pairs placed within a few ulps of the list radius, along awkward directions: the
    predicate must round exactly like the oracle's (no fused multiply-add)."""
    rng = np.random.default_rng(7)
    r = I.EAM["c"] + I.SKIN
    pts = []
    for k in range(400):
        u = rng.normal(size=3)
        u /= np.linalg.norm(u)
        base = rng.uniform(2, 40, size=3)
        dist = r * (1 + rng.integers(-6, 7) * 2.0 ** -52)
        pts += [base, base + dist * u]
    s = I.random_gas(len(pts), 45.0, 0, periodic=(0, 0, 0))
    s.x = np.array(pts)
    sim = sim_of(s)
    sim.md_build_neighbors(force=True)
    check_lists(sim, s)


def test_cross_lists_film():
    s = I.small_film(nx=8, ny=8, nz=5, radius=8.0, gap=-1.5, seed=3, noise=0.05)
    sim = sim_of(s)
    sim.md_build_neighbors(force=True)
    st = sim.md_check()
    assert st["xoverflow"] == 0
    check_lists(sim, s)
    assert check_lists(sim, s, cross=True) > 0
    # the near-atom candidates cover every atom with carbons in range, and stay within two
    # carbon-cell diagonals of a carbon
    xw = O.wrap(s)
    cnt, _ = O.cross_neighbors(s, s.r_list_cross, x=xw, cap=256)
    edge = max(L / max(1, np.floor(L / (s.r_list_cross * (1 + 1e-9)))) for L in s.box_len)
    far, _ = O.cross_neighbors(s, s.r_list_cross + 2 * np.sqrt(3) * edge, x=xw, cap=4096)
    assert (cnt > 0).sum() <= st["nnear"] <= (far > 0).sum()


def test_cross_list_overflow_is_flagged():
    s = I.small_film(nx=8, ny=8, nz=5, radius=8.0, gap=-1.5, seed=3, noise=0.05)
    sim = sim_of(s, xcap=16)
    sim.md_build_neighbors(force=True)
    cnt, _ = O.cross_neighbors(s, s.r_list_cross, x=O.wrap(s), cap=256)
    assert sim.md_check()["xoverflow"] == int(cnt.max()) > 16


def test_list_overflow_is_flagged():
    s = I.config(0)
    sim = sim_of(s, cap=8, xcap=8)
    sim.md_build_neighbors(force=True)
    st = sim.md_check()
    cnt, _ = O.neighbors(s, s.r_list, x=O.wrap(s), cap=64)
    assert st["overflow"] == int(cnt.max())
    assert int(sim.list_counts().max()) == 8
    sim.md_clear_flags()
    assert sim.md_check()["overflow"] == 0


@pytest.mark.parametrize("precision,tpa", [("fp64", 1), ("fp64", 2), ("mixed", 2)])
def test_list_overflow_keeps_the_first_entries(precision, tpa):
    """A list cut at its capacity holds the first cap entries of the whole list, in order."""
    s = I.config(0)
    full = sim_of(s, precision=precision, cap=96, tpa=tpa)
    cut = sim_of(s, precision=precision, cap=8, tpa=tpa)
    for sim in (full, cut):
        sim.md_build_neighbors(force=True)
    assert full.md_check()["overflow"] == 0 and cut.md_check()["overflow"] > 8
    assert np.array_equal(full.id.cpu().numpy(), cut.id.cpu().numpy())
    a, b = full.list_rows(), cut.list_rows()
    assert sum(len(r) > 8 for r in a) > s.n // 2
    for p in range(s.n):
        assert np.array_equal(b[p], a[p][:8]), p


# ------------------------------------------------------------------------------------------
# Forces, densities, energies
# ------------------------------------------------------------------------------------------
def _initial(sim):
    sim.md_build_neighbors(force=True)
    sim.md_eam_forces(md.MD_F_DENSITY | md.MD_F_FORCE | md.MD_F_MORSE | md.MD_F_ENERGY, rho=True)
    st = sim.md_check()
    assert st["overflow"] == 0 and st["xoverflow"] == 0 and st["nonfinite"] == 0, st
    return sim.md_energy()[0], sim.state()[0]


def _assert_obs(obs, ref, tol):
    names = ["e_embed", "e_pair", "e_morse", "e_kin", "w_xx", "w_yy", "w_zz", "w_xy", "w_xz", "w_yz",
             "find_x", "find_y", "find_z"]
    scale_e = max(abs(ref[0]) + abs(ref[1]), 1.0)
    scale_w = max(np.abs(ref[4:10]).max(), 1.0)
    scale_f = max(np.abs(ref[10:13]).max(), 1e-3)
    for k, nm in enumerate(names):
        sc = scale_e if k < 4 else (scale_w if k < 10 else scale_f)
        assert abs(obs[k] - ref[k]) <= tol * sc, (nm, obs[k], ref[k])


def test_density_and_forces_bulk_c0():
    s = I.config(0)
    sim = sim_of(s)
    obs, st = _initial(sim)
    ref = O.evaluate(s, O.wrap(s))
    assert np.allclose(st["rho"], ref["rho"], rtol=1e-13, atol=0)
    assert np.allclose(st["dF"], ref["dF"], rtol=1e-13, atol=0)
    assert_forces(st["f"], ref["f"], FP64_TOL)
    ref_obs = ref["obs"].copy()
    ref_obs[3] = 0.5 * s.mass * np.sum(s.v ** 2) / I.EV_PER_U_TO_A2_FS2
    _assert_obs(obs, ref_obs, 1e-12)


@pytest.mark.parametrize("seed,gap", [(3, -1.5), (9, 0.4)])
def test_forces_film_with_indenter(seed, gap):
    s = I.small_film(nx=8, ny=8, nz=6, radius=8.0, gap=gap, seed=seed, noise=0.05)
    sim = sim_of(s)
    obs, st = _initial(sim)
    ref = O.evaluate(s, O.wrap(s))
    assert_forces(st["f"], ref["f"], FP64_TOL)
    mob = s.fixed == 0
    ref_obs = ref["obs"].copy()
    ref_obs[3] = 0.5 * s.mass * np.sum(s.v[mob] ** 2) / I.EV_PER_U_TO_A2_FS2
    _assert_obs(obs, ref_obs, 1e-12)


def test_morse_standalone_equals_fused():
    s = I.small_film(nx=8, ny=8, nz=6, radius=8.0, gap=-1.0, seed=2, noise=0.05)
    a = sim_of(s)
    a.md_build_neighbors(force=True)
    a.md_eam_forces(md.MD_F_DENSITY | md.MD_F_FORCE | md.MD_F_MORSE | md.MD_F_ENERGY)
    oa = a.md_energy()[0]
    b = sim_of(s)
    b.md_build_neighbors(force=True)
    b.md_eam_forces(md.MD_F_DENSITY | md.MD_F_FORCE | md.MD_F_ENERGY)
    b.md_morse_forces(md.MD_F_ENERGY)
    ob = b.md_energy()[0]
    fa, fb = a.state()[0]["f"], b.state()[0]["f"]
    assert np.allclose(fa, fb, rtol=0, atol=1e-13)
    assert np.allclose(oa[[2, 10, 11, 12]], ob[[2, 10, 11, 12]], rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("shadow", [True, False])
def test_mixed_precision_force_error(shadow):
    """FP32-mixed forces within 1e-5 of the oracle, with separations from the FP32
    cell-local shadow or from rounded FP64 separations."""
    for s in (I.config(0), I.small_film(nx=8, ny=8, nz=6, radius=8.0, gap=-1.0, seed=4, noise=0.05)):
        print(f"[case] {s.name} mixed shadow={shadow}", flush=True)
        sim = md.Simulation(s, precision="mixed", xcap=128, shadow=shadow)
        obs, st = _initial(sim)
        ref = O.evaluate(s, O.wrap(s))
        rel, mx = force_errors(st["f"], ref["f"])
        print(f"  mixed: force rel-RMS {rel:.3e} max/RMS {mx:.3e}", flush=True)
        assert rel <= MIXED_TOL
        assert abs(obs[1] + obs[0] - ref["obs"][0] - ref["obs"][1]) <= 1e-6 * abs(ref["obs"][0])


# ------------------------------------------------------------------------------------------
# Trajectories (Tasks 1-5 over many steps, with list rebuilds)
# ------------------------------------------------------------------------------------------
def _traj(s, nsteps, precision="fp64", fused=True, tpa=1):
    sim = sim_of(s, precision=precision, tpa=tpa)
    sim.initial_forces()
    st = sim.md_check()
    assert st["overflow"] == 0 and st["xoverflow"] == 0, st
    rows = [sim.md_energy()[0]]
    for _ in range(nsteps):
        (sim.step if fused else sim.step_unfused)(energy=True)
        rows.append(sim.md_energy()[0])
    return sim, np.array(rows)


def test_trajectory_c0_100_steps():
    s = I.config(0)
    sim, obs = _traj(s, 100)
    ref = O.md_run(s, 100)
    st = sim.state()[0]
    dx = np.abs(min_image_diff(st["x"], ref["x"], s)).max()
    dv = np.abs(st["v"] - ref["v"]).max()
    print(f"  c0 100 steps: max|dx| {dx:.2e}  max|dv| {dv:.2e}", flush=True)
    assert dx < 1e-9 and dv < 1e-11
    assert_forces(st["f"], ref["f"], 1e-9)
    ro = ref["obs"]
    assert np.array_equal(obs[:, 14], ro[:, 14]), "list rebuild schedule differs"
    etot, rtot = obs[:, 0:4].sum(1), ro[:, 0:4].sum(1)
    assert np.abs(etot - rtot).max() < 1e-9 * np.abs(rtot).max()
    assert sim.md_check()["overflow"] == 0


def test_trajectory_film_with_moving_indenter():
    s = I.small_film(nx=8, ny=8, nz=6, radius=8.0, gap=0.2, seed=12, noise=0.03, steps=60)
    sim, obs = _traj(s, 60)
    ref = O.md_run(s, 60)
    st = sim.state()[0]
    dx = np.abs(min_image_diff(st["x"], ref["x"], s)).max()
    print(f"  film 60 steps: max|dx| {dx:.2e}", flush=True)
    assert dx < 1e-9
    assert np.array_equal(obs[:, 14], ref["obs"][:, 14])
    assert abs(obs[-1, 13] - ref["ind_z"]) < 1e-15
    assert np.abs(obs[:, 10:13] - ref["obs"][:, 10:13]).max() < 1e-9


def test_unfused_step_matches_fused():
    s = I.small_film(nx=8, ny=8, nz=6, radius=8.0, gap=-0.5, seed=5, noise=0.03)
    a, oa = _traj(s, 20, fused=True)
    b, ob = _traj(s, 20, fused=False)
    xa, xb = a.state()[0]["x"], b.state()[0]["x"]
    assert np.abs(xa - xb).max() < 1e-12
    assert np.abs(oa[:, :4] - ob[:, :4]).max() < 1e-9


def test_fixed_atoms_do_not_move():
    s = I.small_film(nx=8, ny=8, nz=5, radius=6.0, gap=0.5, seed=1)
    sim, _ = _traj(s, 30)
    st = sim.state()[0]
    fx = s.fixed.astype(bool)
    assert np.array_equal(st["x"][fx], O.wrap(s)[fx])
    assert np.all(st["v"][fx] == 0)


def test_mixed_trajectory_stays_close():
    s = I.config(0)
    sim, obs = _traj(s, 50, precision="mixed")
    ref = O.md_run(s, 50)
    st = sim.state()[0]
    rel, _ = force_errors(st["f"], ref["f"])
    print(f"  mixed 50 steps: force rel-RMS vs FP64 oracle {rel:.2e}", flush=True)
    assert rel < 1e-3          # chaotic divergence over 50 fs, bounded
    e, er = obs[:, :4].sum(1), ref["obs"][:, :4].sum(1)
    assert np.abs(e - er).max() < 1e-3 * np.abs(er).max()


# ------------------------------------------------------------------------------------------
# The whole-step run (md_run): the two half kicks of consecutive unobserved steps given at
# once and, in FP64, the next step's drift done by the force pass
# ------------------------------------------------------------------------------------------
def _run(s, nsteps, energy_every, precision="fp64", tpa=1):
    import torch
    sim = sim_of(s, precision=precision, tpa=tpa)
    sim.initial_forces()
    st = sim.md_check()
    assert st["overflow"] == 0 and st["xoverflow"] == 0, st
    nobs = nsteps // energy_every if energy_every else 0
    obs = torch.zeros((max(nobs, 1), 1, md.MD_NOBS), dtype=torch.float64, device="cuda")
    print(f"  md_run {nsteps} steps, energies every {energy_every}", flush=True)
    sim.md_run(nsteps, energy_every=energy_every, obs=obs if nobs else None)
    return sim, obs.cpu().numpy()[:nobs, 0]


def _check_run_fp64(sim, obs, s, nsteps, energy_every):
    ref = O.md_run(s, nsteps)
    st = sim.state()[0]
    dx = np.abs(min_image_diff(st["x"], ref["x"], s)).max()
    dv = np.abs(st["v"] - ref["v"]).max()
    print(f"  max|dx| {dx:.2e}  max|dv| {dv:.2e}", flush=True)
    assert dx < 1e-9 and dv < 1e-11
    assert_forces(st["f"], ref["f"], 1e-9)
    flags = sim.md_check()
    assert not (flags["overflow"] or flags["xoverflow"] or flags["nonfinite"]), flags
    ro = ref["obs"][[energy_every * (k + 1) for k in range(len(obs))]]
    assert np.array_equal(obs[:, 14], ro[:, 14]), "list rebuild schedule differs"
    if len(obs):
        etot, rtot = obs[:, 0:4].sum(1), ro[:, 0:4].sum(1)
        assert np.abs(etot - rtot).max() < 1e-9 * np.abs(rtot).max()
        assert np.abs(obs[:, 10:13] - ro[:, 10:13]).max() < 1e-9
        assert abs(obs[-1, 13] - ro[-1, 13]) < 1e-15


@pytest.mark.parametrize("nsteps,energy_every,tpa", [(60, 10, 1), (37, 0, 1), (25, 7, 1), (60, 10, 2),
                                                     (30, 10, 4)])
def test_run_film_with_moving_indenter(nsteps, energy_every, tpa):
    """md_run against the oracle's trajectory: energies every 10 steps, never, and every 7
    steps (the last step then unobserved, its velocities completed by the final half kick);
    with 1, 2 and 4 lanes per atom (the force pass's displacement maxima per lane group)."""
    s = I.small_film(nx=8, ny=8, nz=6, radius=8.0, gap=0.2, seed=12, noise=0.03, steps=nsteps)
    sim, obs = _run(s, nsteps, energy_every, tpa=tpa)
    _check_run_fp64(sim, obs, s, nsteps, energy_every)


def test_run_mixed_film_stays_close():
    s = I.small_film(nx=8, ny=8, nz=6, radius=8.0, gap=0.2, seed=12, noise=0.03, steps=30)
    sim, obs = _run(s, 30, 10, precision="mixed")
    ref = O.md_run(s, 30)
    st = sim.state()[0]
    rel, _ = force_errors(st["f"], ref["f"])
    print(f"  mixed md_run 30 steps: force rel-RMS vs FP64 oracle {rel:.2e}", flush=True)
    assert rel < 1e-3
    ro = ref["obs"][[10, 20, 30]]
    e, er = obs[:, :4].sum(1), ro[:, :4].sum(1)
    assert np.abs(e - er).max() < 1e-3 * np.abs(er).max()


def test_cross_lists_and_run_film_fewer_than_three_cells():
    """An indenter over a 4 x 4-cell film (11.54 A periodic faces): fewer than 3 Cr list
    cells per periodic axis, so the lists come from the per-atom kernel and the Cr-C lists
    from their own launch."""
    s = I.small_film(nx=4, ny=4, nz=4, radius=5.0, gap=-1.5, seed=5, noise=0.05, steps=30)
    sim = sim_of(s)
    sim.md_build_neighbors(force=True)
    st = sim.md_check()
    assert st["overflow"] == 0 and st["xoverflow"] == 0
    check_lists(sim, s)
    assert check_lists(sim, s, cross=True) > 0
    sim, obs = _run(s, 30, 10)
    _check_run_fp64(sim, obs, s, 30, 10)


# ------------------------------------------------------------------------------------------
# Edge cases
# ------------------------------------------------------------------------------------------
def test_dimer_and_single_atom():
    s = I.random_gas(2, 20.0, 0, periodic=(0, 0, 0))
    s.x = np.array([[5.0, 5.0, 5.0], [7.1, 6.0, 5.4]])
    s.v = np.array([[0.001, 0.0, 0.0], [-0.001, 0.0, 0.0]])
    sim, obs = _traj(s, 30)
    ref = O.md_run(s, 30)
    assert np.abs(sim.state()[0]["x"] - ref["x"]).max() < 1e-12
    s1 = I.random_gas(1, 20.0, 0, periodic=(1, 1, 1))
    s1.v = np.array([[0.01, -0.02, 0.005]])
    sim1, _ = _traj(s1, 10)
    ref1 = O.md_run(s1, 10)
    assert np.abs(min_image_diff(sim1.state()[0]["x"], ref1["x"], s1)).max() < 1e-13


def test_empty_system():
    s = I.random_gas(0, 20.0, 0)
    sim, obs = _traj(s, 3)
    assert np.all(obs[:, :13] == 0)
    assert sim.md_check()["nonfinite"] == 0


@pytest.mark.parametrize("tpa", [2, 4, 8])
def test_lanes_per_atom(tpa):
    """T lanes per atom (list interleaved by T): same lists, forces within the FP64 bar,
    same trajectory as the oracle."""
    s = I.small_film(nx=8, ny=8, nz=6, radius=8.0, gap=-0.8, seed=21, noise=0.05)
    sim = sim_of(s, tpa=tpa)
    obs, st = _initial(sim)
    check_lists(sim, s)
    ref = O.evaluate(s, O.wrap(s))
    assert_forces(st["f"], ref["f"], FP64_TOL)
    for mixed in (False, True):
        m = sim_of(s, precision="mixed" if mixed else "fp64", tpa=tpa)
        _, stm = _initial(m)
        rel, _ = force_errors(stm["f"], ref["f"])
        assert rel <= (MIXED_TOL if mixed else FP64_TOL)
    sim2, obs2 = _traj(s, 40, tpa=tpa)
    r2 = O.md_run(s, 40)
    assert np.abs(min_image_diff(sim2.state()[0]["x"], r2["x"], s)).max() < 1e-9
    assert np.array_equal(obs2[:, 14], r2["obs"][:, 14])


def test_lists_atoms_far_outside_the_given_open_extent():
    """Open-axis cell grids follow the atoms: a film whose upper part has moved far above
    the extent given at set-up (and atoms below it) still gets exact lists."""
    s = I.small_film(nx=8, ny=8, nz=6, radius=6.0, gap=0.5, seed=31, noise=0.05)
    x = s.x.copy()
    top = x[:, 2] > 8.0
    x[top, 2] += 150.0 + 0.01 * np.arange(top.sum())
    x[:5, 2] -= 40.0
    s.x = x
    sim = sim_of(s)
    sim.md_build_neighbors(force=True)
    st = sim.md_check()
    assert st["overflow"] == 0 and st["xoverflow"] == 0
    check_lists(sim, s)
    check_lists(sim, s, cross=True)


def test_lists_pairs_at_the_list_radius_across_periodic_faces():
    """Pairs within a few ulps of the list radius whose separation crosses a periodic face
    (the image is taken from the cell stencil on the GPU, from the minimum image in the
    oracle: both must round identically)."""
    rng = np.random.default_rng(17)
    r = I.EAM["c"] + I.SKIN
    L = 30.0
    pts = []
    for k in range(300):
        u = rng.normal(size=3)
        u /= np.linalg.norm(u)
        base = rng.uniform(0.0, L, size=3)
        ax = k % 3
        base[ax] = rng.uniform(0.0, 1.0)          # near the lower face of axis ax
        if u[ax] > 0:
            u[ax] = -u[ax]                          # partner reaches across that face
        dist = r * (1 + rng.integers(-6, 7) * 2.0 ** -52)
        pts += [base, base + dist * u]
    s = I.random_gas(len(pts), L, 0, periodic=(1, 1, 1))
    s.x = np.array(pts)
    sim = sim_of(s, cap=96)
    sim.md_build_neighbors(force=True)
    assert sim.md_check()["overflow"] == 0
    check_lists(sim, s)


# ------------------------------------------------------------------------------------------
# Batched replicas and graph replay
# ------------------------------------------------------------------------------------------
def _small_replicas():
    """Ensemble members of the batched workload, cut to sizes a test can afford."""
    out = []
    for r in (0, 5, 9):
        d = I.replica_draws(r)
        rng = d.pop("rng")
        s = I.film(10 + (d["nx"] - 10) // 4, 10 + (d["ny"] - 10) // 4, 8 + (d["nz"] - 8) // 4,
                   d["radius"], d["gap"], 3000 + r, steps=30, name=f"replica{r}", rng=rng)
        out.append(s)
    return out


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batched_replicas_equal_single_bitwise(precision):
    reps = _small_replicas()
    print(f"[case] batched {len(reps)} replicas sizes {[s.n for s in reps]} {precision}", flush=True)
    b = md.Simulation(reps, precision=precision, cap=64, xcap=160)
    b.initial_forces()
    b.run(30)
    stb = b.state()
    assert b.md_check()["overflow"] == 0
    for r, s in enumerate(reps):
        a = sim_of(s, precision=precision)
        a.initial_forces()
        a.run(30)
        sta = a.state()[0]
        for k in ("x", "v", "f", "dF"):
            assert np.array_equal(sta[k], stb[r][k]), (r, k)


def test_batched_observables_per_replica():
    reps = _small_replicas()
    b = md.Simulation(reps, cap=64, xcap=160)
    b.initial_forces()
    ob = b.md_energy()
    for r, s in enumerate(reps):
        ref = O.evaluate(s, O.wrap(s))
        mob = s.fixed == 0
        ref_obs = ref["obs"].copy()
        ref_obs[3] = 0.5 * s.mass * np.sum(s.v[mob] ** 2) / I.EV_PER_U_TO_A2_FS2
        _assert_obs(ob[r], ref_obs, 1e-12)


def test_graph_replay_equals_eager():
    import torch
    s = I.small_film(nx=10, ny=10, nz=6, radius=8.0, gap=0.2, seed=41, noise=0.03)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        a = sim_of(s)
        a.initial_forces()
        obs_a = torch.zeros((3, 1, md.MD_NOBS), dtype=torch.float64, device="cuda")
        for k in range(3):
            a.md_run(10, energy_every=10, obs=obs_a[k:k + 1])
        b = sim_of(s)
        b.initial_forces()
        obs_b = torch.zeros((1, 1, md.MD_NOBS), dtype=torch.float64, device="cuda")
        g = b.md_graph_create(10, energy_every=10, obs=obs_b)
        rows = []
        for k in range(3):               # eager work and syncs between the replays
            b.md_graph_launch(g)
            torch.cuda.synchronize()
            rows.append(obs_b.cpu().numpy().copy())
            _ = b.md_check()
        torch.cuda.synchronize()
    sa, sb = a.state()[0], b.state()[0]
    for k in ("x", "v", "f"):
        assert np.array_equal(sa[k], sb[k]), k
    oa = obs_a.cpu().numpy()
    for k in range(3):
        assert np.array_equal(oa[k], rows[k][0]), k
    assert a.md_check()["nbuilds"] == b.md_check()["nbuilds"]


# ------------------------------------------------------------------------------------------
# The indenter term of the rebuild rule (Section 2.6 with Task 2)
# ------------------------------------------------------------------------------------------
@pytest.mark.parametrize("nrep,energy_every", [(1, 1), (1, 10), (6, 1), (6, 10)])
def test_rebuild_schedule_indenter_only(nrep, energy_every):
    """Every Cr atom fixed and the indenter moving 0.004 A per step: only the indenter term of
    the half-skin rule fires (every 38 steps).  Rebuild schedule and forces match the oracle
    for one replica (the skin decision taken inside the binning launch) and for six (the
    decision launch, one wavefront per replica), with every step observed or every tenth
    (then the force pass drifts the atoms of the unobserved steps)."""
    import torch

    import tests.test_oracle as T
    nsteps = 120
    reps = [T.indenter_only_film(seed=19 + r, nx=6 + r % 3) for r in range(nrep)]
    print(f"[case] indenter-only nrep={nrep} energy_every={energy_every} sizes {[s.n for s in reps]}",
          flush=True)
    sim = md.Simulation(reps, precision="fp64", xcap=160)
    sim.initial_forces()
    nobs = nsteps // energy_every
    obs = torch.zeros((nobs, nrep, md.MD_NOBS), dtype=torch.float64, device="cuda")
    sim.md_run(nsteps, energy_every=energy_every, obs=obs)
    flags = sim.md_check()
    assert not (flags["overflow"] or flags["xoverflow"] or flags["nonfinite"] or flags["sync_timeout"]), flags
    o = obs.cpu().numpy()
    want = T.expected_indenter_builds(nsteps, reps[0].v_ind, reps[0].dt, 0.5 * reps[0].skin)
    steps = np.arange(1, nobs + 1) * energy_every
    states = sim.state()
    for r, s in enumerate(reps):
        ref = O.md_run(s, nsteps)
        assert np.array_equal(ref["obs"][:, 14], want)
        assert np.array_equal(o[:, r, 14], want[steps]), (r, o[:, r, 14], want[steps])
        assert np.all(o[:, r, 13] == ref["obs"][steps, 13])
        assert_forces(states[r]["f"], ref["f"], FP64_TOL)
        assert np.abs(o[:, r, 10:13] - ref["obs"][steps, 10:13]).max() < 1e-10
    assert flags["nbuilds"] == nrep * int(want[-1])


def test_scan_give_up_is_flagged_and_recovers(monkeypatch):
    """A list build whose cell-count scan gives up its bounded wait (forced from the host:
    MD_SCAN_SPIN_LIMIT=-1 makes every chunk after the first give up at once) is flagged, does
    nothing further, and no build runs until md_clear_flags; then a forced build gives the
    oracle's lists and forces."""
    s = I.small_film(nx=30, ny=30, nz=8, radius=8.0, gap=0.5, seed=51, noise=0.03)
    monkeypatch.setenv("MD_SCAN_SPIN_LIMIT", "-1")
    sim = sim_of(s)
    sim.md_build_neighbors(force=True)
    st = sim.md_check()
    assert st["sync_timeout"] == 1 and st["nbuilds"] == 1, st
    sim.md_build_neighbors(force=True)            # refused while the give-up stands
    monkeypatch.delenv("MD_SCAN_SPIN_LIMIT")
    sim.md_build_neighbors(force=True)
    st = sim.md_check()
    assert st["sync_timeout"] == 1 and st["nbuilds"] == 1, st
    sim.md_clear_flags()
    assert sim.md_check()["sync_timeout"] == 0
    sim.md_build_neighbors(force=True)
    sim.md_eam_forces(md.MD_F_DENSITY | md.MD_F_FORCE | md.MD_F_MORSE)
    st = sim.md_check()
    assert st["sync_timeout"] == 0 and st["nbuilds"] == 2 and st["overflow"] == 0, st
    check_lists(sim, s)
    check_lists(sim, s, cross=True)
    ref = O.evaluate(s, O.wrap(s))
    assert_forces(sim.state()[0]["f"], ref["f"], FP64_TOL)
