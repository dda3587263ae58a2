"""Section 2.6's two-tier lists on the GPU, through the C ABI: an outer list reaching 1.7 r*
(r* = 8.262 A, the paper's cutoff; skin 0.7 r*) rebuilt by the half-skin rule, and an inner
list of the pairs closer than r*, refilled from the outer list before every density pass, over
which the passes run (with the paper's EAM form, as in the paper).

Bars: outer and inner sets bit-exact against the oracle's brute force (the inner set at the
current positions, also after steps without a rebuild); FP64 forces within 1e-10, FP32-mixed
within 1e-5 of the oracle; trajectories as for the one-list path."""
import numpy as np
import pytest

import oracle as O
from paper_1507_07068_amd import inputs as I
from paper_1507_07068_amd import md
from tests.test_gpu_parity import FP64_TOL, MIXED_TOL, assert_forces, force_errors, min_image_diff

pytestmark = pytest.mark.gpu

CAP = 1024    # outer list: about 910 pairs within 1.7 r* in the bulk
ICAP = 256    # inner list: about 180 pairs within r*


def tsim(s, precision="fp64", tpa=1, icap=ICAP, cap=CAP, xcap=160):
    print(f"[case] two-tier {s.name} n={s.n} n_c={s.n_c} precision={precision} tpa={tpa} icap={icap}",
          flush=True)
    return md.Simulation(s, precision=precision, cap=cap, xcap=xcap, tpa=tpa, icap=icap)


def film(seed, gap=-1.0, nx=15, nz=6, steps=50):
    return I.two_tier(I.small_film(nx=nx, ny=nx, nz=nz, radius=7.0, gap=gap, seed=seed, noise=0.05,
                                   steps=steps))


def sets_equal(got, cnt, idx, rows):
    ref = O.neighbor_sets(cnt, idx)
    for t, i in enumerate(rows):
        assert got[i] == ref[t], (i, len(got[i]), len(ref[t]))
    return sum(len(r) for r in ref)


def check_inner(sim, s, rows=None):
    """Inner sets (all atoms, or the ids `rows`) against brute force at r* on the GPU's
    current positions."""
    st = sim.state()[0]
    sel = None if rows is None else np.asarray(rows, dtype=np.int64)
    cnt, idx = O.neighbors(s, s.cutoff, x=st["x"], rows=sel, cap=ICAP)
    got = sim.neighbor_sets(0, inner=True, only=sel)
    return sets_equal(got, cnt, idx, range(s.n) if sel is None else sel.tolist())


def flags_clean(sim):
    st = sim.md_check()
    assert not (st["overflow"] or st["xoverflow"] or st["ioverflow"] or st["nonfinite"] or st["sync_timeout"]), st
    return st


@pytest.mark.parametrize("nc", [10, 15])
def test_two_tier_bulk_sets_and_forces(nc):
    """Periodic bulk of 10 cells (fewer than three list cells per axis: the per-atom list
    kernel) and of 15 (the staged list kernel)."""
    s = I.two_tier(I.bulk(nc, seed=60 + nc, noise=0.06, name=f"two_tier_bulk{nc}"))
    sim = tsim(s, tpa=2)
    sim.md_build_neighbors(force=True)
    sim.md_eam_forces(md.MD_F_DENSITY | md.MD_F_FORCE | md.MD_F_ENERGY, rho=True)
    flags_clean(sim)
    xw = O.wrap(s)
    cnt, idx = O.neighbors(s, s.r_list, x=xw, cap=CAP)
    assert sets_equal(sim.neighbor_sets(0), cnt, idx, range(s.n)) > 800 * s.n
    assert check_inner(sim, s) > 170 * s.n
    ref = O.evaluate(s, xw)
    st = sim.state()[0]
    assert np.allclose(st["rho"], ref["rho"], rtol=1e-12, atol=0)
    assert_forces(st["f"], ref["f"], FP64_TOL)


def test_two_tier_short_periodic_box():
    """A periodic box under 2 (r* + 1) + 1 (6 cells of 3.2 A; an outer skin of 0.9 A keeps it
    over twice the list radius): the inner refill's FP32 screen is off there and every outer
    entry gets the exact test.  Inner sets against brute force at the start and after whole
    steps; forces against the oracle."""
    s = I.two_tier(I.bulk(6, a=3.2, seed=66, noise=0.06, name="two_tier_short_box"))
    s.skin = 0.9
    assert 2 * s.r_list < s.box_len.min() and s.box_len.max() <= 2 * (s.cutoff + 1.0) + 1.0
    sim = tsim(s, tpa=2)
    sim.md_build_neighbors(force=True)
    sim.md_eam_forces(md.MD_F_DENSITY | md.MD_F_FORCE | md.MD_F_ENERGY, rho=True)
    flags_clean(sim)
    assert check_inner(sim, s) > 100 * s.n
    ref = O.evaluate(s, O.wrap(s))
    st = sim.state()[0]
    assert np.allclose(st["rho"], ref["rho"], rtol=1e-12, atol=0)
    assert_forces(st["f"], ref["f"], FP64_TOL)
    sim.md_run(10)
    flags_clean(sim)
    assert check_inner(sim, s) > 100 * s.n


@pytest.mark.parametrize("precision,tpa", [("fp64", 1), ("fp64", 4), ("mixed", 2), ("mixed", 8)])
def test_two_tier_film_with_indenter(precision, tpa):
    s = film(seed=62)
    sim = tsim(s, precision=precision, tpa=tpa)
    sim.md_build_neighbors(force=True)
    sim.md_eam_forces(md.MD_F_DENSITY | md.MD_F_FORCE | md.MD_F_MORSE | md.MD_F_ENERGY, rho=True)
    flags_clean(sim)
    check_inner(sim, s)
    xw = O.wrap(s)
    ref = O.evaluate(s, xw)
    st = sim.state()[0]
    if precision == "fp64":
        assert_forces(st["f"], ref["f"], FP64_TOL)
    else:
        rel, mx = force_errors(st["f"], ref["f"])
        print(f"  two-tier mixed: force rel-RMS {rel:.3e} max/RMS {mx:.3e}", flush=True)
        assert rel <= MIXED_TOL


def test_two_tier_equals_one_list():
    """The passes over the inner list give the forces of the passes over one list reaching r*
    + 0.3 A (only the order of the sums differs)."""
    s = film(seed=63)
    a = tsim(s, tpa=2)
    a.initial_forces()
    one = s.copy()
    one.skin = I.SKIN
    b = md.Simulation(one, precision="fp64", cap=ICAP, xcap=160, tpa=2)
    b.initial_forces()
    fa, fb = a.state()[0]["f"], b.state()[0]["f"]
    assert_forces(fa, fb, 1e-12)
    ea, eb = a.md_energy()[0], b.md_energy()[0]
    assert abs((ea[0] + ea[1]) - (eb[0] + eb[1])) <= 1e-12 * abs(eb[0] + eb[1])


@pytest.mark.parametrize("energy_every", [1, 10])
def test_two_tier_run_against_oracle(energy_every):
    """md_run (inner list refilled every step, outer list by the half-skin rule with the large
    skin: no rebuild in 40 steps) against the oracle's trajectory; the inner sets at the end
    against brute force at the positions reached."""
    import torch
    s = film(seed=64, gap=0.2, steps=40)
    s.v_ind = -0.01
    sim = tsim(s, tpa=2)
    sim.initial_forces()
    nobs = 40 // energy_every
    obs = torch.zeros((nobs, 1, md.MD_NOBS), dtype=torch.float64, device="cuda")
    sim.md_run(40, energy_every=energy_every, obs=obs)
    o = obs.cpu().numpy()[:, 0]
    ref = O.md_run(s, 40)
    st = sim.state()[0]
    dx = np.abs(min_image_diff(st["x"], ref["x"], s)).max()
    print(f"  two-tier md_run: max|dx| {dx:.2e}", flush=True)
    assert dx < 1e-9 and np.abs(st["v"] - ref["v"]).max() < 1e-11
    assert_forces(st["f"], ref["f"], 1e-9)
    steps = np.arange(1, nobs + 1) * energy_every
    ro = ref["obs"][steps]
    assert np.array_equal(o[:, 14], ro[:, 14])
    etot, rtot = o[:, 0:4].sum(1), ro[:, 0:4].sum(1)
    assert np.abs(etot - rtot).max() < 1e-9 * np.abs(rtot).max()
    flags_clean(sim)
    assert check_inner(sim, s) > 0


def test_inner_overflow_is_flagged():
    s = film(seed=65)
    sim = tsim(s, tpa=2, icap=64)
    sim.md_build_neighbors(force=True)
    sim.md_eam_forces(md.MD_F_DENSITY | md.MD_F_FORCE)
    st = sim.md_check()
    assert st["ioverflow"] > 64 and st["overflow"] == 0 and st["nonfinite"] == 0, st
    sim.md_clear_flags()
    assert sim.md_check()["ioverflow"] == 0


def test_two_tier_needs_the_inner_list_arrays():
    s = film(seed=66)
    sim = tsim(s)
    sim.iidx = None
    sim.icnt = None
    sim.icap = 0   # the binding then hands the library no inner-list arrays
    sim._lists_c = None
    with pytest.raises(md.MDError):
        sim.md_eam_forces(md.MD_F_DENSITY)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_two_tier_film_216k_sampled(precision):
    """The 216,000-atom film with the paper's form and two-tier lists at full size: sampled
    outer and inner sets against brute force, sampled forces against the oracle's
    one-atom-at-a-time evaluation, then whole steps with clean status words."""
    s = I.two_tier(I.config(1))
    rng = np.random.default_rng(19)
    rows = set(rng.choice(s.n, size=20, replace=False).tolist())
    tip = s.xc[np.argmin(s.xc[:, 2])]
    d = s.x - tip
    rows |= set(np.argsort(np.einsum("ij,ij->i", d, d))[:6].tolist())
    rows = np.array(sorted(rows), dtype=np.int64)
    sim = tsim(s, precision=precision, tpa=2, cap=1152, xcap=320)   # about 215 carbons within r_M + skin
    sim.initial_forces()
    flags_clean(sim)
    st = sim.state()[0]
    xw = O.wrap(s)
    assert np.array_equal(st["x"], xw)
    cnt, idx = O.neighbors(s, s.r_list, x=xw, rows=rows, cap=1152)
    sets_equal(sim.neighbor_sets(0, only=rows), cnt, idx, rows)
    check_inner(sim, s, rows=rows)
    f, rho, dF = O.sample_forces_paper(s, rows, x=xw)
    rel, mx = force_errors(st["f"][rows], f)
    print(f"  sampled force rel-RMS {rel:.3e} max/RMS {mx:.3e}", flush=True)
    tol = FP64_TOL if precision == "fp64" else MIXED_TOL
    assert rel <= tol and mx <= tol * (10 if tol > FP64_TOL else 1)
    sim.md_run(10)
    flags_clean(sim)
