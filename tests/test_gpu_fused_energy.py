"""md_run's observed steps other than the last take the kinetic energy and the Cr-C sums
inside the force pass, which then also gives the next step's first half kick (and, in FP64,
the drift).  Each velocity sees the same two kicks in the same order as with a kinetic
pass of its own (MD_FUSE_ENERGY=0 at creation).  The runs agree to rounding: the force
pass of an observed step is another build of the kernel (with the drift), whose sums the
compiler may round differently in the last place, and the observables are the same sums
taken in another grouping (per block of the force pass instead of per tile)."""
import numpy as np
import pytest
import torch

from paper_1507_07068_amd import inputs as I
from paper_1507_07068_amd import md

pytestmark = pytest.mark.gpu


def _run(systems, precision, tpa, fuse, monkeypatch, steps, ee):
    monkeypatch.setenv("MD_FUSE_ENERGY", "1" if fuse else "0")
    print(f"[case] fuse={fuse} nrep={len(systems)} precision={precision} tpa={tpa} steps={steps} ee={ee}",
          flush=True)
    sim = md.Simulation(systems, precision=precision, xcap=160, tpa=tpa)
    sim.initial_forces()
    obs = torch.zeros((steps // ee, sim.nrep, md.MD_NOBS), dtype=torch.float64, device="cuda")
    sim.md_run(steps, energy_every=ee, obs=obs)
    st = sim.md_check()
    assert not (st["overflow"] or st["xoverflow"] or st["nonfinite"] or st["sync_timeout"]), st
    out = (sim.state(), obs.cpu().numpy())
    sim.close()
    return out


@pytest.mark.parametrize("precision,tpa,steps,ee", [("fp64", 1, 30, 5), ("fp64", 2, 23, 4), ("mixed", 2, 30, 5)])
def test_fused_energy_steps(precision, tpa, steps, ee, monkeypatch):
    reps = [I.small_film(nx=10 + r, ny=11, nz=5, radius=5.0, gap=0.3, seed=160 + r, noise=0.04)
            for r in range(2)]
    (sa, oa), (sb, ob) = (_run(reps, precision, tpa, f, monkeypatch, steps, ee) for f in (True, False))
    tol = 1e-11 if precision == "fp64" else 1e-5
    for r in range(len(reps)):
        assert np.max(np.abs(sa[r]["x"] - sb[r]["x"])) <= tol
        for k in ("v", "f", "dF"):
            assert np.max(np.abs(sa[r][k] - sb[r][k])) <= tol * np.max(np.abs(sb[r][k])), (r, k)
    # energies, virial, indenter load: each group to tol of its largest magnitude (some
    # components are near-cancelling sums); indenter position and build count exact
    for lo, hi in ((md.MD_E_EMBED, md.MD_W_XX), (md.MD_W_XX, md.MD_F_IND_X), (md.MD_F_IND_X, md.MD_IND_Z)):
        d = np.abs(oa[..., lo:hi] - ob[..., lo:hi])
        assert d.max() <= tol * np.abs(ob[..., lo:hi]).max(), (lo, hi, d.max())
    assert np.array_equal(oa[..., md.MD_IND_Z:md.MD_NBUILDS + 1], ob[..., md.MD_IND_Z:md.MD_NBUILDS + 1])
