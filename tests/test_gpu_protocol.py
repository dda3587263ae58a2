"""The indentation protocol (Section 2.5, Section 4.3) through the C ABI against the oracle run
phase by phase: relax, load at constant speed to a depth, withdraw; the recorded depth and load
(and the trajectory) must match, as whole steps do."""
import numpy as np
import pytest

import oracle as O
from paper_1507_07068_amd import inputs as I
from paper_1507_07068_amd import md
from paper_1507_07068_amd import protocol as P
from tests.test_gpu_parity import min_image_diff

pytestmark = pytest.mark.gpu


def oracle_protocol(s, pr):
    """The oracle trajectory of the three phases, one md_run per phase (each starting from the
    state the previous one ended in): observables after every step."""
    x, v, iz, rows = s.x, s.v, 0.0, []
    for _, n, vel in pr.phases(s):
        t = s.copy()
        t.x, t.v, t.v_ind = x, v, vel
        out = O.md_run(t, n, ind_z=iz)
        rows.append(out["obs"][1:])
        x, v, iz = out["x"], out["v"], out["ind_z"]
    return np.concatenate(rows, axis=0), x, v


@pytest.mark.parametrize("potential", ["fs", "paper"])
def test_protocol_against_oracle(potential):
    s = I.small_film(nx=10, ny=10, nz=5, radius=8.0, gap=0.1, seed=71, noise=0.03)
    s.potential = potential
    pr = P.Protocol(relax_steps=20, speed=0.01, depth=0.25, record_every=5)
    print(f"[case] protocol {potential} n={s.n} phases {pr.phases(s)}", flush=True)
    sim = md.Simulation(s, precision="fp64", cap=256 if potential == "paper" else 64, xcap=160, tpa=2)
    sim.initial_forces()
    rec = P.run(sim, s, pr)
    ref, x_ref, v_ref = oracle_protocol(s, pr)
    k = rec["step"] - 1
    assert np.abs(rec["load"] - ref[k, 12]).max() < 1e-9 * max(1.0, np.abs(ref[:, 12]).max())
    assert np.abs(rec["depth"] - (P.start_depth(s) - ref[k, 13])).max() < 1e-12
    assert np.abs(rec["e_tot"] - ref[k, 0:4].sum(1)).max() < 1e-9 * np.abs(ref[:, 0:4].sum(1)).max()
    st = sim.state()[0]
    assert np.abs(min_image_diff(st["x"], x_ref, s)).max() < 1e-9
    assert np.abs(st["v"] - v_ref).max() < 1e-11
    assert rec["depth"].max() == pytest.approx(0.25, abs=1e-9)
    assert rec["load"].max() > 0.1          # the indenter pressed on the film
    flags = sim.md_check()
    assert not (flags["overflow"] or flags["xoverflow"] or flags["nonfinite"] or flags["sync_timeout"]), flags
