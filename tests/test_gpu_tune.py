"""The launch-shape choices the autotuner makes do not change results: runs with different
list-build work-item targets are bitwise equal (lists are ordered by cell row, along x, then
by slot, whatever the cut into work items), for one film and for a batch.  The tuner returns
a shape from its candidates and serves the second call from its cache."""
import numpy as np
import pytest

from paper_1507_07068_amd import inputs as I
from paper_1507_07068_amd import md
from paper_1507_07068_amd import tune

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("nrep", [1, 4])
def test_list_tgt_does_not_change_results(nrep):
    reps = [I.small_film(nx=14 + r, ny=12, nz=6, radius=6.0, gap=0.3, seed=95 + r, noise=0.04)
            for r in range(nrep)]
    states = []
    for tgt in (64, 160, 224):
        print(f"[case] list_tgt={tgt} nrep={nrep}", flush=True)
        sim = md.Simulation(reps, precision="fp64", xcap=160, tpa=2, list_tgt=tgt)
        sim.initial_forces()
        sim.md_run(40)
        st = sim.md_check()
        assert not (st["overflow"] or st["xoverflow"] or st["nonfinite"] or st["sync_timeout"]), st
        states.append(sim.state())
    for other in states[1:]:
        for r in range(nrep):
            for k in ("x", "v", "f", "dF"):
                assert np.array_equal(states[0][r][k], other[r][k]), (r, k)


def test_tuner_picks_a_candidate_and_caches(tmp_path, monkeypatch):
    monkeypatch.setenv("MD_TUNE_CACHE", str(tmp_path / "tune.json"))
    tune._CACHE.clear()
    ens = [I.small_film(nx=10 + r, ny=10, nz=5, radius=5.0, gap=0.5, seed=97 + r) for r in range(3)]
    r1 = tune.choose(ens, "mixed", steps=10, warmup=3)
    assert r1["tpa"] in tune.TPA and r1["list_tgt"] in tune.LIST_TGT and r1["from_cache"] is None
    assert all(np.isfinite(v) for v in r1["ms_per_step"].values())
    r2 = tune.choose(ens, "mixed")
    assert r2["from_cache"] == "memory" and r2["tpa"] == r1["tpa"]
    tune._CACHE.clear()
    r3 = tune.choose(ens, "mixed")
    assert r3["from_cache"] == "file" and r3["list_tgt"] == r1["list_tgt"]


@pytest.mark.parametrize("nrep", [1, 5])
def test_list_work_distribution_does_not_change_results(nrep, monkeypatch):
    """The list build's two ways of handing out work items (one block per item of the table's
    capacity, or resident blocks taking items from a counter) give bitwise equal runs."""
    reps = [I.small_film(nx=12 + r, ny=12, nz=6, radius=6.0, gap=0.3, seed=120 + r, noise=0.04)
            for r in range(nrep)]
    states = []
    for mode in ("0", "1"):
        monkeypatch.setenv("MD_LIST_PERSISTENT", mode)
        print(f"[case] MD_LIST_PERSISTENT={mode} nrep={nrep}", flush=True)
        sim = md.Simulation(reps, precision="fp64", xcap=160, tpa=2)
        sim.initial_forces()
        sim.md_run(40)
        st = sim.md_check()
        assert not (st["overflow"] or st["xoverflow"] or st["nonfinite"] or st["sync_timeout"]), st
        states.append((sim.state(), [sim.neighbor_sets(r) for r in range(nrep)]))
    (sa, la), (sb, lb) = states
    for r in range(nrep):
        assert la[r] == lb[r]
        for k in ("x", "v", "f", "dF"):
            assert np.array_equal(sa[r][k], sb[r][k]), (r, k)
