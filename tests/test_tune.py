"""The autotuner's keys and its JSON cache (host side; no GPU)."""
import json

from paper_1507_07068_amd import inputs as I
from paper_1507_07068_amd import tune


def test_size_class_and_key_separate_workloads():
    a = [I.small_film(nx=8, ny=8, nz=4)]
    b = [I.small_film(nx=8, ny=8, nz=4) for _ in range(4)]
    c = [I.bulk(6)]
    classes = {tune.size_class(x) for x in (a, b, c)}
    assert len(classes) == 3
    k1 = tune.key(a, "fp64", "gfx950")
    assert k1.startswith("gfx950|") and "|fp64|fs|" in k1
    assert tune.key(a, "mixed", "gfx950") != k1
    p = I.small_film(nx=8, ny=8, nz=4)
    p.potential = "paper"
    assert tune.key([p], "fp64", "gfx950") != k1


def test_cache_file_round_trip(tmp_path, monkeypatch):
    path = tmp_path / "t" / "tune.json"
    monkeypatch.setenv("MD_TUNE_CACHE", str(path))
    assert tune._load() == {}
    tune._store("k1", {"tpa": 2, "list_tgt": 160})
    tune._store("k2", {"tpa": 4, "list_tgt": 224})
    data = json.loads(path.read_text())
    assert data == {"k1": {"tpa": 2, "list_tgt": 160}, "k2": {"tpa": 4, "list_tgt": 224}}
    assert tune._load()["k1"]["list_tgt"] == 160


def test_sources_hash_is_stable():
    assert tune.sources_hash() == tune.sources_hash()
    assert len(tune.sources_hash()) == 12
