"""Host logic of bench.py that runs without a GPU: the one-GPU contract and the pairing of
committed HBM counters with the kernel sources and workload they were taken on."""
import bench


def test_more_than_one_gpu_is_refused(capsys):
    assert bench.main(["--gpus", "2"]) == 2
    assert "one GPU" in capsys.readouterr().err


def _traffic_file(path, sha):
    path.write_text(
        "# counters\n"
        "atoms: 1000\nprecision: fp64\nmean_list: 25.0\n"
        "copy_bytes: 1048576\ncopy_fetch_kib: 512\ncopy_write_kib: 1024\n"
        f"force_fetch_kib: 100\nforce_write_kib: 50\nforce_source_sha256: {sha}\n")


def test_traffic_scaled_by_the_copy_probe(tmp_path, monkeypatch):
    f = tmp_path / "traffic.txt"
    _traffic_file(f, "abc")
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    monkeypatch.setattr(bench, "source_hash", lambda kind: "abc")
    got = bench.measured_traffic("force", 1000, "fp64")
    # the copy moves 1 MiB each way: FETCH_SIZE reads half of that, WRITE_SIZE all of it
    assert got == {"bytes": 100 * 1024 * 2.0 + 50 * 1024 * 1.0, "mean_list": 25.0}


def test_traffic_dropped_when_kernel_or_workload_differ(tmp_path, monkeypatch):
    f = tmp_path / "traffic.txt"
    _traffic_file(f, "abc")
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    monkeypatch.setattr(bench, "source_hash", lambda kind: "abd")
    assert bench.measured_traffic("force", 1000, "fp64") is None      # sources changed
    monkeypatch.setattr(bench, "source_hash", lambda kind: "abc")
    assert bench.measured_traffic("force", 999, "fp64") is None       # other workload
    assert bench.measured_traffic("force", 1000, "mixed") is None     # other precision
    assert bench.measured_traffic("density", 1000, "fp64") is None    # no counters for it


def test_source_hash_ignores_comments(tmp_path, monkeypatch):
    a, b = tmp_path / "a.hip", tmp_path / "b.hip"
    a.write_text("int x = 1;   // one\nint y;\n")
    b.write_text("int x = 1;   // another comment\n\nint y;  \n// only a comment\n")
    monkeypatch.setitem(bench.SOURCES, "t", [str(a)])
    ha = bench.source_hash("t")
    monkeypatch.setitem(bench.SOURCES, "t", [str(b)])
    assert bench.source_hash("t") == ha
