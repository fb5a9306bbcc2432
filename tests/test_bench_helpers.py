"""bench.py helpers that run without a GPU: the HBM-traffic lookup keyed by
the tail kernel's source hash and launch shape."""
import importlib.util
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_source_hash_is_stable(bench):
    h = bench.tail_source_hash()
    assert len(h) == 64 and h == bench.tail_source_hash()


def test_traffic_lookup(bench, tmp_path, monkeypatch):
    h = bench.tail_source_hash()
    prof = tmp_path / "profiles"
    prof.mkdir()
    f = prof / "k_tail_wl_traffic.txt"
    f.write_text("# comment: ignored\nsource_sha256: %s\ntraffic_bytes_per_launch[512,2]: 123456\n" % h)
    # the summary is read from ROOT/profiles; keep the hash of the real sources
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "tail_source_hash", lambda: h)
    assert bench.measured_traffic("wl", 512, 2) == 123456.0
    assert bench.measured_traffic("wl", 1024, 2) is None        # shape not recorded
    assert bench.measured_traffic("other", 512, 2) is None      # no summary
    f.write_text("source_sha256: 0000\ntraffic_bytes_per_launch[512,2]: 123456\n")
    assert bench.measured_traffic("wl", 512, 2) is None         # kernel changed since


def test_more_than_one_gpu_is_refused(bench, monkeypatch, capsys):
    monkeypatch.setattr("sys.argv", ["bench.py", "--gpus", "2"])
    with pytest.raises(SystemExit) as ei:
        bench.main()
    assert ei.value.code == 2
    assert "one GPU" in capsys.readouterr().err
