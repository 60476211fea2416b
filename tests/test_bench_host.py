"""Host-side logic of bench.py (no GPU): the counter-derived traffic is reported only while the
hop kernel sources hash to the value recorded in the committed counter summary, and the
per-reduction hop summary is formed from the timing classes as documented."""
import importlib.util
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def load_bench():
    spec = importlib.util.spec_from_file_location("bench_host", os.path.join(ROOT, "bench.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    return m


def make_tree(b, tmp_path, change_source):
    """A copy of the hop sources and a counter summary whose recorded hash is that of the copy
    (before change_source edits one file)."""
    import hashlib

    csrc = tmp_path / "paper_1103_5103_amd" / "csrc"
    csrc.mkdir(parents=True)
    sha = hashlib.sha256()
    for f in b.KERNEL_SOURCES:
        src = open(os.path.join(ROOT, "paper_1103_5103_amd", "csrc", f), "rb").read()
        sha.update(src)
        (csrc / f).write_bytes(src + (b"\n// changed\n" if change_source and f == b.KERNEL_SOURCES[0] else b""))
    (tmp_path / "profiles").mkdir()
    (tmp_path / "profiles" / "hop_counters_32x64.md").write_text(
        f"traffic_bytes_per_launch: 5.5e+08\nkernel_sources_sha256: {sha.hexdigest()}\n")


def test_traffic_reported_when_sources_match(tmp_path, monkeypatch):
    b = load_bench()
    make_tree(b, tmp_path, change_source=False)
    monkeypatch.setattr(b, "ROOT", str(tmp_path))
    assert b.committed_traffic("32x64") == 5.5e8
    assert b.committed_traffic("no_such_workload") is None


def test_traffic_withheld_when_sources_differ(tmp_path, monkeypatch):
    b = load_bench()
    make_tree(b, tmp_path, change_source=True)
    monkeypatch.setattr(b, "ROOT", str(tmp_path))
    assert b.committed_traffic("32x64") is None


def test_hop_variants_summary():
    b = load_bench()
    # (total ms, launches, bytes) per reduction class: none, zdot, outx, norm
    out = b.hop_variants([(8.0, 100, 4.0e10), (5.0, 50, 3.0e10), (0.0, 0, 0.0), (1.0, 10, 5.0e9)])
    assert set(out) == {"none", "zdot", "norm"}
    assert out["none"] == {"launches": 100, "avg_us": 80.0, "GBps": 5000.0, "bytes_per_launch": 400000000}
    assert out["zdot"]["GBps"] == 6000.0
