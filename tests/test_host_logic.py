"""Host-side logic that needs no GPU: bench.py's reading of the committed counter summary,
its refusal of more than one GPU, and the Python layout's array extents."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def test_traffic_is_read_only_for_the_profiled_sources(tmp_path, monkeypatch):
    import bench

    fp = bench.source_fingerprint()
    assert len(fp) == 16
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "k.md").write_text(f"x\ntraffic_bytes_per_launch: 123456 sources: {fp}\n")
    (prof / "old.md").write_text("traffic_bytes_per_launch: 999 sources: 0000000000000000\n")
    (prof / "none.md").write_text("no counters here\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    # the fingerprint is taken over the package sources under ROOT: give the copy the same ones
    src = os.path.join(ROOT, "paper_2205_00856_amd", "csrc")
    dst = tmp_path / "paper_2205_00856_amd" / "csrc"
    dst.mkdir(parents=True)
    for name in os.listdir(src):
        (dst / name).write_bytes(open(os.path.join(src, name), "rb").read())
    assert bench.measured_traffic("k.md") == 123456.0
    assert bench.measured_traffic("old.md") is None
    assert bench.measured_traffic("none.md") is None
    assert bench.measured_traffic("missing.md") is None
    (dst / "cntri.hip").write_bytes(b"// changed\n")
    assert bench.measured_traffic("k.md") is None


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_layout_extents():
    pytest.importorskip("torch")
    from paper_2205_00856_amd.api import Layout

    L = Layout.contiguous(100, 7)
    assert L.span() == 700 and L.coef_span() == 700 and L.rows() == 700
    S = Layout.contiguous(100, 7, shared_coefficients=True)
    assert S.span() == 700 and S.coef_span() == 100
    I = Layout.interleaved(50, 64, shared_coefficients=True)
    assert I.span() == 50 * 64 and I.coef_span() == 49 * 64 + 1
    U = Layout.uneven([0, 3, 10])
    assert U.span() == 10 and U.coef_span() == 10 and U.rows() == 10
    c = S.c()
    assert c.shared_coefficients == 1 and c.batch_stride == 100
