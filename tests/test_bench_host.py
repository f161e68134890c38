"""Host-side checks of bench.py (no GPU): the lookup of the committed render
counters that fills roofline.traffic, the design bytes of the HBM-bound
stages, and the refusal of more than one GPU."""
import hashlib
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402

COUNTERS = os.path.join(ROOT, "profiles", "k_render_clusters_1M_counters.json")
RENDER_SRC = os.path.join(ROOT, "paper_2605_04844_amd", "csrc", "render.hip")


def test_render_traffic_lookup():
    meta = json.load(open(COUNTERS))
    assert meta["kernels"], "no render shape recorded"
    current = hashlib.sha256(open(RENDER_SRC, "rb").read()).hexdigest() == meta["render_source_sha256"]
    for name, k in meta["kernels"].items():
        assert k["fetch_bytes_per_launch"] > 0 and k["write_bytes_per_launch"] > 0, name
        got = bench.render_traffic("clusters", "quadbox", name)
        want = k["fetch_bytes_per_launch"] + k["write_bytes_per_launch"]
        assert got == (want if current else None), name
    # another shape, workload or mode: no figure
    assert bench.render_traffic("clusters", "quadbox", "k_render<8, false, false>") is None
    assert bench.render_traffic("aniso", "quadbox", next(iter(meta["kernels"]))) is None
    assert bench.render_traffic("clusters", "adr", next(iter(meta["kernels"]))) is None


def test_render_traffic_stale_source(tmp_path, monkeypatch):
    """Counters taken on another render source are not reported."""
    meta = json.load(open(COUNTERS))
    meta["render_source_sha256"] = "0" * 64
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "k_render_clusters_1M_counters.json").write_text(json.dumps(meta))
    src = tmp_path / "paper_2605_04844_amd" / "csrc"
    src.mkdir(parents=True)
    (src / "render.hip").write_bytes(open(RENDER_SRC, "rb").read())
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.render_traffic("clusters", "quadbox", next(iter(meta["kernels"]))) is None


def test_stage_bytes():
    """Design bytes per frame: project 44 + 12 (d+1)^2 B of inputs and 84 B
    of outputs per Gaussian; intersect 164 B per Gaussian and 6 B per pair;
    sort 28 B per pair (two passes)."""
    b = bench.stage_bytes(1_000_000, 3, 26_492_435)
    assert b["project"] == 1_000_000 * (44 + 192 + 84)
    assert b["intersect"] == 1_000_000 * 164 + 26_492_435 * 6
    assert b["sort"] == 26_492_435 * 28
    assert bench.stage_bytes(10, 0, 0)["project"] == 10 * (44 + 12 + 84)


def test_peaks():
    assert bench.VALU_PEAK_TOPS == pytest.approx(157.3 / 2, rel=1e-3)
    assert bench.VALU_SINGLE_ISSUE_TOPS == pytest.approx(39.32, rel=1e-3)
    assert bench.HBM_PEAK_GBS == 8000.0


def test_more_than_one_gpu_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 2
    line = [s for s in r.stdout.splitlines() if s.startswith("{")][-1]
    out = json.loads(line)
    assert out["n_gpus"] == 2 and "one GPU" in out["error"]
