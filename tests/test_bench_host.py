"""Host-side checks of bench.py (no GPU): the lookup of the committed render
counters that fills roofline.traffic, the itemised FLOPs and the roofline
arithmetic, the design bytes of the HBM-bound stages, and the refusal of
more than one GPU."""
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


def _current(meta, k):
    src = os.path.join(ROOT, k["source"])
    return hashlib.sha256(open(src, "rb").read()).hexdigest() == meta["source_sha256"][k["source"]]


def test_render_traffic_lookup():
    """Every render and render-backward launch shape recorded: bytes and VALU
    instructions per launch, reported while its source is unchanged."""
    meta = json.load(open(COUNTERS))
    assert meta["kernels"], "no render shape recorded"
    assert any(n.startswith("k_render_backward<") for n in meta["kernels"])
    for name, k in meta["kernels"].items():
        assert k["fetch_bytes_per_launch"] > 0 and k["write_bytes_per_launch"] > 0, name
        got = bench.render_counters("clusters", "quadbox", name)
        want = k["fetch_bytes_per_launch"] + k["write_bytes_per_launch"]
        if _current(meta, k):
            assert got["traffic"] == want and got["valu_insts"] == k.get("valu_insts_per_launch"), name
        else:
            assert got is None, name
    # another shape, workload or mode: no figure
    assert bench.render_counters("clusters", "quadbox", "k_render<8, false, false>") is None
    assert bench.render_counters("aniso", "quadbox", next(iter(meta["kernels"]))) is None
    assert bench.render_counters("clusters", "adr", next(iter(meta["kernels"]))) is None


def test_views_traffic_lookup():
    """The 32-view step's render and render-backward launches recorded
    (every shape, the launch over all views): bytes and VALU instructions
    per launch, reported while the source is unchanged; the multi-view
    rooflines take them by kernel name."""
    path = os.path.join(ROOT, bench.VIEWS_COUNTERS)
    meta = json.load(open(path))
    names = set(meta["kernels"])
    assert any(n.startswith("k_render_views<") for n in names)
    assert any(n.startswith("k_render_backward_views<") for n in names)
    from paper_2605_04844_amd import quadbox as qb
    for shape in qb.RENDER_VARIANTS:
        assert bench.render_kernel_name(shape, views=True) in names, shape
    for name, k in meta["kernels"].items():
        assert k["fetch_bytes_per_launch"] > 0 and k["write_bytes_per_launch"] > 0, name
        got = bench._counters(bench.VIEWS_COUNTERS, name)
        if _current(meta, k):
            assert got["traffic"] == k["fetch_bytes_per_launch"] + k["write_bytes_per_launch"], name
            assert got["valu_insts"] == k["valu_insts_per_launch"], name
        else:
            assert got is None, name
    assert bench._counters(bench.VIEWS_COUNTERS, "k_render_views<8, false, 0>") is None


def test_render_traffic_stale_source(tmp_path, monkeypatch):
    """Counters taken on another kernel source are not reported."""
    meta = json.load(open(COUNTERS))
    for src in meta["source_sha256"]:
        meta["source_sha256"][src] = "0" * 64
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "k_render_clusters_1M_counters.json").write_text(json.dumps(meta))
    src = tmp_path / "paper_2605_04844_amd" / "csrc"
    src.mkdir(parents=True)
    for f in ("render.hip", "backward.hip"):
        (src / f).write_bytes(open(os.path.join(ROOT, "paper_2605_04844_amd", "csrc", f), "rb").read())
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    for name in meta["kernels"]:
        assert bench.render_counters("clusters", "quadbox", name) is None


def test_counter_fields():
    """The counters' traffic and the VALU issue rate against 78.6 T
    lane-instructions per second."""
    roof = bench.counter_fields({}, {"traffic": 123, "valu_insts": 1_000_000_000}, 1.0,
                                {"examined": 64_000_000_000}, "examined")
    assert roof["traffic"] == 123 and "not in this run" in roof["traffic_source"]
    v = roof["valu_issue"]
    assert v["lane_insts_per_examined"] == 1.0
    assert v["lane_rate_T"] == pytest.approx(64.0, rel=1e-3) and v["frac"] == pytest.approx(64.0 / 78.64, rel=1e-3)
    assert "frac_of_single_issue" not in v
    assert bench.counter_fields({"a": 1}, None, 1.0, {}, "examined") == {"a": 1}


def test_flops_and_roofline_arithmetic():
    """FLOPs per launch: 9 per examined and 11 more per composited entry in
    the render, 9 per entry before the last contributor and 30 more per
    composited entry in the backward; the fraction is FLOP/s over the
    published 157.3 TFLOP/s."""
    work = {"examined": 1000, "composited": 400, "contributors": 700}
    assert bench.render_flops(work) == 9 * 1000 + 11 * 400
    assert bench.backward_flops(work) == 9 * 700 + 30 * 400
    r = bench.alu_roofline(1.573e11, 1.0, "k", work)
    assert r["bound"] == "alu" and r["unit"] == "TFLOP/s" and r["peak"] == 157.3
    assert r["achieved"] == pytest.approx(157.3, rel=1e-6) and r["frac"] == pytest.approx(1.0, rel=1e-4)
    assert r["examined_per_launch"] == 1000 and r["traffic"] is None


def test_stage_bytes():
    """Design bytes per frame: project 44 + 12 (d+1)^2 B of inputs and 88 B
    of outputs (record, rects, count, depth key) per Gaussian; intersect
    148 B per Gaussian (the depth sort takes the projection's keys) and 6 B
    per pair; sort 28 B per pair (two passes); packed pairs 4 and 26 B."""
    b = bench.stage_bytes(1_000_000, 3, 26_492_435)
    assert b["project"] == 1_000_000 * (44 + 192 + 88)
    assert b["intersect"] == 1_000_000 * 148 + 26_492_435 * 6
    assert b["sort"] == 26_492_435 * 28
    assert bench.stage_bytes(10, 0, 0)["project"] == 10 * (44 + 12 + 88)
    # packed pairs: 4 B written per pair by the emission, 26 B per pair sorted
    bp = bench.stage_bytes(1_000_000, 3, 26_492_435, packed=True)
    assert bp["intersect"] == 1_000_000 * 148 + 26_492_435 * 4
    assert bp["sort"] == 26_492_435 * 26


def test_peaks():
    """Published MI355X peaks: FP32 vector 157.3 TFLOP/s (78.6 T lane-FMAs
    per second), HBM 8 TB/s."""
    assert bench.FP32_PEAK_TFLOPS == 157.3
    assert bench.VALU_LANE_PEAK_T == pytest.approx(157.3 / 2, rel=1e-3)
    assert bench.HBM_PEAK_GBS == 8000.0


def test_more_than_one_gpu_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 2
    line = [s for s in r.stdout.splitlines() if s.startswith("{")][-1]
    out = json.loads(line)
    assert out["n_gpus"] == 2 and "one GPU" in out["error"]
