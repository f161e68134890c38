"""Benchmark of the QuadBox rasterizer forward on one MI355X.

Workload: the 1M-Gaussian clustered scene (64 isotropic clusters, SH degree
3) rendered at 1280x720 -- the configuration the headline metric is quoted on.
One step = one whole forward (project -> intersect -> sort -> tile order ->
render) with the Gaussian parameters already resident in HBM.  The pair buffers are sized once
from a warm-up frame, so a step issues no host synchronisation.  Each mode is
timed eagerly (with per-stage HIP events) and as the same frame captured in a
HIP graph and replayed (no host work between launches; every replay is
checked against the eager image); a mode's `ms` is the faster of the two.

Prints one JSON line: FPS of the QuadBox forward (`value`), tile pairs per
frame, the same forward with the 3-sigma AABB and the opacity-aware AABB
boxes, the ablation modes of Table 3 (DualBox, and QuadBox enumerated without
QPass) and QuadBox cut to the 3-sigma tiles, with each mode's image compared
with the QuadBox image, per-stage times from HIP events inside the frame and
each stage's back-to-back launch time (the dominant stage is taken from the
latter), the render's launch time with tiles in work order and in row-major
order, the frame time with
the pair count read back to the host, the achieved bandwidth of the
HBM-bound stages, forward+backward ms per view, the 32-view training step,
the zoom sweep, the roofline of the dominant kernel, and the CPU oracle timed
on a bounded sample.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "FPS & tile pairs/frame (QuadBox vs AABB); fwd+bwd ms/view, 1 GPU"
HBM_PEAK_GBS = 8000.0
# Roofline of the render (Eq. (2)) and its backward, in FLOPs itemised per
# (pixel, list entry) evaluation the algorithm performs, an FMA counting 2
# and exp 1 (compares, min and selects count 0):
#   every examined entry: dx, dy (2), the quadratic form (-b)dy, (-c/2)dy,
#     times dy, two fma (3 + 4) = 9;
#   an entry that composites, in addition: exp, o e, 1 - alpha,
#     T (1 - alpha), alpha T, three fma into the colour = 11.
# The backward examines, per pixel, the entries before its last contributor
# (the same 9 each) and, for each composited one: exp, o e, 1 - alpha, its
# reciprocal, T / (1 - alpha), alpha T, three fma into dL/drgb, the dot
# dL/dC . rgb (5), dL/dalpha (3), the colour-behind update (fma), dpow, the
# opacity share (fma), and its sums dpow, dpow dx, dpow dx^2 (1 + 1 + 1 + 2)
# = 30.
RENDER_FLOPS_EXAMINED, RENDER_FLOPS_COMPOSITED = 9, 11
BACKWARD_FLOPS_EXAMINED, BACKWARD_FLOPS_COMPOSITED = 9, 30
# Published MI355X FP32 vector peak, 157.3 TFLOP/s (256 CUs x 2.4 GHz x 256
# FLOP per clock per CU: 128 lane-FMAs).  In lane operations per second
# that is 78.6 T, the ceiling the measured VALU instruction rate
# (SQ_INSTS_VALU x 64) is read against.  (A quarter-rate reading, one
# 64-lane instruction per SIMD every four clocks, 39.3 T, is no ceiling on
# this chip: the 32-view render issues 46-48 T.)
FP32_PEAK_TFLOPS = 157.3
VALU_LANE_PEAK_T = 256 * 2.4e9 * 128 / 1e12


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="clusters", choices=["clusters", "small"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--trials", type=int, default=3)
    ap.add_argument("--modes", default="quadbox,adr,3sigma,dualbox,quadbox_naive,quadbox_clip3sigma",
                    help="box modes to time; the first one is the headline value")
    ap.add_argument("--no-backward", action="store_true", help="skip the forward+backward timing")
    ap.add_argument("--no-multiview", action="store_true", help="skip the 32-view forward+backward timing")
    ap.add_argument("--no-zoom", action="store_true", help="skip the 3M anisotropic zoom sweep")
    ap.add_argument("--no-rowmajor", action="store_true",
                    help="skip the extra timings (the render with row-major tiles, the frame with the pair count "
                         "read back, standalone stage launches): keeps a kernel trace to the timed frames and the "
                         "work-ordered render launches")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a 1 GiB device copy (counter calibration)")
    return ap.parse_args()


def build_workload(name):
    from paper_2605_04844_amd import scenes
    if name == "small":
        scene, cam = scenes.small_scene()
        cfg = {"workload": "small: 10k Gaussians, 256x256, SH0", "gaussians": scene.n, "width": 256,
               "height": 256, "sh_degree": 0, "seed": 1}
    else:
        scene, cam = scenes.cluster_scene()
        cfg = {"workload": "clusters: 1M Gaussians in 64 clusters, 1280x720, SH3, forward",
               "gaussians": scene.n, "width": cam.width, "height": cam.height, "sh_degree": 3, "seed": 2}
    return scene, cam, cfg


class StageTimer:
    """HIP events on the stream the library launches on (torch's current one)."""

    def __init__(self, torch, names):
        self.torch = torch
        self.names = names
        self.ev = {n: [] for n in names}

    def mark(self):
        e = self.torch.cuda.Event(enable_timing=True)
        e.record()
        return e

    def add(self, name, a, b):
        self.ev[name].append((a, b))

    def ms(self):
        return {n: sum(a.elapsed_time(b) for a, b in v) / max(len(v), 1) for n, v in self.ev.items()}


def run_mode(torch, qb, g, cam, mode, steps, warmup, trials, extras=True):
    # the timed frames leave the sorted 64-bit keys unmaterialised: the render
    # reads only the sorted ids and the ranges
    r = qb.Rasterizer(g.n, cam, write_keys=False)
    r.forward(g, mode)                     # sizes the pair buffers
    torch.cuda.synchronize()
    pairs = r.pairs()
    r._alloc_pairs(pairs)
    r.forward(g, mode, sync_count=False)
    # launch shapes of the intersection, the tile sort and the render for this frame
    isect_shapes = qb.autotune_intersect(r, reps=3, trials=3)
    sort_shapes = qb.autotune_sort(r, reps=3, trials=3)
    shapes = qb.autotune_render(r, reps=10, trials=5)
    for _ in range(warmup):
        r.forward(g, mode, sync_count=False)
    torch.cuda.synchronize()
    trial_ms = []
    timer = StageTimer(torch, ["project", "intersect", "sort", "order", "render"])
    for _ in range(trials):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        start = timer.mark()
        for _ in range(steps):
            e0 = timer.mark()
            r.project(g, mode)
            e1 = timer.mark()
            r.intersect()
            e2 = timer.mark()
            r.sort()
            e3 = timer.mark()
            r.schedule()
            e4 = timer.mark()
            r.render()
            e5 = timer.mark()
            timer.add("project", e0, e1)
            timer.add("intersect", e1, e2)
            timer.add("sort", e2, e3)
            timer.add("order", e3, e4)
            timer.add("render", e4, e5)
        end = timer.mark()
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) * 1e3 / steps
        trial_ms.append((start.elapsed_time(end) / steps, wall))
    assert r.pairs() == pairs, "pair count changed between frames"
    dev = sorted(t[0] for t in trial_ms)[len(trial_ms) // 2]
    wall = sorted(t[1] for t in trial_ms)[len(trial_ms) // 2]
    stage = timer.ms()
    # the same frame captured once in a HIP graph and replayed: no host work
    # between the launches; every replay must reproduce the eager image
    want = r.image.clone()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        r.forward(g, mode, sync_count=False)
    torch.cuda.current_stream().wait_stream(side)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        r.project(g, mode)
        r.intersect()
        r.sort()
        r.schedule()
        r.render()
    graph_trials = []
    for _ in range(trials):
        r.image.fill_(-1.0)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            graph.replay()
        e1.record()
        torch.cuda.synchronize()
        assert torch.equal(r.image, want), "graph replay differs from the eager frame"
        graph_trials.append(e0.elapsed_time(e1) / steps)
    graph_ms = sorted(graph_trials)[len(graph_trials) // 2]
    del graph
    # the render kernel's own launch time (the roofline's denominator):
    # back-to-back launches on this frame's resident buffers, HIP events on
    # the stream the library launches on; the per-stage events above also
    # catch any gap before a stage's first kernel starts
    render_launch_ms = _time(torch, r.render, 20, 2, trials)
    # the same launches with the tiles in row-major order (no qb_tile_order):
    # what the work-ordered dispatch gains
    rowmajor_ms = sync_ms = stage_launch = None
    if extras:
        r.balance = False
        rowmajor_ms = _time(torch, r.render, 20, 2, trials)
        r.balance = True
        # the frame with its pair count read back to the host (one
        # synchronisation per frame, as a caller sizing buffers would)
        sync_ms = _time(torch, lambda: r.forward(g, mode, sync_count=True), steps, 2, trials)
        # back-to-back launches of the HBM-bound stages on the frame's buffers
        stage_launch = {"project": _time(torch, lambda: r.project(g, mode), 20, 2, trials),
                        "intersect": _time(torch, r.intersect, 20, 2, trials),
                        "sort": _time(torch, r.sort, 20, 2, trials),
                        "order": _time(torch, r.schedule, 20, 2, trials),
                        "render": render_launch_ms}
        torch.cuda.synchronize()
    work = render_work(torch, qb, r)
    names = {v: k for k, v in qb.RENDER_VARIANTS.items()}
    snames = {v: k for k, v in qb.SORT_VARIANTS.items()}
    dnames = {v: k for k, v in qb.DEPTH_VARIANTS.items()}
    enames = {v: k for k, v in qb.EMIT_VARIANTS.items()}
    return dict(ms=min(dev, graph_ms), eager_ms=dev, graph_ms=graph_ms, wall_ms=wall, pairs=pairs, stage_ms=stage,
                render_launch_ms=render_launch_ms, render_rowmajor_ms=rowmajor_ms, sync_ms=sync_ms,
                stage_launch_ms=stage_launch, work=work, rast=r,
                render_shape=names[r.render_variant], shape_ms={k: round(v, 4) for k, v in shapes.items()},
                packed=r.packed_id_bits() > 0,
                sort_shape=snames[r.sort_variant], sort_shape_ms={k: round(v, 4) for k, v in sort_shapes.items()},
                intersect_shape=f"{dnames[r.depth_variant]}/{enames[r.emit_variant]}",
                intersect_shape_ms={k: round(v, 4) for k, v in isect_shapes.items()})


def run_fwd_bwd(torch, qb, g, cam, steps, warmup, trials):
    """Forward + backward of an L1 loss against a U(0,1) target (the
    1M-Gaussian 1280x720 SH3 training step of one view): the four forward
    calls, dL/dimage, qb_render_backward and qb_project_backward."""
    from paper_2605_04844_amd import scenes
    r = qb.Rasterizer(g.n, cam, write_keys=False)
    r.forward(g, "quadbox")
    torch.cuda.synchronize()
    r._alloc_pairs(r.pairs())
    target = torch.tensor(scenes.target_image(4, cam.width, cam.height), device="cuda")
    grad2d = torch.empty((g.n, 9), dtype=torch.float32, device="cuda")
    grads = [torch.empty_like(t) for t in g.tensors()]
    inv = 1.0 / float(target.numel())
    dl = torch.empty_like(r.image)
    r.forward(g, "quadbox", sync_count=False)
    qb.autotune_intersect(r, reps=3, trials=2)
    qb.autotune_sort(r, reps=3, trials=2)
    qb.autotune_render(r, reps=5, trials=2)
    r.forward(g, "quadbox", sync_count=False)
    qb.l1_grad([(r.image, target, dl, inv)])
    qb.autotune_backward(r, dl=dl, grad2d=grad2d, reps=3, trials=2)

    def step():
        r.forward(g, "quadbox", sync_count=False)
        qb.l1_grad([(r.image, target, dl, inv)])   # dL/dimage = sign(image - target) / count
        qb.render_backward(r.W, r.H, r.ranges, r.ids_sorted, r.splats, (0.0, 0.0, 0.0), r.final_T, r.n_contrib,
                           dl, g.n, grad2d, r.backward_variant, r.tile_order())
        qb.project_backward(g, cam, r.splats, grad2d, *grads)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    times = []
    for _ in range(trials):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            step()
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1) / steps)
    r.check_capacity()
    # the render backward call on its own, back to back on the last frame's
    # buffers: the 36-byte-per-Gaussian clear of grad2d, then k_render_backward
    qb.l1_grad([(r.image, target, dl, inv)])
    bwd_ms = _time(torch, lambda: qb.render_backward(r.W, r.H, r.ranges, r.ids_sorted, r.splats, (0.0, 0.0, 0.0),
                                                     r.final_T, r.n_contrib, dl, g.n, grad2d, r.backward_variant,
                                                     r.tile_order()), 20, 2, trials)
    names = {v: k for k, v in qb.BACKWARD_VARIANTS.items()}
    return dict(ms=sorted(times)[len(times) // 2], render_backward_ms=bwd_ms, work=render_work(torch, qb, r),
                shape=names[r.backward_variant])


def _time(torch, fn, steps, warmup, trials):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    times = []
    for _ in range(trials):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1) / steps)
    return sorted(times)[len(times) // 2]


def run_multiview(torch, qb, steps, warmup, trials):
    """Forward + backward of an L1 loss over 32 views of 2M Gaussians
    (640x360 / 1280x720 / 1920x1080 by view index), four ways: the
    single-view entry points view after view (gradients summed by torch),
    the batched entry points (quadbox.MultiView forward, l1_grad, backward),
    MultiView.step (each side stream renders and back-propagates its views
    behind their sorts), the last two also captured once in a HIP graph and
    replayed.  Returns ms per view."""
    from paper_2605_04844_amd import scenes
    scene, cams = scenes.multiview_scene()
    g = qb.Gaussians(scene)
    V = len(cams)
    targets = [torch.tensor(scenes.target_image(500 + v, c.width, c.height), device="cuda")
               for v, c in enumerate(cams)]
    mv = qb.MultiView(scene.n, cams)
    pairs = mv.size_pairs(g, "quadbox")
    mv.forward(g)
    loss_items = [(mv.images[v], targets[v], mv.dl[v], 1.0 / mv.images[v].numel()) for v in range(V)]
    qb.l1_grad(loss_items)
    tuned = {"intersect_ms": qb.autotune_intersect(mv, reps=1, trials=2),
             "sort_ms": qb.autotune_sort(mv, reps=1, trials=2),
             "render_ms": qb.autotune_render(mv, reps=3, trials=2),
             "render_backward_ms": qb.autotune_backward(mv, reps=2, trials=2)}
    tuned = {k: {s: round(x, 4) for s, x in v.items()} for k, v in tuned.items()}
    names = {v: k for k, v in qb.RENDER_VARIANTS.items()}
    bnames = {v: k for k, v in qb.BACKWARD_VARIANTS.items()}
    snames = {v: k for k, v in qb.SORT_VARIANTS.items()}
    dnames = {v: k for k, v in qb.DEPTH_VARIANTS.items()}
    enames = {v: k for k, v in qb.EMIT_VARIANTS.items()}
    tuned["picked"] = {"intersect": f"{dnames[mv.depth_variant]}/{enames[mv.emit_variant]}",
                       "sort": snames[mv.sort_variant], "render": names[mv.render_variant],
                       "render_backward": bnames[mv.backward_variant]}
    log("autotune", tuned)

    def batched():
        mv.forward(g)
        qb.l1_grad(loss_items)   # every view's dL/dimage in one launch
        mv.backward(g)

    batched_ms = _time(torch, batched, steps, warmup, trials)
    work = {"examined": 0, "composited": 0, "contributors": 0}
    for v in range(V):
        w = render_work(torch, qb, None, view=(mv, v))
        for k in work:
            work[k] += w[k]
    fwd_ms = tuned["render_ms"][tuned["picked"]["render"]]
    bwd_ms = tuned["render_backward_ms"][tuned["picked"]["render_backward"]]
    rooflines = {"render_views": alu_roofline(render_flops(work), fwd_ms,
                                              render_kernel_name(tuned["picked"]["render"], views=True), work),
                 "render_backward_views": alu_roofline(backward_flops(work), bwd_ms,
                                                       f"k_render_backward_views<{tuned['picked']['render_backward'][0]}>",
                                                       work)}
    # the committed counters of the picked shapes' 32-view launches
    for key, ms, per in (("render_views", fwd_ms, "examined"), ("render_backward_views", bwd_ms, "contributors")):
        counter_fields(rooflines[key], _counters(VIEWS_COUNTERS, rooflines[key]["kernel"]), ms, work, per,
                       source=VIEWS_COUNTERS)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        batched()
    torch.cuda.current_stream().wait_stream(side)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        batched()
    graph_ms = _time(torch, graph.replay, steps, warmup, trials)
    mv.check_capacity()
    del graph

    # the same step from MultiView.step: each side stream renders, takes the
    # loss gradient of and back-propagates its views behind their sorts
    def stepped():
        mv.step(g, targets)

    step_ms = _time(torch, stepped, steps, warmup, trials)
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        stepped()
    torch.cuda.current_stream().wait_stream(side)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        stepped()
    step_graph_ms = _time(torch, graph.replay, steps, warmup, trials)
    mv.check_capacity()
    del graph

    rasts = []
    for c in cams:
        r = qb.Rasterizer(g.n, c, write_keys=False)
        r.forward(g, "quadbox")
        torch.cuda.synchronize()
        r._alloc_pairs(int(r.pairs() * 1.1) + 1024)
        rasts.append(r)
    grad2d = torch.empty((g.n, 9), dtype=torch.float32, device="cuda")
    part = [torch.empty_like(t) for t in g.tensors()]
    total = [torch.empty_like(t) for t in g.tensors()]
    dls = [torch.empty_like(r.image) for r in rasts]

    def per_view():
        for t in total:
            t.zero_()
        for v, r in enumerate(rasts):
            r.forward(g, "quadbox", sync_count=False)
            qb.l1_grad([(r.image, targets[v], dls[v], 1.0 / r.image.numel())])
            qb.render_backward(r.W, r.H, r.ranges, r.ids_sorted, r.splats, (0.0, 0.0, 0.0), r.final_T,
                               r.n_contrib, dls[v], g.n, grad2d, r.backward_variant, r.tile_order())
            qb.project_backward(g, cams[v], r.splats, grad2d, *part)
            for t, p in zip(total, part):
                t.add_(p)

    per_view_ms = _time(torch, per_view, max(1, steps // 4), 1, trials)
    assert all(r.pairs() <= r.capacity for r in rasts)
    return {"workload": "2M Gaussians (64 clusters in [-1,1]^3), 32 views at 640x360 / 1280x720 / 1920x1080, "
                        "SH3, forward + L1 loss gradient + backward",
            "views": V, "gaussians": g.n, "pairs_per_step": int(sum(pairs)),
            "per_view_path_ms_per_view": round(per_view_ms / V, 4),
            "batched_ms_per_view": round(batched_ms / V, 4),
            "batched_graph_ms_per_view": round(graph_ms / V, 4),
            "step_ms_per_view": round(step_ms / V, 4),
            "step_graph_ms_per_view": round(step_graph_ms / V, 4),
            "graph_speedup_vs_per_view": round(per_view_ms / graph_ms, 3),
            "autotune": tuned, "rooflines": rooflines}


def run_zoom_sweep(torch, qb, steps, trials):
    """Forward of the 3M highly anisotropic Gaussians at 1920x1080 with focal
    1920*k, k = 1..8 (the zoom-in sweep): tile pairs per frame and FPS for
    QuadBox, the opacity-aware AABB and the 3-sigma AABB."""
    from paper_2605_04844_amd import scenes
    scene, cams = scenes.aniso_scene()
    g = qb.Gaussians(scene)
    rows = []
    for k, cam in enumerate(cams, start=1):
        row = {"zoom": k}
        for mode in ("quadbox", "adr", "3sigma"):
            res = run_mode(torch, qb, g, cam, mode, steps, 2, trials, extras=False)
            row[mode] = {"pairs": res["pairs"], "fps": round(1000.0 / res["ms"], 2), "ms": round(res["ms"], 4)}
            del res
        row["quadbox_vs_3sigma"] = round(row["3sigma"]["ms"] / row["quadbox"]["ms"], 3)
        log("zoom", row)
        rows.append(row)
    return {"workload": "3M anisotropic Gaussians (major/minor ratio log-uniform in [1,100]), 1920x1080, SH3, "
                        "focal 1920*k, forward", "rows": rows}


def render_work(torch, qb, r, view=None):
    """The render's work on the frame a Rasterizer `r` (or view v of a
    MultiView, view=(mv, v)) holds, from one extra, untimed qb_render_stats
    launch: list entries examined (each pixel's stop index, or its list
    length), entries composited, and the sum of the contributor counts (the
    entries the backward examines)."""
    if view is not None:
        mv, v = view
        W, H = mv.sizes[v]
        args = (mv.ranges[v], mv.ids_sorted[v], mv.splats[v])
        order = None
    else:
        W, H = r.W, r.H
        args = (r.ranges, r.ids_sorted, r.splats)
        order = r.tile_order()
    dev = args[0].device
    img = torch.empty((3, H, W), dtype=torch.float32, device=dev)
    T = torch.empty((H, W), dtype=torch.float32, device=dev)
    nc, nt, nk = (torch.empty((H, W), dtype=torch.int32, device=dev) for _ in range(3))
    qb.render_stats(W, H, *args, (0.0, 0.0, 0.0), img, T, nc, nt, nk, 0, order)
    torch.cuda.synchronize()
    return {"examined": int(nt.to(torch.int64).sum()), "composited": int(nk.to(torch.int64).sum()),
            "contributors": int(nc.to(torch.int64).sum())}


def render_kernel_name(shape, views=False):
    """The k_render (views: k_render_views) instance a render launch shape
    (RENDER_VARIANTS key, e.g. "2px", "1px_rows", "2px_xrow1") runs."""
    rows = "true" if shape.endswith("_rows") else "false"
    xrow = 2 if shape.endswith("_xrow1") else (1 if shape.endswith("_xrow") else 0)
    if views:
        return f"k_render_views<{shape[0]}, {rows}, {xrow}>"
    return f"k_render<{shape[0]}, false, {rows}, {xrow}>"


def render_flops(work):
    return RENDER_FLOPS_EXAMINED * work["examined"] + RENDER_FLOPS_COMPOSITED * work["composited"]


def backward_flops(work):
    return BACKWARD_FLOPS_EXAMINED * work["contributors"] + BACKWARD_FLOPS_COMPOSITED * work["composited"]


def alu_roofline(flops, ms, kernel, work, traffic=None, note=None):
    """FLOPs per launch over the launch time, against the FP32 vector peak."""
    tf = flops / (ms * 1e-3) / 1e12
    out = {"bound": "alu", "achieved": round(tf, 3), "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
           "frac": round(tf / FP32_PEAK_TFLOPS, 4), "traffic": traffic, "kernel": kernel,
           "flops_per_launch": int(flops), "launch_ms": round(ms, 4), **{f"{k}_per_launch": v for k, v in work.items()}}
    if note:
        out["note"] = note
    return out


def stage_bytes(n, sh_degree, pairs, packed=False):
    """Bytes each HBM-bound stage moves by its design, per frame:
    project: the SoA inputs (12 + 12 + 16 + 4 + 12 (d+1)^2 B) read, the 48-byte
      record, 32-byte rects, the count and the 4-byte depth key written, per
      Gaussian;
    intersect: 4 depth-sort passes over the projection's keys (8 B read and
      written, 4 B upsweep read), the count gather (8 B), the offset scan (4 B
      read, 8 written), the emission's reads (rects 32 B, order, count, offset
      16 B) per Gaussian, and 6 B written per pair;
    sort: 2 tile passes of 6 B read and written plus a 2-byte upsweep read,
      per pair.
    With packed pairs (tile << id_bits | id in 4 bytes) the emission writes
    4 B per pair and the sort reads 4 B per pair in each pass's upsweep and
    downsweep, writes 4 B in the first pass and 6 B (tile and id apart) in
    the last: 26 B per pair."""
    proj = n * (44 + 12 * (sh_degree + 1) ** 2 + 88)
    isect = n * (4 * 20 + 8 + 12 + 48) + pairs * (4 if packed else 6)
    sort = pairs * (26 if packed else 28)
    return {"project": proj, "intersect": isect, "sort": sort}


def stage_bandwidth(q, g, copy_gbs):
    """Achieved bandwidth of the HBM-bound stages (design bytes over the
    stage's back-to-back launch time) against the 8 TB/s peak and the
    measured device-copy rate."""
    b = stage_bytes(g.n, g.sh_degree, q["pairs"], q["packed"])
    out = {}
    for k, ms in q["stage_launch_ms"].items():
        if k not in b:
            continue
        gbs = b[k] / (ms * 1e-3) / 1e9
        out[k] = {"bytes": int(b[k]), "ms": round(ms, 4), "gbs": round(gbs, 1),
                  "frac_of_peak": round(gbs / HBM_PEAK_GBS, 3), "frac_of_copy": round(gbs / copy_gbs, 3)}
    return out


def image_delta(torch, img, ref):
    """Max abs difference and PSNR (peak 1) of a mode's image against the
    headline mode's image; DualBox drops real contributions (Table 3)."""
    d = (img - ref).double()
    mse = float((d * d).mean())
    return {"image_max_abs_vs_headline": float(d.abs().max()),
            "psnr_vs_headline": None if mse == 0.0 else round(10.0 * math.log10(1.0 / mse), 2)}


def cpu_baseline(scene, cam, exact_stride=10, trials=3):
    """The oracle (as it stands) on whole frames of the same workload:
    project, all pairs (parallel chunk sort and merge), ranges, and the
    per-pixel render; wall-clock, one untimed warm-up frame, the median of
    `trials` frames on every worker thread the oracle runs, then one frame
    on a single thread.  Also the oracle's exact-sample pair count (tiles
    holding a pixel sample that passes the cutoff) on every
    `exact_stride`-th projected Gaussian: the lower bound of any
    conservative tile set, against the QuadBox, AdR and 3-sigma counts of
    the same sample (untimed)."""
    import numpy as np
    from oracle import oracle as O
    threads = O.threads()

    def frame():
        t0 = time.perf_counter()
        g = O.project(scene, cam, "quadbox")
        t1 = time.perf_counter()
        keys, ids = O.pairs(g, cam.tiles_x)
        rt = O.ranges(keys, cam.num_tiles)
        t2 = time.perf_counter()
        O.render(g, cam.width, cam.height, rt, ids)
        t3 = time.perf_counter()
        return (t3 - t0, t1 - t0, t2 - t1, t3 - t2), g

    frame()
    runs = sorted((frame()[0] for _ in range(trials)), key=lambda t: t[0])
    med = runs[len(runs) // 2]
    O.set_threads(1)
    try:
        one, g = frame()
    finally:
        O.set_threads(threads)
    base = {"value": round(1.0 / med[0], 4), "unit": "frames/s", "cores": threads, "kind": "oracle",
            "sample": f"whole frames of the same workload, median of {trials} after one warm-up on {threads} "
                      f"threads: {med[0]:.2f} s (project {med[1]:.2f}, pairs+sort+ranges {med[2]:.2f}, "
                      f"render {med[3]:.2f}); trials {', '.join(f'{t[0]:.2f}' for t in runs)} s",
            "single_core": {"value": round(1.0 / one[0], 4), "unit": "frames/s", "cores": 1,
                            "sample": f"one frame on 1 thread: {one[0]:.2f} s (project {one[1]:.2f}, "
                                      f"pairs+sort+ranges {one[2]:.2f}, render {one[3]:.2f})"}}
    sub = np.ascontiguousarray(g[::exact_stride])
    missed, exact, _ = O.coverage_audit(sub, cam.width, cam.height)
    quad = int(O.tile_counts(sub, cam.tiles_x).sum())
    exact_pairs = {"estimate": exact * exact_stride, "quadbox_over_exact": round(quad / max(exact, 1), 4),
                   "missed_by_quadbox": missed}
    for mode in ("adr", "3sigma"):
        gm = np.ascontiguousarray(O.project(scene, cam, mode)[::exact_stride])
        exact_pairs[f"{mode}_over_exact"] = round(int(O.tile_counts(gm, cam.tiles_x).sum()) / max(exact, 1), 4)
    exact_pairs.update({
                   "sample": f"every {exact_stride}th Gaussian of the oracle's projection ({len(sub)}), "
                             f"{exact} exact and {quad} QuadBox pairs, scaled by {exact_stride}"})
    return base, exact_pairs


COUNTERS = os.path.join("profiles", "k_render_clusters_1M_counters.json")
VIEWS_COUNTERS = os.path.join("profiles", "k_render_views_multiview_2M_counters.json")


def render_counters(workload, mode, kernel):
    """Counters per launch of the render or render-backward kernel `kernel`
    from the committed summary (every launch shape of the frame; the
    autotuners launch each): HBM bytes (FETCH_SIZE + WRITE_SIZE,
    copy-calibrated) and VALU instructions (SQ_INSTS_VALU), or None when the
    summary was taken on another workload or on a different kernel source
    (the sha256 of each source is recorded)."""
    if workload != "clusters" or mode != "quadbox":
        return None
    return _counters(COUNTERS, kernel)


def _counters(rel, kernel):
    """The entry of `kernel` in the committed counters summary `rel`, or
    None (no summary, no entry, or a different kernel source)."""
    path = os.path.join(ROOT, rel)
    if not os.path.exists(path):
        return None
    meta = json.load(open(path))
    k = meta.get("kernels", {}).get(kernel)
    if k is None:
        return None
    src = k.get("source", "")
    want = meta.get("source_sha256", {}).get(src)
    full = os.path.join(ROOT, src)
    if not want or not os.path.exists(full) or hashlib.sha256(open(full, "rb").read()).hexdigest() != want:
        return None
    return {"traffic": int(k["fetch_bytes_per_launch"] + k["write_bytes_per_launch"]),
            "valu_insts": k.get("valu_insts_per_launch")}


def counter_fields(roof, ctr, ms, work, per, source=COUNTERS):
    """Adds the committed counters' traffic and VALU issue rate to a
    roofline entry (`per`: the work count the lane instructions are divided
    by; `source`: the summary they come from)."""
    if not ctr:
        return roof
    roof["traffic"] = ctr["traffic"]
    roof["traffic_source"] = (f"{source}: FETCH_SIZE + WRITE_SIZE per launch of this kernel, copy-calibrated, "
                              "taken by rocprofv3 on this kernel source (sha256 recorded there), not in this run")
    if ctr.get("valu_insts"):
        lane_rate = ctr["valu_insts"] * 64 / (ms * 1e-3) / 1e12
        roof["valu_issue"] = {"insts_per_launch": int(ctr["valu_insts"]),
                              f"lane_insts_per_{per}": round(ctr["valu_insts"] * 64 / max(work[per], 1), 2),
                              "lane_rate_T": round(lane_rate, 2), "peak_T": round(VALU_LANE_PEAK_T, 2),
                              "frac": round(lane_rate / VALU_LANE_PEAK_T, 4),
                              "source": f"{source}: SQ_INSTS_VALU per launch, not in this run"}
    return roof


def copy_bandwidth(torch, mib=1024, reps=10):
    """Achieved HBM rate of a plain device-to-device copy (bytes read plus
    written per second): the practical ceiling of the HBM-bound stages, next
    to the published 8 TB/s."""
    a = torch.empty(mib << 20, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1)
    ms = _time(torch, lambda: b.copy_(a), reps, 2, 3)
    del a, b
    return round(2.0 * (mib << 20) / (ms * 1e-3) / 1e9, 1)


def calibrate_copy(torch, mib=1024):
    """A plain device copy of known size, for scaling the HBM byte counters."""
    a = torch.empty(mib << 20, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"calibration_copy_bytes": mib << 20}), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this rasterizer runs on one GPU; multi-GPU is not built",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch
    from paper_2605_04844_amd import quadbox as qb
    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    if args.calibrate_copy:
        calibrate_copy(torch)
        return
    qb.lib()
    scene, cam, cfg = build_workload(args.workload)
    g = qb.Gaussians(scene)
    torch.cuda.synchronize()
    results = {}
    modes = args.modes.split(",")
    for mode in modes:
        log("mode", mode)
        results[mode] = run_mode(torch, qb, g, cam, mode, args.steps, args.warmup, args.trials,
                                 extras=not args.no_rowmajor)
        res = results[mode]
        log(mode, f"{res['ms']:.3f} ms/frame, {res['pairs']} pairs, stages",
            {k: round(v, 4) for k, v in res["stage_ms"].items()})
    fwd_bwd = None
    if args.workload == "clusters" and not args.no_backward:
        log("forward + backward")
        fwd_bwd = run_fwd_bwd(torch, qb, g, cam, args.steps, args.warmup, args.trials)
        log(f"fwd+bwd {fwd_bwd['ms']:.3f} ms/view")
    multiview = None
    if args.workload == "clusters" and not args.no_multiview:
        log("multi-view forward + backward")
        multiview = run_multiview(torch, qb, args.steps, args.warmup, args.trials)
        log("multi-view", multiview)
    zoom = None
    if args.workload == "clusters" and not args.no_zoom:
        log("zoom sweep")
        zoom = run_zoom_sweep(torch, qb, max(2, args.steps // 5), 1)
    q = results[modes[0]]
    # the dominant stage by the stages' own back-to-back launch times where
    # they were taken: the in-frame events also charge a stage any gap before
    # its first kernel starts (host issue), which lands on whichever stage
    # the host fell behind on
    stage = q["stage_launch_ms"] if q["stage_launch_ms"] is not None else q["stage_ms"]
    dominant = max(stage, key=stage.get)
    # roofline of the render kernel (qb_render launches k_render alone, so
    # events around back-to-back calls time that kernel)
    render_ms = q["render_launch_ms"]
    kname = render_kernel_name(q["render_shape"])
    ctr = render_counters(args.workload, modes[0], kname)
    roof = alu_roofline(render_flops(q["work"]), render_ms, kname, q["work"])
    roof["flops_per_examined"] = RENDER_FLOPS_EXAMINED
    roof["flops_per_composited"] = RENDER_FLOPS_COMPOSITED
    counter_fields(roof, ctr, render_ms, q["work"], "examined")
    bwd_roof = None
    if fwd_bwd is not None:
        bname = f"k_render_backward<{fwd_bwd['shape'][0]}>"
        bwd_roof = alu_roofline(backward_flops(fwd_bwd["work"]), fwd_bwd["render_backward_ms"], bname,
                                fwd_bwd["work"], note="launch time includes the clear of grad2d (36 B per Gaussian)")
        bwd_roof["flops_per_contributor_entry"] = BACKWARD_FLOPS_EXAMINED
        bwd_roof["flops_per_composited"] = BACKWARD_FLOPS_COMPOSITED
        counter_fields(bwd_roof, render_counters(args.workload, modes[0], bname), fwd_bwd["render_backward_ms"],
                       fwd_bwd["work"], "contributors")
    out = {
        "metric": METRIC,
        "value": round(1000.0 / q["ms"], 2),
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(q["ms"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": cfg,
        "pairs_per_frame": q["pairs"],
        "modes": {m: {"fps": round(1000.0 / r["ms"], 2), "ms": round(r["ms"], 4), "pairs": r["pairs"],
                      "eager_ms": round(r["eager_ms"], 4), "graph_ms": round(r["graph_ms"], 4),
                      "stage_ms": {k: round(v, 4) for k, v in r["stage_ms"].items()},
                      "render_launch_ms": round(r["render_launch_ms"], 4),
                      "render_rowmajor_ms": (round(r["render_rowmajor_ms"], 4)
                                             if r["render_rowmajor_ms"] is not None else None),
                      "ms_with_count_readback": round(r["sync_ms"], 4) if r["sync_ms"] is not None else None,
                      "render_shape": r["render_shape"], "render_shape_ms": r["shape_ms"],
                      "pair_format": "packed" if r["packed"] else "split",
                      "sort_shape": r["sort_shape"], "sort_shape_ms": r["sort_shape_ms"],
                      "intersect_shape": r["intersect_shape"], "intersect_shape_ms": r["intersect_shape_ms"],
                      **image_delta(torch, r["rast"].image, q["rast"].image)}
                  for m, r in results.items()},
        "fwd_bwd_ms_per_view": round(fwd_bwd["ms"], 4) if fwd_bwd is not None else None,
        "render_backward_roofline": bwd_roof,
        "multiview": multiview,
        "zoom_sweep": zoom,
        "quadbox_vs_3sigma": round(results["3sigma"]["ms"] / q["ms"], 3) if "3sigma" in results else None,
        "quadbox_vs_adr": round(results["adr"]["ms"] / q["ms"], 3) if "adr" in results else None,
        "dominant_stage": dominant,
        "stage_launch_ms": ({k: round(v, 4) for k, v in q["stage_launch_ms"].items()}
                            if q["stage_launch_ms"] is not None else None),
        "roofline": roof,
    }
    copy_gbs = copy_bandwidth(torch)
    out["hbm_copy_gbs"] = copy_gbs
    if q["stage_launch_ms"] is not None:
        out["stage_bandwidth"] = stage_bandwidth(q, g, copy_gbs)
    if not args.no_cpu:
        log("cpu baseline")
        out["cpu_baseline"], out["pairs_exact"] = cpu_baseline(scene, cam)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
