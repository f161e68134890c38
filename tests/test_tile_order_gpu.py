"""GPU checks of the tile order (qb_tile_order, qb_tile_order_views) and of
the render and its backward taking tiles in that order.

The order only schedules: every tile is computed exactly as in row-major
order, so the bar is bit-equality with the row-major render (image, final T,
contributor counts) for every launch shape, and the gradients of the render
backward equal up to the order of the float atomic additions (rel 1e-5).
The order itself must be a permutation of the tiles with the clamped work
estimates non-increasing along it.  The work estimate (the number of list
entries a tile's centre pixel examines before its transmittance drops below
1e-4, extrapolated past the first 256 entries) is a heuristic that binary32
log sums evaluate; it is checked against the same definition taken on the
oracle's own projected records, sorted ids and ranges in binary64: within 2
entries or 1% for at least 98% of the tiles, exact for empty tiles."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2605_04844_amd import scenes  # noqa: E402

pytestmark = pytest.mark.gpu

WORK_PREFIX = 256
LOG2_STOP = float(np.log2(1e-4))
ORDER_BINS = 4096


def say(*a):
    print("[order]", *a, flush=True)


@pytest.fixture(scope="module")
def qb():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2605_04844_amd import quadbox
    quadbox.lib()
    return quadbox


def work_reference(g, ids, ranges, W, H):
    """The estimate's definition on the oracle's records (u, v, a, b, c,
    opacity, gamma), sorted ids and ranges, in binary64: the entry at which
    the tile's centre pixel stops within the first WORK_PREFIX entries, else
    the stop extrapolated at the prefix's rate of attenuation (capped at the
    list length; the list length when nothing attenuates)."""
    tiles_x, tiles_y = (W + 15) // 16, (H + 15) // 16
    out = np.zeros(tiles_x * tiles_y, np.float64)
    rg = ranges.reshape(-1, 2).astype(np.int64)
    for t in range(tiles_x * tiles_y):
        s, e = rg[t]
        if e == s:
            continue
        x0, y0 = (t % tiles_x) * 16, (t // tiles_x) * 16
        px = np.float32(x0 + min(16, W - x0) // 2)
        py = np.float32(y0 + min(16, H - y0) // 2)
        rec = g[ids[s:min(e, s + WORK_PREFIX)]]
        dx = (rec["u"].astype(np.float32) - px).astype(np.float64)
        dy = (rec["v"].astype(np.float32) - py).astype(np.float64)
        a, b, c = (rec[k].astype(np.float32).astype(np.float64) for k in ("a", "b", "c"))
        p = (-0.5 * a * dx - b * dy) * dx - 0.5 * c * dy * dy
        gam = rec["gamma"].astype(np.float32).astype(np.float64)
        ok = ~((p > 0.0) | (p < -0.5 * gam))
        alpha = np.where(ok, np.minimum(0.99, rec["opacity"].astype(np.float64) * np.exp(np.minimum(p, 0.0))), 0.0)
        L = np.cumsum(np.log2(1.0 - alpha))
        hit = np.nonzero(L < LOG2_STOP)[0]
        if len(hit):
            out[t] = hit[0] + 1
        elif e - s > WORK_PREFIX and L[-1] < 0.0:
            out[t] = min(WORK_PREFIX * LOG2_STOP / L[-1], e - s)
        else:
            out[t] = e - s
    return out


def check_order(work, order, label):
    n = len(order)
    assert np.array_equal(np.sort(order), np.arange(n)), label + ": not a permutation"
    w = np.minimum(work[order], ORDER_BINS - 1)
    assert np.all(np.diff(w) <= 0), label + ": estimates not non-increasing along the order"


def outputs(r):
    return r.image.clone(), r.final_T.clone(), r.n_contrib.clone()


@pytest.mark.parametrize("seed,n,w,h", [(201, 6000, 333, 250), (202, 20000, 256, 256), (203, 500, 17, 40)])
def test_tile_order_matches_row_major_and_estimate(oracle, qb, seed, n, w, h):
    scene, _ = scenes.random_scene(seed, n, w, h, float(w), sh_degree=2)
    cam = scenes.pinhole(w, h, float(w))
    bg = (0.25, 0.5, 0.75)
    g = qb.Gaussians(scene)
    r = qb.Rasterizer(scene.n, cam)                    # balance on
    r0 = qb.Rasterizer(scene.n, cam, balance=False)    # row-major
    r.forward(g, "quadbox", bg)
    r0.forward(g, "quadbox", bg)
    torch.cuda.synchronize()
    work = r.work.cpu().numpy().view(np.uint32).astype(np.int64)
    order = r.order.cpu().numpy().view(np.uint32).astype(np.int64)
    label = f"seed {seed} {w}x{h}"
    check_order(work, order, label)
    ref = oracle.forward(scene, cam, "quadbox", bg)
    assert np.array_equal(r.ranges.cpu().numpy().view(np.uint32).ravel(), ref["ranges"].ravel()), label
    want = work_reference(ref["g"], ref["ids"], ref["ranges"], w, h)
    lens = np.diff(ref["ranges"].reshape(-1, 2).astype(np.int64), axis=1)[:, 0]
    d = np.abs(work - want)
    close = d <= np.maximum(2.0, 0.01 * want)
    say(label, f"tiles {len(order)}, work max {work.max()}, close on {np.mean(close):.4f}, max diff {d.max():.1f}")
    assert np.all(work[lens == 0] == 0), label
    assert np.all(work <= lens), label
    assert np.mean(close) >= 0.98, label
    for name, v in qb.RENDER_VARIANTS.items():
        r.render_variant = r0.render_variant = v
        r.render(bg)
        r0.render(bg)
        torch.cuda.synchronize()
        for a, b in zip(outputs(r), outputs(r0)):
            assert torch.equal(a, b), (label, name)
    # backward in the forward's order against row-major
    dl = torch.tensor(scenes.target_image(seed, w, h), device="cuda") - r.image
    for name, v in qb.BACKWARD_VARIANTS.items():
        g1 = torch.empty((scene.n, 9), dtype=torch.float32, device="cuda")
        g0 = torch.empty_like(g1)
        qb.render_backward(w, h, r.ranges, r.ids_sorted, r.splats, bg, r.final_T, r.n_contrib, dl.contiguous(),
                           scene.n, g1, v, r.order)
        qb.render_backward(w, h, r0.ranges, r0.ids_sorted, r0.splats, bg, r0.final_T, r0.n_contrib,
                           dl.contiguous(), scene.n, g0, v, None)
        torch.cuda.synchronize()
        den = float(torch.linalg.norm(g0))
        rel = float(torch.linalg.norm(g1 - g0)) / max(den, 1e-30)
        assert rel <= 1e-5, (label, name, rel)


def test_tile_order_empty_frame(qb):
    """No visible Gaussian: every estimate is 0 and the order still covers
    every tile."""
    scene, _ = scenes.random_scene(204, 100, 64, 48, 64.0, sh_degree=0)
    scene.means[2] = -5.0   # behind the camera
    cam = scenes.pinhole(64, 48, 64.0)
    g = qb.Gaussians(scene)
    r = qb.Rasterizer(scene.n, cam)
    r.forward(g, "quadbox")
    torch.cuda.synchronize()
    assert r.pairs() == 0
    work = r.work.cpu().numpy()
    assert np.all(work == 0)
    check_order(work.astype(np.int64), r.order.cpu().numpy().astype(np.int64), "empty frame")


def test_tile_order_full_size_clusters(qb):
    """The headline frame (1M Gaussians, 1280x720) as the bench times it:
    the order is a permutation with non-increasing estimates and the render
    in that order equals the row-major render bit for bit."""
    scene, cam = scenes.cluster_scene()
    g = qb.Gaussians(scene)
    r = qb.Rasterizer(scene.n, cam, write_keys=False)
    r.forward(g, "quadbox")
    torch.cuda.synchronize()
    work = r.work.cpu().numpy().view(np.uint32).astype(np.int64)
    order = r.order.cpu().numpy().view(np.uint32).astype(np.int64)
    check_order(work, order, "clusters 1M")
    lens = np.diff(r.ranges.cpu().numpy().view(np.uint32).reshape(-1, 2).astype(np.int64), axis=1)[:, 0]
    assert np.all(work <= lens)
    say("clusters 1M: work mean", float(work.mean()), "max", int(work.max()), "heaviest tile", int(order[0]))
    ordered = outputs(r)
    r.balance = False
    r.render()
    torch.cuda.synchronize()
    for a, b in zip(ordered, outputs(r)):
        assert torch.equal(a, b)


def test_tile_order_views(qb):
    """One order over every tile of several views (different sizes): a
    permutation of all global tiles, each view's estimates equal to the
    single-view call's, images equal to the row-major batched render."""
    scene, _ = scenes.cluster_scene(seed=61, n=20_000, clusters=16, sigma=0.2, cube_centres=True)
    rng = np.random.Generator(np.random.PCG64(62))
    cams = []
    for w, h in [(96, 64), (160, 90), (200, 120), (123, 77)]:
        d = rng.normal(size=3)
        cams.append(scenes.look_at(3.0 * d / np.linalg.norm(d), width=w, height=h, focal=float(w)))
    g = qb.Gaussians(scene)
    mv = qb.MultiView(scene.n, cams)
    mv0 = qb.MultiView(scene.n, cams, balance=False)
    mv.size_pairs(g)
    mv0.size_pairs(g)
    mv.forward(g)
    mv0.forward(g)
    torch.cuda.synchronize()
    work = mv.work.cpu().numpy().view(np.uint32).astype(np.int64)
    check_order(work, mv.order.cpu().numpy().view(np.uint32).astype(np.int64), "views")
    o = 0
    for v, cam in enumerate(cams):
        r = qb.Rasterizer(scene.n, cam)
        r.forward(g, "quadbox")
        torch.cuda.synchronize()
        t = mv.num_tiles[v]
        assert np.array_equal(work[o:o + t], r.work.cpu().numpy().view(np.uint32).astype(np.int64)), v
        o += t
        assert torch.equal(mv.images[v], mv0.images[v]), v
        assert torch.equal(mv.n_contrib[v], mv0.n_contrib[v]), v


def test_tile_order_in_graph_replay(qb):
    """A single-view forward captured in a HIP graph recomputes the tile
    order on every replay: with the order overwritten between replays (every
    entry tile 0: in range, not a permutation) the replayed image still
    equals the eager one, and the estimates are rewritten."""
    scene, _ = scenes.random_scene(205, 8000, 300, 180, 300.0, sh_degree=1)
    cam = scenes.pinhole(300, 180, 300.0)
    g = qb.Gaussians(scene)
    r = qb.Rasterizer(scene.n, cam, write_keys=False)
    r.forward(g, "quadbox")
    torch.cuda.synchronize()
    r._alloc_pairs(r.pairs() + 1024)
    r.forward(g, "quadbox", sync_count=False)
    torch.cuda.synchronize()
    want, want_work = r.image.clone(), r.work.clone()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        r.forward(g, "quadbox", sync_count=False)
    torch.cuda.current_stream().wait_stream(side)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        r.forward(g, "quadbox", sync_count=False)
    for rep in range(3):
        r.image.fill_(-1.0)
        r.order.zero_()
        r.work.fill_(7)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(r.image, want), rep
        assert torch.equal(r.work, want_work), rep
        check_order(r.work.cpu().numpy().astype(np.int64), r.order.cpu().numpy().astype(np.int64), f"replay {rep}")
