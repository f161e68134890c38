"""qb_intersect_noalloc (the intersection for callers that cannot allocate)
against qb_intersect with a workspace: the same pair count, the same pairs
in the same order (bit for bit), on two calls in a row -- the 1M-Gaussian
clustered scene at 1280x720, then the 10k-Gaussian scene at 256x256 -- so
the second call runs over the first call's leftovers in the static scratch.
The sorted lists built from the no-alloc pairs also equal the oracle's."""
import numpy as np
import pytest
import torch

from paper_2605_04844_amd import quadbox as qb
from paper_2605_04844_amd import scenes

pytestmark = pytest.mark.gpu


def say(*a):
    print("[noalloc]", *a, flush=True)


def run_both(scene, cam, mode):
    g = qb.Gaussians(scene)
    r = qb.Rasterizer(scene.n, cam, write_keys=True)
    r.packed = False     # the reference pairs in qb_intersect's own format
    r.forward(g, mode)   # projection, and the reference pairs from qb_intersect
    torch.cuda.synchronize()
    P = r.pairs()
    assert 0 < P <= r.capacity
    want_tiles = r.pair_tiles[:P].clone()
    want_ids = r.pair_ids[:P].clone()
    tiles = torch.full((r.capacity,), -1, dtype=torch.int16, device="cuda")
    ids = torch.full((r.capacity,), -1, dtype=torch.int32, device="cuda")
    num = torch.full((1,), -5, dtype=torch.int64, device="cuda")
    qb.intersect_noalloc(scene.n, r.splats, r.rects, r.counts, r.W, r.H, r.capacity, tiles, ids, num, mode)
    torch.cuda.synchronize()
    assert int(num.item()) == P
    assert torch.equal(tiles[:P], want_tiles)
    assert torch.equal(ids[:P], want_ids)
    # the sort of the no-alloc pairs gives the oracle's sorted list
    r.pair_tiles.copy_(tiles)
    r.pair_ids.copy_(ids)
    r.num_pairs.copy_(num)
    r.sort()
    torch.cuda.synchronize()
    return r, P


def test_noalloc_matches_workspace_path_twice(oracle):
    scene, cam = scenes.cluster_scene()
    say("call 1: 1M Gaussians, 1280x720")
    r, P = run_both(scene, cam, "quadbox")
    say(f"call 1: {P} pairs equal qb_intersect's")
    del r
    scene, cam = scenes.small_scene()
    say("call 2: 10k Gaussians, 256x256")
    r, P = run_both(scene, cam, "quadbox")
    ref = oracle.forward(scene, cam, "quadbox")
    assert P == len(ref["keys"])
    assert np.array_equal(r.keys_sorted[:P].cpu().numpy().view(np.uint64), ref["keys"])
    assert np.array_equal(r.ids_sorted[:P].cpu().numpy().view(np.uint32), ref["ids"])
    say(f"call 2: {P} pairs equal qb_intersect's, sorted list equals the oracle's")


def test_noalloc_naive_and_empty():
    """The naive traversal mode, and n = 0 (writes a zero count)."""
    scene, cam = scenes.small_scene(n=3000)
    run_both(scene, cam, "quadbox_naive")
    num = torch.full((1,), 77, dtype=torch.int64, device="cuda")
    qb.intersect_noalloc(0, None, None, None, 256, 256, 0, None, None, num)
    torch.cuda.synchronize()
    assert int(num.item()) == 0
