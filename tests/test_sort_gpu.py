"""GPU checks of qb_sort on synthetic pair lists, against the definition of
SortPairs (Sec. 2): the pairs arrive in emission order, so the sorted ids are
the stable sort of that order by tile, and the ranges are the oracle's
per-tile first/last-index definition over the sorted keys.  The tile patterns
stress the radix passes where they differ: every pair in one tile (one digit
everywhere, the longest runs of equal digits in the histogram pass), a
sawtooth over all tiles (every neighbour a different digit), runs of 37
equal tiles (runs that straddle the 8-pair lane groups and the 4096-pair
workgroups), and uniform random tiles; counts from 1 to 1M include ragged
tails that are not whole lane groups or workgroups.  Every launch shape of
qb_sort_ex (radix workgroups of 4096 to 8192 pairs) is checked, on split
pairs and, where tile and id fit 32 bits, on packed ones; 3M packed pairs
over 1000 tiles take more radix workgroups than one workgroup's prologue
scans itself (the scan launches).  Bit-exact."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def qb():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2605_04844_amd import quadbox
    quadbox.lib()
    return quadbox


def patterns(seed, n, tiles):
    rng = np.random.Generator(np.random.PCG64(seed))
    yield "one tile", np.full(n, tiles - 1, np.uint16)
    yield "sawtooth", (np.arange(n) % tiles).astype(np.uint16)
    yield "runs of 37", np.repeat(rng.integers(0, tiles, n // 37 + 1), 37)[:n].astype(np.uint16)
    yield "random", rng.integers(0, tiles, n).astype(np.uint16)


@pytest.mark.parametrize("n,tiles", [(1, 1), (5, 1), (4095, 3600), (4096 * 3 + 17, 3600), (200_003, 65536),
                                     (1_000_000, 3600), (1_000_000, 64), (3_000_017, 1000)])
def test_sort_synthetic_tiles(oracle, qb, n, tiles):
    cap = n + 100
    ws = torch.empty(qb.sort_workspace_size(cap), dtype=torch.uint8, device="cuda")
    num_pairs = torch.tensor([n], dtype=torch.int64, device="cuda")
    ids_in = np.arange(n, dtype=np.uint32)   # emission order
    for name, t in patterns(n, n, tiles):
        print(f"[sort] n {n} tiles {tiles} {name}", flush=True)
        pt = torch.zeros(cap, dtype=torch.int16, device="cuda")
        pt[:n] = torch.from_numpy(t.view(np.int16)).cuda()
        pi = torch.zeros(cap, dtype=torch.int32, device="cuda")
        pi[:n] = torch.from_numpy(ids_in.view(np.int32)).cuda()
        order = np.argsort(t, kind="stable")
        want_ids = ids_in[order]
        want_ranges = oracle.ranges(t[order].astype(np.uint64) << np.uint64(32), tiles)
        for shape, variant in qb.SORT_VARIANTS.items():
            ids = torch.full((cap,), -1, dtype=torch.int32, device="cuda")
            ranges = torch.full((tiles * 2,), -1, dtype=torch.int32, device="cuda")
            qb.sort(cap, num_pairs, tiles, pt, pi, None, None, ids, ranges, ws, variant)
            torch.cuda.synchronize()
            got_ids = ids.cpu().numpy().view(np.uint32)[:n]
            assert np.array_equal(got_ids, want_ids), (n, tiles, name, shape)
            assert np.array_equal(ranges.cpu().numpy().view(np.uint32).reshape(-1, 2), want_ranges), \
                (n, tiles, name, shape)
            # the input lists are left as they were
            assert np.array_equal(pt[:n].cpu().numpy().view(np.uint16), t), (n, tiles, name, shape)
        # the same pairs packed as tile << bits | id (where they fit 32 bits)
        bits = max(1, int(np.ceil(np.log2(max(n, 2)))))
        tbits = int(np.ceil(np.log2(tiles))) if tiles > 1 else 0
        if bits + tbits > 32:
            continue
        packed = (t.astype(np.uint64) << np.uint64(bits)) | ids_in.astype(np.uint64)
        pk = torch.zeros(cap, dtype=torch.int32, device="cuda")
        pk[:n] = torch.from_numpy(packed.astype(np.uint32).view(np.int32)).cuda()
        for shape, variant in qb.SORT_VARIANTS.items():
            ids = torch.full((cap,), -1, dtype=torch.int32, device="cuda")
            ranges = torch.full((tiles * 2,), -1, dtype=torch.int32, device="cuda")
            qb.sort(cap, num_pairs, tiles, None, pk, None, None, ids, ranges, ws, variant, bits)
            torch.cuda.synchronize()
            got_ids = ids.cpu().numpy().view(np.uint32)[:n]
            assert np.array_equal(got_ids, want_ids), (n, tiles, name, shape, "packed")
            assert np.array_equal(ranges.cpu().numpy().view(np.uint32).reshape(-1, 2), want_ranges), \
                (n, tiles, name, shape, "packed")
