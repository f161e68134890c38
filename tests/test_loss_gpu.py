"""qb_l1_grad against torch's sign: the image gradient of the L1 loss that
drives the render backward in training (Sec. 4.1), value for value, over items of
several sizes in one launch (vector and scalar paths, equal values and
signed zeros)."""
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


def test_l1_grad_matches_torch_sign(qb):
    rng = np.random.default_rng(3)
    dev = torch.device("cuda")
    sizes = [3 * 360 * 640, 1001, 0, 3 * 720 * 1280, 7, 4]
    items, want = [], []
    base = torch.empty(4 + sum(sizes), dtype=torch.float32, device=dev)   # room for a misaligned slice
    for k, m in enumerate(sizes):
        img = torch.from_numpy(rng.uniform(0, 1, m).astype(np.float32)).to(dev)
        tgt = torch.from_numpy(rng.uniform(0, 1, m).astype(np.float32)).to(dev)
        if m:
            eq = torch.from_numpy(rng.random(m) < 0.1).to(dev)
            tgt = torch.where(eq, img, tgt)                    # equal values: sign 0
            img[: min(m, 2)] = torch.tensor([0.0, -0.0], device=dev)[: min(m, 2)]
            tgt[: min(m, 2)] = torch.tensor([-0.0, 0.0], device=dev)[: min(m, 2)]
        if k == 1:   # one item misaligned by one element: the scalar path
            img = base[1:1 + m].copy_(img)
        grad = torch.full((m,), 7.0, dtype=torch.float32, device=dev)
        scale = 1.0 / max(m, 1)
        items.append((img, tgt, grad, scale))
        want.append(torch.sign(img - tgt) * scale)
    qb.l1_grad(items)
    torch.cuda.synchronize()
    for (img, tgt, grad, scale), w in zip(items, want):
        got, ref = grad.cpu().numpy(), w.cpu().numpy()
        # exactly +scale, -scale or zero where torch has them (its zero may
        # carry a sign; qb_l1_grad writes +0)
        assert np.array_equal(got, ref), (img.numel(), np.nonzero(got != ref)[0][:5])
        assert not np.signbit(got[got == 0]).any()
