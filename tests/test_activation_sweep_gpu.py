"""Exhaustive agreement of the projection's transcendental activations with
the oracle (bit for bit), on every binary32 value of the ranges that decide
keys and cutoffs: gamma = 2 ln(255 o) (Eq. (3)) for every o in (1/255, 1]
(the opacity-aware cull boundary and everything above it), the sigmoid for
every logit in [-5.6, 17], and exp for every log-scale in [-20, 5].  Both
sides evaluate in binary64 and round once, each with its own exp and log;
they could differ only where a last-ulp binary64 difference straddles a
binary32 rounding boundary.  The library evaluates the same device
functions qb_project uses (qb_activations)."""
import ctypes as C

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

CHUNK = 1 << 26


def bits_of(x):
    return int(np.float32(x).view(np.uint32))


def ranges():
    # (activation, first bit pattern, one past the last): binary32 patterns
    # of non-negative floats ascend with the value, of negative floats with
    # the magnitude
    one_255 = bits_of(np.float32(1.0) / np.float32(255.0))
    return [
        ("gamma", one_255 - 16, bits_of(1.0) + 1),
        ("opacity", 0, bits_of(17.0) + 1),
        ("opacity", 0x80000000, bits_of(-5.6) + 1),
        ("scale", 0, bits_of(5.0) + 1),
        ("scale", 0x80000000, bits_of(-20.0) + 1),
    ]


def test_activation_sweep_exhaustive(oracle):
    from paper_2605_04844_amd import quadbox as qb
    L = qb.lib()
    which = {"scale": 0, "opacity": 1, "gamma": 2}
    total = 0
    for name, lo, hi in ranges():
        bad = 0
        for a in range(lo, hi, CHUNK):
            b = min(hi, a + CHUNK)
            x = np.arange(a, b, dtype=np.uint32).view(np.float32)
            xg = torch.arange(a, b, dtype=torch.int64, device="cuda").to(torch.int32).view(torch.float32)
            out = torch.empty_like(xg)
            st = L.qb_activations(b - a, C.c_void_p(xg.data_ptr()), which[name], C.c_void_p(out.data_ptr()),
                                  C.c_void_p(torch.cuda.current_stream().cuda_stream))
            assert st == 0, st
            want = oracle.activations(x, name)
            got = out.cpu().numpy()
            diff = got.view(np.uint32) != want.view(np.uint32)
            if diff.any():
                i = np.nonzero(diff)[0][:5]
                print(f"[sweep] {name}: x {x[i]} gpu {got[i]} oracle {want[i]}", flush=True)
            bad += int(diff.sum())
        n = hi - lo
        total += n
        print(f"[sweep] {name} on {n} binary32 inputs [{np.uint32(lo).view(np.float32)}, "
              f"{np.uint32(hi - 1).view(np.float32)}]: {bad} differ", flush=True)
        assert bad == 0, (name, bad)
    print(f"[sweep] {total} inputs in all", flush=True)
