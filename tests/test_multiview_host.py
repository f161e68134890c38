"""Host logic of MultiView (no GPU): each per-view call gets the workspaces
of the side stream it is issued on."""
import contextlib
import os
import sys

import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from paper_2605_04844_amd import quadbox as qb  # noqa: E402


def test_per_view_passes_the_stream_it_issues_on(monkeypatch):
    """A call's workspace slot is the stream it is issued on (two streams
    sharing one workspace would race), every view once."""
    class FakeStream:
        def __init__(self, i):
            self.i = i

        def wait_stream(self, other):
            pass

    current = []

    @contextlib.contextmanager
    def on(stream):
        current.append(stream.i)
        yield
        current.pop()

    monkeypatch.setattr(torch.cuda, "stream", on)
    monkeypatch.setattr(torch.cuda, "current_stream", lambda: FakeStream(-1))
    for V, S in [(9, 4), (32, 4), (3, 3)]:
        mv = qb.MultiView.__new__(qb.MultiView)
        mv.V, mv.S = V, S
        mv.streams = [FakeStream(i) for i in range(S)]
        seen = []
        mv._per_view(lambda v, slot: seen.append((v, slot, current[-1])))
        assert sorted(v for v, _, _ in seen) == list(range(V))
        assert all(slot == st for _, slot, st in seen)
    # without side streams every call runs on the current stream, slot 0
    mv.streams = []
    seen = []
    mv._per_view(lambda v, slot: seen.append((v, slot)))
    assert seen == [(v, 0) for v in range(mv.V)]
