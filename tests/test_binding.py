"""Host-side checks of the Python binding (no GPU): the autograd function refuses to
differentiate a forward call whose saved fragment lists a later forward overwrote.

The library's compute entry points are replaced by stand-ins that return success without
launching anything, so only the binding's own bookkeeping runs."""
import ctypes
import os

import pytest


def _tp(monkeypatch):
    import paper_2401_06003_amd as tp
    if not os.path.exists(tp.LIB_PATH):
        pytest.skip("libtrips.so not built")
    real = tp.lib()

    class NoLaunch:
        def __getattr__(self, name):
            return getattr(real, name)

        def trips_forward(self, *args):
            return 0

        def trips_backward(self, *args):
            return 0

    monkeypatch.setattr(tp, "_lib", NoLaunch())
    monkeypatch.setattr(tp, "_stream", lambda: ctypes.c_void_p(0))
    return tp


def _inputs(n, D):
    import torch
    t = [torch.rand(n, requires_grad=True) for _ in range(5)]
    t.append(torch.rand(n, D, requires_grad=True))
    return t


def _cam():
    import scenes
    return scenes.camera([[1, 0, 0], [0, 1, 0], [0, 0, 1]], (0, 0, 3), 32, 24)


def test_stale_saved_lists_raise(monkeypatch):
    tp = _tp(monkeypatch)
    r = tp.Renderer([_cam()], 3, 4, 10, device="cpu")
    a = _inputs(10, 4)
    first = tp.render(*a, r)
    second = tp.render(*a, r)
    second.sum().backward()  # the latest forward: fine
    with pytest.raises(RuntimeError, match="overwritten"):
        first.sum().backward()


def test_shared_buffers_share_the_check(monkeypatch):
    tp = _tp(monkeypatch)
    r = tp.Renderer([_cam()], 3, 4, 10, device="cpu")
    r2 = tp.Renderer([_cam()], 3, 4, 10, device="cpu", share_buffers_with=r)
    assert r2.saved is r.saved
    a = _inputs(10, 4)
    out = tp.render(*a, r)
    tp.render(*a, r2).sum().backward()
    with pytest.raises(RuntimeError, match="overwritten"):
        out.sum().backward()


def test_backward_twice_of_the_same_forward(monkeypatch):
    tp = _tp(monkeypatch)
    r = tp.Renderer([_cam()], 3, 4, 10, device="cpu")
    a = _inputs(10, 4)
    out = tp.render(*a, r)
    out.sum().backward(retain_graph=True)
    out.sum().backward()  # nothing overwrote the lists in between


def test_separate_buffers_do_not_interfere(monkeypatch):
    tp = _tp(monkeypatch)
    r = tp.Renderer([_cam()], 3, 4, 10, device="cpu")
    r2 = tp.Renderer([_cam()], 3, 4, 10, device="cpu")
    a = _inputs(10, 4)
    out = tp.render(*a, r)
    tp.render(*a, r2)
    out.sum().backward()
