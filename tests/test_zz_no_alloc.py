"""The forward entry point that allocates nothing (trips_forward_noalloc): through the C ABI,
against trips_forward on the same inputs, two calls in a row with the second smaller (the
static per-GPU scratch keeps the first call's contents): bit-identical pyramid, coverage,
list lengths and kept fragments, and a backward from its saved lists equal to the one from
trips_forward's."""
import numpy as np
import pytest

import scenes
from gpu_util import PARAMS, renderer, to_device

pytestmark = pytest.mark.gpu


def _pair(sc, dev):
    import torch
    a = renderer(sc, dev)
    b = renderer(sc, dev)
    t = to_device(sc["points"], dev)
    args = [t[k] for k in PARAMS]
    ca = torch.full((a.texels,), -1.0, device=dev)
    cb = torch.full((b.texels,), -1.0, device=dev)
    want = a.forward(*args, alpha_out=ca)
    got = b.forward_noalloc(*args, alpha_out=cb)
    wc, wi = a.export_fragments()
    gc, gi = b.export_fragments()
    G = torch.from_numpy(scenes.upstream_gradient(9, a.pyramid_numel())).to(dev)
    wg = a.backward(*args, G)
    gg = b.backward(*args, G)
    torch.cuda.synchronize()
    assert torch.equal(got, want)
    assert torch.equal(cb, ca)
    assert torch.equal(gc, wc) and torch.equal(gi, wi)
    for x, y in zip(gg, wg):
        assert torch.equal(x, y)
    return int(wc.sum())


def test_noalloc_forward_matches_forward_twice(gpu):
    big = scenes.cluster_scene(2)  # 2M points, 1920x1080, 8 layers
    small = scenes.unit_cube(1)    # 4096 points, 256x256, 5 layers
    print("noalloc: 2M points 1920x1080, then 4096 points 256x256", flush=True)
    assert _pair(big, gpu) > 10_000_000
    assert _pair(small, gpu) > 10_000
