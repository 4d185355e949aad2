"""Batched views: one call over several views of different resolutions equals per-view calls
(bitwise), and the HIP-graph plan replays equal the eager calls."""
import numpy as np
import pytest

import scenes
from gpu_util import PARAMS, gpu_forward, renderer, to_device
from oracle import oracle

pytestmark = pytest.mark.gpu


def _views_scene():
    sc = scenes.multiview_scene(4, n=30000, views=6, nlayers=6)
    return sc


def test_batched_equals_per_view_forward(gpu):
    sc = _views_scene()
    batched, _, _ = gpu_forward(sc, gpu)
    for v, cam in enumerate(sc["cams"]):
        single, _, _ = gpu_forward(sc, gpu, cams=[cam])
        for k in range(3):
            assert np.array_equal(batched[v][k], single[0][k]), (v, k)


def test_batched_backward_is_sum_of_views(gpu):
    import torch
    sc = _views_scene()
    rb = renderer(sc, gpu)
    t = to_device(sc["points"], gpu)
    rb.forward(*[t[k] for k in PARAMS])
    G = torch.from_numpy(scenes.upstream_gradient(9, rb.pyramid_numel())).to(gpu)
    gb = rb.backward(*[t[k] for k in PARAMS], G)
    acc = None
    o = 0
    for v, cam in enumerate(sc["cams"]):
        rv = renderer(sc, gpu, cams=[cam])
        rv.forward(*[t[k] for k in PARAMS])
        n = rv.pyramid_numel()
        gv = rv.backward(*[t[k] for k in PARAMS], G[o:o + n].contiguous())
        o += n
        acc = [g.clone() for g in gv] if acc is None else [a + g for a, g in zip(acc, gv)]
    torch.cuda.synchronize()
    for k, a, b in zip(PARAMS, acc, gb):
        assert torch.equal(a, b), k


def test_graph_plan_replays_match_eager(gpu):
    import torch
    import paper_2401_06003_amd as tp
    sc = _views_scene()
    r = renderer(sc, gpu)
    t = to_device(sc["points"], gpu)
    args = [t[k] for k in PARAMS]
    ref = r.forward(*args).clone()
    G = torch.from_numpy(scenes.upstream_gradient(9, r.pyramid_numel())).to(gpu)
    gref = [g.clone() for g in r.backward(*args, G)]
    pyr = torch.empty_like(ref)
    grads = [torch.empty_like(g) for g in gref]
    plan = tp.Plan(r, *args, pyr, G, grads)
    for rep in range(3):
        pyr.fill_(-1.0)
        for g in grads:
            g.fill_(-1.0)
        plan.launch(forward=True, backward=True)
        torch.cuda.synchronize()
        assert torch.equal(pyr, ref), rep
        for a, b in zip(grads, gref):
            assert torch.equal(a, b), rep
        _ = (ref * 2).sum().item()  # unrelated eager work between replays


def test_sixteen_mixed_views_against_oracle(gpu):
    """16 views with mixed resolutions and uneven visible counts (near and far cameras)."""
    sc = scenes.multiview_scene(4, n=40000, views=16, nlayers=8)
    res, _, _ = gpu_forward(sc, gpu)
    for v, cam in enumerate(sc["cams"]):
        pyr, counts, ids = oracle.forward(sc["points"], cam, sc["nlayers"])
        assert np.array_equal(res[v][1], counts), v
        assert np.array_equal(res[v][2], ids), v
        assert np.all(np.abs(res[v][0] - pyr) <= 1e-5 * np.abs(pyr)), v


def test_autotuner_picks_a_candidate(gpu, tmp_path):
    import paper_2401_06003_amd as tp
    sc = scenes.unit_cube(8, n=5000, W=160, H=120, nlayers=5)
    t = to_device(sc["points"], gpu)
    cands = [(16, 4096, 4096), (32, 1024, 2048), (8, 2048, 8192)]
    cache = str(tmp_path / "tune.json")
    best, ms = tp.autotune(sc["cams"], sc["nlayers"], sc["D"], *[t[k] for k in PARAMS],
                           candidates=cands, reps=2, cache_path=cache, device=gpu)
    chosen = (best.tile_w, best.points_per_block, best.item_entries)
    assert chosen in cands and all(v > 0 for v in ms.values())
    assert chosen == min(ms, key=ms.get)
    again, _ = tp.autotune(sc["cams"], sc["nlayers"], sc["D"], *[t[k] for k in PARAMS],
                           candidates=cands, reps=2, cache_path=cache, device=gpu)  # from cache
    assert (again.tile_w, again.points_per_block, again.item_entries) == chosen
