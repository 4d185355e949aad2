"""GPU parity at the full sizes of the target workloads, through the C ABI, against the oracle
on the same seeded inputs (Sec. 3.1-3.2, Eq. 2-7; the adjoint of Eq. 6-7 through Eq. 2-5):

- 8M points at 1920x1080, 8 layers, D = 4, forward + backward: every texel's list length
  and kept ids exactly, every colour within 1e-5, every gradient of every point;
- the 16-view, 4M-point batched workload at full size with a non-default launch shape: four
  of its views (the largest and smallest resolution, the nearest and farthest camera) on a
  random 2% of their texels, and every point's gradient exactly for that texel set (the
  upstream gradient is zero elsewhere);
- clouds that write nothing (no points, every point culled), forward and backward;
- a view with more tiles than the scatter pass can stage in LDS (its unstaged path)."""
import numpy as np
import pytest

import scenes
from gpu_util import (GRAD_KEY, PARAMS, assert_lists, assert_pyramid, grad_close, renderer,
                      to_device)
from oracle import oracle, parallel

pytestmark = pytest.mark.gpu


def _run(sc, dev, G, tuning=None, cams=None):
    """Forward, export and backward of one call; numpy results."""
    import torch
    r = renderer(sc, dev, tuning, cams)
    t = to_device(sc["points"], dev)
    args = [t[k] for k in PARAMS]
    pyr = r.forward(*args)
    counts, ids = r.export_fragments()
    g = torch.from_numpy(np.ascontiguousarray(G, dtype=np.float32).reshape(-1)).to(dev)
    outs = r.backward(*args, g)
    torch.cuda.synchronize()
    got = {"pyr": pyr.cpu().numpy().astype(np.float64).reshape(-1, sc["D"]),
           "counts": counts.cpu().numpy(), "ids": ids.cpu().numpy().astype(np.int64)}
    for k, o in zip(PARAMS, outs):
        got[k] = o.cpu().numpy().astype(np.float64)
    return got, r


def test_target_8m_points_1080p(gpu):
    sc = scenes.cluster_scene(2, n=8_000_000)
    cam, nl, D = sc["cams"][0], sc["nlayers"], sc["D"]
    P = oracle.num_pixels(cam["W"], cam["H"], nl)
    G = scenes.upstream_gradient(3, P * D).reshape(P, D)
    got, _ = _run(sc, gpu, G)
    f = parallel.forward(sc["points"], cam, nl)
    assert_lists(got["counts"], got["ids"], f["counts"], f["ids"], "8M")
    assert_pyramid(got["pyr"], f["pyr"], "8M")
    assert f["counts"].sum() > 40_000_000  # the fragments of 8M points were compared
    b = parallel.backward(sc["points"], cam, nl, G.astype(np.float64))
    for k in PARAMS:
        grad_close(got[k], b[GRAD_KEY[k]].reshape(got[k].shape), "8M " + k)


def _eye(cam):
    R = np.asarray(cam["R"], dtype=np.float64).reshape(3, 3)
    return -R.T @ np.asarray(cam["t"], dtype=np.float64).reshape(3)


def test_multiview_4m_points_16_views_sampled(gpu):
    import paper_2401_06003_amd as tp
    sc = scenes.multiview_scene(4, n=4_000_000, views=16, nlayers=8)
    pts, cams, nl, D = sc["points"], sc["cams"], sc["nlayers"], sc["D"]
    area = [c["W"] * c["H"] for c in cams]
    dist = [float(np.linalg.norm(_eye(c))) for c in cams]
    checked = sorted({int(np.argmax(area)), int(np.argmin(area)), int(np.argmin(dist)),
                      int(np.argmax(dist))})
    sizes = [oracle.num_pixels(c["W"], c["H"], nl) for c in cams]
    offs = np.cumsum([0] + sizes)
    rng = np.random.default_rng(44)
    masks = {v: (rng.random(sizes[v]) < 0.02).astype(np.uint8) for v in checked}
    G = np.zeros((offs[-1], D), dtype=np.float32)
    for v in checked:
        sel = np.nonzero(masks[v])[0]
        G[offs[v] + sel] = rng.standard_normal((len(sel), D)).astype(np.float32)
    got, _ = _run(sc, gpu, G, tuning=tp.make_tuning(32, 8192, 16384))
    want = {k: 0.0 for k in PARAMS}
    kept = 0
    for v in checked:
        m = masks[v].astype(bool)
        a, b = offs[v], offs[v + 1]
        f = parallel.forward(pts, cams[v], nl, mask=masks[v])
        assert_lists(got["counts"][a:b][m], got["ids"][a:b][m], f["counts"][m], f["ids"][m],
                     "view %d" % v)
        assert_pyramid(got["pyr"][a:b][m], f["pyr"][m], "view %d" % v)
        kept += int((f["ids"][m] >= 0).sum())
        g = parallel.backward(pts, cams[v], nl, G[a:b].astype(np.float64), mask=masks[v])
        for k in PARAMS:
            want[k] = want[k] + g[GRAD_KEY[k]].reshape(got[k].shape)
    assert kept > 10000
    for k in PARAMS:
        grad_close(got[k], want[k], k)


@pytest.mark.parametrize("case", ["no_points", "all_culled"])
def test_clouds_that_write_nothing(gpu, case):
    """Forward and backward of a cloud with no fragments: empty lists, a zero pyramid (with a
    background: the background itself), zero point and camera gradients, and the whole
    upstream gradient on the background."""
    import torch
    sc = scenes.random_small(5, n=0 if case == "no_points" else 200, W=70, H=45, nlayers=5)
    if case == "all_culled":
        sc["points"]["z"][:] = -1.0
    r = renderer(sc, gpu)
    t = to_device(sc["points"], gpu)
    args = [t[k] for k in PARAMS]
    P, D, n = r.texels, sc["D"], len(sc["points"]["x"])
    rng = np.random.default_rng(6)
    bg = torch.from_numpy(rng.uniform(0, 1, P * D).astype(np.float32)).to(gpu)
    G = torch.from_numpy(rng.standard_normal(P * D).astype(np.float32)).to(gpu)
    for with_bg in (False, True):
        alpha = torch.full((P,), -1.0, device=gpu)
        pyr = r.forward(*args, background=bg if with_bg else None, alpha_out=alpha)
        counts, ids = r.export_fragments()
        gbg = torch.full((P * D,), -1.0, device=gpu)
        gcam = torch.full((1, 16), -1.0, device=gpu)
        outs = r.backward(*args, G, background=bg if with_bg else None, grad_background=gbg,
                          grad_camera=gcam)
        torch.cuda.synchronize()
        assert torch.equal(pyr, bg if with_bg else torch.zeros_like(pyr))
        assert torch.all(alpha == 0) and torch.all(counts == 0) and torch.all(ids == -1)
        assert torch.equal(gbg, G) and torch.all(gcam == 0)
        for o in outs:
            assert o.numel() == n * (D if o.dim() == 2 else 1) and torch.all(o == 0)


def test_view_beyond_staged_scatter(gpu):
    """3200x1600, 8 layers: 26,704 tiles of 16x16, more than the scatter pass stages in LDS,
    so the block's bin positions are read per entry; lists, colours and gradients."""
    sc = scenes.random_small(12, n=20000, W=3200, H=1600, nlayers=8, s_lo=0.3, s_hi=80.0)
    cam, nl, D = sc["cams"][0], sc["nlayers"], sc["D"]
    tiles = sum(-(-w // 16) * -(-h // 16) for w, h in oracle.layer_dims(cam["W"], cam["H"], nl))
    assert 26214 < tiles <= 32768, tiles
    P = oracle.num_pixels(cam["W"], cam["H"], nl)
    G = scenes.upstream_gradient(13, P * D).reshape(P, D)
    got, _ = _run(sc, gpu, G)
    f = parallel.forward(sc["points"], cam, nl)
    assert_lists(got["counts"], got["ids"], f["counts"], f["ids"], "unstaged")
    assert_pyramid(got["pyr"], f["pyr"], "unstaged")
    b = parallel.backward(sc["points"], cam, nl, G.astype(np.float64))
    for k in PARAMS:
        grad_close(got[k], b[GRAD_KEY[k]].reshape(got[k].shape), k)
