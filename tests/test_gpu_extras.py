"""GPU parity of the optional terms through the C ABI: a background composited behind the
kept fragments, the coverage 1 - T_K, their gradients and the camera gradient, against the
oracle's extended entry points on the same seeded inputs; batched views equal per-view
calls bit for bit, and a captured plan equals the eager calls bit for bit."""
import numpy as np
import pytest

import scenes
from gpu_util import GRAD_KEY, PARAMS, assert_lists, assert_pyramid, grad_close, renderer, to_device
from oracle import oracle

pytestmark = pytest.mark.gpu

# coverage = 1 - T_K with T_K a product of at most 16 single-precision factors
ALPHA_ATOL = 1e-5


def _inputs(P, D, seed):
    rng = np.random.default_rng(seed)
    bg = rng.uniform(0.0, 1.0, (P, D)).astype(np.float32)
    G = scenes.upstream_gradient(seed, P * D).reshape(P, D).astype(np.float32)
    Ga = rng.standard_normal(P).astype(np.float32)
    return bg, G, Ga


def _gpu(sc, dev, bg, G, Ga, tuning=None, cams=None):
    import torch
    r = renderer(sc, dev, tuning, cams)
    t = to_device(sc["points"], dev)
    args = [t[k] for k in PARAMS]
    P, D = r.texels, sc["D"]
    bgt = torch.from_numpy(np.ascontiguousarray(bg).reshape(-1)).to(dev)
    alpha = torch.empty(P, device=dev)
    pyr = r.forward(*args, background=bgt, alpha_out=alpha)
    counts, ids = r.export_fragments()
    g = torch.from_numpy(np.ascontiguousarray(G).reshape(-1)).to(dev)
    ga = torch.from_numpy(np.ascontiguousarray(Ga)).to(dev)
    gbg = torch.empty(P * D, device=dev)
    gcam = torch.empty((r.V, 16), device=dev)
    outs = r.backward(*args, g, background=bgt, grad_alpha=ga, grad_background=gbg,
                      grad_camera=gcam)
    torch.cuda.synchronize()
    res = {"pyr": pyr.cpu().numpy().astype(np.float64).reshape(P, D),
           "coverage": alpha.cpu().numpy().astype(np.float64), "counts": counts.cpu().numpy(),
           "ids": ids.cpu().numpy().astype(np.int64),
           "gbg": gbg.cpu().numpy().astype(np.float64).reshape(P, D),
           "gcam": gcam.cpu().numpy().astype(np.float64)}
    for k, o in zip(PARAMS, outs):
        res[k] = o.cpu().numpy().astype(np.float64)
    return res


def _check_view(got, sc, cam, bg, G, Ga, where=""):
    nl = sc["nlayers"]
    f = oracle.forward_ex(sc["points"], cam, nl, background=bg.astype(np.float64))
    assert_lists(got["counts"], got["ids"], f["counts"], f["ids"], where)
    assert_pyramid(got["pyr"], f["pyr"], where)
    assert np.abs(got["coverage"] - f["alpha"]).max() <= ALPHA_ATOL, where
    b = oracle.backward_ex(sc["points"], cam, nl, G.astype(np.float64),
                           background=bg.astype(np.float64), grad_alpha=Ga.astype(np.float64))
    for k in PARAMS:
        grad_close(got[k], b[GRAD_KEY[k]].reshape(got[k].shape), where + k)
    grad_close(got["gbg"], b["gbg"], where + "gbg")
    # camera: sums over every point of products with mixed signs
    grad_close(got["gcam"].reshape(-1), b["gcam"], where + "gcam", rtol_norm=1e-4, rtol=1e-2,
               atol_rel=1e-4)


@pytest.mark.parametrize("seed", [0, 1])
@pytest.mark.parametrize("tile_w", [8, 16])
def test_small_scenes(gpu, seed, tile_w):
    import paper_2401_06003_amd as tp
    sc = scenes.random_small(300 + seed, n=500, W=90, H=70, nlayers=5, s_lo=0.3, s_hi=24.0)
    cam = sc["cams"][0]
    P = oracle.num_pixels(cam["W"], cam["H"], sc["nlayers"])
    bg, G, Ga = _inputs(P, sc["D"], seed + 10)
    got = _gpu(sc, gpu, bg, G, Ga, tp.make_tuning(tile_w, 0, 0))
    got["gcam"] = got["gcam"][0]
    _check_view(got, sc, cam, bg, G, Ga)


def test_heavy_lists_items(gpu):
    """Long lists cut into several work items (partial lists merged)."""
    import paper_2401_06003_amd as tp
    sc = scenes.random_small(9, n=5000, W=40, H=30, nlayers=4, s_lo=2.0, s_hi=12.0)
    cam = sc["cams"][0]
    P = oracle.num_pixels(cam["W"], cam["H"], sc["nlayers"])
    bg, G, Ga = _inputs(P, sc["D"], 21)
    got = _gpu(sc, gpu, bg, G, Ga, tp.make_tuning(16, 256, 256))
    got["gcam"] = got["gcam"][0]
    _check_view(got, sc, cam, bg, G, Ga)


def test_descriptor_width_8_rotated_camera(gpu):
    sc = scenes.unit_cube(6, n=2000, W=120, H=90, nlayers=5, D=8)
    cam = dict(sc["cams"][0])
    a = 0.2
    cam["R"] = np.array([[np.cos(a), 0, np.sin(a)], [0, 1, 0], [-np.sin(a), 0, np.cos(a)]])
    sc = dict(sc, cams=[cam])
    P = oracle.num_pixels(cam["W"], cam["H"], sc["nlayers"])
    bg, G, Ga = _inputs(P, 8, 22)
    got = _gpu(sc, gpu, bg, G, Ga)
    got["gcam"] = got["gcam"][0]
    _check_view(got, sc, cam, bg, G, Ga)


def _three_cams(sc):
    c0 = sc["cams"][0]
    c1 = dict(c0, t=np.asarray(c0["t"], dtype=np.float64) + np.array([0.05, -0.03, 0.1]))
    c2 = scenes.camera(np.eye(3), (0.02, 0.01, 0.0), 64, 48, 50.0)
    return [c0, c1, c2]


def test_batched_equals_per_view_bitwise(gpu):
    sc = scenes.random_small(31, n=800, W=80, H=60, nlayers=5, s_lo=0.3, s_hi=20.0)
    cams = _three_cams(sc)
    Ps = [oracle.num_pixels(c["W"], c["H"], sc["nlayers"]) for c in cams]
    ins = [_inputs(P, sc["D"], 40 + v) for v, P in enumerate(Ps)]
    bg = np.concatenate([i[0] for i in ins])
    G = np.concatenate([i[1] for i in ins])
    Ga = np.concatenate([i[2] for i in ins])
    batched = _gpu(sc, gpu, bg, G, Ga, cams=cams)
    o = 0
    for v, (c, P) in enumerate(zip(cams, Ps)):
        one = _gpu(sc, gpu, ins[v][0], ins[v][1], ins[v][2], cams=[c])
        for k in ("pyr", "coverage", "gbg", "counts", "ids"):
            assert np.array_equal(batched[k][o:o + P], one[k]), (v, k)
        assert np.array_equal(batched["gcam"][v], one["gcam"][0]), v
        o += P


def test_plan_replays_equal_eager(gpu):
    import torch
    import paper_2401_06003_amd as tp
    sc = scenes.random_small(32, n=600, W=70, H=50, nlayers=5)
    cams = _three_cams(sc)[:2]
    r = renderer(sc, gpu, cams=cams)
    t = to_device(sc["points"], gpu)
    args = [t[k] for k in PARAMS]
    P, D, n = r.texels, sc["D"], len(sc["points"]["x"])
    bg, G, Ga = (torch.from_numpy(np.ascontiguousarray(a).reshape(-1)).to(gpu)
                 for a in _inputs(P, D, 50))
    eager_alpha = torch.empty(P, device=gpu)
    eager_pyr = r.forward(*args, background=bg, alpha_out=eager_alpha).clone()
    eg = torch.empty(P * D, device=gpu)
    ec = torch.empty((2, 16), device=gpu)
    eager = [o.clone() for o in r.backward(*args, G, background=bg, grad_alpha=Ga,
                                           grad_background=eg, grad_camera=ec)]
    pyr = torch.empty(P * D, device=gpu)
    alpha = torch.empty(P, device=gpu)
    gbg = torch.empty(P * D, device=gpu)
    gcam = torch.empty((2, 16), device=gpu)
    grads = [torch.empty(n, device=gpu) for _ in range(5)] + [torch.empty((n, D), device=gpu)]
    plan = tp.Plan(r, *args, pyr, G, grads, background=bg, alpha_out=alpha, grad_alpha=Ga,
                   grad_background=gbg, grad_camera=gcam)
    for _ in range(3):
        for x in (pyr, alpha, gbg, gcam, *grads):
            x.fill_(-7.0)
        plan.launch(forward=True, backward=True)
        torch.cuda.synchronize()
        assert torch.equal(pyr, eager_pyr) and torch.equal(alpha, eager_alpha)
        assert torch.equal(gbg, eg) and torch.equal(gcam, ec)
        for a, b in zip(grads, eager):
            assert torch.equal(a, b)


def test_full_size_coverage_and_camera_gradient(gpu):
    """The 2M-point 1080p scene (forward + backward, Sec. 3.1-3.2, Eq. 6-7) with a
    background, against the oracle evaluated on every texel: every texel's list length and
    kept ids exactly, its colour and coverage, and every gradient (all six point arrays, the
    background and the camera, a sum over all points)."""
    from oracle import parallel
    sc = scenes.cluster_scene(2)
    cam, nl, D = sc["cams"][0], sc["nlayers"], sc["D"]
    P = oracle.num_pixels(cam["W"], cam["H"], nl)
    bg, G, Ga = _inputs(P, D, 60)
    got = _gpu(sc, gpu, bg, G, Ga)
    f = parallel.forward(sc["points"], cam, nl, background=bg.astype(np.float64))
    assert_lists(got["counts"], got["ids"], f["counts"], f["ids"], "full size")
    assert np.abs(got["coverage"] - f["alpha"]).max() <= ALPHA_ATOL
    assert_pyramid(got["pyr"], f["pyr"], "full size")
    b = parallel.backward(sc["points"], cam, nl, G.astype(np.float64),
                          background=bg.astype(np.float64), grad_alpha=Ga.astype(np.float64))
    for k in PARAMS:
        grad_close(got[k], b[GRAD_KEY[k]].reshape(got[k].shape), k)
    grad_close(got["gcam"][0], b["gcam"], "gcam", rtol_norm=1e-4, rtol=1e-2, atol_rel=1e-4)
    grad_close(got["gbg"], b["gbg"], "gbg")
