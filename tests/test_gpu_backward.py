"""GPU backward parity: gradients for positions, sizes, opacities and descriptors against the
oracle's adjoint (double precision from the same single-precision fragments) and against
central finite differences of the double-precision oracle (relative error <= 1e-3)."""
import numpy as np
import pytest

import scenes
from gpu_util import GRAD_KEY, PARAMS, grad_close, renderer, to_device
from oracle import oracle
from test_oracle_backward import _fd_scene, _loss

pytestmark = pytest.mark.gpu


def _gpu_grads(sc, dev, G, tuning=None, cams=None):
    import torch
    r = renderer(sc, dev, tuning, cams)
    t = to_device(sc["points"], dev)
    r.forward(*[t[k] for k in PARAMS])
    g = torch.from_numpy(np.ascontiguousarray(G, dtype=np.float32).reshape(-1)).to(dev)
    outs = r.backward(*[t[k] for k in PARAMS], g)
    torch.cuda.synchronize()
    return {k: o.cpu().numpy().astype(np.float64) for k, o in zip(PARAMS, outs)}


def _check(sc, dev, seed=0, tuning=None):
    cam, nl = sc["cams"][0], sc["nlayers"]
    P = oracle.num_pixels(cam["W"], cam["H"], nl)
    G = scenes.upstream_gradient(seed, P * sc["D"]).reshape(P, sc["D"])
    got = _gpu_grads(sc, dev, G, tuning)
    ref = oracle.backward(sc["points"], cam, nl, G.astype(np.float64))
    for k in PARAMS:
        grad_close(got[k], ref[GRAD_KEY[k]].reshape(got[k].shape), k)
    return got


@pytest.mark.parametrize("seed", [0, 1])
@pytest.mark.parametrize("tile_w", [8, 16, 64])
def test_small_scenes(gpu, seed, tile_w):
    import paper_2401_06003_amd as tp
    sc = scenes.random_small(200 + seed, n=500, W=90, H=70, nlayers=5, s_lo=0.3, s_hi=24.0)
    _check(sc, gpu, seed, tp.make_tuning(tile_w, 0, 0))


def test_heavy_lists_items(gpu):
    import paper_2401_06003_amd as tp
    sc = scenes.random_small(8, n=5000, W=40, H=30, nlayers=4, s_lo=2.0, s_hi=12.0)
    _check(sc, gpu, 3, tp.make_tuning(16, 256, 256))


def test_unit_cube_4096(gpu):
    _check(scenes.unit_cube(1), gpu, 1)


def test_unit_cube_4096_small_launch_shape(gpu):
    """At the autotuner's launch shape for this workload (8x32 tiles, 512-point blocks,
    256-entry items)."""
    import paper_2401_06003_amd as tp
    _check(scenes.unit_cube(1), gpu, 1, tp.make_tuning(8, 512, 256))


def test_spatially_ordered_points(gpu):
    """A Morton-ordered cluster scene (consecutive points crowd the same texels) with work
    items small enough that heavy tiles are cut into several."""
    import paper_2401_06003_amd as tp
    sc = scenes.morton_sorted(scenes.cluster_scene(6, n=30_000, W=240, H=136, nlayers=5,
                                                   s_hi=48.0))
    _check(sc, gpu, 4, tp.make_tuning(16, 0, 512))


def test_descriptor_width_8(gpu):
    _check(scenes.unit_cube(5, n=2000, W=120, H=90, nlayers=5, D=8), gpu, 2)


def test_matches_central_differences(gpu):
    """The gradient accuracy bar: GPU gradients within 1e-3 of FP64 central differences."""
    seed, sc = _fd_scene()
    cam, n = sc["cams"][0], sc["nlayers"]
    P = oracle.num_pixels(cam["W"], cam["H"], n)
    G = np.random.default_rng(seed + 1000).standard_normal((P, sc["D"])).astype(np.float32)
    got = _gpu_grads(sc, gpu, G)
    pts = {k: np.asarray(v, dtype=np.float64).copy() for k, v in sc["points"].items()}
    G64 = G.astype(np.float64)
    for name in PARAMS:
        arr = pts[name]
        fd = np.zeros_like(arr)
        flat, fdf = arr.reshape(-1), fd.reshape(-1)
        for k in range(flat.size):
            old = flat[k]
            h = 1e-6 * max(1.0, abs(old))
            flat[k] = old + h
            lp = _loss(pts, cam, n, G64)
            flat[k] = old - h
            lm = _loss(pts, cam, n, G64)
            flat[k] = old
            fdf[k] = (lp - lm) / (2 * h)
        g = got[name].reshape(fd.shape)
        rel = np.linalg.norm(g - fd) / np.linalg.norm(fd)
        assert rel <= 1e-3, (name, rel)


def test_backward_twice_bitwise(gpu):
    sc = scenes.unit_cube(3, n=3000, W=128, H=96)
    cam = sc["cams"][0]
    P = oracle.num_pixels(cam["W"], cam["H"], sc["nlayers"])
    G = scenes.upstream_gradient(4, P * 4).reshape(P, 4)
    a = _gpu_grads(sc, gpu, G)
    b = _gpu_grads(sc, gpu, G)
    for k in PARAMS:
        assert np.array_equal(a[k], b[k]), k


def test_culled_points_get_zero(gpu):
    sc = scenes.random_small(9, n=300, W=64, H=48, nlayers=4)
    sc["points"]["z"][:20] = -1.0
    got = _check(sc, gpu, 5)
    for k in PARAMS:
        assert np.all(got[k][:20] == 0)


def test_cluster_scene_full_size_sampled_points(gpu):
    """2M points at 1920x1080: gradients of a sample of points, each exact in the oracle
    because every texel the point writes is evaluated."""
    sc = scenes.cluster_scene(2)
    cam, nl = sc["cams"][0], sc["nlayers"]
    P = oracle.num_pixels(cam["W"], cam["H"], nl)
    G = scenes.upstream_gradient(3, P * 4).reshape(P, 4)
    got = _gpu_grads(sc, gpu, G)
    rng = np.random.default_rng(1)
    pick = rng.choice(len(sc["points"]["x"]), 400, replace=False)
    sub = {k: v[pick] for k, v in sc["points"].items()}
    fr = oracle.fragments(sub, cam, nl)
    mask = np.zeros(P, dtype=np.uint8)
    mask[oracle.texel_index(cam, nl, fr["L"], fr["i"], fr["j"])] = 1
    ref = oracle.backward(sc["points"], cam, nl, G.astype(np.float64), mask=mask)
    for k in PARAMS:
        grad_close(got[k][pick], ref[GRAD_KEY[k]][pick].reshape(got[k][pick].shape), k)
