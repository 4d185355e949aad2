"""Pins of the oracle's analytic adjoint.

The paper states the renderer is differentiable in point positions, sizes, descriptors
and opacities but prints no gradient formulas; the adjoint is pinned by
  - central finite differences of the double-precision oracle forward on a 64-point,
    32x32 subset drawn by the cluster recipe (kinks kept away from the step), and
  - closed forms of one- and two-fragment texels (Eq. 6-7 differentiated by hand).
"""
import math

import numpy as np
import pytest

import exact_points as ep
import scenes
from oracle import oracle

PARAMS = ("x", "y", "z", "sw", "alpha", "desc")
GRAD_OF = {"x": "gx", "y": "gy", "z": "gz", "sw": "gsw", "alpha": "galpha", "desc": "gdesc"}


def _margins_ok(pts, cam, nlayers, margin=1e-3, zgap=1e-4):
    """True if no fragment is within `margin` of a kink or discontinuity (double precision)."""
    valid, xyzs = oracle.project(pts, cam, nlayers, fp32=False)
    if not valid.all():
        return False
    W, H = cam["W"], cam["H"]
    smax = 2.0 ** (nlayers - 1)
    for p in range(len(valid)):
        x, y, z, s = xyzs[p]
        if abs(s - 1.0) <= margin or s >= smax - margin:
            return False
        if s >= 1.0:
            e = math.floor(math.log2(s))
            t = s / 2.0 ** e
            if abs(t - 1.0) <= margin or abs(t - 2.0) <= margin:
                return False
            layers = [e, e + 1]
        else:
            layers = [0]
        for L in layers:
            for q, ext in ((x, W), (y, H)):
                u = q / 2.0 ** L - 0.5
                f = u - math.floor(u)
                if f <= margin or f >= 1.0 - margin:
                    return False
    fr = oracle.fragments(pts, cam, nlayers, fp32=False)
    dims = oracle.layer_dims(W, H, nlayers)
    base = np.cumsum([0] + [w * h for w, h in dims])
    pix = base[fr["L"]] + fr["j"] * np.array([dims[L][0] for L in fr["L"]]) + fr["i"]
    for p in np.unique(pix):
        zz = fr["z"][pix == p]
        if len(zz) > 16:
            return False
        if len(zz) > 1 and np.min(np.diff(np.sort(zz))) <= zgap:
            return False
    return True


def _fd_scene():
    for seed in range(33, 333):
        sc = scenes.fd_candidate(seed)
        if _margins_ok(sc["points"], sc["cams"][0], sc["nlayers"]):
            return seed, sc
    raise RuntimeError("no candidate passed the kink margins")


def _loss(pts, cam, nlayers, G):
    pyr, _, _ = oracle.forward(pts, cam, nlayers, fp32=False)
    return float(np.sum(G * pyr))


def test_adjoint_matches_central_differences():
    seed, sc = _fd_scene()
    cam, n = sc["cams"][0], sc["nlayers"]
    pts = {k: np.asarray(v, dtype=np.float64).copy() for k, v in sc["points"].items()}
    P = oracle.num_pixels(cam["W"], cam["H"], n)
    G = np.random.default_rng(seed + 1000).standard_normal((P, sc["D"]))
    grads = oracle.backward(pts, cam, n, G, fp32=False)
    pyr, counts, _ = oracle.forward(pts, cam, n, fp32=False)
    assert counts.sum() > 200 and counts.max() > 4
    for name in PARAMS:
        arr = pts[name]
        fd = np.zeros_like(arr)
        flat, fdf = arr.reshape(-1), fd.reshape(-1)
        for k in range(flat.size):
            old = flat[k]
            h = 1e-6 * max(1.0, abs(old))
            flat[k] = old + h
            lp = _loss(pts, cam, n, G)
            flat[k] = old - h
            lm = _loss(pts, cam, n, G)
            flat[k] = old
            fdf[k] = (lp - lm) / (2 * h)
        g = grads[GRAD_OF[name]].reshape(fd.shape)
        rel = np.linalg.norm(g - fd) / np.linalg.norm(fd)
        # central differences in double precision are accurate to ~1e-9 here
        assert rel <= 1e-6, (name, rel)
        assert np.all(np.abs(g - fd) <= 1e-5 * np.abs(fd) + 1e-7 * np.abs(fd).max()), name


def test_one_fragment_closed_forms():
    """C = gamma tau with gamma = alpha at a texel centre (beta = iota = 1)."""
    c = ep.cam(64, 64)
    tau = np.array([0.2, 0.4, 0.6, 0.8])
    pts = ep.points(c, [10.5], [20.5], [1.0], [2.0], [0.7], [tau])
    P = oracle.num_pixels(64, 64, 3)
    G = np.zeros((P, 4))
    g = np.array([1.0, -2.0, 0.5, 3.0])
    G[20 * 64 + 10] = g
    out = oracle.backward(pts, c, 3, G)
    a = float(np.float32(0.7))
    np.testing.assert_allclose(out["gdesc"][0], a * g, rtol=1e-15)            # dC/dtau = gamma
    np.testing.assert_allclose(out["galpha"][0], g @ tau.astype(np.float32), rtol=1e-12)


def test_two_fragment_closed_forms():
    """C = a1 c1 + (1 - a1) a2 c2: dC/da1 = c1 - a2 c2, dC/da2 = (1 - a1) c2."""
    c = ep.cam(64, 64)
    c1 = np.array([1.0, 0.5, 0.25, 0.0])
    c2 = np.array([0.0, 0.25, 0.5, 1.0])
    # point 1 is nearer (depth 1) but has the larger index
    pts = ep.points(c, [10.5, 10.5], [20.5, 20.5], [1.0, 1.0], [2.0, 1.0], [0.3, 0.6], [c2, c1])
    P = oracle.num_pixels(64, 64, 3)
    G = np.zeros((P, 4))
    g = np.array([0.3, -1.0, 2.0, 0.7])
    G[20 * 64 + 10] = g
    out = oracle.backward(pts, c, 3, G)
    a1, a2 = float(np.float32(0.6)), float(np.float32(0.3))
    c1f, c2f = c1.astype(np.float32).astype(np.float64), c2.astype(np.float32).astype(np.float64)
    np.testing.assert_allclose(out["galpha"][1], g @ (c1f - a2 * c2f), rtol=1e-12)
    np.testing.assert_allclose(out["galpha"][0], g @ ((1 - a1) * c2f), rtol=1e-12)
    np.testing.assert_allclose(out["gdesc"][1], a1 * g, rtol=1e-15)
    np.testing.assert_allclose(out["gdesc"][0], (1 - a1) * a2 * g, rtol=1e-15)


def test_fragments_beyond_clamp_get_no_gradient():
    c = ep.cam(64, 64)
    depth = 2.0 ** np.arange(20)
    rng = np.random.default_rng(5)
    pts = ep.points(c, [10.5] * 20, [20.5] * 20, [1.0] * 20, depth, rng.uniform(0.1, 0.5, 20),
                    rng.uniform(0, 1, (20, 4)))
    P = oracle.num_pixels(64, 64, 3)
    G = np.zeros((P, 4))
    G[20 * 64 + 10] = [1.0, 1.0, 1.0, 1.0]
    out = oracle.backward(pts, c, 3, G)
    assert np.all(out["galpha"][16:] == 0) and np.all(out["gdesc"][16:] == 0)
    assert np.all(out["galpha"][:16] != 0)
