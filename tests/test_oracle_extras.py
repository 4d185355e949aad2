"""Pins of the oracle's optional terms: a background seen through the transmittance the kept
fragments leave (where the environment map E of Eq. 1 enters), the coverage 1 - T_K, and
the gradients with respect to the background and to the camera (R, t, fx, fy, cx, cy of
Eq. 2).

  - an empty scene shows the background exactly and passes G straight through;
  - the coverage equals the blend (Eq. 6-7) of a constant-1 descriptor, computed by the
    plain forward with no coverage code involved;
  - a one-fragment texel gives gamma tau + (1 - gamma) bg;
  - dL/dbg = (1 - coverage) G, from the forward's own coverage;
  - translating every point by d equals translating the camera by R d, so the summed
    point gradients equal R^T dL/dt;
  - central finite differences of the double-precision forward for the gradients through
    the background, the coverage and every camera parameter.
"""
import copy

import numpy as np

import exact_points as ep
import scenes
from oracle import oracle
from test_oracle_backward import _fd_scene

CAM_KEYS = ["R%d" % k for k in range(9)] + ["t0", "t1", "t2", "fx", "fy", "cx", "cy"]


def _cam_get(cam, key):
    if key[0] == "R":
        return float(np.asarray(cam["R"], dtype=np.float64).reshape(9)[int(key[1])])
    if key[0] == "t":
        return float(np.asarray(cam["t"], dtype=np.float64).reshape(3)[int(key[1])])
    return float(cam[key])


def _cam_set(cam, key, value):
    c = copy.deepcopy(cam)
    if key[0] in "Rt":
        n = 9 if key[0] == "R" else 3
        arr = np.asarray(c[key[0]], dtype=np.float64).reshape(n).copy()
        arr[int(key[1])] = value
        c[key[0]] = arr.reshape(3, 3) if n == 9 else arr
    else:
        c[key] = value
    return c


def test_empty_scene_shows_background():
    sc = scenes.random_small(3, n=16)
    cam, nl, D = sc["cams"][0], sc["nlayers"], sc["D"]
    pts = {k: np.asarray(v, dtype=np.float64).copy() for k, v in sc["points"].items()}
    pts["z"] = -pts["z"]  # every point behind the camera: culled
    P = oracle.num_pixels(cam["W"], cam["H"], nl)
    rng = np.random.default_rng(1)
    bg = rng.uniform(-1, 1, (P, D))
    G = rng.standard_normal((P, D))
    f = oracle.forward_ex(pts, cam, nl, background=bg)
    assert np.array_equal(f["pyr"], bg) and not f["alpha"].any() and not f["counts"].any()
    b = oracle.backward_ex(pts, cam, nl, G, background=bg, grad_alpha=rng.standard_normal(P))
    assert np.array_equal(b["gbg"], G)
    assert not b["gcam"].any() and not b["gx"].any() and not b["gdesc"].any()


def test_coverage_is_the_blend_of_a_constant_one():
    sc = scenes.random_small(4, n=600)
    cam, nl = sc["cams"][0], sc["nlayers"]
    f = oracle.forward_ex(sc["points"], cam, nl)
    ones = dict(sc["points"])
    ones["desc"] = np.ones_like(sc["points"]["desc"])
    pyr1, counts, _ = oracle.forward(ones, cam, nl)
    assert counts.sum() > 100 and counts.max() > 16
    np.testing.assert_allclose(f["alpha"], pyr1[:, 0], rtol=0, atol=1e-14)
    assert np.array_equal(f["alpha"] > 0, counts > 0)


def test_one_fragment_texel_with_background():
    c = ep.cam(64, 64)
    tau = np.array([0.2, 0.4, 0.6, 0.8])
    pts = ep.points(c, [10.5], [20.5], [1.0], [2.0], [0.7], [tau])
    P = oracle.num_pixels(64, 64, 3)
    bg = np.random.default_rng(2).uniform(0, 1, (P, 4))
    f = oracle.forward_ex(pts, c, 3, background=bg)
    pix = 20 * 64 + 10
    a = float(np.float32(0.7))
    np.testing.assert_allclose(f["alpha"][pix], a, rtol=1e-15)
    np.testing.assert_allclose(f["pyr"][pix], a * tau.astype(np.float32).astype(np.float64) + (1 - a) * bg[pix],
                               rtol=1e-14)
    others = np.ones(P, dtype=bool)
    others[pix] = False
    assert np.array_equal(f["pyr"][others], bg[others])


def test_background_gradient_is_transmittance_times_g():
    sc = scenes.random_small(5, n=96)
    cam, nl, D = sc["cams"][0], sc["nlayers"], sc["D"]
    P = oracle.num_pixels(cam["W"], cam["H"], nl)
    rng = np.random.default_rng(6)
    bg, G = rng.uniform(0, 1, (P, D)), rng.standard_normal((P, D))
    f = oracle.forward_ex(sc["points"], cam, nl, background=bg)
    b = oracle.backward_ex(sc["points"], cam, nl, G, background=bg)
    np.testing.assert_allclose(b["gbg"], (1.0 - f["alpha"])[:, None] * G, rtol=1e-12, atol=1e-15)


def test_translation_gradient_equals_summed_point_gradients():
    sc = scenes.random_small(7, n=96)
    cam, nl, D = sc["cams"][0], sc["nlayers"], sc["D"]
    # a rotated camera, so R^T is not the identity
    ang = 0.3
    R = np.array([[np.cos(ang), 0, np.sin(ang)], [0, 1, 0], [-np.sin(ang), 0, np.cos(ang)]])
    cam = dict(cam, R=R, t=np.array([0.2, -0.1, 0.3]))
    P = oracle.num_pixels(cam["W"], cam["H"], nl)
    G = np.random.default_rng(8).standard_normal((P, D))
    b = oracle.backward_ex(sc["points"], cam, nl, G, fp32=False)
    summed = np.array([b["gx"].sum(), b["gy"].sum(), b["gz"].sum()])
    assert np.abs(b["gcam"][9:12]).max() > 1e-3
    np.testing.assert_allclose(summed, R.T @ b["gcam"][9:12], rtol=1e-10, atol=1e-12)


def _loss(pts, cam, nl, G, bg, Ga):
    f = oracle.forward_ex(pts, cam, nl, background=bg, fp32=False)
    return float(np.sum(G * f["pyr"]) + np.sum(Ga * f["alpha"]))


def test_extras_match_central_differences():
    seed, sc = _fd_scene()
    cam, nl, D = sc["cams"][0], sc["nlayers"], sc["D"]
    pts = {k: np.asarray(v, dtype=np.float64).copy() for k, v in sc["points"].items()}
    P = oracle.num_pixels(cam["W"], cam["H"], nl)
    rng = np.random.default_rng(seed + 2000)
    G, Ga, bg = rng.standard_normal((P, D)), rng.standard_normal(P), rng.uniform(0, 1, (P, D))
    b = oracle.backward_ex(pts, cam, nl, G, background=bg, grad_alpha=Ga, fp32=False)
    # point parameters, through the background and coverage terms as well
    for name, gname in (("x", "gx"), ("sw", "gsw"), ("alpha", "galpha")):
        arr = pts[name]
        fd = np.zeros_like(arr)
        for k in range(arr.size):
            old = arr[k]
            h = 1e-6 * max(1.0, abs(old))
            arr[k] = old + h
            lp = _loss(pts, cam, nl, G, bg, Ga)
            arr[k] = old - h
            lm = _loss(pts, cam, nl, G, bg, Ga)
            arr[k] = old
            fd[k] = (lp - lm) / (2 * h)
        rel = np.linalg.norm(b[gname] - fd) / np.linalg.norm(fd)
        assert rel <= 1e-6, (name, rel)
    # the background (the loss is linear in it)
    for pix in rng.choice(P, 24, replace=False):
        for d in range(D):
            old = bg[pix, d]
            bg[pix, d] = old + 1e-3
            lp = _loss(pts, cam, nl, G, bg, Ga)
            bg[pix, d] = old - 1e-3
            lm = _loss(pts, cam, nl, G, bg, Ga)
            bg[pix, d] = old
            np.testing.assert_allclose(b["gbg"][pix, d], (lp - lm) / 2e-3, rtol=1e-8, atol=1e-12)
    # every camera parameter
    fd = np.zeros(16)
    for k, key in enumerate(CAM_KEYS):
        old = _cam_get(cam, key)
        h = 1e-7 * max(1.0, abs(old))
        lp = _loss(pts, _cam_set(cam, key, old + h), nl, G, bg, Ga)
        lm = _loss(pts, _cam_set(cam, key, old - h), nl, G, bg, Ga)
        fd[k] = (lp - lm) / (2 * h)
    rel = np.linalg.norm(b["gcam"] - fd) / np.linalg.norm(fd)
    assert rel <= 1e-6, rel
    assert np.all(np.abs(b["gcam"] - fd) <= 1e-5 * np.abs(fd) + 1e-6 * np.abs(fd).max()), (b["gcam"], fd)
