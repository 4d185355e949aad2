"""Pins of the oracle's coarser-layer inclusion (Sec. 3.6): the list a texel
blends also holds the fragments of the texels of every coarser layer that cover it.

The paper gives the rule no more detail than that it is done the usual way; the reading
pinned here: texel (i, j) of layer L takes in the fragments of texel (i >> k, j >> k) of
layer L + k for every k >= 1, each with its own gamma; the union is ordered by depth,
point index, then layer (finer first) and clamped to 16.

  - one layer, and the coarsest layer of any pyramid, are unchanged by inclusion;
  - brute force: the union lists built in Python from the pinned fragment list
    (oracle_fragments), blended by Eq. 6-7, give the oracle's lists and colours;
  - closed forms: a large near point written only to layer 2 occludes a small far point
    of layer 0 (C = a tA + (1 - a) b tB and its derivatives), and nothing outside the
    large point's covering texel sees it;
  - a texel mask gives the unmasked result on the masked texels (the ancestors are found);
  - central finite differences of the double-precision forward, with a background and
    the coverage, for every point parameter and the camera.
"""
import numpy as np

import exact_points as ep
import scenes
from oracle import oracle
from test_oracle_backward import GRAD_OF, PARAMS, _margins_ok
from test_oracle_extras import CAM_KEYS, _cam_get, _cam_set


def _union_lists(pts, cam, nl, fp32=True):
    """For every texel (pyramid row), the fragment rows of its inclusion list in blend order,
    from the fragment list alone."""
    fr = oracle.fragments(pts, cam, nl, fp32=fp32)
    dims = oracle.layer_dims(cam["W"], cam["H"], nl)
    lists = []
    for L, (WL, HL) in enumerate(dims):
        for j in range(HL):
            for i in range(WL):
                k = fr["L"] - L
                sel = (k >= 0) & ((i >> np.maximum(k, 0)) == fr["i"]) & ((j >> np.maximum(k, 0)) == fr["j"])
                rows = np.nonzero(sel)[0]
                order = np.lexsort((fr["L"][rows], fr["idx"][rows], fr["z"][rows]))
                lists.append(rows[order][:16])
    return fr, lists


def test_single_layer_and_coarsest_layer_unchanged():
    sc = scenes.random_small(11, n=96)
    cam, D = sc["cams"][0], sc["D"]
    for nl in (1, 4):
        a = oracle.forward_ex(sc["points"], cam, nl)
        b = oracle.forward_ex(sc["points"], cam, nl, coarser=True)
        dims = oracle.layer_dims(cam["W"], cam["H"], nl)
        last = sum(w * h for w, h in dims[:-1])
        assert np.array_equal(a["pyr"][last:], b["pyr"][last:])
        assert np.array_equal(a["ids"][last:], b["ids"][last:])
        assert np.array_equal(a["counts"], b["counts"])  # own fragments in both modes
        if nl == 1:
            assert np.array_equal(a["pyr"], b["pyr"]) and np.array_equal(a["alpha"], b["alpha"])
        else:
            assert not np.array_equal(a["pyr"], b["pyr"])  # inclusion changes finer layers


def test_brute_force_union_lists():
    for seed, nl in ((12, 4), (13, 3)):
        sc = scenes.random_small(seed, n=400, depth_ties=(seed == 13))
        cam, D = sc["cams"][0], sc["D"]
        pts = sc["points"]
        rng = np.random.default_rng(seed)
        P = oracle.num_pixels(cam["W"], cam["H"], nl)
        bg = rng.uniform(-1, 1, (P, D))
        out = oracle.forward_ex(pts, cam, nl, background=bg, coarser=True)
        fr, lists = _union_lists(pts, cam, nl)
        desc = np.asarray(pts["desc"], dtype=np.float32).astype(np.float64)
        longest = 0
        for pix, rows in enumerate(lists):
            ids = np.full(16, -1)
            ids[:len(rows)] = fr["idx"][rows]
            assert np.array_equal(out["ids"][pix], ids), pix
            T, C = 1.0, np.zeros(D)
            for r in rows:
                C += T * fr["gamma"][r] * desc[fr["idx"][r]]
                T *= 1.0 - fr["gamma"][r]
            np.testing.assert_allclose(out["pyr"][pix], C + T * bg[pix], rtol=1e-13, atol=1e-15)
            np.testing.assert_allclose(out["alpha"][pix], 1.0 - T, rtol=1e-13, atol=1e-15)
            longest = max(longest, len(rows))
        assert longest == 16  # the clamp is exercised


def _occluder_scene(near_is_large):
    c = ep.cam(32, 32)
    tA = np.array([1.0, 0.5, 0.25, 0.125])
    tB = np.array([0.0, 0.25, 0.75, 1.0])
    # A: screen size 4 (layer 2 only, iota 1) centred on layer-2 texel (2, 2);
    # B: screen size 1 (layer 0 only, iota 1) centred on layer-0 texel (9, 10)
    dA, dB = (1.0, 2.0) if near_is_large else (2.0, 1.0)
    pts = ep.points(c, [10.0, 9.5], [10.0, 10.5], [4.0, 1.0], [dA, dB], [0.6, 0.3], [tA, tB])
    pts["alpha"] = np.array([0.6, 0.3], dtype=np.float32)
    return c, pts


def test_closed_form_occluder():
    for near_is_large in (True, False):
        c, pts = _occluder_scene(near_is_large)
        nl = 3
        a, b = float(np.float32(0.6)), float(np.float32(0.3))
        tA = pts["desc"][0].astype(np.float64)
        tB = pts["desc"][1].astype(np.float64)
        out = oracle.forward_ex(pts, c, nl, coarser=True)
        plain = oracle.forward_ex(pts, c, nl)
        t9_10 = oracle.texel_index(c, nl, 0, 9, 10)
        want = a * tA + (1 - a) * b * tB if near_is_large else b * tB + (1 - b) * a * tA
        np.testing.assert_allclose(out["pyr"][t9_10], want, rtol=1e-15)
        np.testing.assert_allclose(plain["pyr"][t9_10], b * tB, rtol=1e-15)
        # every layer-0 texel of rows/columns 8..11 and layer-1 texel of 4..5 sees A
        for L, lo in ((0, 8), (1, 4)):
            span = 4 >> L
            for j in range(lo, lo + span):
                for i in range(lo, lo + span):
                    t = oracle.texel_index(c, nl, L, i, j)
                    if (L, i, j) == (0, 9, 10):
                        continue
                    np.testing.assert_allclose(out["pyr"][t], a * tA, rtol=1e-15)
            for (i, j) in ((lo - 1, lo), (lo + span, lo), (lo, lo - 1), (lo, lo + span)):
                t = oracle.texel_index(c, nl, L, i, j)
                assert not out["pyr"][t].any()
        # gradients of g . C at texel (0, 9, 10)
        P = oracle.num_pixels(32, 32, nl)
        G = np.zeros((P, 4))
        g = np.array([0.5, -1.0, 2.0, 0.25])
        G[t9_10] = g
        gr = oracle.backward_ex(pts, c, nl, G, coarser=True)
        if near_is_large:
            dA, dB, wA, wB = g @ (tA - b * tB), g @ ((1 - a) * tB), a, (1 - a) * b
        else:
            dA, dB, wA, wB = g @ ((1 - b) * tA), g @ (tB - a * tA), (1 - b) * a, b
        np.testing.assert_allclose(gr["galpha"], [dA, dB], rtol=1e-14)
        np.testing.assert_allclose(gr["gdesc"][0], wA * g, rtol=1e-14)
        np.testing.assert_allclose(gr["gdesc"][1], wB * g, rtol=1e-14)


def test_mask_finds_ancestors():
    sc = scenes.random_small(14, n=80)
    cam, nl, D = sc["cams"][0], 4, sc["D"]
    P = oracle.num_pixels(cam["W"], cam["H"], nl)
    rng = np.random.default_rng(14)
    mask = rng.random(P) < 0.2
    G = rng.standard_normal((P, D))
    full = oracle.forward_ex(sc["points"], cam, nl, coarser=True)
    part = oracle.forward_ex(sc["points"], cam, nl, coarser=True, mask=mask)
    assert np.array_equal(part["pyr"][mask], full["pyr"][mask])
    assert np.array_equal(part["ids"][mask], full["ids"][mask])
    assert not part["pyr"][~mask].any()
    a = oracle.backward_ex(sc["points"], cam, nl, G * mask[:, None], coarser=True)
    b = oracle.backward_ex(sc["points"], cam, nl, G, coarser=True, mask=mask)
    for k in ("gx", "gy", "gz", "gsw", "galpha", "gdesc"):
        np.testing.assert_allclose(b[k], a[k], rtol=1e-12, atol=1e-14)


def _fd_scene_coarser():
    """A cluster subset whose inclusion lists stay below the clamp and keep distinct points
    apart in depth, so the loss is smooth in every parameter."""
    for seed in range(40, 400):
        sc = scenes.fd_candidate(seed, n=24, nlayers=5)
        pts, cam, nl = sc["points"], sc["cams"][0], sc["nlayers"]
        if not _margins_ok(pts, cam, nl):
            continue
        fr, lists = _union_lists(pts, cam, nl, fp32=False)
        ok = True
        for rows in lists:
            if len(rows) >= 16:
                ok = False
                break
            z, idx = fr["z"][rows], fr["idx"][rows]
            for u in range(len(rows)):
                for v in range(u + 1, len(rows)):
                    if idx[u] != idx[v] and abs(z[u] - z[v]) <= 1e-4:
                        ok = False
        if ok and max(len(r) for r in lists) >= 4:
            return seed, sc
    raise RuntimeError("no candidate passed the margins")


def test_adjoint_matches_central_differences():
    seed, sc = _fd_scene_coarser()
    cam, nl, D = sc["cams"][0], sc["nlayers"], sc["D"]
    pts = {k: np.asarray(v, dtype=np.float64).copy() for k, v in sc["points"].items()}
    P = oracle.num_pixels(cam["W"], cam["H"], nl)
    rng = np.random.default_rng(seed + 7)
    G = rng.standard_normal((P, D))
    Ga = rng.standard_normal(P)
    bg = rng.uniform(-1, 1, (P, D))

    def loss(p, c):
        f = oracle.forward_ex(p, c, nl, background=bg, fp32=False, coarser=True)
        return float(np.sum(G * f["pyr"]) + np.sum(Ga * f["alpha"]))

    gr = oracle.backward_ex(pts, cam, nl, G, background=bg, grad_alpha=Ga, fp32=False,
                            coarser=True)
    plain = oracle.backward_ex(pts, cam, nl, G, background=bg, grad_alpha=Ga, fp32=False)
    assert not np.allclose(gr["galpha"], plain["galpha"])  # inclusion matters here
    for name in PARAMS:
        arr = pts[name]
        fd = np.zeros_like(arr)
        flat, fdf = arr.reshape(-1), fd.reshape(-1)
        for k in range(flat.size):
            old = flat[k]
            h = 1e-6 * max(1.0, abs(old))
            flat[k] = old + h
            lp = loss(pts, cam)
            flat[k] = old - h
            lm = loss(pts, cam)
            flat[k] = old
            fdf[k] = (lp - lm) / (2 * h)
        g = gr[GRAD_OF[name]].reshape(fd.shape)
        assert np.linalg.norm(g - fd) <= 1e-6 * np.linalg.norm(fd), name
    for key in CAM_KEYS:
        v = _cam_get(cam, key)
        h = 1e-6 * max(1.0, abs(v))
        fd = (loss(pts, _cam_set(cam, key, v + h)) - loss(pts, _cam_set(cam, key, v - h))) / (2 * h)
        k = CAM_KEYS.index(key)
        assert abs(gr["gcam"][k] - fd) <= 1e-6 * max(1.0, abs(fd)), key
    np.testing.assert_allclose(gr["gbg"], (1.0 - oracle.forward_ex(
        pts, cam, nl, background=bg, fp32=False, coarser=True)["alpha"])[:, None] * G, rtol=1e-12)
