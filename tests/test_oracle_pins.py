"""Pins of the CPU oracle against what the paper and the mathematics fix.

The paper prints no worked example, so the oracle is pinned by closed forms,
invariants, special cases and an independent brute-force formulation:
  - layer weights of Eq. 5 form a partition of unity (Sec. 3.1);
  - bilinear weights of Eq. 4 sum to one; the trilinear mass is 1 (or eps + (1-eps) s);
  - a point at a texel centre of layer L with size 2^L is exactly one fragment, gamma = alpha;
  - textbook pinhole projection (Eq. 2);
  - gather formulation (oracle/gather.py) == scatter formulation (oracle/oracle.py);
  - clamp to the 16 front-most elements (Sec. 3.2) and the front-to-back blend closed
    forms (Eq. 6-7);
  - permutation and shift covariance.
"""
import math

import numpy as np
import pytest

import exact_points as ep
import scenes
from oracle import gather, oracle


def _one_point(c, sx, sy, s, depth=1.0, alpha=0.7, desc=(0.25, 0.5, 0.75, 1.0)):
    return ep.points(c, [sx], [sy], [s], [depth], alpha, [desc])


# --------------------------------------------------------------------- Eq. 5
def test_iota_partition_of_unity_random_sizes():
    rng = np.random.default_rng(11)
    n = 6
    c = ep.cam(4096, 4096)
    for s in rng.uniform(1.0, 2.0 ** (n - 1), 300).astype(np.float32):
        if float(s) == 2.0 ** math.floor(math.log2(float(s))):
            continue
        pts = _one_point(c, 2048.5, 2048.5, float(s))
        fr = oracle.fragments(pts, c, n)
        layers = sorted(set(fr["L"].tolist()))
        e = math.floor(math.log2(float(s)))
        assert layers == [e, e + 1], (s, layers)
        io = {L: fr["iota"][fr["L"] == L][0] for L in layers}
        assert io[e] + io[e + 1] == 1.0  # exact: 2 - t and t - 1 with t in (1, 2)
        # Eq. 5 literally: iota = 1 - |s - 2^L| / (2^Lup - 2^Llo)
        for L in layers:
            lit = 1.0 - abs(float(s) - 2.0 ** L) / (2.0 ** (e + 1) - 2.0 ** e)
            assert io[L] == pytest.approx(lit, rel=0, abs=1e-15)


def test_iota_special_cases():
    n = 5
    c = ep.cam(1024, 1024)
    # s < 1: layer 0 only, iota = eps + (1 - eps) s  (eps = 0.25)
    for s in (0.001, 0.25, 0.5, 0.999):
        s = float(np.float32(s))
        fr = oracle.fragments(_one_point(c, 500.25, 500.75, s), c, n)
        assert set(fr["L"].tolist()) == {0}
        assert np.all(fr["iota"] == 0.25 + 0.75 * s)
    # s exactly a power of two below the coarsest layer: one layer, iota = 1
    for L in range(n):
        fr = oracle.fragments(_one_point(c, 500.25, 500.75, 2.0 ** L), c, n)
        assert set(fr["L"].tolist()) == {L} and np.all(fr["iota"] == 1.0)
    # s at or beyond the coarsest texel size: clamp to the coarsest layer, iota = 1
    for s in (2.0 ** (n - 1), 2.0 ** (n - 1) * 1.5, 1000.0):
        fr = oracle.fragments(_one_point(c, 500.25, 500.75, s), c, n)
        assert set(fr["L"].tolist()) == {n - 1} and np.all(fr["iota"] == 1.0)
    # continuity at s = 1 from below: eps + (1 - eps) * 1 = 1
    assert 0.25 + 0.75 * 1.0 == 1.0


# --------------------------------------------------------------------- Eq. 3-4
def test_beta_and_trilinear_mass():
    rng = np.random.default_rng(12)
    n = 6
    c = ep.cam(4096, 4096)
    for _ in range(200):
        sx, sy = rng.uniform(1500, 2500, 2)
        s = float(np.float32(math.exp(rng.uniform(math.log(0.2), math.log(2.0 ** (n - 1))))))
        alpha = 0.6
        pts = _one_point(c, float(np.float32(sx)), float(np.float32(sy)), s, alpha=alpha)
        fr = oracle.fragments(pts, c, n)
        for L in set(fr["L"].tolist()):
            assert abs(fr["beta"][fr["L"] == L].sum() - 1.0) <= 4e-16
        mass = float((fr["beta"] * fr["iota"]).sum())
        want = 0.25 + 0.75 * s if s < 1 else 1.0
        assert abs(mass - want) <= 1e-15, (s, mass, want)
        # gamma = beta * iota * alpha
        np.testing.assert_allclose(fr["gamma"], fr["beta"] * fr["iota"] * np.float32(alpha),
                                   rtol=1e-15)


def test_single_texel_special_case_every_layer():
    """A point at the centre of texel (i, j) of layer L with s = 2^L is exactly one fragment."""
    n = 6
    W, H = 640, 384
    c = ep.cam(W, H)
    dims = oracle.layer_dims(W, H, n)
    for L in range(n):
        WL, HL = dims[L]
        i, j = WL // 3, HL // 2
        sx, sy = (i + 0.5) * 2 ** L, (j + 0.5) * 2 ** L
        tau = (0.1, 0.2, 0.3, 0.4)
        pts = _one_point(c, sx, sy, 2.0 ** L, alpha=0.7, desc=tau)
        fr = oracle.fragments(pts, c, n)
        assert len(fr["L"]) == 1
        assert (fr["L"][0], fr["i"][0], fr["j"][0]) == (L, i, j)
        assert fr["gamma"][0] == np.float64(np.float32(0.7))
        pyr, counts, ids = oracle.forward(pts, c, n)
        layer = oracle.split_layers(pyr, c, n)[L]
        want = np.float64(np.float32(0.7)) * np.asarray(tau, dtype=np.float32).astype(np.float64)
        assert np.array_equal(layer[j, i], want)
        assert np.count_nonzero(pyr) == 4 and counts.sum() == 1 and ids[counts > 0][0, 0] == 0
    # s < 1 at a layer-0 texel centre: one fragment with gamma = (0.25 + 0.75 s) alpha
    s = 0.375
    pts = _one_point(c, 100.5, 200.5, s, alpha=0.5)
    fr = oracle.fragments(pts, c, n)
    assert len(fr["L"]) == 1 and fr["L"][0] == 0 and (fr["i"][0], fr["j"][0]) == (100, 200)
    assert fr["gamma"][0] == (0.25 + 0.75 * s) * 0.5


# --------------------------------------------------------------------- Eq. 2
def test_projection_pinhole():
    rng = np.random.default_rng(13)
    # on-axis point with R = I, t = 0 maps to the principal point
    c = scenes.camera(np.eye(3), (0, 0, 0), 640, 480)
    pts = {"x": np.zeros(3, np.float32), "y": np.zeros(3, np.float32),
           "z": np.array([0.5, 1, 7], np.float32), "sw": np.full(3, 0.01, np.float32)}
    valid, xyzs = oracle.project(pts, c, 5)
    assert valid.all() and np.all(xyzs[:, 0] == 320) and np.all(xyzs[:, 1] == 240)
    # general pose against the textbook K (R X + t), evaluated in double precision
    for trial in range(5):
        q, r = np.linalg.qr(rng.standard_normal((3, 3)))
        R = (q * np.sign(np.diag(r))).astype(np.float32)
        t = rng.uniform(-1, 1, 3).astype(np.float32) + np.float32([0, 0, 4])
        c = scenes.camera(R, t, 1920, 1080)
        # non-square pixels and an off-centre principal point
        c["fy"] = np.float32(float(c["fx"]) * 0.8)
        c["cy"] = np.float32(float(c["cy"]) + 13.25)
        X = rng.uniform(-1, 1, (500, 3)).astype(np.float32)
        sw = rng.uniform(0.001, 0.05, 500).astype(np.float32)
        pts = {"x": X[:, 0].copy(), "y": X[:, 1].copy(), "z": X[:, 2].copy(), "sw": sw}
        Rd, td = R.astype(np.float64).reshape(3, 3), t.astype(np.float64)
        Xc = X.astype(np.float64) @ Rd.T + td
        K = np.array([[float(c["fx"]), 0, float(c["cx"])], [0, float(c["fy"]), float(c["cy"])],
                      [0, 0, 1]])
        h = Xc @ K.T
        ref = np.stack([h[:, 0] / h[:, 2], h[:, 1] / h[:, 2], Xc[:, 2],
                        float(c["fx"]) * sw.astype(np.float64) / Xc[:, 2]], axis=1)
        for fp32, tol in ((True, 2e-6), (False, 1e-12)):
            valid, xyzs = oracle.project(pts, c, 8, fp32=fp32)
            assert valid.all()
            scale = np.array([2000.0, 2000.0, 10.0, 1.0]) * np.maximum(1, np.abs(ref))
            assert np.all(np.abs(xyzs - ref) <= tol * scale), (fp32, np.max(np.abs(xyzs - ref)))
    # behind the near plane and non-finite inputs are culled
    c = scenes.camera(np.eye(3), (0, 0, 0), 64, 64)
    pts = {"x": np.array([0, 0, np.nan, 0], np.float32), "y": np.zeros(4, np.float32),
           "z": np.array([-1, 0.005, 1, 1], np.float32),
           "sw": np.array([0.1, 0.1, 0.1, np.inf], np.float32)}
    valid, _ = oracle.project(pts, c, 4)
    assert not valid.any()


# --------------------------------------------------------------------- Sec. 3.2 lists
@pytest.mark.parametrize("seed,ties", [(0, False), (1, False), (2, True), (3, True), (4, False)])
def test_gather_equals_scatter(seed, ties):
    sc = scenes.random_small(seed, n=48, W=24, H=20, nlayers=4, depth_ties=ties)
    pts, c = sc["points"], sc["cams"][0]
    a = oracle.forward(pts, c, 4)
    b = gather.render(pts, c, 4)
    assert np.array_equal(a[1], b[1]), "per-texel list lengths differ"
    assert np.array_equal(a[2], b[2]), "kept ids or their order differ"
    assert np.array_equal(a[0], b[0]), "blended values differ"
    assert a[1].sum() > 100


def test_gather_equals_scatter_non_square_pixels():
    sc = scenes.random_small(5, n=48, W=24, H=20, nlayers=4)
    pts, c = sc["points"], dict(sc["cams"][0])
    c["fy"] = np.float32(float(c["fx"]) * 0.7)
    c["cy"] = np.float32(8.5)
    a = oracle.forward(pts, c, 4)
    b = gather.render(pts, c, 4)
    assert a[1].sum() > 50
    for k in range(3):
        assert np.array_equal(a[k], b[k])


def test_gather_equals_scatter_clamped_lists():
    # many points on a small view so lists exceed 16
    sc = scenes.random_small(7, n=160, W=12, H=10, nlayers=3, s_lo=2.0, s_hi=6.0)
    pts, c = sc["points"], sc["cams"][0]
    a = oracle.forward(pts, c, 3)
    b = gather.render(pts, c, 3)
    assert a[1].max() > 16
    for k in range(3):
        assert np.array_equal(a[k], b[k])


def test_clamp_to_16_front_most():
    L, n = 1, 4
    c = ep.cam(64, 64)
    rng = np.random.default_rng(14)
    order = rng.permutation(20)          # point p has depth 2^order[p]
    depth = 2.0 ** order
    alpha = rng.uniform(0.05, 0.9, 20).astype(np.float32)
    tau = rng.uniform(0, 1, (20, 4)).astype(np.float32)
    i, j = 5, 9
    sx, sy = (i + 0.5) * 2 ** L, (j + 0.5) * 2 ** L
    pts = ep.points(c, [sx] * 20, [sy] * 20, [2.0 ** L] * 20, depth, alpha, tau)
    pyr, counts, ids = oracle.forward(pts, c, n)
    dims = oracle.layer_dims(64, 64, n)
    pix = dims[0][0] * dims[0][1] + j * dims[1][0] + i
    assert counts[pix] == 20 and counts.sum() == 20
    front = np.argsort(order)[:16]       # the 16 nearest, nearest first
    assert np.array_equal(ids[pix], front)
    want = np.zeros(4)
    T = 1.0
    for p in front:
        want += T * float(alpha[p]) * tau[p].astype(np.float64)
        T *= 1.0 - float(alpha[p])
    np.testing.assert_allclose(pyr[pix], want, rtol=1e-15)


# --------------------------------------------------------------------- Eq. 6-7
def test_blend_closed_forms():
    c = ep.cam(64, 64)
    # two fragments: a1 c1 + (1 - a1) a2 c2, nearer first regardless of index
    pts = ep.points(c, [10.5, 10.5], [20.5, 20.5], [1.0, 1.0], [4.0, 2.0], [0.3, 0.6],
                    [[1, 0, 0, 0], [0, 1, 0, 0]])
    pyr, counts, ids = oracle.forward(pts, c, 3)
    pix = 20 * 64 + 10
    a1, a2 = float(np.float32(0.6)), float(np.float32(0.3))
    np.testing.assert_allclose(pyr[pix], [(1 - a1) * a2, a1, 0, 0], rtol=1e-15)
    assert list(ids[pix, :2]) == [1, 0]
    # constant descriptor 1: C = 1 - prod_m (1 - gamma_m) over the kept fragments
    sc = scenes.random_small(21, n=120, W=16, H=12, nlayers=3, s_lo=1.0, s_hi=5.0)
    pts, c = sc["points"], sc["cams"][0]
    pts["desc"] = np.ones_like(pts["desc"])
    pyr, counts, ids = oracle.forward(pts, c, 3)
    fr = oracle.fragments(pts, c, 3)
    dims = oracle.layer_dims(c["W"], c["H"], 3)
    base = np.cumsum([0] + [w * h for w, h in dims])
    pix_of = base[fr["L"]] + fr["j"] * np.array([dims[L][0] for L in fr["L"]]) + fr["i"]
    want = np.zeros(len(counts))
    for p in np.unique(pix_of):
        g = fr["gamma"][pix_of == p][:16]   # fragments come sorted by depth within a texel
        want[p] = 1.0 - np.prod(1.0 - g)
    np.testing.assert_allclose(pyr[:, 0], want, rtol=1e-13, atol=1e-15)
    assert counts.max() > 16


# --------------------------------------------------------------------- covariance
def test_permutation_invariance():
    sc = scenes.random_small(31, n=80, W=20, H=16, nlayers=4)
    pts, c = sc["points"], sc["cams"][0]
    perm = np.random.default_rng(3).permutation(80)
    pts2 = {k: v[perm] for k, v in pts.items()}
    a = oracle.forward(pts, c, 4)
    b = oracle.forward(pts2, c, 4)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    mapped = np.where(b[2] >= 0, perm[np.maximum(b[2], 0)], -1)
    assert np.array_equal(a[2], mapped)


def test_shift_covariance_exact():
    """Moving the principal point by 2^(n-1) px moves layer L by 2^(n-1-L) texels.  Screen
    coordinates stay inside one binade, so single-precision rounding commutes with the shift."""
    n = 5
    shift = 2 ** (n - 1)
    W = H = 1024
    rng = np.random.default_rng(15)
    cnt = 200
    c0 = ep.cam(W, H, cx=512.0, cy=512.0)
    sx = rng.uniform(600, 800, cnt).astype(np.float32).astype(np.float64)
    sy = rng.uniform(600, 800, cnt).astype(np.float32).astype(np.float64)
    s = rng.uniform(0.3, 24, cnt).astype(np.float32).astype(np.float64)
    pts = ep.points(c0, sx, sy, s, np.ones(cnt), rng.uniform(0.1, 1, cnt),
                    rng.uniform(0, 1, (cnt, 4)))
    c1 = dict(c0, cx=np.float32(512.0 + shift), cy=np.float32(512.0 + shift))
    a = oracle.split_layers(oracle.forward(pts, c0, n)[0], c0, n)
    b = oracle.split_layers(oracle.forward(pts, c1, n)[0], c1, n)
    for L in range(n):
        k = shift >> L
        assert np.array_equal(b[L][k:, k:], a[L][:-k, :-k]), L
        assert np.count_nonzero(a[L]) > 0


# --------------------------------------------------------------------- generators
def test_generators_deterministic():
    a = scenes.unit_cube(1)
    b = scenes.unit_cube(1)
    for k in a["points"]:
        assert np.array_equal(a["points"][k], b["points"][k])
    c = scenes.unit_cube(2)
    assert not np.array_equal(a["points"]["x"], c["points"]["x"])
    s = scenes.cluster_scene(2, n=10000)
    assert s["points"]["x"].dtype == np.float32 and s["points"]["desc"].shape == (10000, 4)
