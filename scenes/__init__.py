"""Seeded synthetic scenes and cameras for trilinear point splatting.

Both the GPU tests and the CPU oracle tests feed the arrays made here to their
side; this module holds none of the renderer's arithmetic (no projection of
points to layers, no weights, no blending).  The paper's datasets (Tanks and
Temples, Mip-NeRF 360, Boat, Office) are not available, so these stand in for
them with the paper's scales: 1.8M-72.5M points, 1920x1080 views, up to 8
pyramid layers, 4-8 descriptor channels, position noise 0.01.

All draws use numpy's PCG64 generator seeded explicitly; every array is
float32 (the renderer's precision).  A scene is a dict
  {"points": {"x","y","z","sw","alpha": [N], "desc": [N, D]},
   "cams": [camera, ...], "nlayers": n, "D": D}
and a camera is {"R": [9] row-major world->camera, "t": [3], "fx", "fy", "cx",
"cy", "W", "H", "znear"} with the OpenCV convention (x right, y down, z forward).
"""
import math

import numpy as np

RESOLUTIONS = [(640, 480), (800, 600), (1024, 768), (1280, 720), (1600, 900), (1920, 1080)]


def intrinsics(W, H, hfov_deg):
    """Square-pixel pinhole intrinsics with horizontal field of view hfov."""
    fx = (W / 2.0) / math.tan(math.radians(hfov_deg) / 2.0)
    return fx, fx, W / 2.0, H / 2.0


def camera(R, t, W, H, hfov_deg=60.0, znear=0.01):
    fx, fy, cx, cy = intrinsics(W, H, hfov_deg)
    return {"R": np.asarray(R, dtype=np.float32).reshape(9), "t": np.asarray(t, dtype=np.float32),
            "fx": np.float32(fx), "fy": np.float32(fy), "cx": np.float32(cx), "cy": np.float32(cy),
            "W": int(W), "H": int(H), "znear": np.float32(znear)}


def look_at(eye, target, W, H, hfov_deg=60.0, up=(0.0, -1.0, 0.0)):
    """Camera at eye looking at target; world->camera rotation rows are the camera axes."""
    eye = np.asarray(eye, dtype=np.float64)
    fwd = np.asarray(target, dtype=np.float64) - eye
    fwd /= np.linalg.norm(fwd)
    up = np.asarray(up, dtype=np.float64)
    if abs(float(np.dot(up, fwd))) > 0.99:
        up = np.array([0.0, 0.0, 1.0]) if abs(fwd[2]) < 0.9 else np.array([1.0, 0.0, 0.0])
    right = np.cross(up, fwd)  # x axis (right) for a y-down camera
    right /= np.linalg.norm(right)
    down = np.cross(fwd, right)
    R = np.stack([right, down, fwd])
    t = -R @ eye
    return camera(R, t, W, H, hfov_deg)


def _depth(cam, xyz):
    """Camera depth used only to pick world sizes with a given screen-size spread."""
    R = np.asarray(cam["R"], dtype=np.float64).reshape(3, 3)
    return xyz.astype(np.float64) @ R[2] + float(cam["t"][2])


def _log_uniform(rng, lo, hi, n):
    return np.exp(rng.uniform(math.log(lo), math.log(hi), n))


def _random_rotation(rng):
    q, r = np.linalg.qr(rng.standard_normal((3, 3)))
    q *= np.sign(np.diag(r))
    return q


def cluster_points(rng, n, n_clusters=64, plane_frac=0.3, n_planes=8):
    """Mixture of anisotropic Gaussian clusters plus points on random planar patches."""
    n_plane = int(round(n * plane_frac))
    n_clu = n - n_plane
    centres = rng.uniform(-1.0, 1.0, (n_clusters, 3))
    rots = np.stack([_random_rotation(rng) for _ in range(n_clusters)])
    sig = _log_uniform(rng, 0.01, 0.2, n_clusters * 3).reshape(n_clusters, 3)
    cid = rng.integers(0, n_clusters, n_clu)
    local = rng.standard_normal((n_clu, 3)) * sig[cid]
    pts_c = centres[cid] + np.einsum("nij,nj->ni", rots[cid], local)
    parts = [pts_c]
    if n_plane:
        pc = rng.uniform(-1.0, 1.0, (n_planes, 3))
        normals = rng.standard_normal((n_planes, 3))
        normals /= np.linalg.norm(normals, axis=1, keepdims=True)
        e1 = np.cross(normals, rng.standard_normal((n_planes, 3)))
        e1 /= np.linalg.norm(e1, axis=1, keepdims=True)
        e2 = np.cross(normals, e1)
        side = rng.uniform(0.5, 2.0, n_planes)
        pid = rng.integers(0, n_planes, n_plane)
        a = rng.uniform(-0.5, 0.5, (n_plane, 2)) * side[pid, None]
        parts.append(pc[pid] + a[:, :1] * e1[pid] + a[:, 1:] * e2[pid])
    xyz = np.concatenate(parts, axis=0)
    xyz = xyz[rng.permutation(n)]  # no spatial order in the point index
    return xyz, centres


def _points(xyz, sw, alpha, desc):
    return {"x": np.ascontiguousarray(xyz[:, 0], dtype=np.float32),
            "y": np.ascontiguousarray(xyz[:, 1], dtype=np.float32),
            "z": np.ascontiguousarray(xyz[:, 2], dtype=np.float32),
            "sw": np.ascontiguousarray(sw, dtype=np.float32),
            "alpha": np.ascontiguousarray(alpha, dtype=np.float32),
            "desc": np.ascontiguousarray(desc, dtype=np.float32)}


def unit_cube(seed=1, n=4096, W=256, H=256, nlayers=5, D=4, s_lo=0.5, s_hi=32.0,
              alpha_lo=0.2, dist=2.5):
    """Points uniform in [-0.5, 0.5]^3 seen from `dist` along -z; projected sizes
    log-uniform in [s_lo, s_hi] px (4096 points, 256x256, 5 layers: the CPU-sized case)."""
    rng = np.random.default_rng(seed)
    xyz = rng.uniform(-0.5, 0.5, (n, 3))
    cam = camera(np.eye(3), (0.0, 0.0, dist), W, H, 60.0)
    s_star = _log_uniform(rng, s_lo, s_hi, n)
    sw = s_star * _depth(cam, xyz) / float(cam["fx"])
    alpha = rng.uniform(alpha_lo, 1.0, n)
    desc = rng.uniform(0.0, 1.0, (n, D))
    return {"points": _points(xyz, sw, alpha, desc), "cams": [cam], "nlayers": nlayers, "D": D}


def cluster_scene(seed=2, n=2_000_000, W=1920, H=1080, nlayers=8, D=4, s_lo=0.5, s_hi=128.0,
                  alpha_lo=0.1, dist=3.0):
    """Surface-like scene: 70% anisotropic clusters, 30% planar patches, one camera
    at `dist` along -z; projected sizes log-uniform in [s_lo, s_hi] px."""
    rng = np.random.default_rng(seed)
    xyz, _ = cluster_points(rng, n)
    cam = camera(np.eye(3), (0.0, 0.0, dist), W, H, 60.0)
    s_star = _log_uniform(rng, s_lo, s_hi, n)
    sw = s_star * _depth(cam, xyz) / float(cam["fx"])
    alpha = rng.uniform(alpha_lo, 1.0, n)
    desc = rng.uniform(0.0, 1.0, (n, D))
    return {"points": _points(xyz, sw, alpha, desc), "cams": [cam], "nlayers": nlayers, "D": D}


def morton_sorted(sc, bits=10):
    """The same scene with its points reordered along a Morton (Z-order) curve of their
    positions, 3 x `bits` bits: the order of a spatially coherent cloud, where consecutive
    points are neighbours in space and on screen."""
    p = sc["points"]
    xyz = np.stack([p["x"], p["y"], p["z"]], axis=1).astype(np.float64)
    lo, hi = xyz.min(axis=0), xyz.max(axis=0)
    q = ((xyz - lo) / np.maximum(hi - lo, 1e-30) * ((1 << bits) - 1)).astype(np.uint64)
    code = np.zeros(len(xyz), dtype=np.uint64)
    for b in range(bits):
        for a in range(3):
            code |= ((q[:, a] >> np.uint64(b)) & np.uint64(1)) << np.uint64(3 * b + a)
    order = np.argsort(code, kind="stable")
    out = dict(sc)
    out["points"] = {k: np.ascontiguousarray(v[order]) for k, v in p.items()}
    return out


def upstream_gradient(seed, n_values):
    """Upstream pyramid gradient, N(0, 1) float32."""
    return np.random.default_rng(seed).standard_normal(n_values).astype(np.float32)


def fd_candidate(seed, n=64, res=32, nlayers=5, D=4):
    """A 64-point subset drawn by the cluster recipe, camera fitted so the points fill a
    res x res view, projected sizes log-uniform in [0.5, 16] px.  The finite-difference
    test rejects candidates whose fragments sit near a kink and asks for the next seed."""
    rng = np.random.default_rng(seed)
    xyz, _ = cluster_points(rng, 4096)
    xyz = xyz[rng.choice(len(xyz), n, replace=False)]
    c = xyz.mean(axis=0)
    ext = float(np.max(np.abs(xyz[:, :2] - c[:2])))
    dist = 1.2 * ext / math.tan(math.radians(30.0)) + float(np.ptp(xyz[:, 2]))
    cam = camera(np.eye(3), (-c[0], -c[1], -c[2] + dist), res, res, 60.0)
    s_star = _log_uniform(rng, 0.5, 16.0, n)
    sw = s_star * _depth(cam, xyz) / float(cam["fx"])
    alpha = rng.uniform(0.1, 1.0, n)
    desc = rng.uniform(0.0, 1.0, (n, D))
    return {"points": _points(xyz, sw, alpha, desc), "cams": [cam], "nlayers": nlayers, "D": D}


def multiview_scene(seed=4, n=4_000_000, views=16, nlayers=8, D=4, sw_lo=0.002, sw_hi=0.05):
    """Clusters only, fixed world sizes; `views` cameras with mixed resolutions, directions
    uniform on the sphere, distance log-uniform in [1.2, 8], each looking at a random
    cluster centre (near cameras see few large splats, far cameras see all points small)."""
    rng = np.random.default_rng(seed)
    xyz, centres = cluster_points(rng, n, plane_frac=0.0)
    sw = _log_uniform(rng, sw_lo, sw_hi, n)
    alpha = rng.uniform(0.1, 1.0, n)
    desc = rng.uniform(0.0, 1.0, (n, D))
    cams = []
    for _ in range(views):
        W, H = RESOLUTIONS[int(rng.integers(0, len(RESOLUTIONS)))]
        d = rng.standard_normal(3)
        d /= np.linalg.norm(d)
        dist = float(_log_uniform(rng, 1.2, 8.0, 1)[0])
        target = centres[int(rng.integers(0, len(centres)))]
        cams.append(look_at(target + dist * d, target, W, H))
    return {"points": _points(xyz, sw, alpha, desc), "cams": cams, "nlayers": nlayers, "D": D}


def ring_scene(seed=5, n=8_000_000, views=8, W=2560, H=1440, nlayers=8, D=8, radius=3.0,
               elevation_deg=15.0):
    """Optimisation workload: the cluster recipe at 8M points, 8 cameras on a ring of radius 3,
    45 degrees apart at 15 degrees elevation, 2560x1440, 8 descriptor channels."""
    rng = np.random.default_rng(seed)
    xyz, _ = cluster_points(rng, n)
    cams = []
    el = math.radians(elevation_deg)
    for k in range(views):
        az = 2.0 * math.pi * k / views
        eye = radius * np.array([math.cos(el) * math.sin(az), -math.sin(el), -math.cos(el) * math.cos(az)])
        cams.append(look_at(eye, (0.0, 0.0, 0.0), W, H))
    s_star = _log_uniform(rng, 0.5, 128.0, n)
    sw = s_star * radius / float(cams[0]["fx"])
    alpha = rng.uniform(0.1, 1.0, n)
    desc = rng.uniform(0.0, 1.0, (n, D))
    return {"points": _points(xyz, sw, alpha, desc), "cams": cams, "nlayers": nlayers, "D": D}


def perturbed(points, seed, sigma=0.01, size_lo=0.5, size_hi=2.0):
    """Copy with xyz += N(0, sigma^2) and world sizes scaled by U[size_lo, size_hi]."""
    rng = np.random.default_rng(seed)
    n = len(points["x"])
    out = {k: v.copy() for k, v in points.items()}
    for k in ("x", "y", "z"):
        out[k] = (out[k] + rng.normal(0.0, sigma, n)).astype(np.float32)
    out["sw"] = (out["sw"] * rng.uniform(size_lo, size_hi, n)).astype(np.float32)
    return out


def random_small(seed, n=64, W=32, H=24, nlayers=4, D=4, s_lo=0.3, s_hi=12.0, depth_ties=False):
    """Tiny random scenes for parity tests (several tiles plus ragged edges).  With
    depth_ties, points share a handful of exact depths so index tie-breaks matter."""
    rng = np.random.default_rng(seed)
    cam = camera(np.eye(3), (0.0, 0.0, 0.0), W, H, 60.0)
    fx = float(cam["fx"])
    if depth_ties:
        z = rng.choice(np.array([1.0, 1.5, 2.0, 3.0], dtype=np.float64), n)
    else:
        z = rng.uniform(1.0, 3.0, n)
    # screen positions a little beyond the borders so edge and outside cases occur
    sx = rng.uniform(-0.1 * W, 1.1 * W, n)
    sy = rng.uniform(-0.1 * H, 1.1 * H, n)
    x = (sx - W / 2.0) * z / fx
    y = (sy - H / 2.0) * z / float(cam["fy"])
    s_star = _log_uniform(rng, s_lo, s_hi, n)
    sw = s_star * z / fx
    alpha = rng.uniform(0.05, 1.0, n)
    desc = rng.uniform(0.0, 1.0, (n, D))
    xyz = np.stack([x, y, z], axis=1)
    return {"points": _points(xyz, sw, alpha, desc), "cams": [cam], "nlayers": nlayers, "D": D}


def decoder_weights(seed, nlayers, D=4, out_dim=3, features=32):
    """Seeded weights of the reconstruction network (trained weights are not available):
    per layer a 3x3 kernel [3, 3, C_in, 2 features] with C_in = D for the coarsest layer and
    D + features otherwise, drawn N(0, 1 / (9 C_in)) and rounded to binary16 (the kernels are
    given in that format), and a bias [2 features] N(0, 0.1^2) float32; the output layer
    [features, out_dim] N(0, 1 / features) and its bias, float32."""
    rng = np.random.default_rng(seed)
    w, b = [], []
    for L in range(nlayers):
        cin = D if L == nlayers - 1 else D + features
        k = rng.standard_normal((3, 3, cin, 2 * features)) / math.sqrt(9.0 * cin)
        w.append(k.astype(np.float16))
        b.append((0.1 * rng.standard_normal(2 * features)).astype(np.float32))
    wo = (rng.standard_normal((features, out_dim)) / math.sqrt(features)).astype(np.float32)
    bo = (0.1 * rng.standard_normal(out_dim)).astype(np.float32)
    return {"w": w, "b": b, "wo": wo, "bo": bo}


def feature_pyramid(seed, W, H, nlayers, D=4, empty_frac=0.2):
    """A seeded stand-in for a rendered pyramid: per layer [H_L, W_L, D] float32 with
    W_L = ceil(W / 2^L), values U[0, 1], and a fraction of texels zero (holes)."""
    rng = np.random.default_rng(seed)
    out = []
    for L in range(nlayers):
        w_l, h_l = -(-W // (1 << L)), -(-H // (1 << L))
        a = rng.uniform(0.0, 1.0, (h_l, w_l, D)).astype(np.float32)
        a[rng.random((h_l, w_l)) < empty_frac] = 0.0
        out.append(a)
    return out
