"""Points placed so that their single-precision projection is exact.

Camera: R = I, t = 0, fx = fy = 256 (a power of two), so a point at depth Z = 2^k with
X = (x - cx) * Z / 256 lands exactly on screen x, and world size sw = s * Z / 256 gives
screen size exactly s.  Used by the closed-form pins."""
import numpy as np


def cam(W, H, cx=None, cy=None):
    return {"R": np.eye(3, dtype=np.float32).reshape(9), "t": np.zeros(3, dtype=np.float32),
            "fx": np.float32(256.0), "fy": np.float32(256.0),
            "cx": np.float32(W / 2.0 if cx is None else cx),
            "cy": np.float32(H / 2.0 if cy is None else cy), "W": int(W), "H": int(H),
            "znear": np.float32(0.01)}


def points(c, sx, sy, s, depth, alpha, desc):
    """Exact world coordinates for screen positions sx, sy, sizes s, depths (powers of two)."""
    sx, sy, s, depth = (np.atleast_1d(np.asarray(v, dtype=np.float64)) for v in (sx, sy, s, depth))
    n = len(sx)
    X = (sx - float(c["cx"])) * depth / 256.0
    Y = (sy - float(c["cy"])) * depth / 256.0
    sw = s * depth / 256.0
    for arr in (X, Y, sw):
        assert np.all(arr.astype(np.float32).astype(np.float64) == arr), "not exactly representable"
    return {"x": X.astype(np.float32), "y": Y.astype(np.float32), "z": depth.astype(np.float32),
            "sw": sw.astype(np.float32),
            "alpha": np.broadcast_to(np.asarray(alpha, dtype=np.float32), (n,)).copy(),
            "desc": np.asarray(desc, dtype=np.float32).reshape(n, -1)}
