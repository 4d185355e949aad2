"""ctypes wrapper around the C oracle (trips_oracle.c).

TEST INFRASTRUCTURE ONLY.  Only tests, the smoke check and the benchmark's
CPU-baseline leg may import this module.

Scene convention (plain dicts of numpy arrays, shared with the GPU tests through
the seeded generators, which hold none of the method's arithmetic):
  points: x, y, z, sw, alpha  -> [N] arrays; desc -> [N, D]
  camera: R (9, row-major world->camera), t (3), fx, fy, cx, cy, W, H, znear
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "trips_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force=False):
    """Compile the oracle with gcc (no fast-math, no FP contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
                               "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        override = os.environ.get("TRIPS_ORACLE_LIB")
        if override:  # a test build of the oracle (see tests/test_oracle_mutations.py)
            _lib = _configure(ctypes.CDLL(override))
        else:
            build()
            _lib = _configure(ctypes.CDLL(_LIB))
    return _lib


class use_library:
    """Context manager: route every call of this module to another build of the oracle
    (used by the tests that plant mistakes in a copy of the source)."""

    def __init__(self, path):
        self.path = path

    def __enter__(self):
        global _lib
        self.saved = _lib
        _lib = _configure(ctypes.CDLL(self.path))
        return _lib

    def __exit__(self, *exc):
        global _lib
        _lib = self.saved
        return False


def _configure(L):
    if True:
        dp = ctypes.POINTER(ctypes.c_double)
        i32p = ctypes.POINTER(ctypes.c_int32)
        i64p = ctypes.POINTER(ctypes.c_int64)
        i64, c_int, c_double = ctypes.c_int64, ctypes.c_int, ctypes.c_double
        L.oracle_num_pixels.argtypes = [c_int, c_int, c_int]
        L.oracle_num_pixels.restype = i64
        L.oracle_project.argtypes = [i64, dp, dp, dp, dp, dp, c_int, c_int, c_int, c_double, c_int,
                                     i32p, dp]
        L.oracle_project.restype = c_int
        L.oracle_fragments.argtypes = [i64, dp, dp, dp, dp, dp, dp, c_int, c_int, c_int, c_double,
                                       c_int, i64, i64p, dp]
        L.oracle_fragments.restype = i64
        u8p = ctypes.c_void_p
        L.oracle_forward.argtypes = [i64, dp, dp, dp, dp, dp, dp, c_int, dp, c_int, c_int, c_int,
                                     c_int, c_double, c_int, u8p, dp, i32p, i64p]
        L.oracle_forward.restype = c_int
        L.oracle_backward.argtypes = [i64, dp, dp, dp, dp, dp, dp, c_int, dp, c_int, c_int, c_int,
                                      c_int, c_double, c_int, u8p, dp, dp, dp, dp, dp, dp, dp]
        L.oracle_backward.restype = c_int
        L.oracle_forward_ex.argtypes = [i64, dp, dp, dp, dp, dp, dp, c_int, dp, c_int, c_int,
                                        c_int, c_int, c_double, c_int, c_int, u8p, u8p, dp, i32p,
                                        i64p, u8p]
        L.oracle_forward_ex.restype = c_int
        L.oracle_backward_ex.argtypes = [i64, dp, dp, dp, dp, dp, dp, c_int, dp, c_int, c_int,
                                         c_int, c_int, c_double, c_int, c_int, u8p, u8p, dp, u8p,
                                         dp, dp, dp, dp, dp, dp, u8p, u8p]
        L.oracle_backward_ex.restype = c_int
    return L


def _d(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _ptr(a, ct=ctypes.c_double):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def cam_vector(cam):
    """R(9), t(3), fx, fy, cx, cy, znear as float64 (17 values)."""
    v = np.zeros(17, dtype=np.float64)
    v[0:9] = np.asarray(cam["R"], dtype=np.float64).reshape(9)
    v[9:12] = np.asarray(cam["t"], dtype=np.float64).reshape(3)
    v[12], v[13], v[14], v[15] = cam["fx"], cam["fy"], cam["cx"], cam["cy"]
    v[16] = cam.get("znear", 0.01)
    return v


def layer_dims(W, H, nlayers):
    """[(W_L, H_L)] with W_L = ceil(W / 2^L)."""
    return [(-(-W // (1 << L)), -(-H // (1 << L))) for L in range(nlayers)]


def num_pixels(W, H, nlayers):
    return int(lib().oracle_num_pixels(int(W), int(H), int(nlayers)))


def project(pts, cam, nlayers, eps=0.25, fp32=True):
    n = len(pts["x"])
    X, Y, Z, S = (_d(pts[k]) for k in ("x", "y", "z", "sw"))
    cv = cam_vector(cam)
    valid = np.zeros(n, dtype=np.int32)
    out = np.zeros((n, 4), dtype=np.float64)
    rc = lib().oracle_project(n, _ptr(X), _ptr(Y), _ptr(Z), _ptr(S), _ptr(cv), int(cam["W"]),
                              int(cam["H"]), int(nlayers), float(eps), int(fp32),
                              _ptr(valid, ctypes.c_int32), _ptr(out))
    assert rc == 0, rc
    return valid.astype(bool), out


def fragments(pts, cam, nlayers, eps=0.25, fp32=True):
    """All fragments in (layer pixel, depth, index) order.

    Returns dict with idx, L, i, j (int64) and gamma, beta, iota, z (float64)."""
    n = len(pts["x"])
    X, Y, Z, S, A = (_d(pts[k]) for k in ("x", "y", "z", "sw", "alpha"))
    cv = cam_vector(cam)
    cap = 8 * max(n, 1)
    ints = np.zeros((cap, 4), dtype=np.int64)
    reals = np.zeros((cap, 4), dtype=np.float64)
    nf = lib().oracle_fragments(n, _ptr(X), _ptr(Y), _ptr(Z), _ptr(S), _ptr(A), _ptr(cv),
                                int(cam["W"]), int(cam["H"]), int(nlayers), float(eps), int(fp32),
                                cap, _ptr(ints, ctypes.c_int64), _ptr(reals))
    assert nf >= 0, nf
    return {"idx": ints[:nf, 0], "L": ints[:nf, 1], "i": ints[:nf, 2], "j": ints[:nf, 3],
            "gamma": reals[:nf, 0], "beta": reals[:nf, 1], "iota": reals[:nf, 2],
            "z": reals[:nf, 3]}


def _mask_ptr(mask, P):
    if mask is None:
        return None, ctypes.c_void_p(0)
    m = np.ascontiguousarray(np.asarray(mask, dtype=np.uint8))
    assert m.shape == (P,)
    return m, ctypes.c_void_p(m.ctypes.data)


def forward(pts, cam, nlayers, maxlist=16, eps=0.25, fp32=True, mask=None):
    """One view.  Returns (pyr [P, D] float64, counts [P] int32, ids [P, maxlist] int64).

    Rows are the texels of all layers concatenated, each layer row-major.  With a [P]
    boolean mask only those texels are evaluated (others stay 0 / -1)."""
    n = len(pts["x"])
    X, Y, Z, S, A = (_d(pts[k]) for k in ("x", "y", "z", "sw", "alpha"))
    desc = _d(pts["desc"]).reshape(n, -1) if n else np.zeros((0, pts["desc"].shape[-1]))
    D = desc.shape[1]
    cv = cam_vector(cam)
    P = num_pixels(cam["W"], cam["H"], nlayers)
    pyr = np.zeros((P, D), dtype=np.float64)
    counts = np.zeros(P, dtype=np.int32)
    ids = np.zeros((P, maxlist), dtype=np.int64)
    keep, mp = _mask_ptr(mask, P)
    rc = lib().oracle_forward(n, _ptr(X), _ptr(Y), _ptr(Z), _ptr(S), _ptr(A), _ptr(desc), D,
                              _ptr(cv), int(cam["W"]), int(cam["H"]), int(nlayers), int(maxlist),
                              float(eps), int(fp32), mp, _ptr(pyr), _ptr(counts, ctypes.c_int32),
                              _ptr(ids, ctypes.c_int64))
    assert rc == 0, rc
    return pyr, counts, ids


def backward(pts, cam, nlayers, G, maxlist=16, eps=0.25, fp32=True, mask=None):
    """One view: gradients of sum(G * pyramid).  G is [P, D].  With a texel mask only
    those texels contribute (exact for points whose texels are all in the mask).

    Returns dict gx, gy, gz, gsw, galpha [N] and gdesc [N, D] (float64)."""
    n = len(pts["x"])
    X, Y, Z, S, A = (_d(pts[k]) for k in ("x", "y", "z", "sw", "alpha"))
    desc = _d(pts["desc"]).reshape(n, -1)
    D = desc.shape[1]
    cv = cam_vector(cam)
    Gd = _d(G).reshape(-1, D)
    assert Gd.shape[0] == num_pixels(cam["W"], cam["H"], nlayers)
    out = {k: np.zeros(n, dtype=np.float64) for k in ("gx", "gy", "gz", "gsw", "galpha")}
    out["gdesc"] = np.zeros((n, D), dtype=np.float64)
    keep, mp = _mask_ptr(mask, Gd.shape[0])
    rc = lib().oracle_backward(n, _ptr(X), _ptr(Y), _ptr(Z), _ptr(S), _ptr(A), _ptr(desc), D,
                               _ptr(cv), int(cam["W"]), int(cam["H"]), int(nlayers), int(maxlist),
                               float(eps), int(fp32), mp, _ptr(Gd), _ptr(out["gx"]), _ptr(out["gy"]),
                               _ptr(out["gz"]), _ptr(out["gsw"]), _ptr(out["galpha"]),
                               _ptr(out["gdesc"]))
    assert rc == 0, rc
    return out


def _opt(a):
    """(keep-alive array, void pointer) of an optional float64 array."""
    if a is None:
        return None, ctypes.c_void_p(0)
    a = _d(a)
    return a, ctypes.c_void_p(a.ctypes.data)


def forward_ex(pts, cam, nlayers, background=None, maxlist=16, eps=0.25, fp32=True, mask=None,
               coarser=False):
    """forward() with the optional terms: background [P, D] composited behind the kept
    list with the transmittance it leaves; coarser: every texel also blends the fragments
    of the coarser layers' texels that cover it.  Returns dict pyr [P, D], counts (own
    fragments), ids (the blended list) and alpha [P] (the coverage 1 - T_K)."""
    n = len(pts["x"])
    X, Y, Z, S, A = (_d(pts[k]) for k in ("x", "y", "z", "sw", "alpha"))
    desc = _d(pts["desc"]).reshape(n, -1) if n else np.zeros((0, pts["desc"].shape[-1]))
    D = desc.shape[1]
    cv = cam_vector(cam)
    P = num_pixels(cam["W"], cam["H"], nlayers)
    out = {"pyr": np.zeros((P, D)), "counts": np.zeros(P, dtype=np.int32),
           "ids": np.zeros((P, maxlist), dtype=np.int64), "alpha": np.zeros(P)}
    keep, mp = _mask_ptr(mask, P)
    bgk, bgp = _opt(None if background is None else np.asarray(background).reshape(P, D))
    rc = lib().oracle_forward_ex(n, _ptr(X), _ptr(Y), _ptr(Z), _ptr(S), _ptr(A), _ptr(desc), D,
                                 _ptr(cv), int(cam["W"]), int(cam["H"]), int(nlayers),
                                 int(maxlist), float(eps), int(fp32), int(bool(coarser)), mp, bgp,
                                 _ptr(out["pyr"]),
                                 _ptr(out["counts"], ctypes.c_int32),
                                 _ptr(out["ids"], ctypes.c_int64),
                                 ctypes.c_void_p(out["alpha"].ctypes.data))
    assert rc == 0, rc
    return out


def backward_ex(pts, cam, nlayers, G, background=None, grad_alpha=None, maxlist=16, eps=0.25,
                fp32=True, mask=None, coarser=False):
    """backward() with the optional terms: the background the forward composited, the
    upstream gradient of the coverage, and the gradients of the background (gbg [P, D])
    and of the camera (gcam [16]: dR row-major, dt, dfx, dfy, dcx, dcy); coarser as in
    forward_ex."""
    n = len(pts["x"])
    X, Y, Z, S, A = (_d(pts[k]) for k in ("x", "y", "z", "sw", "alpha"))
    desc = _d(pts["desc"]).reshape(n, -1)
    D = desc.shape[1]
    cv = cam_vector(cam)
    Gd = _d(G).reshape(-1, D)
    P = Gd.shape[0]
    assert P == num_pixels(cam["W"], cam["H"], nlayers)
    out = {k: np.zeros(n) for k in ("gx", "gy", "gz", "gsw", "galpha")}
    out["gdesc"] = np.zeros((n, D))
    out["gbg"] = np.zeros((P, D))
    out["gcam"] = np.zeros(16)
    keep, mp = _mask_ptr(mask, P)
    bgk, bgp = _opt(None if background is None else np.asarray(background).reshape(P, D))
    gak, gap = _opt(None if grad_alpha is None else np.asarray(grad_alpha).reshape(P))
    rc = lib().oracle_backward_ex(n, _ptr(X), _ptr(Y), _ptr(Z), _ptr(S), _ptr(A), _ptr(desc), D,
                                  _ptr(cv), int(cam["W"]), int(cam["H"]), int(nlayers),
                                  int(maxlist), float(eps), int(fp32), int(bool(coarser)), mp, bgp,
                                  _ptr(Gd), gap,
                                  _ptr(out["gx"]), _ptr(out["gy"]), _ptr(out["gz"]),
                                  _ptr(out["gsw"]), _ptr(out["galpha"]), _ptr(out["gdesc"]),
                                  ctypes.c_void_p(out["gbg"].ctypes.data),
                                  ctypes.c_void_p(out["gcam"].ctypes.data))
    assert rc == 0, rc
    return out


def texel_index(cam, nlayers, L, i, j):
    """Row of texel (i, j) of layer L in the concatenated pyramid of one view."""
    dims = layer_dims(cam["W"], cam["H"], nlayers)
    base = np.cumsum([0] + [w * h for w, h in dims])
    L = np.asarray(L)
    W = np.array([w for w, _ in dims])[L]
    return base[L] + np.asarray(j) * W + np.asarray(i)


def split_layers(flat, cam, nlayers):
    """Split a [P, ...] per-texel array into per-layer [H_L, W_L, ...] views."""
    outs, o = [], 0
    for (wl, hl) in layer_dims(cam["W"], cam["H"], nlayers):
        outs.append(flat[o:o + wl * hl].reshape((hl, wl) + flat.shape[1:]))
        o += wl * hl
    return outs
