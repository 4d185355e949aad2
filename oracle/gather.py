"""Brute-force *gather* oracle for tiny scenes (pure Python, exact rational arithmetic).

TEST INFRASTRUCTURE ONLY.  Only tests may import this module.

This is a second, independent formulation of the same definition as the C
scatter oracle: instead of emitting each point's footprint, it visits every texel
of every layer and asks every point how much it contributes there, evaluating the
paper's formulas directly:
  - layer pair floor(log2 s), ceil(log2 s) and iota = 1 - |s - 2^L| / (2^Lup - 2^Llo)
    (Sec. 3.1, Eq. 5), s < 1 -> layer 0 with eps + (1 - eps) s;
  - beta = (1 - |u - i|)(1 - |v - j|) for the texel centre at integer (i, j) in
    layer-texel units, non-zero iff |u - i| < 1 and |v - j| < 1 (Eq. 4);
  - gamma = beta * iota * alpha (Eq. 3);
  - the list of the texel is sorted by depth then index and clamped to 16
    (Sec. 3.2), and blended front to back (Eq. 6-7).
Single-precision steps (the projection and u, v) are evaluated as exact rationals
and rounded once to the nearest binary32 value, ties to even, which is what IEEE
single precision arithmetic (including a fused multiply-add) defines.
"""
from fractions import Fraction as Fr
import math

import numpy as np

_F32_MAX_EXP = 127
_F32_MIN_EXP = -126
_F32_MANT = 23


def round_f32(q):
    """Round an exact rational to the nearest binary32 value (ties to even)."""
    q = Fr(q)
    if q == 0:
        return Fr(0)
    sign = -1 if q < 0 else 1
    a = -q if q < 0 else q
    # exponent e with 2^e <= a < 2^(e+1)
    e = math.frexp(float(a))[1] - 1
    while Fr(2) ** e > a:
        e -= 1
    while Fr(2) ** (e + 1) <= a:
        e += 1
    if e < _F32_MIN_EXP:
        quantum = Fr(2) ** (_F32_MIN_EXP - _F32_MANT)
    else:
        quantum = Fr(2) ** (e - _F32_MANT)
    m = a / quantum
    lo = m.numerator // m.denominator
    rem = m - lo
    if rem > Fr(1, 2) or (rem == Fr(1, 2) and lo % 2 == 1):
        lo += 1
    r = lo * quantum
    if r >= Fr(2) ** (_F32_MAX_EXP + 1):
        return None  # overflow -> infinity
    return sign * r


def f32(x):
    return Fr(float(np.float32(x)))


def _op(q):
    r = round_f32(q)
    if r is None:
        raise OverflowError
    return r


def project_point(X, Y, Z, sw, cam):
    """Single-precision pinhole projection with the fixed operation order:
    Xc = fma(R0, X, fma(R1, Y, fma(R2, Z, t0))) (likewise Yc, Zc), x = fma(fx, Xc/Zc, cx),
    y = fma(fy, Yc/Zc, cy), s = (fx * sw) / Zc.  Returns None when culled."""
    R = [f32(r) for r in np.asarray(cam["R"]).reshape(9)]
    t = [f32(v) for v in np.asarray(cam["t"]).reshape(3)]
    fx, fy, cx, cy = f32(cam["fx"]), f32(cam["fy"]), f32(cam["cx"]), f32(cam["cy"])
    X, Y, Z, sw = f32(X), f32(Y), f32(Z), f32(sw)
    try:
        rows = []
        for r in range(3):
            inner = _op(R[3 * r + 2] * Z + t[r])
            mid = _op(R[3 * r + 1] * Y + inner)
            rows.append(_op(R[3 * r + 0] * X + mid))
        Xc, Yc, Zc = rows
        if not (Zc > f32(cam.get("znear", 0.01))):
            return None
        x = _op(fx * _op(Xc / Zc) + cx)
        y = _op(fy * _op(Yc / Zc) + cy)
        s = _op(_op(fx * sw) / Zc)
    except OverflowError:
        return None
    if not (s > 0):
        return None
    return x, y, Zc, s


def layer_weights(s, nlayers, eps):
    """{layer: iota} for screen size s (exact rational)."""
    if s < 1:
        return {0: float(Fr(eps) + (1 - Fr(eps)) * s)}
    smax = Fr(2) ** (nlayers - 1)
    if s >= smax:
        return {nlayers - 1: 1.0}
    lo = 0
    while Fr(2) ** (lo + 1) <= s:
        lo += 1
    up = lo if Fr(2) ** lo == s else lo + 1
    if lo == up:
        return {lo: 1.0}
    den = Fr(2) ** up - Fr(2) ** lo
    return {L: float(1 - abs(s - Fr(2) ** L) / den) for L in (lo, up)}


def render(pts, cam, nlayers, maxlist=16, eps=0.25):
    """Returns (pyr [P, D], counts [P], ids [P, maxlist]) like oracle.forward (fp32 mode)."""
    n = len(pts["x"])
    desc = np.asarray(pts["desc"], dtype=np.float64).reshape(n, -1)
    D = desc.shape[1]
    W, H = int(cam["W"]), int(cam["H"])
    proj = []
    for p in range(n):
        r = project_point(pts["x"][p], pts["y"][p], pts["z"][p], pts["sw"][p], cam)
        if r is None:
            proj.append(None)
            continue
        x, y, z, s = r
        proj.append((x, y, z, layer_weights(s, nlayers, eps)))
    dims = [(-(-W // (1 << L)), -(-H // (1 << L))) for L in range(nlayers)]
    P = sum(w * h for w, h in dims)
    pyr = np.zeros((P, D))
    counts = np.zeros(P, dtype=np.int32)
    ids = np.full((P, maxlist), -1, dtype=np.int64)
    base = 0
    for L, (WL, HL) in enumerate(dims):
        # single-precision texel coordinates u = x / 2^L - 0.5 of every point in this layer
        uv = {}
        for p, pr in enumerate(proj):
            if pr is None or L not in pr[3]:
                continue
            x, y, z, lw = pr
            u = _op(x / Fr(2) ** L - Fr(1, 2))
            v = _op(y / Fr(2) ** L - Fr(1, 2))
            uv[p] = (u, v, z, lw[L])
        for j in range(HL):
            for i in range(WL):
                lst = []
                for p, (u, v, z, iota) in uv.items():
                    du, dv = abs(u - i), abs(v - j)
                    if du < 1 and dv < 1:
                        wx, wy = float(1 - du), float(1 - dv)
                        gamma = ((wx * wy) * iota) * float(np.float32(pts["alpha"][p]))
                        lst.append((z, p, gamma))
                lst.sort(key=lambda e: (e[0], e[1]))
                pix = base + j * WL + i
                counts[pix] = len(lst)
                T = 1.0
                for m, (z, p, gamma) in enumerate(lst[:maxlist]):
                    ids[pix, m] = p
                    w = T * gamma
                    for d in range(D):
                        pyr[pix, d] += w * float(np.float32(desc[p, d]))
                    T = T * (1.0 - gamma)
        base += WL * HL
    return pyr, counts, ids
