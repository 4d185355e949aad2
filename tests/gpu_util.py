"""Helpers for the GPU parity tests: run the HIP path through the C ABI and the oracle on
the same seeded inputs."""
import numpy as np

from oracle import oracle

PARAMS = ("x", "y", "z", "sw", "alpha", "desc")
GRAD_KEY = {"x": "gx", "y": "gy", "z": "gz", "sw": "gsw", "alpha": "galpha", "desc": "gdesc"}

# Pyramid tolerance.  Every term of a blended texel is non-negative (gamma, T, tau >= 0),
# so the single-precision result has a relative error of at most about
# (4 roundings of gamma + 16 of T + 16 of the sum) * 2^-24 < 3e-6; the bar is 1e-5.
PYR_RTOL = 1e-5


def to_device(pts, dev):
    import torch
    return {k: torch.from_numpy(np.ascontiguousarray(pts[k])).to(dev) for k in PARAMS}


def renderer(sc, dev, tuning=None, cams=None, include_coarser=False):
    import paper_2401_06003_amd as tp
    cams = sc["cams"] if cams is None else cams
    return tp.Renderer(cams, sc["nlayers"], sc["D"], len(sc["points"]["x"]), tuning=tuning,
                       device=dev, include_coarser=include_coarser)


def gpu_forward(sc, dev, tuning=None, cams=None):
    """(per-view pyramids [P_v, D], counts, ids) from one batched call over `cams`."""
    import torch
    r = renderer(sc, dev, tuning, cams)
    t = to_device(sc["points"], dev)
    out = r.forward(*[t[k] for k in PARAMS])
    counts, ids = r.export_fragments()
    torch.cuda.synchronize()
    out = out.cpu().numpy().astype(np.float64).reshape(-1, sc["D"])
    counts = counts.cpu().numpy()
    ids = ids.cpu().numpy().astype(np.int64)
    res, o = [], 0
    for pv in r.view_texels:
        res.append((out[o:o + pv], counts[o:o + pv], ids[o:o + pv]))
        o += pv
    return res, r, t


def assert_pyramid(got, want, where=""):
    bad = ~(np.abs(got - want) <= PYR_RTOL * np.abs(want))
    if bad.any():
        k = np.argwhere(bad)[0]
        raise AssertionError("%s pyramid differs at %s: gpu %r oracle %r (%d bad)" %
                             (where, tuple(k), got[tuple(k)], want[tuple(k)], int(bad.sum())))


def assert_lists(counts, ids, ocounts, oids, where=""):
    if not np.array_equal(counts, ocounts):
        k = int(np.argmax(counts != ocounts))
        raise AssertionError("%s list length differs at texel %d: gpu %d oracle %d" %
                             (where, k, counts[k], ocounts[k]))
    if not np.array_equal(ids, oids):
        k = int(np.argmax(np.any(ids != oids, axis=1)))
        raise AssertionError("%s kept fragments differ at texel %d: gpu %s oracle %s" %
                             (where, k, ids[k], oids[k]))


def check_forward(sc, dev, tuning=None):
    res, r, t = gpu_forward(sc, dev, tuning)
    for v, cam in enumerate(sc["cams"]):
        pyr, counts, ids = oracle.forward(sc["points"], cam, sc["nlayers"])
        assert_lists(res[v][1], res[v][2], counts, ids, "view %d" % v)
        assert_pyramid(res[v][0], pyr, "view %d" % v)
    return res, r, t


def grad_close(g, o, name, rtol_norm=1e-4, rtol=1e-3, atol_rel=1e-5):
    """Gradients: single precision, fixed-order sums, against the double-precision adjoint.
    Per tensor ||g - o|| <= rtol_norm ||o||; per element |g - o| <= rtol |o| + atol_rel max|o|."""
    g = np.asarray(g, dtype=np.float64)
    o = np.asarray(o, dtype=np.float64)
    no = np.linalg.norm(o)
    if no == 0:
        assert np.all(g == 0), name
        return 0.0
    e = np.linalg.norm(g - o) / no
    assert e <= rtol_norm, (name, e)
    bad = np.abs(g - o) > rtol * np.abs(o) + atol_rel * np.abs(o).max()
    assert not bad.any(), (name, int(bad.sum()), g[bad][:4], o[bad][:4])
    return e
