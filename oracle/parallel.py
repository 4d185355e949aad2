"""The oracle on several host cores, by texel masks.

TEST INFRASTRUCTURE ONLY.  Only tests, the smoke check and the benchmark's CPU-baseline leg
may import this module.

The pyramid is cut into `workers` interleaved texel sets (texel k goes to set k mod workers,
so the long lists of the coarse layers spread over every set); each set is evaluated by an
unchanged call of the oracle with that set as its mask, in a thread of its own (ctypes
releases the interpreter lock for the call).  Nothing of the oracle's arithmetic is touched:
- forward: a texel's list, length, ids and colour depend only on that texel's own fragments
  (Sec. 3.2, Eq. 6-7), so every texel is taken from the one call that evaluated it;
- backward: the gradient of sum(G * pyramid) is a sum over texels of each texel's adjoint,
  and the chain rule through the projection is linear in the per-point sums, so the
  gradients of the calls add up to the gradient of the whole pyramid (in double precision,
  up to the order of the final additions).
Coarser-layer inclusion is not split this way (a texel's list reaches into other texels).
"""
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

from oracle import oracle


def default_workers():
    """Host threads to use: OMP_NUM_THREADS when set (the CPU share of a GPU host), else
    every core, at most 16."""
    env = os.environ.get("OMP_NUM_THREADS")
    n = int(env) if env and env.isdigit() and int(env) > 0 else (os.cpu_count() or 1)
    return max(1, min(16, n))


def _masks(P, workers, mask=None):
    k = np.arange(P) % workers
    base = np.ones(P, dtype=bool) if mask is None else np.asarray(mask).astype(bool)
    return [((k == w) & base).astype(np.uint8) for w in range(workers)]


def forward(pts, cam, nlayers, workers=None, mask=None, **kw):
    """oracle.forward_ex over `workers` threads; same result dict (pyr, counts, ids, alpha)."""
    workers = workers or default_workers()
    P = oracle.num_pixels(cam["W"], cam["H"], nlayers)
    masks = _masks(P, workers, mask)
    with ThreadPoolExecutor(workers) as ex:
        parts = list(ex.map(lambda m: oracle.forward_ex(pts, cam, nlayers, mask=m, **kw), masks))
    out = {k: np.array(v, copy=True) for k, v in parts[0].items()}
    for m, part in zip(masks[1:], parts[1:]):
        sel = m.astype(bool)
        for k in out:
            out[k][sel] = part[k][sel]
    return out


def backward(pts, cam, nlayers, G, workers=None, mask=None, **kw):
    """oracle.backward_ex over `workers` threads; same result dict (gradients summed over
    the texel sets; gbg taken per texel)."""
    workers = workers or default_workers()
    P = oracle.num_pixels(cam["W"], cam["H"], nlayers)
    masks = _masks(P, workers, mask)
    with ThreadPoolExecutor(workers) as ex:
        parts = list(ex.map(lambda m: oracle.backward_ex(pts, cam, nlayers, G, mask=m, **kw),
                            masks))
    out = {k: np.zeros_like(v) for k, v in parts[0].items()}
    for m, part in zip(masks, parts):
        sel = m.astype(bool)
        for k, v in part.items():
            if k == "gbg":
                out[k][sel] = v[sel]
            else:
                out[k] += v
    return out
