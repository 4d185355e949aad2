"""The reconstruction network of Sec. 3.3 (Fig. conv) in plain numpy, double precision.

TEST INFRASTRUCTURE ONLY.  Only tests, the smoke check and the benchmark's CPU-baseline leg
may import this module; the GPU library never does.

The network turns the renderer's feature pyramid (n layers of D channels) into one
full-resolution image.  The paper describes it in words and a figure only; the readings
taken here (each is one branch or constant below):
- one block per pyramid layer, run from the coarsest layer to the finest, F = 32 features;
- a block's input is its layer's D feature channels followed, for every layer but the
  coarsest, by the 32 channels of the next coarser block's output upsampled to this layer;
- a block is one gated convolution (the gating of Yu et al., "free-form inpainting"):
  a 3x3 convolution, stride 1, zero padding 1, with 2F outputs, the first F passed through
  ELU, the last F through the logistic sigmoid, multiplied channel by channel;
- the self-bypass adds the block's upsampled input features to its output (every block but
  the coarsest, which has no such input);
- upsampling by two is bilinear with texel centres at half-integer positions (texel k of the
  coarser layer is centred where texels 2k and 2k+1 of the finer layer meet, the pyramid's
  texel convention), edge texels repeated, cropped to the finer layer's size;
- the finest block's features go through a 1x1 convolution to `out_dim` output channels.

Precision: with fp16=True every value the GPU stores in binary16 is rounded to binary16
(nearest, ties to even) at the same point: the layer's features and the upsampled features
as a block reads them, and every block's output; the arithmetic between those points is
double precision.  With fp16=False nothing is rounded.

Weights: per layer L a kernel `w[L]` of shape [3, 3, C_in(L), 2F] (tap row, tap column, input
channel, output channel; outputs 0..F-1 are the feature half, F..2F-1 the gate half) with
C_in = D for the coarsest layer and D + F otherwise (the layer's features first), a bias
`b[L]` [2F]; the output layer `wo` [F, out_dim] and `bo` [out_dim].
"""
import numpy as np

F = 32


def r16(a, on=True):
    """Round to binary16 (nearest even) and back to double, when on."""
    a = np.asarray(a, dtype=np.float64)
    return a.astype(np.float16).astype(np.float64) if on else a


def elu(x):
    """ELU with unit scale: x for x > 0, exp(x) - 1 otherwise."""
    return np.where(x > 0, x, np.expm1(np.minimum(x, 0.0)))


def sigmoid(x):
    """Logistic function 1 / (1 + exp(-x)), in the form that never overflows."""
    x = np.asarray(x, dtype=np.float64)
    e = np.exp(-np.abs(x))
    return np.where(x >= 0, 1.0 / (1.0 + e), e / (1.0 + e))


def _up_axis(a, n_out, axis):
    """Bilinear doubling along one axis: finer texel i sits at coarser position i/2 - 1/4,
    so an even i takes 1/4 of texel i/2 - 1 and 3/4 of texel i/2, an odd i takes 3/4 of
    texel (i-1)/2 and 1/4 of texel (i+1)/2; indices past either edge repeat the edge."""
    n_in = a.shape[axis]
    i = np.arange(n_out)
    k = i // 2
    near = np.clip(k, 0, n_in - 1)
    far = np.clip(np.where(i % 2 == 0, k - 1, k + 1), 0, n_in - 1)
    return 0.75 * np.take(a, near, axis=axis) + 0.25 * np.take(a, far, axis=axis)


def upsample2(h, H_out, W_out):
    """[H1, W1, C] -> [H_out, W_out, C] with H_out in {2 H1 - 1, 2 H1} (likewise W)."""
    h = np.asarray(h, dtype=np.float64)
    return _up_axis(_up_axis(h, H_out, 0), W_out, 1)


def conv3x3(x, w, b):
    """Cross-correlation with zero padding 1: out[y, x, o] = b[o] + sum over the 3x3 taps
    (dy, dx) and input channels c of xpad[y + dy, x + dx, c] w[dy, dx, c, o] (one matrix
    product per tap)."""
    x = np.asarray(x, dtype=np.float64)
    H, W, C = x.shape
    xp = np.zeros((H + 2, W + 2, C))
    xp[1:-1, 1:-1] = x
    out = np.broadcast_to(np.asarray(b, dtype=np.float64), (H, W, w.shape[3])).copy()
    for dy in range(3):
        for dx in range(3):
            out += xp[dy:dy + H, dx:dx + W].reshape(H * W, C).dot(
                np.asarray(w[dy, dx], dtype=np.float64)).reshape(H, W, -1)
    return out


def gated(x, w, b):
    """One gated convolution: ELU of the feature half times the sigmoid of the gate half."""
    a = conv3x3(x, w, b)
    return elu(a[..., :F]) * sigmoid(a[..., F:])


def block(feat, coarse, w, b, fp16=True):
    """One layer's block.  feat [H, W, D] (the layer's features), coarse [H1, W1, F] or None
    (the coarser block's output); returns the block's output [H, W, F] (rounded to binary16
    when fp16)."""
    feat = r16(feat, fp16)
    H, W, _ = feat.shape
    if coarse is None:
        return r16(gated(feat, w, b), fp16)
    up = r16(upsample2(coarse, H, W), fp16)
    return r16(gated(np.concatenate([feat, up], axis=2), w, b) + up, fp16)


def output_layer(h, wo, bo):
    """1x1 convolution of the finest block's features: [H, W, F] -> [H, W, out_dim]."""
    H, W, _ = h.shape
    return (h.reshape(H * W, F).dot(np.asarray(wo, dtype=np.float64)) +
            np.asarray(bo, dtype=np.float64)).reshape(H, W, -1)


def decode(layers, weights, fp16=True):
    """layers: the pyramid as a list of [H_L, W_L, D] arrays, finest first.  Returns
    (image [H_0, W_0, out_dim], [block outputs, finest first])."""
    n = len(layers)
    hs = [None] * n
    for L in range(n - 1, -1, -1):
        hs[L] = block(layers[L], hs[L + 1] if L + 1 < n else None, weights["w"][L],
                      weights["b"][L], fp16)
    return output_layer(hs[0], weights["wo"], weights["bo"]), hs
