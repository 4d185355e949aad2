"""Pins of the reconstruction-network oracle (Sec. 3.3, Fig. conv) against what the
mathematics fixes: a brute-force loop convolution, a library correlation, a library
bilinear upsampling, exact reproduction of affine functions, the limits of the gate, closed
forms of the self-bypass and of the channel order, and binary16 storage.  The paper prints
no numbers for the network (and no trained weights exist), so the structural readings
themselves are unpinned against the paper; planted mistakes in copies of the functions must
each fail a pin here."""
import numpy as np
import pytest

import scenes
from oracle import decoder as dec

F = dec.F


def brute_conv(x, w, b):
    """Pure-Python loops: out[y][x][o] = b[o] + sum x[y+dy-1][x+dx-1][c] w[dy][dx][c][o]."""
    H, W, C = x.shape
    O = w.shape[3]
    out = np.zeros((H, W, O))
    for yy in range(H):
        for xx in range(W):
            for o in range(O):
                s = float(b[o])
                for dy in range(3):
                    for dx in range(3):
                        sy, sx = yy + dy - 1, xx + dx - 1
                        if 0 <= sy < H and 0 <= sx < W:
                            for c in range(C):
                                s += float(x[sy, sx, c]) * float(w[dy, dx, c, o])
                out[yy, xx, o] = s
    return out


def test_conv_matches_brute_force_loops():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((4, 5, 3))
    w = rng.standard_normal((3, 3, 3, 2))
    b = rng.standard_normal(2)
    assert np.allclose(dec.conv3x3(x, w, b), brute_conv(x, w, b), rtol=1e-13, atol=1e-13)


def test_conv_matches_library_correlation():
    from scipy.signal import correlate2d
    rng = np.random.default_rng(2)
    x = rng.standard_normal((7, 6, 4))
    w = rng.standard_normal((3, 3, 4, 3))
    b = np.zeros(3)
    got = dec.conv3x3(x, w, b)
    for o in range(3):
        ref = sum(correlate2d(x[..., c], w[..., c, o], mode="same", boundary="fill")
                  for c in range(4))
        assert np.allclose(got[..., o], ref, rtol=1e-13, atol=1e-13)


def test_conv_delta_places_the_kernel():
    """A unit impulse at (y0, x0) gives w[dy, dx] at output (y0 + 1 - dy, x0 + 1 - dx)."""
    w = np.arange(9 * 2, dtype=np.float64).reshape(3, 3, 1, 2)
    x = np.zeros((5, 5, 1))
    x[2, 2, 0] = 1.0
    out = dec.conv3x3(x, w, np.zeros(2))
    for dy in range(3):
        for dx in range(3):
            assert np.array_equal(out[3 - dy, 3 - dx], w[dy, dx, 0])
    x[:] = 0
    x[0, 0, 0] = 1.0  # at the corner only the taps that stay inside exist (zero padding)
    out = dec.conv3x3(x, w, np.zeros(2))
    assert np.count_nonzero(np.abs(out).sum(axis=2)) == 4


def test_upsample_matches_library_bilinear():
    import torch
    rng = np.random.default_rng(3)
    h = rng.standard_normal((5, 7, 3))
    t = torch.from_numpy(h.transpose(2, 0, 1)[None].copy())
    ref = torch.nn.functional.interpolate(t, scale_factor=2, mode="bilinear",
                                          align_corners=False)[0].numpy().transpose(1, 2, 0)
    assert np.allclose(dec.upsample2(h, 10, 14), ref, rtol=1e-14, atol=1e-14)
    # an odd finer size is the doubled layer cropped (ceil(W / 2^L) halves to ceil(W_L / 2))
    assert np.allclose(dec.upsample2(h, 9, 13), ref[:9, :13], rtol=1e-14, atol=1e-14)


def test_upsample_reproduces_affine_functions_inside():
    """Coarse texel k is centred at finer position 2k + 1 (finer texel i at i + 1/2), so an
    affine function sampled at the coarse centres comes back exactly at the finer centres
    that have coarse neighbours on both sides."""
    ky, kx = np.meshgrid(np.arange(6), np.arange(8), indexing="ij")
    f = lambda py, px: 0.5 + 0.25 * py - 0.125 * px
    h = f(2 * ky + 1.0, 2 * kx + 1.0)[..., None]
    up = dec.upsample2(h, 12, 16)[..., 0]
    iy, ix = np.meshgrid(np.arange(12), np.arange(16), indexing="ij")
    want = f(iy + 0.5, ix + 0.5)
    inner = (iy >= 1) & (iy <= 10) & (ix >= 1) & (ix <= 14)
    assert np.array_equal(up[inner], want[inner])
    const = np.full((3, 4, 2), 0.3)
    assert np.array_equal(dec.upsample2(const, 5, 8), np.full((5, 8, 2), 0.3))


def test_activations():
    x = np.array([-50.0, -1.0, 0.0, 0.5, 3.0])
    assert np.array_equal(dec.elu(x)[2:], x[2:])
    assert abs(dec.elu(np.array([-1.0]))[0] - (np.exp(-1.0) - 1.0)) < 1e-16
    assert abs(dec.elu(np.array([-50.0]))[0] + 1.0) < 1e-15
    assert dec.sigmoid(np.array([0.0]))[0] == 0.5
    assert abs(dec.sigmoid(np.array([2.0]))[0] - np.exp(2.0) / (1.0 + np.exp(2.0))) < 1e-15
    assert abs(dec.sigmoid(np.array([-3.0]))[0] - 1.0 / (1.0 + np.exp(3.0))) < 1e-16


def test_gate_limits():
    """A gate held open passes ELU of the feature half; a gate held shut gives 0."""
    rng = np.random.default_rng(4)
    x = rng.standard_normal((4, 6, 5))
    w = rng.standard_normal((3, 3, 5, 2 * F)) * 0.2
    w[..., F:] = 0.0
    b = np.zeros(2 * F)
    b[F:] = 60.0
    feat = dec.conv3x3(x, w, b)[..., :F]
    assert np.allclose(dec.gated(x, w, b), dec.elu(feat), rtol=1e-15, atol=1e-15)
    b[F:] = -800.0
    assert np.all(np.abs(dec.gated(x, w, b)) < 1e-300)


def test_block_closed_form_channel_order_and_bypass():
    """Identity from each upsampled feature channel to the matching feature output at the
    centre tap, gate open: the block gives ELU(up) + up (= 2 up for up > 0), exactly; the
    layer's own channels come first, then the upsampled ones."""
    D = 4
    rng = np.random.default_rng(5)
    feat = rng.uniform(0, 1, (6, 7, D))
    coarse = rng.uniform(0.1, 1, (3, 4, F))
    w = np.zeros((3, 3, D + F, 2 * F))
    for c in range(F):
        w[1, 1, D + c, c] = 1.0
    b = np.zeros(2 * F)
    b[F:] = 60.0
    up = dec.upsample2(coarse, 6, 7)
    got = dec.block(feat, coarse, w, b, fp16=False)
    assert np.allclose(got, 2 * up, rtol=1e-15, atol=0)
    # the layer's own channel d to output d, with the gate open: ELU(feat) + up
    w[:] = 0
    for d in range(D):
        w[1, 1, d, d] = 1.0
    got = dec.block(feat, coarse, w, b, fp16=False)
    assert np.allclose(got[..., :D], feat + up[..., :D], rtol=1e-15, atol=0)
    assert np.allclose(got[..., D:], up[..., D:], rtol=1e-15, atol=0)


def test_decoder_constant_propagation():
    """All kernels zero, the coarsest layer's feature bias c > 0 with its gate open: every
    block outputs c (the gated term of the other blocks is ELU(0) sigmoid(0) = 0 and the
    bypass carries c up), so the image is c sum(wo) + bo everywhere."""
    nl, D, c = 4, 4, 0.375
    wt = scenes.decoder_weights(6, nl, D)
    for L in range(nl):
        wt["w"][L] = np.zeros_like(wt["w"][L])
        wt["b"][L] = np.zeros_like(wt["b"][L])
    wt["b"][nl - 1][:F] = c
    wt["b"][nl - 1][F:] = 60.0
    pyr = scenes.feature_pyramid(7, 37, 21, nl, D)
    img, hs = dec.decode(pyr, wt, fp16=True)
    for h in hs:
        assert np.all(h == c)
    assert img.shape == (21, 37, 3)
    assert np.allclose(img, c * wt["wo"].astype(np.float64).sum(axis=0) + wt["bo"], rtol=1e-14)


def test_binary16_storage():
    nl, D = 3, 4
    wt = scenes.decoder_weights(8, nl, D)
    pyr = scenes.feature_pyramid(9, 20, 13, nl, D)
    _, hs = dec.decode(pyr, wt, fp16=True)
    for h in hs:
        assert np.array_equal(h, h.astype(np.float16).astype(np.float64))
    img64, hs64 = dec.decode(pyr, wt, fp16=False)
    img16, _ = dec.decode(pyr, wt, fp16=True)
    # storage rounding moves the result by a few binary16 ulps of its scale, no more
    scale = np.abs(img64).max()
    assert np.abs(img16 - img64).max() < 2e-2 * scale
    assert np.abs(img16 - img64).max() > 0


# ---- planted mistakes: each must make a pin above fail ----

def _shifted_up(a, n_out, axis):  # texel centres at integers (no half-texel phase)
    n_in = a.shape[axis]
    i = np.arange(n_out)
    k0 = np.clip(i // 2, 0, n_in - 1)
    k1 = np.clip(i // 2 + (i % 2), 0, n_in - 1)
    return 0.5 * np.take(a, k0, axis=axis) + 0.5 * np.take(a, k1, axis=axis)


def _flipped_conv(x, w, b):  # convolution instead of correlation
    return _ORIG_CONV(x, np.ascontiguousarray(w[::-1, ::-1]), b)


def _swapped_gated(x, w, b):  # feature and gate halves swapped
    a = _ORIG_CONV(x, w, b)
    return dec.elu(a[..., F:]) * dec.sigmoid(a[..., :F])


def _no_bypass_block(feat, coarse, w, b, fp16=True):
    feat = dec.r16(feat, fp16)
    H, W, _ = feat.shape
    if coarse is None:
        return dec.r16(dec.gated(feat, w, b), fp16)
    up = dec.r16(dec.upsample2(coarse, H, W), fp16)
    return dec.r16(dec.gated(np.concatenate([feat, up], axis=2), w, b), fp16)


def _swapped_order_block(feat, coarse, w, b, fp16=True):
    feat = dec.r16(feat, fp16)
    H, W, _ = feat.shape
    if coarse is None:
        return dec.r16(dec.gated(feat, w, b), fp16)
    up = dec.r16(dec.upsample2(coarse, H, W), fp16)
    return dec.r16(dec.gated(np.concatenate([up, feat], axis=2), w, b) + up, fp16)


_ORIG_CONV = dec.conv3x3

PINS = [test_conv_matches_brute_force_loops, test_conv_matches_library_correlation,
        test_conv_delta_places_the_kernel, test_upsample_matches_library_bilinear,
        test_upsample_reproduces_affine_functions_inside, test_activations, test_gate_limits,
        test_block_closed_form_channel_order_and_bypass, test_decoder_constant_propagation,
        test_binary16_storage]


@pytest.mark.parametrize("name,attr,fn", [
    ("half-texel phase dropped", "_up_axis", _shifted_up),
    ("convolution for correlation", "conv3x3", _flipped_conv),
    ("feature and gate halves swapped", "gated", _swapped_gated),
    ("no self-bypass", "block", _no_bypass_block),
    ("upsampled channels first", "block", _swapped_order_block),
])
def test_planted_mistake_is_caught(monkeypatch, name, attr, fn):
    monkeypatch.setattr(dec, attr, fn)
    failed = 0
    for pin in PINS:
        try:
            pin()
        except AssertionError:
            failed += 1
    assert failed > 0, name
