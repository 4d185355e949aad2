"""GPU parity of the reconstruction network (Sec. 3.3, Fig. conv) through the C ABI, against
the double-precision oracle (oracle/decoder.py) in its binary16-storage mode, on the same
seeded inputs (weights and pyramids from scenes/; no input comes from the GPU).

Tolerances, from the arithmetic:
- one block, same inputs: both sides round the same quantities to binary16 at the same
  points; between them the GPU accumulates 9 (D + 32) products of binary16 values (exact in
  float32) in float32 (relative error at most K 2^-24 of the sum of absolute terms) and takes
  float32 ELU and sigmoid; the doubled features are formed with float32 fused multiply-adds.
  So a stored value may round to the neighbouring binary16 value: the bar is one binary16
  spacing of the reference plus K 2^-24 times the sum of absolute terms, plus one spacing of
  the doubled value the bypass adds.
- the whole network: such one-spacing differences (about 3 in 10^4 values per block) feed
  the next blocks; a CPU emulation of the GPU's float32 arithmetic at 300x170, 6 layers, gives
  a largest image difference of 1.9e-3 of the image's mean magnitude and a norm-wise relative
  difference of 3.5e-5; the bars are 2^-6 of the mean magnitude per element (8x) and 1e-3
  norm-wise."""
import numpy as np
import pytest

import scenes
from oracle import decoder as dec

pytestmark = pytest.mark.gpu
F = dec.F


def _decoder(W, H, nl, D, seed, out_dim=3, dev=None):
    import paper_2401_06003_amd as tp
    wt = scenes.decoder_weights(seed, nl, D, out_dim)
    return tp.Decoder(W, H, nl, D, wt, device=dev), wt


def _block_bar(x_abs, w, b, ref):
    """One binary16 spacing of the reference plus the float32 accumulation bound."""
    K = 9 * w.shape[2] + 1
    s = dec.conv3x3(x_abs, np.abs(w.astype(np.float64)), np.abs(b.astype(np.float64)))
    spacing = np.spacing(np.abs(ref).astype(np.float16)).astype(np.float64)
    return spacing + K * 2.0 ** -24 * (s[..., :F] + s[..., F:] + np.abs(ref))


@pytest.mark.parametrize("D", [4, 8])
@pytest.mark.parametrize("W,H", [(53, 37), (16, 16), (5, 3), (129, 66)])
def test_block_parity(gpu, D, W, H):
    """A block below the coarsest layer and the coarsest block, on sizes that span several
    16x16 tiles with ragged edges, one tile, and less than a tile."""
    import torch
    nl = 3
    W0, H0 = 2 * W, 2 * H  # layer 1 of a W0 x H0 view is W x H
    d, wt = _decoder(W0, H0, nl, D, 21 + D, dev=gpu)
    rng = np.random.default_rng(31)
    for L in (1, nl - 1):
        Wl, Hl = d.dims[L]
        feat = rng.uniform(0, 1, (Hl, Wl, D)).astype(np.float32)
        feat[rng.random((Hl, Wl)) < 0.2] = 0
        coarse = None
        if L + 1 < nl:
            Wc, Hc = d.dims[L + 1]
            coarse = rng.uniform(-0.5, 1.5, (Hc, Wc, F)).astype(np.float16)
        got = d.block(L, torch.from_numpy(feat).to(gpu),
                      None if coarse is None else torch.from_numpy(coarse).to(gpu))
        got = got.cpu().numpy().astype(np.float64)
        ref = dec.block(feat, coarse, wt["w"][L], wt["b"][L], fp16=True)
        x = dec.r16(feat)
        if coarse is not None:
            up = dec.r16(dec.upsample2(coarse, Hl, Wl))
            x = np.concatenate([x, up], axis=2)
        bar = _block_bar(np.abs(x), wt["w"][L], wt["b"][L], ref)
        if coarse is not None:  # the bypass adds a doubled value that may be one spacing off
            bar += np.spacing(np.abs(up).astype(np.float16)).astype(np.float64)
        bad = np.abs(got - ref) > bar
        assert not bad.any(), (L, int(bad.sum()), got[bad][:4], ref[bad][:4])


@pytest.mark.parametrize("D", [4, 8])
def test_output_layer(gpu, D):
    """The finest block with the 1x1 output convolution applied (float32 out)."""
    import torch
    nl, W, H = 2, 45, 29
    d, wt = _decoder(W, H, nl, D, 41, out_dim=5, dev=gpu)
    rng = np.random.default_rng(42)
    feat = rng.uniform(0, 1, (H, W, D)).astype(np.float32)
    Wc, Hc = d.dims[1]
    coarse = rng.uniform(-0.5, 1.5, (Hc, Wc, F)).astype(np.float16)
    got = d.block(0, torch.from_numpy(feat).to(gpu), torch.from_numpy(coarse).to(gpu),
                  final=True).cpu().numpy().astype(np.float64)
    h = dec.block(feat, coarse, wt["w"][0], wt["b"][0], fp16=True)
    ref = dec.output_layer(h, wt["wo"], wt["bo"])
    # h may differ by one binary16 spacing in a few values (block bar); the 1x1 layer then
    # moves the output by at most that spacing times sum |wo|, plus float32 rounding
    x = np.concatenate([dec.r16(feat), dec.r16(dec.upsample2(coarse, H, W))], axis=2)
    hb = _block_bar(np.abs(x), wt["w"][0], wt["b"][0], h)
    bar = hb.max(axis=2, keepdims=True) * np.abs(wt["wo"]).sum(axis=0) + 1e-6
    assert np.all(np.abs(got - ref) <= bar)


def _net_check(img, ref):
    scale = np.abs(ref).mean()
    err = np.abs(img - ref)
    assert err.max() <= 2.0 ** -6 * scale, (err.max(), scale)
    assert np.linalg.norm(img - ref) <= 1e-3 * np.linalg.norm(ref)


@pytest.mark.parametrize("D,W,H,nl", [(4, 300, 170, 6), (8, 97, 61, 4), (4, 7, 5, 1),
                                      (8, 33, 17, 5)])
def test_network_parity(gpu, D, W, H, nl):
    import torch
    d, wt = _decoder(W, H, nl, D, 51 + nl, dev=gpu)
    pyr = scenes.feature_pyramid(52 + nl, W, H, nl, D)
    flat = torch.from_numpy(np.concatenate([p.reshape(-1) for p in pyr])).to(gpu)
    img = d.forward(flat).cpu().numpy().astype(np.float64)
    ref, _ = dec.decode(pyr, wt, fp16=True)
    _net_check(img, ref)


def test_network_1080p(gpu):
    """The full-resolution view of the headline workload: 1920x1080, 8 layers, D = 4."""
    import torch
    W, H, nl, D = 1920, 1080, 8, 4
    d, wt = _decoder(W, H, nl, D, 61, dev=gpu)
    pyr = scenes.feature_pyramid(62, W, H, nl, D)
    flat = torch.from_numpy(np.concatenate([p.reshape(-1) for p in pyr])).to(gpu)
    img = d.forward(flat).cpu().numpy().astype(np.float64)
    ref, _ = dec.decode(pyr, wt, fp16=True)
    _net_check(img, ref)


def test_rendered_pyramid_decodes(gpu):
    """Renderer then network on the 4096-point scene: the GPU's image from the GPU's pyramid
    against the oracle network on the oracle's pyramid."""
    import torch
    from gpu_util import gpu_forward
    from oracle import oracle
    sc = scenes.unit_cube(1)
    cam, nl, D = sc["cams"][0], sc["nlayers"], sc["D"]
    res, r, _ = gpu_forward(sc, gpu)
    d, wt = _decoder(cam["W"], cam["H"], nl, D, 71, dev=gpu)
    pyr_gpu = torch.from_numpy(res[0][0].astype(np.float32).reshape(-1)).to(gpu)
    img = d.forward(pyr_gpu).cpu().numpy().astype(np.float64)
    opyr, _, _ = oracle.forward(sc["points"], cam, nl)
    layers, o = [], 0
    for (w, h) in oracle.layer_dims(cam["W"], cam["H"], nl):
        layers.append(opyr[o:o + w * h].reshape(h, w, D))
        o += w * h
    ref, _ = dec.decode(layers, wt, fp16=True)
    _net_check(img, ref)
