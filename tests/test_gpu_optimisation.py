"""Optimisation loop through the autograd function: targets are rendered by the CPU oracle
from a perturbed copy of the scene (positions + N(0, 0.01^2), world sizes x U[0.5, 2]); the
GPU renderer optimises positions, log-sizes, opacities and descriptors with Adam from the
unperturbed scene.  The loss (mean squared error per layer, normalised by the layer's
size) must fall."""
import numpy as np
import pytest

import scenes
from oracle import oracle

pytestmark = pytest.mark.gpu


def test_adam_loop_reduces_loss(gpu):
    import torch
    import paper_2401_06003_amd as tp
    sc = scenes.ring_scene(5, n=30000, views=2, W=160, H=96, nlayers=5, D=8)
    pts, cams, nl, D = sc["points"], sc["cams"], sc["nlayers"], sc["D"]
    truth = scenes.perturbed(pts, seed=55)
    targets = [torch.from_numpy(oracle.forward(truth, c, nl)[0].astype(np.float32).reshape(-1))
               for c in cams]
    target = torch.cat(targets).to(gpu)
    r = tp.Renderer(cams, nl, D, len(pts["x"]), device=gpu)
    # per-element weights: each layer's squared error is normalised by W_L * H_L * D
    wts = []
    for c in cams:
        dims, _ = tp.layer_layout(c, nl)
        for (w, h) in dims:
            wts.append(torch.full((w * h * D,), 1.0 / (w * h * D)))
    wts = torch.cat(wts).to(gpu)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(gpu)
    xyz = [dev(pts[k]).requires_grad_(True) for k in ("x", "y", "z")]
    log_sw = torch.log(dev(pts["sw"])).requires_grad_(True)
    alpha = dev(pts["alpha"]).requires_grad_(True)
    desc = dev(pts["desc"]).requires_grad_(True)
    opt = torch.optim.Adam([{"params": xyz, "lr": 1e-4}, {"params": [log_sw], "lr": 1e-2},
                            {"params": [desc], "lr": 1e-2}, {"params": [alpha], "lr": 1e-2}],
                           betas=(0.9, 0.999))
    losses = []
    for it in range(40):
        opt.zero_grad()
        out = tp.render(*xyz, torch.exp(log_sw), alpha, desc, r)
        loss = ((out - target) ** 2 * wts).sum()
        loss.backward()
        opt.step()
        with torch.no_grad():
            alpha.clamp_(0.0, 1.0)
        losses.append(loss.item())
    assert np.all(np.isfinite(losses))
    first, last = np.mean(losses[:3]), np.mean(losses[-3:])
    assert last < 0.7 * first, (first, last)
    smooth = np.convolve(losses, np.ones(5) / 5, mode="valid")
    assert np.all(np.diff(smooth) < 0.02 * first), "loss does not fall steadily"
