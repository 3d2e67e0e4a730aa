"""Pins of the oracle's U-Net (Section 4.3), its loss and gradient (Section 4.4)
and Adam (Section 5) against library routines (torch CPU float64),
finite differences and structural special cases.  CPU only."""
import numpy as np
import pytest
import torch
import torch.nn.functional as F

from synth.weights import he_normal_params, n_params, unet_layers


def torch_unet(params, levels, base, guide_bhwc, features=False):
    """The same network built from torch.nn.functional float64 CPU ops
    (features=True: the decoder output, the head's input, NCHW)."""
    p = params if isinstance(params, torch.Tensor) else torch.as_tensor(np.asarray(params, np.float64))
    layers = unet_layers(levels, base)
    ws, off = [], 0
    for _, ci, co, k in layers:
        w = p[off: off + co * ci * k * k].reshape(co, ci, k, k)
        off += co * ci * k * k
        b = p[off: off + co]
        off += co
        ws.append((w, b, k))
    x = guide_bhwc.permute(0, 3, 1, 2)
    it = iter(ws)

    def conv(x):
        w, b, k = next(it)
        return F.conv2d(x, w, b, padding=k // 2)

    skips = []
    for _ in range(levels - 1):
        x = F.relu(conv(x))
        x = F.relu(conv(x))
        skips.append(x)
        x = F.max_pool2d(x, 2)
    x = F.relu(conv(x))
    x = F.relu(conv(x))
    for l in range(levels - 2, -1, -1):
        x = torch.cat([skips[l], F.interpolate(x, scale_factor=2, mode="nearest")], dim=1)
        x = F.relu(conv(x))
        x = F.relu(conv(x))
    if features:
        return x
    z = conv(x)
    return torch.sigmoid(z).permute(0, 2, 3, 1), z.permute(0, 2, 3, 1)


def test_param_count_matches_generator(orc):
    for L, b in ((2, 2), (3, 16), (4, 32), (4, 48)):
        assert orc.unet_param_count(L, b) == n_params(L, b)


@pytest.mark.parametrize("levels,base,B,H,W", [(2, 2, 1, 6, 10), (3, 4, 2, 16, 8), (3, 16, 1, 32, 32)])
def test_forward_matches_torch(orc, levels, base, B, H, W):
    params = he_normal_params(levels, base, seed=levels * 10 + base, bias="uniform")
    rng = np.random.default_rng(base)
    guide = rng.random((B, H, W, 3)) * np.array([2.0, 1.0, 3.0])
    lm, logits = orc.unet_forward(params, levels, base, guide)
    tl, tz = torch_unet(params, levels, base, torch.as_tensor(guide))
    np.testing.assert_allclose(logits, tz.numpy(), rtol=1e-10, atol=1e-11)
    np.testing.assert_allclose(lm, tl.numpy(), rtol=1e-10, atol=1e-12)


def test_zero_weights_head_bias_sets_channel_order(orc):
    levels, base = 3, 4
    params = np.zeros(n_params(levels, base), np.float32)
    bias = np.array([-2.0, -1.0, 0.0, 0.5, 1.0, 3.0], np.float32)
    params[-6:] = bias
    guide = np.random.default_rng(0).random((8, 12, 3))
    lm, _ = orc.unet_forward(params, levels, base, guide)
    np.testing.assert_array_equal(lm, np.broadcast_to(1.0 / (1.0 + np.exp(-bias.astype(np.float64))), lm.shape))


def test_delta_first_layer_is_a_shift(orc):
    """With identity-like kernels the first conv reproduces a shifted input;
    pinned through a 2-level net whose other layers pass channel 0 through."""
    levels, base = 2, 1
    layers = unet_layers(levels, base)
    params = np.zeros(n_params(levels, base), np.float32)
    off = 0
    idx = {}
    for name, ci, co, k in layers:
        idx[name] = off
        off += co * ci * k * k + co
    # enc0a: out = guide channel 0 shifted right by one pixel (kernel tap dx = 0)
    params[idx["enc0a"] + (0 * 3 + 1) * 3 + 0] = 1.0  # W[o=0][c=0][dy=1][dx=0]
    params[idx["enc0b"] + 4] = 1.0  # centre tap
    params[idx["dec0a"] + 4] = 1.0  # skip channel centre tap (c = 0 of 2)
    params[idx["dec0b"] + 4] = 1.0
    params[idx["head"]: idx["head"] + 6] = 1.0  # every output = logit of channel 0
    guide = np.random.default_rng(1).random((4, 6, 3))
    _, logits = orc.unet_forward(params, levels, base, guide)
    want = np.zeros((4, 6))
    want[:, 1:] = guide[:, :-1, 0]
    for c in range(6):
        np.testing.assert_allclose(logits[..., c], want, atol=1e-15)


@pytest.mark.parametrize("levels,base,B,H,W", [(2, 2, 2, 4, 6), (3, 3, 1, 8, 8)])
def test_gradient_matches_torch_autograd(orc, levels, base, B, H, W):
    params = he_normal_params(levels, base, seed=3, bias="uniform")
    rng = np.random.default_rng(7)
    guide = rng.random((B, H, W, 3))
    target = rng.random((B, H, W, 6))
    loss, grad = orc.unet_loss_grad(params, levels, base, guide, target)
    p = torch.tensor(params.astype(np.float64), requires_grad=True)
    pred, _ = torch_unet(p, levels, base, torch.as_tensor(guide))
    tl = torch.mean((pred - torch.as_tensor(target)) ** 2)
    tl.backward()
    assert loss == pytest.approx(tl.item(), rel=1e-12)
    np.testing.assert_allclose(grad, p.grad.numpy(), rtol=1e-9, atol=1e-13)


def test_gradient_matches_finite_differences(orc):
    levels, base = 2, 2
    params = he_normal_params(levels, base, seed=5, bias="uniform")
    rng = np.random.default_rng(9)
    guide = rng.random((1, 4, 4, 3))
    target = rng.random((1, 4, 4, 6))
    _, grad = orc.unet_loss_grad(params, levels, base, guide, target)
    # finite differences in float64 via torch (the oracle takes fp32 params,
    # so perturbing them by 1e-6 would be lost to rounding)
    p0 = torch.tensor(params.astype(np.float64))
    eps = 1e-6
    picks = np.random.default_rng(2).choice(params.size, 25, replace=False)
    for i in picks:
        e = torch.zeros_like(p0)
        e[i] = eps
        lp = torch.mean((torch_unet(p0 + e, levels, base, torch.as_tensor(guide))[0] - torch.as_tensor(target)) ** 2)
        lm = torch.mean((torch_unet(p0 - e, levels, base, torch.as_tensor(guide))[0] - torch.as_tensor(target)) ** 2)
        fd = (lp - lm).item() / (2 * eps)
        assert grad[i] == pytest.approx(fd, rel=1e-5, abs=1e-10)


def test_maxpool_gradient_goes_to_first_maximum(orc):
    """Ties inside a pooling window: the whole gradient goes to the first
    maximum in raster order (fixed rule), checked on a net whose first-level
    output is constant per 2x2 window."""
    levels, base = 2, 1
    layers = unet_layers(levels, base)
    params = np.zeros(n_params(levels, base), np.float32)
    idx, off = {}, 0
    for name, ci, co, k in layers:
        idx[name] = off
        off += co * ci * k * k + co
    params[idx["enc0a"] + 9] = 1.0  # bias of enc0a = 1: constant positive map
    params[idx["enc0b"] + 4] = 1.0
    params[idx["bot1a"] + 4] = 1.0
    params[idx["bot1b"] + 4] = 1.0
    params[idx["dec0a"] + 9 + 4] = 1.0  # up channel centre tap
    params[idx["dec0b"] + 4] = 1.0
    params[idx["head"]: idx["head"] + 6] = 1.0
    guide = np.zeros((1, 4, 4, 3))
    target = np.zeros((1, 4, 4, 6))
    _, grad = orc.unet_loss_grad(params, levels, base, guide, target)
    p = torch.tensor(params.astype(np.float64), requires_grad=True)
    pred, _ = torch_unet(p, levels, base, torch.as_tensor(guide))
    torch.mean(pred**2).backward()
    # torch routes ties to one element too; the totals per layer must agree
    np.testing.assert_allclose(grad, p.grad.numpy(), rtol=1e-9, atol=1e-13)


def test_adam_matches_torch(orc):
    rng = np.random.default_rng(4)
    p = rng.standard_normal(50)
    m = np.zeros(50)
    v = np.zeros(50)
    tp = torch.tensor(p.copy(), requires_grad=True)
    opt = torch.optim.Adam([tp], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    for t in range(1, 6):
        g = rng.standard_normal(50)
        p, m, v = orc.adam(p, g, m, v, t)
        opt.zero_grad()
        tp.grad = torch.tensor(g)
        opt.step()
        np.testing.assert_allclose(p, tp.detach().numpy(), rtol=1e-12, atol=1e-15)


def test_window_interior_is_border_free(orc):
    """Locality of the 4-level network (two 3x3 convolutions per level, 2x2
    max-pools, nearest upsampling): on a window whose offset is a multiple
    of 8, the outputs 48 or more pixels inside it equal the whole image's
    (the GPU comparison at 1024x1024 relies on this, with a 64-pixel margin);
    with a 24-pixel margin they do not."""
    p = he_normal_params(4, 8, seed=3, bias="uniform")
    g = np.random.default_rng(5).random((1, 256, 256, 3))
    full, _ = orc.unet_forward(p, 4, 8, g)
    y0, x0, C = 48, 64, 160
    win, _ = orc.unet_forward(p, 4, 8, g[:, y0:y0 + C, x0:x0 + C])
    d = np.abs(win[0] - full[0, y0:y0 + C, x0:x0 + C])
    assert d[48:C - 48, 48:C - 48].max() == 0.0
    assert d[24:C - 24, 24:C - 24].max() > 1e-6
