"""Pins of the oracle's channel adapters (Section 4.3: four NAFBlock adapters
on the decoder output, one per output group) against torch CPU float64
library routines, the identity initialisation of the block, per-image
pooling and the group-to-channel routing; and of their training gradient
(orc_adapters_loss_grad: the network with the adapters in place of its
head) against torch float64 autograd, central differences and the zeros
the identity initialisation and the target-less group force.  CPU only."""
import numpy as np
import torch
import torch.nn.functional as F

from synth.weights import adapter_param_count, adapter_params, adapter_tensors, he_normal_params, unet_layers


def _split(params, c):
    """Per-adapter dict of float64 torch tensors."""
    p = torch.as_tensor(np.asarray(params, np.float64))
    out, off = [], 0
    for _ in range(4):
        d = {}
        for name, shape, _ in adapter_tensors(c):
            n = int(np.prod(shape))
            d[name] = p[off: off + n].reshape(shape)
            off += n
        out.append(d)
    assert off == p.numel()
    return out


def _ln2d(x, w, b):
    """Layer norm over the channels of each pixel of an NCHW tensor."""
    y = F.layer_norm(x.permute(0, 2, 3, 1), (x.shape[1],), w, b, eps=1e-6)
    return y.permute(0, 3, 1, 2)


def torch_adapter(d, x):
    """One NAFBlock + head from torch.nn.functional ops; x NCHW float64."""
    c = x.shape[1]
    t = _ln2d(x, d["ln1_w"], d["ln1_b"])
    t = F.conv2d(t, d["conv1_w"][:, :, None, None], d["conv1_b"])
    t = F.conv2d(t, d["dw_w"][:, None], d["dw_b"], padding=1, groups=2 * c)
    t1, t2 = t.chunk(2, dim=1)
    t = t1 * t2
    s = F.conv2d(F.adaptive_avg_pool2d(t, 1), d["sca_w"][:, :, None, None], d["sca_b"])
    t = t * s
    t = F.conv2d(t, d["conv3_w"][:, :, None, None], d["conv3_b"])
    y = x + t * d["beta"][None, :, None, None]
    t = F.conv2d(_ln2d(y, d["ln2_w"], d["ln2_b"]), d["conv4_w"][:, :, None, None], d["conv4_b"])
    t1, t2 = t.chunk(2, dim=1)
    t = F.conv2d(t1 * t2, d["conv5_w"][:, :, None, None], d["conv5_b"])
    out = y + t * d["gamma"][None, :, None, None]
    return torch.sigmoid(F.conv2d(out, d["head_w"][:, :, None, None], d["head_b"]))


def torch_adapters(params, c, feat_bhwc):
    x = torch.as_tensor(np.asarray(feat_bhwc, np.float64)).permute(0, 3, 1, 2)
    outs = [torch_adapter(d, x).permute(0, 2, 3, 1).numpy() for d in _split(params, c)]
    lm = np.concatenate([outs[1], outs[2], outs[0]], axis=-1)  # (+X, -X), (+Y, -Y), (+Z, -Z)
    return lm, outs[3]


def test_param_count(orc):
    for c in (4, 16, 32, 48):
        assert orc.adapter_param_count(c) == adapter_param_count(c) == 4 * (7 * c * c + 35 * c + 2)


def test_adapters_match_torch(orc):
    rng = np.random.default_rng(3)
    for c, B, H, W in ((8, 2, 6, 5), (4, 1, 9, 7)):
        params = adapter_params(c, seed=c)
        feat = np.maximum(rng.normal(size=(B, H, W, c)), 0.0)  # post-ReLU features
        lm, ex = orc.adapters_forward(params, c, feat)
        tlm, tex = torch_adapters(params, c, feat)
        np.testing.assert_allclose(lm, tlm, rtol=1e-11, atol=1e-13)
        np.testing.assert_allclose(ex, tex, rtol=1e-11, atol=1e-13)


def test_identity_initialisation_reduces_to_heads(orc):
    """beta = gamma = 0 makes each NAFBlock the identity, so every output is
    sigmoid(head(feat)) of its group."""
    c, B, H, W = 8, 1, 5, 4
    params = adapter_params(c, seed=1, init="identity")
    rng = np.random.default_rng(1)
    feat = rng.random((B, H, W, c))
    lm, ex = orc.adapters_forward(params, c, feat)
    per = 7 * c * c + 35 * c + 2
    dst = {0: (lm, (4, 5)), 1: (lm, (0, 1)), 2: (lm, (2, 3)), 3: (ex, (0, 1))}
    for g in range(4):
        hw = params[g * per + per - 2 * c - 2: g * per + per - 2].astype(np.float64).reshape(2, c)
        hb = params[g * per + per - 2: g * per + per].astype(np.float64)
        want = 1.0 / (1.0 + np.exp(-(feat @ hw.T + hb)))
        arr, ch = dst[g]
        np.testing.assert_allclose(arr[..., list(ch)], want, rtol=1e-13, atol=1e-15)


def test_channel_attention_pools_each_image(orc):
    """Image b's outputs depend on image b only (the attention's mean is over
    one image, not the batch)."""
    c = 4
    params = adapter_params(c, seed=9)
    rng = np.random.default_rng(9)
    feat = rng.random((2, 6, 6, c))
    lm2, ex2 = orc.adapters_forward(params, c, feat)
    lm1, ex1 = orc.adapters_forward(params, c, feat[1:])
    np.testing.assert_array_equal(lm2[1:], lm1)
    np.testing.assert_array_equal(ex2[1:], ex1)
    feat_b = feat.copy()
    feat_b[0] *= 3.0
    lm3, _ = orc.adapters_forward(params, c, feat_b)
    np.testing.assert_array_equal(lm3[1], lm2[1])
    assert np.abs(lm3[0] - lm2[0]).max() > 1e-3


def test_group_routing(orc):
    """Head biases +-20 with zero head weights put sigmoid(+-20) exactly where
    each group's channels belong."""
    c = 4
    params = adapter_params(c, seed=2).astype(np.float64)
    per = 7 * c * c + 35 * c + 2
    sig = {+1: 1.0 / (1.0 + np.exp(-20.0)), -1: 1.0 / (1.0 + np.exp(20.0))}
    signs = [(+1, -1), (-1, +1), (+1, +1), (-1, -1)]
    for g in range(4):
        params[g * per + per - 2 * c - 2: g * per + per - 2] = 0.0
        params[g * per + per - 2: g * per + per] = [20.0 * s for s in signs[g]]
    lm, ex = orc.adapters_forward(params.astype(np.float32), c, np.ones((1, 3, 3, c)))
    want_lm = [sig[s] for s in (signs[1] + signs[2] + signs[0])]
    np.testing.assert_allclose(lm[0, 1, 1], want_lm, rtol=1e-15)
    np.testing.assert_allclose(ex[0, 1, 1], [sig[s] for s in signs[3]], rtol=1e-15)


def test_unet_features_are_the_head_input(orc):
    """Applying the plain 1x1 head to the features gives the U-Net's logits."""
    levels, base = 3, 4
    params = he_normal_params(levels, base, seed=4, bias="uniform")
    rng = np.random.default_rng(4)
    guide = rng.random((2, 8, 8, 3))
    feat = orc.unet_features(params, levels, base, guide)
    _, logits = orc.unet_forward(params, levels, base, guide)
    n_head = 6 * base + 6
    hw = params[-n_head:-6].astype(np.float64).reshape(6, base)
    hb = params[-6:].astype(np.float64)
    np.testing.assert_allclose(feat @ hw.T + hb, logits, rtol=1e-12, atol=1e-13)
    assert feat.min() >= 0.0 and unet_layers(levels, base)[-1][1] == base


def _torch_joint_loss(params, levels, base, ad_params, guide, target):
    """Loss of the network with the adapters in place of its head, and
    torch autograd's gradients of both parameter vectors."""
    from tests.test_oracle_unet import torch_unet

    p = torch.tensor(np.asarray(params, np.float64), requires_grad=True)
    a = torch.tensor(np.asarray(ad_params, np.float64), requires_grad=True)
    x = torch_unet(p, levels, base, torch.as_tensor(guide), features=True)
    c = base
    outs = []
    off = 0
    for _ in range(4):
        d = {}
        for name, shape, _ in adapter_tensors(c):
            n = int(np.prod(shape))
            d[name] = a[off: off + n].reshape(shape)
            off += n
        outs.append(torch_adapter(d, x).permute(0, 2, 3, 1))
    lm = torch.cat([outs[1], outs[2], outs[0]], dim=-1)
    loss = torch.mean((lm - torch.as_tensor(target)) ** 2)
    loss.backward()
    return loss.item(), p.grad.numpy(), a.grad.numpy()


def test_joint_gradient_matches_torch_autograd(orc):
    levels, base, B, H, W = 2, 4, 2, 6, 4
    rng = np.random.default_rng(11)
    params = he_normal_params(levels, base, seed=11, bias="uniform")
    ad = adapter_params(base, seed=12)
    guide = rng.random((B, H, W, 3))
    target = rng.random((B, H, W, 6))
    loss, g, ga = orc.adapters_loss_grad(params, levels, base, ad, guide, target)
    tl, tg, tga = _torch_joint_loss(params, levels, base, ad, guide, target)
    assert abs(loss - tl) <= 1e-13 * max(1.0, abs(tl))
    np.testing.assert_allclose(g, tg, rtol=1e-9, atol=1e-13)
    np.testing.assert_allclose(ga, tga, rtol=1e-9, atol=1e-13)
    assert np.abs(ga).max() > 1e-4 and np.abs(g).max() > 1e-4


def test_joint_gradient_central_differences(orc):
    """A few entries of each adapter tensor and of the trunk against central
    differences of the oracle's own loss (fp64 on fp32-rounded parameters:
    the step moves a parameter by a representable amount)."""
    levels, base, B, H, W = 2, 4, 1, 4, 6
    rng = np.random.default_rng(13)
    params = he_normal_params(levels, base, seed=13, bias="uniform").astype(np.float32)
    ad = adapter_params(base, seed=14).astype(np.float32)
    guide = rng.random((B, H, W, 3))
    target = rng.random((B, H, W, 6))
    _, g, ga = orc.adapters_loss_grad(params, levels, base, ad, guide, target)
    h = np.float32(2.0 ** -10)
    per = len(ad) // 4
    off = 0
    picks = []
    for name, shape, _ in adapter_tensors(base):
        n = int(np.prod(shape))
        picks.append(off + n // 2)  # one entry of each tensor of group 1
        off += n
    for i in [per + k for k in picks]:
        up, dn = ad.copy(), ad.copy()
        up[i] += h
        dn[i] -= h
        lu = orc.adapters_loss_grad(params, levels, base, up, guide, target)[0]
        ld = orc.adapters_loss_grad(params, levels, base, dn, guide, target)[0]
        fd = (lu - ld) / (float(up[i]) - float(dn[i]))
        assert abs(fd - ga[i]) <= 2e-4 * max(abs(fd), 1e-3), (i, fd, ga[i])
    for i in (0, len(params) // 3, len(params) - 7 * base - 20):
        up, dn = params.copy(), params.copy()
        up[i] += h
        dn[i] -= h
        lu = orc.adapters_loss_grad(up, levels, base, ad, guide, target)[0]
        ld = orc.adapters_loss_grad(dn, levels, base, ad, guide, target)[0]
        fd = (lu - ld) / (float(up[i]) - float(dn[i]))
        assert abs(fd - g[i]) <= 2e-4 * max(abs(fd), 1e-3), (i, fd, g[i])


def test_joint_gradient_structural_zeros(orc):
    """The alpha/emissive group has no target, so its slice takes no
    gradient, and the unused plain head neither; with the identity
    initialisation (beta = gamma = 0) no gradient reaches the block's inner
    layers, while beta and gamma themselves do get one."""
    levels, base, B, H, W = 2, 4, 1, 4, 4
    rng = np.random.default_rng(15)
    params = he_normal_params(levels, base, seed=15, bias="uniform")
    guide = rng.random((B, H, W, 3))
    target = rng.random((B, H, W, 6))
    per = 7 * base * base + 35 * base + 2
    for init in ("random", "identity"):
        ad = adapter_params(base, seed=16, init=init)
        _, g, ga = orc.adapters_loss_grad(params, levels, base, ad, guide, target)
        assert np.all(ga[3 * per:] == 0.0)
        assert np.all(g[-(6 * base + 6):] == 0.0)
    off, spans = 0, {}
    for name, shape, _ in adapter_tensors(base):
        n = int(np.prod(shape))
        spans[name] = (off, off + n)
        off += n
    for grp in range(3):
        for name in ("ln1_w", "ln1_b", "conv1_w", "conv1_b", "dw_w", "dw_b", "sca_w", "sca_b", "conv3_w", "conv3_b",
                     "ln2_w", "ln2_b", "conv4_w", "conv4_b", "conv5_w", "conv5_b"):
            lo, hi = spans[name]
            assert np.all(ga[grp * per + lo: grp * per + hi] == 0.0), (grp, name)
        for name in ("beta", "gamma", "head_w", "head_b"):
            lo, hi = spans[name]
            assert np.abs(ga[grp * per + lo: grp * per + hi]).max() > 0.0, (grp, name)
