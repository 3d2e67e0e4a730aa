"""Pins of the oracle's channel adapters (Section 4.3: four NAFBlock adapters
on the decoder output, one per output group) against torch CPU float64
library routines, the identity initialisation of the block, per-image
pooling and the group-to-channel routing.  CPU only."""
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
