"""Parity of the HIP channel adapters (lnm_infer_adapters: U-Net trunk + four
NAFBlock adapters, Section 4.3) with the fp64 oracle (orc_unet_features +
orc_adapters_forward)."""
import numpy as np
import pytest

from synth.weights import adapter_params, he_normal_params
from tests.helpers import NET_ABS, log, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2604_03748_amd import lnm

    return lnm.Context(0)


def _guide_like(B, H, W, seed):
    rng = np.random.default_rng(seed)
    g = rng.random((B, H, W, 3)) * np.array([2.5, 1.0, 3.5])
    g[..., 2] *= rng.random((B, H, W)) > 0.3
    return g.astype(np.float32)


def _both(ctx, orc, levels, base, B, H, W, seed, precision=0, init="random"):
    from paper_2604_03748_amd import lnm

    log(f"adapters L{levels} b{base} B{B} {H}x{W} precision {precision} init {init}")
    params = he_normal_params(levels, base, seed=seed, bias="uniform")
    ap = adapter_params(base, seed=seed + 1, init=init)
    g = _guide_like(B, H, W, seed)
    net = lnm.Net(ctx, levels, base, params, precision=precision)
    ad = lnm.Adapters(net, ap)
    lm, ex = ad.infer(to_dev(g))
    feat = orc.unet_features(params, levels, base, g.astype(np.float64))
    rlm, rex = orc.adapters_forward(ap, base, feat)
    return to_host(lm), to_host(ex), rlm, rex


@pytest.mark.parametrize("levels,base,B,H,W", [(3, 16, 2, 32, 32), (4, 32, 1, 24, 40), (3, 48, 1, 16, 24),
                                               (2, 64, 2, 10, 6), (4, 32, 2, 72, 104), (3, 64, 1, 40, 72)])
def test_adapters_fp32_match_oracle(ctx, orc, levels, base, B, H, W):
    lm, ex, rlm, rex = _both(ctx, orc, levels, base, B, H, W, seed=levels * 7 + base)
    d_lm, d_ex = np.abs(lm - rlm).max(), np.abs(ex - rex).max()
    log(f"max |lightmaps - oracle| {d_lm:.3g}, max |alpha/emissive - oracle| {d_ex:.3g}")
    assert d_lm <= NET_ABS and d_ex <= NET_ABS
    assert rlm.std() > 1e-2  # outputs are not saturated


def test_identity_adapters_equal_group_heads(ctx, orc):
    lm, ex, rlm, rex = _both(ctx, orc, 3, 16, 1, 16, 16, seed=5, init="identity")
    assert np.abs(lm - rlm).max() <= NET_ABS and np.abs(ex - rex).max() <= NET_ABS


def test_identity_adapters_reproduce_the_plain_head_at_every_precision(ctx):
    """With beta = gamma = 0 each NAFBlock is the identity, so adapters whose
    heads are the plain head's rows must give the plain network's lightmaps:
    this checks that the adapters read the fp32, bf16 and e4m3 trunk
    features (and the e4m3 scale) exactly as the plain head does."""
    from paper_2604_03748_amd import lnm
    from synth.weights import adapter_tensors

    levels, base, B, H, W = 3, 16, 2, 32, 24
    params = he_normal_params(levels, base, seed=3, bias="uniform")
    hw = params[-(6 * base + 6):-6].reshape(6, base)
    hb = params[-6:]
    ap = adapter_params(base, seed=4, init="identity")
    per = len(ap) // 4
    rows = {0: (4, 5), 1: (0, 1), 2: (2, 3), 3: (0, 1)}
    for grp, (r0, r1) in rows.items():
        end = (grp + 1) * per
        ap[end - 2 * base - 2: end - 2] = np.concatenate([hw[r0], hw[r1]])
        ap[end - 2: end] = [hb[r0], hb[r1]]
    g = to_dev(_guide_like(B, H, W, 3))
    amax = lnm.Net(ctx, levels, base, params).calibrate_amax(g)
    for prec in (lnm.FP32, lnm.BF16, lnm.FP8_E4M3):
        net = lnm.Net(ctx, levels, base, params, precision=prec, act_scales=amax if prec == lnm.FP8_E4M3 else None)
        plain = to_host(net.infer(g))
        lm, ex = lnm.Adapters(net, ap).infer(g)
        d = np.abs(to_host(lm) - plain).max()
        log(f"precision {prec}: identity adapters vs plain head max abs {d:.3g}")
        assert d <= 2e-6
        np.testing.assert_allclose(to_host(ex), plain[..., [0, 1]], rtol=0, atol=2e-6)
    assert [t[0] for t in adapter_tensors(base)][-2:] == ["head_w", "head_b"]


def test_adapter_errors(ctx):
    from paper_2604_03748_amd import lnm

    net = lnm.Net(ctx, 3, 16, he_normal_params(3, 16))
    with pytest.raises(lnm.LnmError):
        lnm.Adapters(net, np.zeros(10, np.float32))
    bad = adapter_params(16)
    bad[3] = np.nan
    with pytest.raises(lnm.LnmError):
        lnm.Adapters(net, bad)
    ad = lnm.Adapters(net, adapter_params(16))
    with pytest.raises(lnm.LnmError):
        ad.infer(to_dev(_guide_like(1, 10, 12, 0)))  # not divisible by 4
