"""An image's lightmaps do not depend on the batch it is inferred in: the
conv tiling takes its split-K factor (which sets the order of each output's
sums) from one image's workgroup count, and every other choice the batch
size affects (tile height, the bf16 large-layer form) keeps that order.
The served frames rely on this (a frame is the same alone and in a mix)."""
import numpy as np
import pytest

from tests.helpers import log, to_dev, to_host
from synth.scene import headline
from synth.weights import he_normal_params

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2604_03748_amd import lnm

    return lnm.Context(0)


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp8"])
def test_image_same_alone_and_in_batch(ctx, prec):
    import torch

    from paper_2604_03748_amd import lnm

    wl = headline()  # 4 levels, base 32, 256x256: deep layers split at batch 1
    params = he_normal_params(wl.levels, wl.base, seed=1, bias="uniform")
    rng = np.random.default_rng(5)
    gs = [(rng.random((1, 256, 256, 3)) * np.array([2.5, 1.0, 3.5])).astype(np.float32) for _ in range(2)]
    amax = None
    if prec == "fp8":
        amax = lnm.Net(ctx, wl.levels, wl.base, params).calibrate_amax(to_dev(gs[0][0]))
    p = {"fp32": lnm.FP32, "bf16": lnm.BF16, "fp8": lnm.FP8_E4M3}[prec]
    net = lnm.Net(ctx, wl.levels, wl.base, params, precision=p, act_scales=amax)
    log(f"{prec}: one image alone and in a batch of three")
    alone = to_host(net.infer(to_dev(gs[0])))[0]
    batch = to_host(net.infer(torch.cat([to_dev(gs[0]), to_dev(gs[1]), to_dev(gs[0])], 0)))
    assert np.array_equal(batch[0], alone) and np.array_equal(batch[2], alone)
    assert not np.array_equal(batch[1], alone)
