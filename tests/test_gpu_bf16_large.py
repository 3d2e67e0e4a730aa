"""The bf16 large-layer conv form (8 x 16 pixels x 64 output channels per
workgroup, one LDS buffer) against the default form (8 x 16 x 32, two
buffers).  Both sum every output over the same chunks, taps and MFMA
steps in the same order, so their results are equal bit for bit.  The
tiling picks the large form from the workgroup count, which grows with the
batch, so one image run alone (default form) and in a batch of two (large
form) must give the same lightmaps; the configurations below keep every
layer unsplit at both batch sizes, so nothing else changes between the two
runs."""
import numpy as np
import pytest

from tests.helpers import log, to_dev, to_host
from synth.weights import he_normal_params

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2604_03748_amd import lnm

    return lnm.Context(0)


@pytest.mark.parametrize("levels,base,H,W", [
    (2, 64, 256, 256),  # level 1 at 128^2: four 32-channel tiles, pooled and plain gathers
    (2, 48, 256, 384),  # level 1 at 128x192: three tiles (the odd tile count)
])
def test_large_form_equals_default_form(ctx, levels, base, H, W):
    import torch

    from paper_2604_03748_amd import lnm

    log(f"bf16 large form: levels {levels} base {base} {W}x{H}, batch 1 against batch 2")
    rng = np.random.default_rng(11)
    g = (rng.random((1, H, W, 3)) * np.array([2.5, 1.0, 3.5])).astype(np.float32)
    params = he_normal_params(levels, base, seed=3, bias="uniform")
    net = lnm.Net(ctx, levels, base, params, precision=lnm.BF16)
    one = to_host(net.infer(to_dev(g)))
    two = to_host(net.infer(torch.cat([to_dev(g), to_dev(g)], 0)))
    assert one.shape == (1, H, W, 6) and two.shape == (2, H, W, 6)
    assert np.array_equal(two[0], one[0]) and np.array_equal(two[1], one[0])
    assert one.std() > 1e-3  # not a constant map
