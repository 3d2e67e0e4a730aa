"""BF16 form of the U-Net (bf16 weights/activations, fp32 accumulation on
MFMA) against the fp64 oracle: max abs error per lightmap channel <= 2e-2 on
the [0, 1] lightmaps, mean abs error reported."""
import numpy as np
import pytest

from tests.helpers import log, to_dev, to_host
from synth.weights import he_normal_params

pytestmark = pytest.mark.gpu

BF16_MAX_ABS = 2e-2  # trained network (the method's use), per channel
# Untrained He-normal networks amplify rounding more (no layer has learned to
# be contractive): bf16 rounds each layer's activations by up to 2^-9
# relative, which compounds over the 14 convolutions; the bound used for them
# is twice the trained-network one.
BF16_MAX_ABS_UNTRAINED = 4e-2
BF16_MEAN_ABS_UNTRAINED = 5e-3


@pytest.fixture(scope="module")
def ctx():
    from paper_2604_03748_amd import lnm

    return lnm.Context(0)


def _guide_like(B, H, W, seed):
    rng = np.random.default_rng(seed)
    g = rng.random((B, H, W, 3)) * np.array([2.5, 1.0, 3.5])
    g[..., 2] *= rng.random((B, H, W)) > 0.3
    return g.astype(np.float32)


def per_channel(lm, ref):
    d = np.abs(lm - ref).reshape(-1, 6)
    return d.max(axis=0), d.mean(axis=0)


@pytest.mark.parametrize("levels,base,B,H,W", [(3, 16, 2, 40, 72), (4, 32, 2, 64, 48), (4, 48, 1, 32, 40),
                                                (4, 32, 1, 256, 256)])
def test_bf16_vs_oracle(ctx, orc, levels, base, B, H, W):
    from paper_2604_03748_amd import lnm

    params = he_normal_params(levels, base, seed=7, bias="uniform")
    g = _guide_like(B, H, W, 11)
    net = lnm.Net(ctx, levels, base, params, precision=lnm.BF16)
    lm = to_host(net.infer(to_dev(g)))
    ref, _ = orc.unet_forward(params, levels, base, g.astype(np.float64))
    mx, mean = per_channel(lm, ref)
    log(f"bf16 L{levels}b{base} B{B} {H}x{W}: max abs per channel {np.round(mx, 5).tolist()}, "
        f"mean {np.round(mean, 6).tolist()}")
    assert np.all(mx <= BF16_MAX_ABS_UNTRAINED), mx
    assert np.all(mean <= BF16_MEAN_ABS_UNTRAINED), mean
    # the reduced precision is visible (the bf16 path is not a disguised fp32 one)
    assert mx.max() > 1e-5


def test_bf16_frame_matches_fp32_frame(ctx):
    """Same frame through both precisions: the march is shared (fp32), the
    lightmaps agree within the bf16 bound."""
    from paper_2604_03748_amd import lnm
    from synth.scene import headline

    wl = headline()
    params = he_normal_params(wl.levels, wl.base, seed=0, bias="uniform")
    n32 = lnm.Net(ctx, wl.levels, wl.base, params)
    n16 = lnm.Net(ctx, wl.levels, wl.base, params, precision=lnm.BF16)
    dens = to_dev(wl.volume())
    p = lnm.make_params(wl.step_voxels, seed=0)
    g32, l32, _ = n32.frame(dens, 8.0, wl.camera, p, shade=False)
    g16, l16, _ = n16.frame(dens, 8.0, wl.camera, p, shade=False)
    assert np.array_equal(to_host(g32), to_host(g16))
    mx, _ = per_channel(to_host(l16), to_host(l32))
    log(f"bf16 vs fp32 frame: max abs per channel {np.round(mx, 5).tolist()}")
    assert np.all(mx <= BF16_MAX_ABS_UNTRAINED)


def test_bf16_trained_network_on_guiding_maps(ctx, orc):
    """The stated bound on the method's use: the network trained by the
    oracle (tests/golden/trained_L3b16.npy) on guiding maps of held-out
    scenes.  Per lightmap channel: max abs <= 2e-2; mean abs reported."""
    import os

    from paper_2604_03748_amd import lnm
    from synth.scene import Camera, PERSPECTIVE, make_volume

    params = np.load(os.path.join(os.path.dirname(__file__), "golden", "trained_L3b16.npy"))
    guides = []
    for s in range(900, 904):
        vol = make_volume(32, 6, s)
        cam = Camera(PERSPECTIVE, (2.6, 0.7 + 0.1 * (s - 900), 0.9), fov_y_deg=40.0, width=64, height=64)
        g, _, _ = orc.march(vol, 8.0, cam, 2.0, seed=s)
        guides.append(g)
    g = np.stack(guides).astype(np.float32)
    ref, _ = orc.unet_forward(params, 3, 16, g.astype(np.float64))
    net = lnm.Net(ctx, 3, 16, params, precision=lnm.BF16)
    lm = to_host(net.infer(to_dev(g)))
    mx, mean = per_channel(lm, ref)
    log(f"bf16 trained L3b16 on guiding maps: max abs per channel {np.round(mx, 5).tolist()}, "
        f"mean {np.round(mean, 6).tolist()}")
    assert np.all(mx <= BF16_MAX_ABS), mx
