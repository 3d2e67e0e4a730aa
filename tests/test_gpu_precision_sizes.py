"""The precision forms at the configured full sizes: the 512x512 guiding map
of the precision configuration (headline volume and camera) through the
fp32, bf16 and fp8 networks against the fp64 oracle's network on the same
guiding map, and the dynamic scene's 1024x1024 frame through the base-48
bf16 network against the fp32 one (a property that holds at any size: the
two differ only by the bf16 roundings)."""
import numpy as np
import pytest

from synth.scene import dynamic, headline, make_volume_torch, orbit_camera
from synth.weights import he_normal_params
from tests.helpers import NET_ABS, log, to_dev, to_host

pytestmark = pytest.mark.gpu

BF16_MAX_ABS_UNTRAINED = 4e-2  # He-normal networks, per channel (see test_gpu_bf16)
FP8_MEAN_ABS_UNTRAINED = 0.05  # gross-failure bound for untrained fp8 networks (see test_gpu_fp8)


@pytest.fixture(scope="module")
def ctx():
    from paper_2604_03748_amd import lnm

    return lnm.Context(0)


def per_channel(lm, ref):
    d = np.abs(lm - ref).reshape(-1, 6)
    return d.max(axis=0), d.mean(axis=0)


def test_precision_forms_at_512(ctx, orc):
    from paper_2604_03748_amd import lnm

    wl = headline(res=512)
    log(f"precision forms on {wl.name}")
    params = he_normal_params(wl.levels, wl.base, seed=0, bias="uniform")
    dens = to_dev(wl.volume())
    g = ctx.march(dens, 8.0, wl.camera, lnm.make_params(wl.step_voxels, seed=0))
    ref, _ = orc.unet_forward(params, wl.levels, wl.base, to_host(g).astype(np.float64))
    n32 = lnm.Net(ctx, wl.levels, wl.base, params)
    calib = [ctx.march(dens, 8.0, wl.camera, lnm.make_params(wl.step_voxels, seed=0, frame=f)) for f in (1, 2)]
    amax = np.max([n32.calibrate_amax(c) for c in calib], axis=0)
    nets = {"fp32": n32, "bf16": lnm.Net(ctx, wl.levels, wl.base, params, precision=lnm.BF16),
            "fp8": lnm.Net(ctx, wl.levels, wl.base, params, precision=lnm.FP8_E4M3, act_scales=amax)}
    errs = {}
    for k, net in nets.items():
        mx, mean = per_channel(to_host(net.infer(g)), ref)
        errs[k] = (mx, mean)
        log(f"{k} at 512x512: max abs per channel {np.round(mx, 5).tolist()}, mean {np.round(mean, 6).tolist()}")
    assert np.all(errs["fp32"][0] <= NET_ABS)
    assert np.all(errs["bf16"][0] <= BF16_MAX_ABS_UNTRAINED)
    assert np.all(errs["fp8"][1] <= FP8_MEAN_ABS_UNTRAINED)
    assert errs["fp8"][0].max() > errs["bf16"][0].max() > errs["fp32"][0].max()


def test_dynamic_frame_bf16_against_fp32(ctx):
    from paper_2604_03748_amd import lnm

    wl = dynamic()
    log(f"bf16 against fp32 on {wl.name}")
    params = he_normal_params(wl.levels, wl.base, seed=0, bias="uniform")
    dens = make_volume_torch(wl.grid, wl.n_blobs, wl.seed, wl.noise_amp, frame=5, obstacle_radius=0.15)
    cam = orbit_camera(5)
    p = lnm.make_params(wl.step_voxels, seed=0, frame=5)
    n32 = lnm.Net(ctx, wl.levels, wl.base, params)
    n16 = lnm.Net(ctx, wl.levels, wl.base, params, precision=lnm.BF16)
    g32, l32, _ = n32.frame(dens, 8.0, cam, p, shade=False)
    g16, l16, _ = n16.frame(dens, 8.0, cam, p, shade=False)
    assert np.array_equal(to_host(g32), to_host(g16))
    mx, mean = per_channel(to_host(l16), to_host(l32))
    log(f"bf16 vs fp32, 1024x1024 base 48: max abs per channel {np.round(mx, 5).tolist()}, "
        f"mean {np.round(mean, 6).tolist()}")
    assert np.all(mx <= BF16_MAX_ABS_UNTRAINED)
    assert mx.max() > 1e-5
