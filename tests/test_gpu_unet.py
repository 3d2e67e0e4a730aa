"""Parity of the HIP U-Net (lnm_infer), the frame (lnm_frame) and the six-way
shading (lnm_composite) with the fp64 oracle."""
import numpy as np
import pytest

from synth.scene import headline, light_direction, small_ortho
from synth.weights import he_normal_params
from tests.helpers import check_march, check_net, fp32_ray_allowance, log, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2604_03748_amd import lnm

    return lnm.Context(0)


def _guide_like(B, H, W, seed):
    """Inputs with the value ranges of guiding maps (L~ in [0,3], T, D)."""
    rng = np.random.default_rng(seed)
    g = rng.random((B, H, W, 3)) * np.array([2.5, 1.0, 3.5])
    g[..., 2] *= rng.random((B, H, W)) > 0.3
    return g.astype(np.float32)


def _infer_both(ctx, orc, levels, base, B, H, W, seed, what):
    from paper_2604_03748_amd import lnm

    log(f"case {what}: L{levels} base {base} B{B} {H}x{W}")
    params = he_normal_params(levels, base, seed=seed, bias="uniform")
    net = lnm.Net(ctx, levels, base, params)
    g = _guide_like(B, H, W, seed)
    import torch

    logits = torch.empty((B, H, W, 6), dtype=torch.float32, device="cuda")
    lm = net.infer(to_dev(g), logits=logits)
    lm_ref, lo_ref = orc.unet_forward(params, levels, base, g.astype(np.float64))
    return check_net(to_host(lm), lm_ref, to_host(logits), lo_ref, what)


def test_small_net(ctx, orc):
    _infer_both(ctx, orc, 3, 16, 1, 64, 64, 1, "L3b16_64px")


def test_ragged_batch(ctx, orc):
    # W not a multiple of the 16-pixel tile, H not a multiple of 8
    _infer_both(ctx, orc, 3, 16, 2, 44, 72, 2, "L3b16_B2_44x72")


def test_headline_net_small_image(ctx, orc):
    _infer_both(ctx, orc, 4, 32, 2, 64, 48, 3, "L4b32_B2_64x48")


def test_wide_net_padded_channel_tile(ctx, orc):
    # base 48: output widths not a multiple of the 32-channel tile
    _infer_both(ctx, orc, 4, 48, 1, 32, 40, 4, "L4b48_32x40")


def test_headline_net_full_size(ctx, orc):
    _infer_both(ctx, orc, 4, 32, 1, 256, 256, 0, "L4b32_256px")


def test_workspace_and_shape_errors(ctx):
    from paper_2604_03748_amd import lnm
    import torch

    params = he_normal_params(3, 16, seed=0)
    net = lnm.Net(ctx, 3, 16, params)
    g = to_dev(_guide_like(1, 32, 32, 0))
    ws = net.workspace(1, 32, 32)
    with pytest.raises(lnm.LnmError) as e:
        net.infer(g, workspace=ws[: ws.numel() // 2])
    assert e.value.status == lnm.LNM_ERR_SHAPE
    with pytest.raises(lnm.LnmError) as e:
        net.infer(to_dev(_guide_like(1, 30, 32, 0)))  # 30 not divisible by 4
    assert e.value.status == lnm.LNM_ERR_SHAPE
    with pytest.raises(lnm.LnmError) as e:
        lnm.Net(ctx, 3, 16, params[:-1])
    assert e.value.status == lnm.LNM_ERR_SHAPE
    with pytest.raises(lnm.LnmError) as e:
        lnm.Net(ctx, 3, 16, params, precision=lnm.FP8_E4M3 + 7)
    torch.cuda.synchronize()


@pytest.mark.parametrize("wl_fn", [small_ortho, headline])
def test_frame_end_to_end(ctx, orc, wl_fn):
    """lnm_frame = march -> U-Net -> six-way shading, against the oracle's
    three stages run on the same inputs."""
    from paper_2604_03748_amd import lnm

    wl = wl_fn()
    log(f"case frame {wl.name}")
    vol = wl.volume()
    params = he_normal_params(wl.levels, wl.base, seed=0, bias="uniform")
    net = lnm.Net(ctx, wl.levels, wl.base, params)
    lights = [(tuple(light_direction(0)), (1.0, 0.9, 0.8)), ((0.3, 1.0, -0.2), (0.2, 0.25, 0.3))]
    p = lnm.make_params(wl.step_voxels, seed=0)
    g, lm, rgba = net.frame(to_dev(vol), 8.0, wl.camera, p, lights=lights)
    g, lm, rgba = to_host(g), to_host(lm), to_host(rgba)
    gr, m, _ = orc.march(vol, 8.0, wl.camera, wl.step_voxels, seed=0)
    allow = fp32_ray_allowance(orc, vol, 8.0, wl.camera, wl.step_voxels, seed=0)
    check_march(g, gr, m, 0.1, 0, f"frame {wl.name}", allow=allow)
    # the network sees the GPU's own guide so the comparison isolates it
    lm_ref, _ = orc.unet_forward(params, wl.levels, wl.base, g)
    check_net(lm, lm_ref, what=f"frame {wl.name}")
    rgba_ref = orc.composite(lm, g, wl.camera, lights)
    d = np.abs(rgba - rgba_ref)
    log(f"composite max abs {d.max():.3g}")
    assert d.max() <= 1e-5 * max(1.0, np.abs(rgba_ref).max())
    # whole path from the oracle's own guide: the same lightmaps within tolerance
    lm_full, _ = orc.unet_forward(params, wl.levels, wl.base, gr)
    check_net(lm, lm_full, what=f"frame {wl.name} (oracle guide)")


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp8"])
def test_frame_shading_equals_separate_composite(ctx, prec):
    """lnm_frame shades in its head launch; the result must be bit-identical
    to lnm_composite run on the frame's own lightmaps and guide."""
    from paper_2604_03748_amd import lnm

    wl = small_ortho()
    vol = to_dev(wl.volume())
    params = he_normal_params(wl.levels, wl.base, seed=2, bias="uniform")
    lights = [(tuple(light_direction(1)), (1.0, 0.9, 0.8)), ((-0.3, 1.0, 0.2), (0.2, 0.25, 0.3))]
    p = lnm.make_params(wl.step_voxels, seed=0)
    amax = None
    if prec == "fp8":
        amax = lnm.Net(ctx, wl.levels, wl.base, params).calibrate_amax(ctx.march(vol, 8.0, wl.camera, p))
    code = {"fp32": lnm.FP32, "bf16": lnm.BF16, "fp8": lnm.FP8_E4M3}[prec]
    net = lnm.Net(ctx, wl.levels, wl.base, params, precision=code, act_scales=amax)
    g, lm, rgba = net.frame(vol, 8.0, wl.camera, p, lights=lights)
    sep = ctx.composite(wl.camera, lights, lm[None], g[None])[0]
    log(f"{prec}: frame shading vs separate composite, max abs {np.abs(to_host(rgba) - to_host(sep)).max():.3g}")
    assert np.array_equal(to_host(rgba), to_host(sep))


def test_composite_matches_oracle(ctx, orc):
    wl = small_ortho()
    rng = np.random.default_rng(5)
    lm = rng.random((2, 16, 24, 6)).astype(np.float32)
    g = rng.random((2, 16, 24, 3)).astype(np.float32)
    cam = wl.camera.resized(24, 16)
    lights = [((0.2, -0.7, 0.4), (1.0, 0.5, 0.25)), ((-1.0, 0.0, 0.0), (0.1, 0.2, 0.3)), ((0, 0, 1), (1, 1, 1))]
    out = to_host(ctx.composite(cam, lights, to_dev(lm), to_dev(g)))
    for b in range(2):
        ref = orc.composite(lm[b], g[b], cam, lights)
        assert np.abs(out[b] - ref).max() <= 2e-6
