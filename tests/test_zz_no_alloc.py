"""lnm_frame_static (the frame in the library's static workspace, for callers
that cannot allocate) against lnm_frame with a caller workspace: the same
frame bit for bit, on two calls in a row, the second smaller; frames beyond
the static workspace are refused."""
import numpy as np
import pytest

from synth.scene import headline, light_direction, small_ortho
from synth.weights import he_normal_params
from tests.helpers import log, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2604_03748_amd import lnm

    return lnm.Context(0)


def _case(ctx, wl, prec, seed):
    import torch

    from paper_2604_03748_amd import lnm

    code = {"fp32": lnm.FP32, "bf16": lnm.BF16}[prec]
    params = he_normal_params(wl.levels, wl.base, seed=seed, bias="uniform")
    net = lnm.Net(ctx, wl.levels, wl.base, params, precision=code)
    vol = to_dev(wl.volume())
    lights = [(tuple(light_direction(seed)), (1.0, 0.9, 0.8)), ((0.3, 1.0, -0.2), (0.2, 0.25, 0.3))]
    p = lnm.make_params(wl.step_voxels, seed=seed)
    H, W = wl.camera.height, wl.camera.width
    need = net.frame_workspace(vol, 8.0, wl.camera, p).numel()
    log(f"case {wl.name} {prec}: frame workspace {need} bytes of {lnm.STATIC_SCRATCH_BYTES}")
    assert need <= lnm.STATIC_SCRATCH_BYTES
    outs = [torch.full((H, W, c), float("nan"), dtype=torch.float32, device="cuda") for c in (3, 6, 4)]
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    net.frame_static(vol, 8.0, wl.camera, p, outs[0], outs[1], lights=lights, rgba=outs[2])
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == before
    ref = net.frame(vol, 8.0, wl.camera, p, lights=lights)
    for name, a, b in zip(("guide", "lightmaps", "rgba"), outs, ref):
        a, b = to_host(a), to_host(b)
        log(f"  {name}: max abs diff {np.abs(a - b).max():.3g}")
        assert np.isfinite(a).all()
        assert np.array_equal(a, b), name


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_two_calls_second_smaller(ctx, prec):
    # the configured 128^3 / 256x256 frame, then the 32^3 / 64x64 one: the
    # second call reads the workspace the first one left behind
    _case(ctx, headline(), prec, 0)
    _case(ctx, small_ortho(), prec, 1)


def test_frame_beyond_static_workspace_is_refused(ctx):
    import torch

    from paper_2604_03748_amd import lnm

    wl = headline(res=512)
    params = he_normal_params(wl.levels, wl.base, seed=0)
    net = lnm.Net(ctx, wl.levels, wl.base, params)
    vol = to_dev(wl.volume())
    p = lnm.make_params(wl.step_voxels, seed=0)
    g = torch.zeros((512, 512, 3), dtype=torch.float32, device="cuda")
    lm = torch.zeros((512, 512, 6), dtype=torch.float32, device="cuda")
    with pytest.raises(lnm.LnmError) as e:
        net.frame_static(vol, 8.0, wl.camera, p, g, lm)
    assert e.value.status == lnm.LNM_ERR_SHAPE and "static workspace" in str(e.value)
    torch.cuda.synchronize()
    assert not g.any() and not lm.any()  # nothing was enqueued
