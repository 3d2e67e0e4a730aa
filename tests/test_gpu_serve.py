"""Continuous-batching server on the GPU: a request's frame is bit-identical
alone and in a mix of instances with different grid and view sizes; the HBM
budget is respected; latency percentiles are reported."""
import numpy as np
import pytest

from synth.scene import light_direction, make_volume_torch
from synth.weights import he_normal_params
from tests.helpers import log, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup():
    from paper_2604_03748_amd import lnm
    from paper_2604_03748_amd.serve import Backend, Instance

    ctx = lnm.Context(0)
    params = he_normal_params(3, 16, seed=0, bias="uniform")
    net = lnm.Net(ctx, 3, 16, params, precision=lnm.BF16)
    grids, views = (32, 48, 64), (32, 64, 96)
    insts = {}
    for k in range(6):
        n = grids[k % 3]
        insts[k] = Instance(k, make_volume_torch(n, 8, 1000 + k, 0.3, device="cuda"), views[(k // 2) % 3],
                            step_voxels=2.0, start_deg=37.0 * k, seed=1000 + k,
                            light=(tuple(light_direction(1000 + k)), (1.0, 1.0, 1.0)))
    return lnm, ctx, net, insts, Backend


def test_frame_identical_alone_and_in_mix(setup):
    from paper_2604_03748_amd.serve import Request, Scheduler, poisson_requests

    lnm, ctx, net, insts, Backend = setup
    reqs = poisson_requests(len(insts), rate_hz=400, duration_s=0.25, seed=11)
    keep = [r.rid for r in reqs[:: max(1, len(reqs) // 8)]]
    be = Backend(ctx, net, n_streams=3)
    one = max(be.request_bytes(v.res) + be.batch_bytes([Request(0, k, 0, 0.0)], insts) for k, v in insts.items())
    budget = 4 * one  # tight enough that admission binds
    sch = Scheduler(be, insts, budget, max_batch=6, keep_ids=keep)
    st = sch.run(reqs)
    log(f"mix: {st}")
    assert st["requests"] == len(reqs) and st["failed"] == 0 and st["rejected"] == 0
    assert sch.peak_in_use <= budget
    assert st["mean_batch"] > 1.0  # requests really were batched together
    mixed = {rid: tuple(to_host(t) for t in be.keep[rid]) for rid in keep}
    byid = {r.rid: r for r in reqs}
    for rid in keep:
        r = byid[rid]
        be1 = Backend(ctx, net, n_streams=1)
        alone = Scheduler(be1, insts, budget, max_batch=1, keep_ids=[rid])
        alone.run([Request(rid, r.instance, r.frame, 0.0)])
        solo = tuple(to_host(t) for t in be1.keep[rid])
        for a, b in zip(mixed[rid], solo):
            assert np.array_equal(a, b), rid
    log(f"{len(keep)} frames bit-identical alone and in the mix")


def test_composite_batch_equals_per_image_composite(setup):
    """One shading launch for a batch, each image with its own camera and
    lights, equals lnm_composite on each image alone, bit for bit."""
    import torch

    lnm, ctx, net, insts, Backend = setup
    rng = np.random.default_rng(3)
    B, H, W = 5, 24, 40
    lm = torch.as_tensor(rng.random((B, H, W, 6)).astype(np.float32), device="cuda")
    g = torch.as_tensor(rng.random((B, H, W, 3)).astype(np.float32), device="cuda")
    from synth.scene import Camera, PERSPECTIVE

    cams = [Camera(PERSPECTIVE, (0.5 + 2 * np.cos(b), 0.6, 0.5 + 2 * np.sin(b)), width=W, height=H) for b in range(B)]
    lights = [[(tuple(light_direction(10 + b + k)), (1.0, 0.5 + 0.1 * k, 0.25)) for k in range(1 + b % 3)]
              for b in range(B)]
    got = to_host(ctx.composite_batch(cams, lights, lm, g))
    for b in range(B):
        one = to_host(ctx.composite(cams[b], lights[b], lm[b], g[b]))
        assert np.array_equal(got[b], one), b
    with pytest.raises(lnm.LnmError):
        ctx.composite_batch(cams[:-1] + [Camera(PERSPECTIVE, (2.5, 0.5, 0.5), width=W + 1, height=H)], lights, lm, g)


@pytest.mark.timeout(600)
def test_serving_configuration_frames_identical_alone_and_in_mix():
    """The serving configuration's grids (64^3 .. 256^3) and views (128^2 ..
    512^2) with the 4-level base-32 bf16 network and resident brick copies:
    sampled frames of a held, batched mix equal the same frames served alone."""
    from paper_2604_03748_amd import lnm
    from paper_2604_03748_amd.serve import Backend, Instance, Request, Scheduler, poisson_requests

    ctx = lnm.Context(0)
    net = lnm.Net(ctx, 4, 32, he_normal_params(4, 32, seed=0, bias="uniform"), precision=lnm.BF16)
    grids, views = (64, 96, 128, 192, 256), (128, 256, 512)
    insts = {}
    for k in range(10):
        insts[k] = Instance(k, make_volume_torch(grids[k % 5], 24, 1000 + k, 0.3, device="cuda"), views[k % 3],
                            start_deg=37.0 * k, seed=1000 + k,
                            light=(tuple(light_direction(1000 + k)), (1.0, 1.0, 1.0)))
        insts[k].prepare(ctx)
    reqs = poisson_requests(len(insts), rate_hz=2000, duration_s=0.1, seed=13)
    keep = [r.rid for r in reqs[:: max(1, len(reqs) // 12)]]
    be = Backend(ctx, net, n_streams=4)
    sch = Scheduler(be, insts, 64 * 2**30, max_batch=16, keep_ids=keep, hold_s=2e-3)
    st = sch.run(reqs)
    log(f"serving-configuration mix: {st}")
    assert st["requests"] == len(reqs) and st["failed"] == 0 and st["rejected"] == 0
    assert st["mean_batch"] > 1.0
    byid = {r.rid: r for r in reqs}
    for rid in keep:
        r = byid[rid]
        be1 = Backend(ctx, net, n_streams=1)
        Scheduler(be1, insts, 64 * 2**30, max_batch=1, keep_ids=[rid]).run([Request(rid, r.instance, r.frame, 0.0)])
        for a, b in zip(be.keep[rid], be1.keep[rid]):
            assert np.array_equal(to_host(a), to_host(b)), rid
    log(f"{len(keep)} frames bit-identical alone and in the mix")
