"""Reference lightmaps on the GPU, and what the trained network gains.

The network is trained on the GPU (library forward/backward kernels) on
guiding maps and fine-step reference lightmaps of seeded synthetic scenes,
then compared on held-out scenes with (ii) the method without the network:
each lightmap channel predicted from the guiding map's in-scatter channel by
a per-channel least-squares affine fit on the training set, and (iii) the
same network untrained."""
import math

import numpy as np
import pytest

from synth.scene import Camera, ORTHOGRAPHIC, PERSPECTIVE, make_volume
from synth.rng import substream
from synth.weights import he_normal_params
from tests.helpers import log, to_dev, to_host

pytestmark = pytest.mark.gpu

N, RES, STEP, REF_STEP = 32, 64, 2.0, 0.5


@pytest.fixture(scope="module")
def ctx():
    from paper_2604_03748_amd import lnm

    return lnm.Context(0)


def scene(seed):
    """32^3 volume of 6 blobs and a camera on a random orbit around it."""
    vol = make_volume(N, 6, seed)
    u = substream(seed, "view").uniform(3)
    az, el = 2 * math.pi * u[0], 0.5 * (u[1] - 0.5)
    d = 2.5
    eye = (0.5 + d * math.cos(el) * math.cos(az), 0.5 + d * math.sin(el), 0.5 + d * math.cos(el) * math.sin(az))
    proj = PERSPECTIVE if u[2] < 0.5 else ORTHOGRAPHIC
    cam = Camera(proj, eye, fov_y_deg=40.0, ortho_half_extent=0.8, width=RES, height=RES)
    return vol, cam


def test_reference_lightmaps_match_oracle(ctx, orc):
    vol, cam = scene(3)
    ref = orc.reference_lightmaps(vol, 8.0, cam, REF_STEP)
    got = to_host(ctx.reference_lightmaps(to_dev(vol), 8.0, cam, REF_STEP))
    d = np.abs(got - ref)
    tol = 1e-4 * np.abs(ref) + 2e-5
    log(f"reference lightmaps: max abs {d.max():.3g}, worst ratio {(d / tol).max():.3g}")
    assert np.all(d <= tol)
    srgb = to_host(ctx.reference_lightmaps(to_dev(vol), 8.0, cam, REF_STEP, srgb=True))
    assert np.abs(srgb - orc.srgb_encode(got)).max() <= 1e-5


def make_set(ctx, seeds):
    import torch
    from paper_2604_03748_amd import lnm

    gs, ts = [], []
    for s in seeds:
        vol, cam = scene(s)
        dens = to_dev(vol)
        gs.append(ctx.march(dens, 8.0, cam, lnm.make_params(STEP, seed=s)))
        ts.append(ctx.reference_lightmaps(dens, 8.0, cam, REF_STEP, srgb=True))
    return torch.stack(gs), torch.stack(ts)


def psnr(pred, ref):
    mse = float(np.mean((pred - ref) ** 2))
    return 10 * math.log10(1.0 / mse), mse


def test_trained_network_beats_method_without_it(ctx):
    import torch
    from paper_2604_03748_amd import lnm

    tr_g, tr_t = make_set(ctx, range(100, 196))
    te_g, te_t = make_set(ctx, range(1000, 1016))
    params = he_normal_params(3, 16, seed=0)
    # (iii) untrained network
    net0 = lnm.Net(ctx, 3, 16, params)
    p_untrained = to_host(net0.infer(te_g))
    # (ii) the method without the network: per-channel affine fit of L~
    Gh, Th = to_host(tr_g), to_host(tr_t)
    A = np.stack([Gh[..., 0].ravel(), np.ones(Gh[..., 0].size)], axis=1)
    coef = [np.linalg.lstsq(A, Th[..., c].ravel(), rcond=None)[0] for c in range(6)]
    Ge = to_host(te_g)
    p_affine = np.stack([np.clip(coef[c][0] * Ge[..., 0] + coef[c][1], 0, 1) for c in range(6)], axis=-1)
    # (i) trained network: Adam, lr 1e-3, batch 12
    tr = lnm.Trainer(ctx, 3, 16, params)
    rng = np.random.default_rng(0)
    n = tr_g.shape[0]
    loss = torch.empty(1, dtype=torch.float32, device=tr_g.device)
    hist = []
    for it in range(600):
        idx = torch.as_tensor(rng.choice(n, 12, replace=False), device=tr_g.device)
        tr.step(tr_g[idx].contiguous(), tr_t[idx].contiguous(), lr=1e-3, loss=loss)
        if it % 100 == 0 or it == 599:
            hist.append(float(to_host(loss)[0]))
    p_trained = to_host(tr.infer(te_g))
    ref = to_host(te_t)
    (ps_tr, mse_tr), (ps_af, mse_af), (ps_un, mse_un) = psnr(p_trained, ref), psnr(p_affine, ref), psnr(p_untrained, ref)
    log(f"training loss {hist}")
    log(f"held-out PSNR / MSE: trained {ps_tr:.2f} dB / {mse_tr:.5f}; without network (affine on L~) "
        f"{ps_af:.2f} dB / {mse_af:.5f}; untrained {ps_un:.2f} dB / {mse_un:.5f}")
    assert ps_tr >= ps_af + 3.0
    assert ps_tr >= ps_un + 3.0
