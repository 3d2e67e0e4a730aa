"""Parity of the HIP guiding-map march (lnm_march) with the fp64 oracle."""
import math

import numpy as np
import pytest

from synth.scene import Camera, ORTHOGRAPHIC, PERSPECTIVE, dynamic, headline, make_volume, small_ortho
from tests.helpers import check_march, fp32_ray_allowance, log, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2604_03748_amd import lnm

    return lnm.Context(0)


def _run(ctx, vol, ss, cam, step, **kw):
    from paper_2604_03748_amd import lnm

    p = lnm.make_params(step, depth_tau=kw.get("depth_tau", 0.1), ert_eps=kw.get("ert_eps", 1e-6),
                        jitter=kw.get("jitter", True), seed=kw.get("seed", 0), frame=kw.get("frame", 0),
                        quadrature=kw.get("quadrature", 0), light_w=kw.get("light_w", (1.0, 1.0, 1.0)),
                        light_set=kw.get("light_set", 0), work_order=kw.get("work_order", 0))
    g = ctx.march(to_dev(vol), ss, cam, p)
    return to_host(g)


def _both(ctx, orc, vol, ss, cam, step, what, stride=1, **kw):
    log(f"case {what}: grid {vol.shape} image {cam.width}x{cam.height} step {step} {kw}")
    gg = _run(ctx, vol, ss, cam, step, **kw)
    gr, m, cnt = orc.march(vol, ss, cam, step, stride=stride, **kw)
    allow = fp32_ray_allowance(orc, vol, ss, cam, step, stride=stride, **kw)
    if stride > 1:
        gg, gr, m, allow = (a[::stride, ::stride] for a in (gg, gr, m, allow))
    check_march(gg, gr, m, kw.get("depth_tau", 0.1), step / max(vol.shape), what, allow=allow)
    return gg, gr, cnt


def test_small_ortho(ctx, orc):
    wl = small_ortho()
    _, gr, cnt = _both(ctx, orc, wl.volume(), 8.0, wl.camera, wl.step_voxels, "ortho32_64px")
    assert cnt[1] > cnt[0] > 0
    assert (gr[..., 1] < 0.5).sum() > 100  # the scene is not trivial


def test_headline_full_image(ctx, orc):
    wl = headline()
    _both(ctx, orc, wl.volume(), 8.0, wl.camera, wl.step_voxels, "persp128_256px")


def test_ragged_sizes_oblique_camera(ctx, orc):
    vol = make_volume((20, 28, 36), 5, 17, noise_amp=0.3)
    cam = Camera(PERSPECTIVE, (-1.3, 2.1, 1.7), target=(0.55, 0.45, 0.5), up=(0.2, 0.1, 1.0), fov_y_deg=48.0,
                 width=45, height=37)
    _both(ctx, orc, vol, 6.0, cam, 1.5, "ragged", seed=5, frame=3)
    cam_o = Camera(ORTHOGRAPHIC, (0.4, -2.0, 0.7), target=(0.5, 0.5, 0.5), up=(0.0, 0.0, 1.0),
                   ortho_half_extent=0.8, width=33, height=50)
    _both(ctx, orc, vol, 6.0, cam_o, 0.75, "ragged_ortho", seed=9)


def test_riemann_weights_and_light_mix(ctx, orc):
    wl = small_ortho()
    _both(ctx, orc, wl.volume(), 8.0, wl.camera, 2.0, "riemann", quadrature=1, light_w=(0.5, 2.0, 0.0))
    _both(ctx, orc, wl.volume(), 8.0, wl.camera, 2.0, "top_only", light_w=(0.0, 1.0, 0.0), jitter=False)


def test_left_right_light_set(ctx, orc):
    """The guiding-light ablation's (left, right) side lights (Section 5)."""
    wl = small_ortho()
    _both(ctx, orc, wl.volume(), 8.0, wl.camera, 2.0, "left_right", light_set=1)
    _both(ctx, orc, wl.volume(), 8.0, wl.camera, 2.0, "left_only", light_set=1, light_w=(0.0, 1.0, 0.0))
    vol = make_volume((20, 28, 36), 5, 17, noise_amp=0.3)
    cam = Camera(PERSPECTIVE, (-1.3, 2.1, 1.7), target=(0.55, 0.45, 0.5), up=(0.2, 0.1, 1.0), fov_y_deg=48.0,
                 width=45, height=37)
    _both(ctx, orc, vol, 6.0, cam, 1.5, "left_right_oblique", seed=5, light_set=1, light_w=(0.3, 0.5, 1.2))


def test_ert_off_and_dense(ctx, orc):
    wl = small_ortho()
    _both(ctx, orc, wl.volume(), 8.0, wl.camera, 2.0, "ert_off", ert_eps=0.0)
    _, gr, _ = _both(ctx, orc, wl.volume() * 6.0, 8.0, wl.camera, 1.0, "dense")
    assert (gr[..., 1] == 0.0).sum() > 100  # many rays terminated early


def test_empty_volume_and_miss(ctx, orc):
    wl = small_ortho()
    g = _run(ctx, np.zeros((32, 32, 32), np.float32), 8.0, wl.camera, 2.0)
    assert np.all(g[..., 0] == 0) and np.all(g[..., 1] == 1) and np.all(g[..., 2] == 0)
    away = Camera(PERSPECTIVE, (3.0, 0.5, 0.5), target=(4.0, 0.5, 0.5), width=24, height=24)
    g = _run(ctx, wl.volume(), 8.0, away, 2.0)
    assert np.all(g[..., 0] == 0) and np.all(g[..., 1] == 1) and np.all(g[..., 2] == 0)


def test_degenerate_view_along_z(ctx, orc):
    """w parallel to the world z axis: the side lights fall back to w x x."""
    vol = make_volume(24, 5, 2)
    cam = Camera(ORTHOGRAPHIC, (0.5, 0.5, 3.0), target=(0.5, 0.5, 0.5), up=(0.0, 1.0, 0.0), width=24, height=24)
    _both(ctx, orc, vol, 8.0, cam, 1.0, "view_along_z", light_w=(0.0, 1.0, 0.5))


def test_tiny_grid_and_image(ctx, orc):
    vol = np.full((1, 1, 1), 0.7, np.float32)
    cam = Camera(PERSPECTIVE, (2.0, 0.6, 0.4), width=1, height=1)
    _both(ctx, orc, vol, 3.0, cam, 0.1, "1voxel_1px")
    vol2 = make_volume((2, 3, 2), 2, 1)
    cam2 = Camera(ORTHOGRAPHIC, (0.5, 0.5, 2.5), target=(0.5, 0.5, 0.5), up=(0.0, 1.0, 0.0),
                  ortho_half_extent=0.6, width=3, height=2)
    _both(ctx, orc, vol2, 5.0, cam2, 0.5, "2x3x2_3x2px")


def test_dynamic_scene_full_size_sampled(ctx, orc):
    """256^3 grid with the sphere obstacle, 1024^2 orbit view: a 1-in-16
    pixel lattice is checked against the oracle."""
    wl = dynamic()
    vol = wl.volume(frame=37, obstacle_radius=0.15)
    from synth.scene import orbit_camera

    cam = orbit_camera(37)
    _both(ctx, orc, vol, 8.0, cam, wl.step_voxels, "dynamic256_1024px_stride16", stride=16, frame=37)
    # this grid takes the z order by default; the band order gives the same map at every pixel
    from paper_2604_03748_amd import lnm

    a = _run(ctx, vol, 8.0, cam, wl.step_voxels, frame=37)
    b = _run(ctx, vol, 8.0, cam, wl.step_voxels, frame=37, work_order=lnm.ORDER_BANDS)
    assert np.array_equal(a, b)


def _bricks_numpy(vol):
    """The bricked layout as documented for lnm_make_bricks, built with numpy."""
    nz, ny, nx = vol.shape
    nb = [(n >> 2) + 1 for n in (nx, ny, nz)]
    pad = np.zeros((4 * nb[2] + 1, 4 * nb[1] + 1, 4 * nb[0] + 1), np.float32)
    pad[1:nz + 1, 1:ny + 1, 1:nx + 1] = vol
    out = np.zeros((nb[2], nb[1], nb[0], 128), np.float32)
    for bz in range(nb[2]):
        for by in range(nb[1]):
            for bx in range(nb[0]):
                blk = pad[4 * bz:4 * bz + 5, 4 * by:4 * by + 5, 4 * bx:4 * bx + 5]
                out[bz, by, bx, :125] = blk.ravel()
    return out.ravel()


def test_prebuilt_bricks(ctx, orc):
    """lnm_make_bricks writes the documented layout, and a march on prebuilt
    bricks equals the march that builds them itself, with a smaller workspace."""
    from paper_2604_03748_amd import lnm

    for shape in ((20, 28, 36), (5, 3, 9), (64, 64, 64)):
        vol = make_volume(shape, 5, 17, noise_amp=0.3)
        log(f"bricks of {shape}")
        dens = to_dev(vol)
        br = ctx.make_bricks(dens)
        assert np.array_equal(to_host(br), _bricks_numpy(vol))
        cam = Camera(PERSPECTIVE, (-1.3, 2.1, 1.7), target=(0.55, 0.45, 0.5), up=(0.2, 0.1, 1.0), width=45, height=37)
        p = lnm.make_params(1.5, seed=5)
        a = to_host(ctx.march(dens, 6.0, cam, p))
        b = to_host(ctx.march(dens, 6.0, cam, p, bricks=br))
        assert np.array_equal(a, b)
        assert ctx.march_workspace_bytes(dens, 6.0, cam, p, bricks=br) < ctx.march_workspace_bytes(dens, 6.0, cam, p)


def cases_cam_odd():
    return Camera(PERSPECTIVE, (1.9, -1.2, 1.4), target=(0.5, 0.5, 0.45), up=(0.0, 0.0, 1.0), fov_y_deg=50.0,
                  width=41, height=35)


def test_work_orders_agree(ctx, orc):
    """The light marches' work order (screen bands, records sorted by brick
    layer and taken by each XCD in turn, or records sorted by z cell with the
    cell's grid planes read from LDS) changes nothing in the guiding map: bit
    for bit equal, on cameras whose side lights stay in z planes and on ones
    whose lights do not (view along z, left/right set)."""
    from paper_2604_03748_amd import lnm

    wl = headline()
    ragged = make_volume((20, 28, 36), 5, 17, noise_amp=0.3)
    cases = [
        ("headline", wl.volume(), 8.0, wl.camera, wl.step_voxels, {}),
        ("ragged", ragged, 6.0, Camera(PERSPECTIVE, (-1.3, 2.1, 1.7), target=(0.55, 0.45, 0.5), up=(0.2, 0.1, 1.0),
                                        fov_y_deg=48.0, width=45, height=37), 1.5, {"seed": 5, "frame": 3}),
        ("view_along_z", make_volume(24, 5, 2), 8.0,
         Camera(ORTHOGRAPHIC, (0.5, 0.5, 3.0), target=(0.5, 0.5, 0.5), up=(0.0, 1.0, 0.0), width=24, height=24),
         1.0, {"light_w": (0.0, 1.0, 0.5)}),
        ("left_right", ragged, 6.0, Camera(ORTHOGRAPHIC, (0.4, -2.0, 0.7), up=(0.0, 0.0, 1.0), ortho_half_extent=0.8,
                                           width=33, height=50), 0.75, {"light_set": 1, "seed": 9}),
        ("dense_riemann", small_ortho().volume() * 6.0, 8.0, small_ortho().camera, 1.0, {"quadrature": 1}),
        # no axis a multiple of four: the cell order stages its planes value
        # by value instead of in groups of four
        ("odd_rows", make_volume((19, 26, 33), 4, 11, noise_amp=0.3), 6.0, cases_cam_odd(), 1.25, {"seed": 2}),
    ]
    for what, vol, ss, cam, step, kw in cases:
        log(f"work orders: {what}")
        a = _run(ctx, vol, ss, cam, step, work_order=lnm.ORDER_BANDS, **kw)
        b = _run(ctx, vol, ss, cam, step, work_order=lnm.ORDER_Z, **kw)
        assert np.array_equal(a, b), what
        c = _run(ctx, vol, ss, cam, step, work_order=lnm.ORDER_CELLS, **kw)
        d = np.abs(a - c)
        log(f"  cells vs bands: max abs {d.max():.3g} over {int((d > 0).sum())} values")
        assert np.array_equal(a, c), what
        assert np.array_equal(a, _run(ctx, vol, ss, cam, step, **kw)), what  # auto (bands or cells)
    dens = to_dev(ragged)
    cam = cases[1][3]
    pb, pz = lnm.make_params(1.5, work_order=lnm.ORDER_BANDS), lnm.make_params(1.5, work_order=lnm.ORDER_Z)
    assert ctx.march_workspace_bytes(dens, 6.0, cam, pz) > ctx.march_workspace_bytes(dens, 6.0, cam, pb)
    with pytest.raises(lnm.LnmError):
        ctx.march(dens, 6.0, cam, lnm.make_params(1.5, work_order=4))
    # cell order needs a cell's two grid planes in LDS: 144 x 144 planes do not fit
    big = to_dev(make_volume((16, 144, 144), 3, 1))
    with pytest.raises(lnm.LnmError) as e:
        ctx.march(big, 6.0, cam, lnm.make_params(1.5, work_order=lnm.ORDER_CELLS))
    assert e.value.status == lnm.LNM_ERR_UNSUPPORTED


def test_march_batch_equals_single_marches(ctx):
    """lnm_march_batch (ragged: own grid, camera, step and seed per map)
    gives each map bit for bit what lnm_march gives it alone; a bad entry
    anywhere fails the call before anything is enqueued."""
    import torch

    from paper_2604_03748_amd import lnm

    vols = [make_volume((20, 28, 36), 5, 17, noise_amp=0.3), make_volume(64, 8, 3, noise_amp=0.3),
            make_volume((5, 3, 9), 2, 4)]
    cams = [Camera(PERSPECTIVE, (-1.3, 2.1, 1.7), target=(0.55, 0.45, 0.5), up=(0.2, 0.1, 1.0), width=45, height=37),
            headline().camera.resized(96, 64),
            Camera(ORTHOGRAPHIC, (0.4, -2.0, 0.7), up=(0.0, 0.0, 1.0), ortho_half_extent=0.8, width=33, height=50)]
    prms = [lnm.make_params(1.5, seed=5, frame=3), lnm.make_params(4.0, seed=0), lnm.make_params(0.75, seed=9)]
    dens = [to_dev(v) for v in vols]
    log("march batch of 3 ragged maps")
    got = ctx.march_batch(dens, [6.0, 8.0, 3.0], cams, prms)
    for i, (d, ss, c, p) in enumerate(zip(dens, [6.0, 8.0, 3.0], cams, prms)):
        assert np.array_equal(to_host(got[i]), to_host(ctx.march(d, ss, c, p))), i
    # a zero field of view in the last-but-one entry: error, and the first
    # guide untouched
    from dataclasses import replace

    outs = [torch.full((c.height, c.width, 3), float("nan"), device="cuda") for c in cams]
    bad = [cams[0], replace(cams[1], fov_y_deg=0.0), cams[2]]
    with pytest.raises(lnm.LnmError):
        ctx.march_batch(dens, [6.0, 8.0, 3.0], bad, prms, outs=outs,
                        workspace=torch.empty(64 << 20, dtype=torch.uint8, device="cuda"))
    torch.cuda.synchronize()
    assert np.isnan(to_host(outs[0])).all()
