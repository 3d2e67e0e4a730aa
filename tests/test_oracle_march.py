"""Pins of the oracle's guiding-map march (Algorithm 1, Section 4.2), its
reference lightmaps and the six-way shading (Section 3) against closed forms,
invariants and textbook special cases.  CPU only."""
import math
import os

import numpy as np
import pytest

from synth.scene import Camera, ORTHOGRAPHIC, PERSPECTIVE, make_volume, ortho_camera, small_ortho

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows


# ------------------------------------------------------------------ hashing
def test_splitmix64_known_answers(orc):
    want = [int(r[0], 16) for r in _golden("splitmix64_seed0.txt")]
    gamma = 0x9E3779B97F4A7C15
    got = [orc.splitmix64((k * gamma) & (2**64 - 1)) for k in range(4)]
    assert got == want


def test_jitter_is_uniform_24bit(orc):
    u = np.array([orc.jitter(7, 3, p) for p in range(20000)])
    assert np.all(u >= 0) and np.all(u < 1)
    assert np.all(u * 2**24 == np.floor(u * 2**24))  # exact in fp32
    assert abs(u.mean() - 0.5) < 0.01
    hist = np.histogram(u, bins=10, range=(0, 1))[0]
    assert hist.min() > 1800 and hist.max() < 2200
    assert orc.jitter(7, 3, 5) != orc.jitter(7, 4, 5) != orc.jitter(8, 3, 5)


def test_jitter_key_roles(orc):
    """The key mix, a reading (the paper fixes no generator): the frame
    enters the key shifted into the high 32 bits and the pixel index into
    the low ones, both XORed into the seed.  So a frame is the same as a
    seed with the frame in its high word, a pixel the same as a seed with
    the pixel in its low word, and a swap of seed and frame (or frame and
    pixel) changes the value."""
    M = 2**64 - 1
    for seed, frame, pixel in ((7, 3, 5), (0, 1, 0), (123456789, 77, 65535), (2**40 + 9, 2**31 - 1, 2**20)):
        u = orc.jitter(seed, frame, pixel)
        assert u == orc.jitter((seed ^ (frame << 32)) & M, 0, pixel)
        assert u == orc.jitter((seed ^ pixel) & M, frame, 0)
        # 24 high bits of SplitMix64 of the key, as a fraction
        key = (seed ^ (frame << 32) ^ pixel) & M
        assert u == (orc.splitmix64(key) >> 40) / 2**24
    assert orc.jitter(3, 7, 5) != orc.jitter(7, 3, 5)
    assert orc.jitter(7, 5, 3) != orc.jitter(7, 3, 5)


# ------------------------------------------------------------------ sampling
def test_sigma_trilinear_special_cases(orc):
    rng = np.random.default_rng(1)
    v = rng.random((5, 6, 7)).astype(np.float32)
    nz, ny, nx = v.shape
    # on a voxel centre the sample is the voxel value times sigma_scale
    for (i, j, k) in [(0, 0, 0), (3, 2, 1), (6, 5, 4)]:
        p = ((i + 0.5) / nx, (j + 0.5) / ny, (k + 0.5) / nz)
        assert orc.sigma_at(v, 3.0, p) == pytest.approx(3.0 * float(v[k, j, i]), rel=1e-12)
    # midway between two x-neighbours: their mean
    p = ((2 + 1.0) / nx, (1 + 0.5) / ny, (3 + 0.5) / nz)
    assert orc.sigma_at(v, 1.0, p) == pytest.approx(0.5 * (float(v[3, 1, 2]) + float(v[3, 1, 3])), rel=1e-12)
    # zero border: the support box face is exactly zero, half way to it is half
    p_face = (-0.5 / nx, (1 + 0.5) / ny, (2 + 0.5) / nz)
    assert orc.sigma_at(v, 1.0, p_face) == 0.0
    p_half = (0.0, (1 + 0.5) / ny, (2 + 0.5) / nz)
    assert orc.sigma_at(v, 1.0, p_half) == pytest.approx(0.5 * float(v[2, 1, 0]), rel=1e-12)
    assert orc.sigma_at(v, 1.0, (2.0, 0.5, 0.5)) == 0.0


# ------------------------------------------------------------------ closed forms
def test_empty_volume_is_exactly_transparent(orc):
    wl = small_ortho()
    g, _, cnt = orc.march(np.zeros((32, 32, 32), np.float32), 8.0, wl.camera, 2.0)
    assert np.all(g[..., 0] == 0.0) and np.all(g[..., 1] == 1.0) and np.all(g[..., 2] == 0.0)
    assert cnt[0] > 0  # the rays did cross the support box


def _aligned_cube_camera(n):
    """Orthographic camera looking down -x whose pixel rays pass through voxel
    centres and whose samples (h = 1 voxel, no jitter) land on voxel centres.
    Pixel (i, j) sees voxel row y = n-1-j and column z = n-1-i."""
    return Camera(ORTHOGRAPHIC, (3.0 + 0.5 / n, 0.5, 0.5), target=(0.5 + 0.5 / n, 0.5, 0.5),
                  up=(0.0, 1.0, 0.0), ortho_half_extent=0.5, width=n, height=n)


@pytest.mark.parametrize("w", [(1.0, 1.0, 1.0), (1.0, 0.0, 0.0), (0.0, 1.0, 0.0), (0.0, 0.0, 1.0)])
def test_uniform_cube_closed_form(orc, w):
    n, c, ss = 12, 0.35, 4.0
    vol = np.full((n, n, n), c, np.float32)
    cam = _aligned_cube_camera(n)
    g, _, _ = orc.march(vol, ss, cam, 1.0, depth_tau=0.1, ert_eps=0.0, jitter=False, light_w=w)
    q = math.exp(-ss * float(np.float32(c)) / n)
    for j in range(n):
        # front light: sum_k q^(k-1)(1-q) q^(k-1); top = w x z = -y (voxels below
        # row y = n-1-j: n-1-j of them); bottom = +y (j voxels above)
        want = w[0] * (1 - q ** (2 * n)) / (1 + q) + (1 - q**n) * (w[1] * q ** (n - 1 - j) + w[2] * q**j)
        np.testing.assert_allclose(g[j, :, 0], want, rtol=1e-12)
    np.testing.assert_allclose(g[..., 1], math.exp(-ss * float(np.float32(c))), rtol=1e-12)
    # first interior sample is x = 1 - dx/2, at t = 2 + 1/n: index 2n + 1
    np.testing.assert_allclose(g[..., 2], (2 * n + 1) / n, rtol=1e-12)


def test_uniform_cube_riemann_quadrature(orc):
    n, c, ss = 10, 0.5, 3.0
    vol = np.full((n, n, n), c, np.float32)
    cam = _aligned_cube_camera(n)
    g, _, _ = orc.march(vol, ss, cam, 1.0, ert_eps=0.0, jitter=False, quadrature=1, unit_radiance=True)
    s = ss * float(np.float32(c))
    q = math.exp(-s / n)
    # A_k = T_{k-1} sigma h = q^(k-1) s/n
    np.testing.assert_allclose(g[..., 0], (s / n) * (1 - q**n) / (1 - q), rtol=1e-12)


def test_uniform_slab_transmittance_converges_to_beer_lambert(orc):
    """exp(-sigma_t L) for a slab crossed by an oblique ray, as h -> 0."""
    n = 16
    vol = np.zeros((n, n, n), np.float32)
    vol[:, :, 4:12] = 0.25  # slab 4 <= x-index < 12
    ss = 6.0
    # orthographic rays along -x: optical depth through the slab of trilinear
    # density = 0.25 * ss * (8 voxels) exactly (ramps integrate symmetrically)
    cam = _aligned_cube_camera(n)
    errs = []
    for h in (2.0, 1.0, 0.5, 0.25, 0.125):
        g, _, _ = orc.march(vol, ss, cam, h, ert_eps=0.0, jitter=True, seed=3)
        T = g[4:12, 4:12, 1]
        errs.append(np.abs(T - math.exp(-0.25 * ss * 8 / n)).max())
    assert errs[-1] < 1e-12 or errs[-1] < errs[0]
    assert errs[-1] < 1e-9  # the trilinear ramp is integrated exactly by h | 1/2 voxel lattices


def test_alpha_identity(orc):
    wl = small_ortho()
    vol = wl.volume()
    g, _, _ = orc.march(vol, 8.0, wl.camera, 2.0, ert_eps=0.0, unit_radiance=True)
    np.testing.assert_allclose(g[..., 0], 1.0 - g[..., 1], atol=1e-13)


def test_front_transmittance_is_previous_primary(orc):
    wl = small_ortho()
    gap = orc.front_identity_gap(wl.volume(), 8.0, wl.camera, 2.0, jitter=True, seed=5)
    assert gap < 1e-12


def test_ert_bounds_the_dropped_tail(orc):
    wl = small_ortho()
    vol = wl.volume() * 4.0
    g0, _, _ = orc.march(vol, 8.0, wl.camera, 2.0, ert_eps=0.0)
    g1, _, _ = orc.march(vol, 8.0, wl.camera, 2.0, ert_eps=1e-6)
    term = g1[..., 1] == 0.0
    assert term.sum() > 50  # the scene is dense enough to terminate rays
    # transmittance is only cut where it had fallen below eps; L~ loses at most
    # 3 eps (three unit lights times the leftover transmittance)...
    assert np.all(g0[..., 1][term] < 1e-6)
    np.testing.assert_allclose(g1[..., 1][~term], g0[..., 1][~term], rtol=1e-12)
    # ...plus what the shortened secondary marches cut (each <= eps)
    assert np.abs(g1[..., 0] - g0[..., 0]).max() < 6e-6


# ------------------------------------------------------------------ invariants
def test_convergence_in_step(orc):
    vol = make_volume(24, 5, 11)
    cam = ortho_camera(24, 24)
    ref, _, _ = orc.march(vol, 8.0, cam, 1.0 / 16, ert_eps=0.0, jitter=False)
    errs = []
    for h in (4.0, 2.0, 1.0, 0.5):
        g, _, _ = orc.march(vol, 8.0, cam, h, ert_eps=0.0, jitter=False)
        errs.append(np.sqrt(np.mean((g[..., :2] - ref[..., :2]) ** 2)))
    assert all(a > b for a, b in zip(errs, errs[1:])), errs
    order = math.log2(errs[1] / errs[3]) / 2
    assert 0.6 < order < 1.6, (errs, order)


def test_mirror_symmetry(orc):
    n = 24
    base = make_volume(n, 5, 21)
    vol = (base + base[::-1, :, :]).astype(np.float32)  # symmetric about z = 1/2
    cam = ortho_camera(20, 18)  # looks down -x: image right = -z
    g, _, _ = orc.march(vol, 8.0, cam, 1.5, jitter=False)
    np.testing.assert_allclose(g, g[:, ::-1, :], atol=1e-12)
    lm = orc.reference_lightmaps(vol, 8.0, cam, 1.0)
    np.testing.assert_allclose(lm[..., 0], lm[:, ::-1, 1], atol=1e-12)
    for a in (2, 3, 4, 5):
        np.testing.assert_allclose(lm[..., a], lm[:, ::-1, a], atol=1e-12)


def test_rotation_about_world_z(orc):
    """Rotating volume and camera by 90 degrees about the z axis (which fixes
    the surrogate lights' w x z construction) leaves the guiding map unchanged."""
    n = 20
    vol = make_volume(n, 5, 4)
    rot = np.ascontiguousarray(vol[:, ::-1, :].transpose(0, 2, 1))  # (x, y) -> (1 - y, x)
    for proj, extra in ((ORTHOGRAPHIC, {}), (PERSPECTIVE, {"fov_y_deg": 50.0})):
        cam = Camera(proj, (2.9, 0.61, 0.37), target=(0.45, 0.52, 0.55), up=(0.1, 1.0, 0.2), width=22,
                     height=16, **extra)
        R = lambda p: (1.0 - p[1], p[0], p[2])
        Rv = lambda v: (-v[1], v[0], v[2])
        cam_r = Camera(proj, R(cam.eye), target=R(cam.target), up=Rv(cam.up), width=22, height=16, **extra)
        g, _, _ = orc.march(vol, 8.0, cam, 2.0, jitter=True, seed=9)
        gr, _, _ = orc.march(rot, 8.0, cam_r, 2.0, jitter=True, seed=9)
        np.testing.assert_allclose(gr, g, atol=1e-11)


def test_left_right_lights_are_the_quarter_turned_top_bottom(orc):
    """Guiding-light ablation (Section 5): viewing along -x, top = w x z = -y
    and left = w x top = -z.  Turning the volume and the camera's up vector
    by 90 degrees about the view axis (y -> z) makes the top light of the
    turned scene the left light of the original, pixel for pixel."""
    n = 20
    vol = make_volume(n, 5, 11)
    # V'(x, y, z) = V(x, 1 - z, y): V'[k][j][i] = V[j][n-1-k][i]
    turned = np.ascontiguousarray(vol.transpose(1, 0, 2)[::-1, :, :])
    cam_y = ortho_camera(18, 18)
    cam_z = Camera(ORTHOGRAPHIC, cam_y.eye, up=(0.0, 0.0, 1.0), ortho_half_extent=cam_y.ortho_half_extent,
                   width=18, height=18)
    for w in ((0.0, 1.0, 0.0), (0.0, 0.0, 1.0), (0.4, 0.7, 0.2)):
        lr, _, _ = orc.march(vol, 8.0, cam_z, 1.5, jitter=True, seed=2, light_w=w, light_set=1)
        tb, _, _ = orc.march(turned, 8.0, cam_y, 1.5, jitter=True, seed=2, light_w=w, light_set=0)
        np.testing.assert_allclose(lr, tb, atol=1e-11)
    # the two sets differ on a generic volume, and agree with front light only
    a = orc.march(vol, 8.0, cam_y, 1.5, jitter=False, light_set=0)[0]
    b = orc.march(vol, 8.0, cam_y, 1.5, jitter=False, light_set=1)[0]
    assert np.abs(a[..., 0] - b[..., 0]).max() > 1e-3
    np.testing.assert_array_equal(a[..., 1:], b[..., 1:])
    f0 = orc.march(vol, 8.0, cam_y, 1.5, jitter=False, light_w=(1, 0, 0), light_set=0)[0]
    f1 = orc.march(vol, 8.0, cam_y, 1.5, jitter=False, light_w=(1, 0, 0), light_set=1)[0]
    np.testing.assert_array_equal(f0, f1)


def test_perspective_projection_of_a_point(orc):
    """A compact blob shows up at the pinhole projection of its centre."""
    n = 64
    centre = np.array([0.62, 0.71, 0.33])
    zs = (np.arange(n) + 0.5) / n
    Z, Y, X = np.meshgrid(zs, zs, zs, indexing="ij")
    vol = np.exp(-((X - centre[0]) ** 2 + (Y - centre[1]) ** 2 + (Z - centre[2]) ** 2) / (2 * 0.02**2))
    cam = Camera(PERSPECTIVE, (2.7, 0.9, 1.4), target=(0.5, 0.5, 0.5), up=(0.0, 1.0, 0.0), fov_y_deg=40.0,
                 width=96, height=64)
    g, _, _ = orc.march(vol.astype(np.float32), 20.0, cam, 0.5, jitter=False)
    eye = np.array(cam.eye)
    f = np.array(cam.target) - eye
    f /= np.linalg.norm(f)
    r = np.cross(f, cam.up)
    r /= np.linalg.norm(r)
    u = np.cross(r, f)
    p = centre - eye
    t = math.tan(math.radians(cam.fov_y_deg) / 2)
    sx = (p @ r) / (p @ f) / (t * cam.width / cam.height)
    sy = (p @ u) / (p @ f) / t
    i_want = (sx + 1) * cam.width / 2 - 0.5
    j_want = (1 - sy) * cam.height / 2 - 0.5
    alpha = 1 - g[..., 1]
    jj, ii = np.unravel_index(np.argmax(alpha), alpha.shape)
    assert abs(ii - i_want) <= 1.0 and abs(jj - j_want) <= 1.0
    # centroid of opacity agrees to a fraction of a pixel
    J, I = np.mgrid[: cam.height, : cam.width]
    assert abs((alpha * I).sum() / alpha.sum() - i_want) < 0.3
    assert abs((alpha * J).sum() / alpha.sum() - j_want) < 0.3


def test_depth_is_first_threshold_crossing(orc):
    n = 16
    vol = np.zeros((n, n, n), np.float32)
    vol[:, :, 5:] = 1.0  # dense for x-index >= 5
    cam = _aligned_cube_camera(n)
    g, m, _ = orc.march(vol, 1.0, cam, 1.0, depth_tau=0.5, jitter=False)
    # samples at x = (n - 1/2 - k')/n ... first with sigma > 0.5 is x-index n-1,
    # reached at t = 2 + 1/n, i.e. sample index 2n + 1
    np.testing.assert_allclose(g[..., 2], (2 * n + 1) / n, rtol=1e-12)
    g2, _, _ = orc.march(vol, 1.0, cam, 1.0, depth_tau=2.0, jitter=False)
    assert np.all(g2[..., 2] == 0.0)  # never crosses: no surface


# ------------------------------------------------------------------ reference lightmaps
def test_reference_lightmaps_uniform_cube(orc):
    n, c, ss = 10, 0.3, 5.0
    vol = np.full((n, n, n), c, np.float32)
    cam = _aligned_cube_camera(n)
    lm = orc.reference_lightmaps(vol, ss, cam, 1.0, ert_eps=0.0)
    q = math.exp(-ss * float(np.float32(c)) / n)
    a = 1 - q**n
    J, I = np.mgrid[:n, :n]
    np.testing.assert_allclose(lm[..., 0], a * q ** (n - 1 - I), rtol=1e-12)  # +X = right = -z
    np.testing.assert_allclose(lm[..., 1], a * q**I, rtol=1e-12)
    np.testing.assert_allclose(lm[..., 2], a * q**J, rtol=1e-12)  # +Y = up
    np.testing.assert_allclose(lm[..., 3], a * q ** (n - 1 - J), rtol=1e-12)
    np.testing.assert_allclose(lm[..., 4], (1 - q ** (2 * n)) / (1 + q), rtol=1e-12)  # toward camera
    np.testing.assert_allclose(lm[..., 5], n * (1 - q) * q ** (n - 1), rtol=1e-12)  # away


def test_reference_plus_z_is_front_only_guide(orc):
    wl = small_ortho()
    vol = wl.volume()
    lm = orc.reference_lightmaps(vol, 8.0, wl.camera, 0.5, ert_eps=0.0)
    g, _, _ = orc.march(vol, 8.0, wl.camera, 0.5, ert_eps=0.0, jitter=False, light_w=(1.0, 0.0, 0.0))
    np.testing.assert_allclose(lm[..., 4], g[..., 0], atol=1e-12)


# ------------------------------------------------------------------ shading
def test_srgb_points(orc):
    for enc, lin in ((float(a), float(b)) for a, b in _golden("srgb_points.txt")):
        assert orc.srgb_decode(enc) == pytest.approx(lin, rel=1e-9, abs=1e-15)
        assert orc.srgb_encode(lin) == pytest.approx(enc, rel=1e-6, abs=1e-15)
    x = np.linspace(0, 1, 101)
    np.testing.assert_allclose(orc.srgb_decode(orc.srgb_encode(x)), x, atol=1e-12)


def test_composite_axis_lights_select_channels(orc):
    rng = np.random.default_rng(3)
    H, W = 5, 7
    lm = rng.random((H, W, 6))
    guide = rng.random((H, W, 3))
    cam = ortho_camera(W, H)  # right = -z, up = +y, toward camera = +x
    lin = orc.srgb_decode(lm)
    axes = {0: (0, 0, -1), 1: (0, 0, 1), 2: (0, 1, 0), 3: (0, -1, 0), 4: (1, 0, 0), 5: (-1, 0, 0)}
    for ch, d in axes.items():
        out = orc.composite(lm, guide, cam, [(d, (1.0, 0.5, 2.0))])
        np.testing.assert_allclose(out[..., 0], lin[..., ch], rtol=1e-12)
        np.testing.assert_allclose(out[..., 2], 2.0 * lin[..., ch], rtol=1e-12)
        np.testing.assert_allclose(out[..., 3], 1.0 - guide[..., 1], rtol=1e-12)
    d = np.array([1.0, -2.0, -2.0]) / 3.0  # camera frame (2/3 right... ) = (r, u, z) = (2/3, -2/3, 1/3)
    out = orc.composite(lm, guide, cam, [(d, (1, 1, 1)), ((0, 1, 0), (1, 1, 1))])
    want = (2 / 3) * lin[..., 0] + (2 / 3) * lin[..., 3] + (1 / 3) * lin[..., 4] + lin[..., 2]
    np.testing.assert_allclose(out[..., 1], want, rtol=1e-12)
