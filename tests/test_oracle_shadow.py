"""Pins of the oracle's depth-based obstacle shadowing (Section 4.5): the
shadow map of a sphere against a world-space ray-sphere solve, per-pixel
visibility against brute-force occlusion along the light ray, the D = 0
special case, and the shadowed composite against the plain one.  CPU only."""
import math

import numpy as np

from synth.scene import PERSPECTIVE, perspective_camera


def _basis(cam):
    eye, tgt, up = (np.array(v, dtype=np.float64) for v in (cam.eye, cam.target, cam.up))
    f = tgt - eye
    f /= np.linalg.norm(f)
    r = np.cross(f, up)
    r /= np.linalg.norm(r)
    u = np.cross(r, f)
    return eye, f, r, u


def _ray(cam, i, j):
    """Pinhole ray of pixel (i, j) through its centre (Section 4.2's camera)."""
    assert cam.projection == PERSPECTIVE
    eye, f, r, u = _basis(cam)
    sx = 2.0 * (i + 0.5) / cam.width - 1.0
    sy = 1.0 - 2.0 * (j + 0.5) / cam.height
    th = math.tan(math.radians(cam.fov_y_deg) / 2.0)
    d = f + th * (sx * cam.width / cam.height * r + sy * u)
    return eye, d / np.linalg.norm(d)


def _light_frame(l):
    l = np.asarray(l, dtype=np.float64) / np.linalg.norm(l)
    a = np.array([1.0, 0.0, 0.0]) if abs(l[1]) > 0.99 else np.array([0.0, 1.0, 0.0])
    e1 = np.cross(a, l)
    e1 /= np.linalg.norm(e1)
    return e1, np.cross(l, e1), l


LIGHT = np.array([0.3, 0.8, -0.5]) / np.linalg.norm([0.3, 0.8, -0.5])
CENTRE = np.array([0.5, 0.5, 0.5])
RADIUS = 0.15
ORIGIN = np.array([0.42, 0.57, 0.5])  # off the sphere centre, so a wrong basis shows
E = 0.9
S = 96


def test_shadow_map_matches_world_space_ray_sphere(orc):
    depth = orc.shadow_map_sphere(S, E, ORIGIN, LIGHT, CENTRE, RADIUS)
    e1, e2, l = _light_frame(LIGHT)
    hit = 0
    for j in range(0, S, 2):
        for i in range(0, S, 2):
            u = -E + 2 * E * (i + 0.5) / S
            v = -E + 2 * E * (j + 0.5) / S
            # ray from far out on the light side, travelling along -l
            p0 = ORIGIN + u * e1 + v * e2 + 10.0 * l
            oc = p0 - CENTRE
            b = np.dot(oc, -l)
            disc = b * b - (np.dot(oc, oc) - RADIUS * RADIUS)
            if disc < 0:
                assert depth[j, i] == -np.inf
                continue
            s_hit = -b - math.sqrt(disc)  # first hit
            z_hit = np.dot(p0 + s_hit * -l - ORIGIN, l)
            assert abs(depth[j, i] - z_hit) < 1e-12
            hit += 1
    assert hit > 40, hit


def test_light_basis_is_right_handed_orthonormal():
    for l in (LIGHT, np.array([0.0, 1.0, 0.0]), np.array([0.05, -0.999, 0.0])):
        e1, e2, ll = _light_frame(l)
        m = np.stack([e1, e2, ll])
        assert np.allclose(m @ m.T, np.eye(3), atol=1e-12)
        assert np.allclose(np.cross(e1, e2), ll, atol=1e-12)


def _scene(res=96):
    """A smoke slab x < 0.3 behind the sphere obstacle, seen from +x."""
    cam = perspective_camera(res, res)
    n = 32
    vol = np.zeros((n, n, n), dtype=np.float32)
    vol[:, :, : int(0.3 * n)] = 1.0
    return cam, vol


# toward the light: mostly from the camera side, so the sphere shadows the slab
LIGHT_SLAB = np.array([0.9, 0.3, 0.2]) / np.linalg.norm([0.9, 0.3, 0.2])


def test_visibility_matches_brute_force_occlusion(orc):
    cam, vol = _scene()
    g = orc.march(vol, 8.0, cam, 1.0, jitter=False)[0]
    depth = orc.shadow_map_sphere(S, E, ORIGIN, LIGHT_SLAB, CENTRE, RADIUS)
    bias = 1e-3
    vis = orc.shadow_visibility(g, cam, LIGHT_SLAB, depth, E, ORIGIN, bias)
    e1, e2, l = _light_frame(LIGHT_SLAB)
    texel = 2 * E / S
    checked = shadowed = 0
    for j in range(cam.height):
        for i in range(cam.width):
            D = g[j, i, 2]
            if D == 0.0:
                assert vis[j, i] == 1.0
                continue
            o, d = _ray(cam, i, j)
            P = o + D * d
            q = P - CENTRE
            r_perp = np.linalg.norm(q - np.dot(q, l) * l)
            # skip points where texel snapping or the bias can decide
            if abs(r_perp - RADIUS) < 1.5 * texel or np.linalg.norm(q) < RADIUS + 0.02:
                continue
            s = np.linspace(1e-3, 2.0, 4001)
            pts = P[None, :] + s[:, None] * l[None, :]
            occluded = bool(np.any(np.sum((pts - CENTRE) ** 2, axis=1) < RADIUS * RADIUS))
            assert vis[j, i] == (0.0 if occluded else 1.0), (i, j)
            checked += 1
            shadowed += occluded
    assert checked > 800 and shadowed > 30, (checked, shadowed)


def test_no_obstacle_means_fully_visible(orc):
    cam, vol = _scene(24)
    g = orc.march(vol, 8.0, cam, 1.0, jitter=False)[0]
    depth = np.full((S, S), -np.inf)
    vis = orc.shadow_visibility(g, cam, LIGHT, depth, E, ORIGIN, 1e-3)
    assert np.all(vis == 1.0)


def test_shadowed_composite_reduces_to_plain_composite(orc):
    rng = np.random.default_rng(5)
    H, W = 6, 7
    cam = perspective_camera(W, H)
    lm = rng.uniform(0, 1, (H, W, 6))
    guide = np.stack([rng.uniform(0, 1, (H, W)), rng.uniform(0, 1, (H, W)), rng.uniform(0, 2, (H, W))], -1)
    lights = [(LIGHT, (1.0, 0.9, 0.8)), ((-0.6, 0.2, 0.77), (0.2, 0.3, 0.5))]
    ones = np.ones((2, H, W))
    full = orc.composite(lm, guide, cam, lights)
    assert np.allclose(orc.composite_shadowed(lm, guide, cam, lights, ones), full, rtol=0, atol=1e-14)
    zero = orc.composite_shadowed(lm, guide, cam, lights, np.zeros((2, H, W)))
    assert np.all(zero[..., :3] == 0.0) and np.array_equal(zero[..., 3], full[..., 3])
    mask = rng.integers(0, 2, (2, H, W)).astype(np.float64)
    got = orc.composite_shadowed(lm, guide, cam, lights, mask)
    want = sum(mask[k][..., None] * orc.composite(lm, guide, cam, [lights[k]])[..., :3] for k in range(2))
    assert np.allclose(got[..., :3], want, rtol=0, atol=1e-14)
