"""Seeded synthetic smoke volumes, cameras and lights.

The paper trains and measures on LBM-simulated smoke rendered by an offline
path tracer (Section 5, "Data Generation"); neither the simulator nor the data
ships with it.  These procedural fields stand in for that data with the same
structure: a scattering-coefficient grid with soft blobs, small-scale
modulation, optional motion and an obstacle mask.

Recipe (all draws from ``synth.rng`` substreams of the scene seed):

* blob b: centre c_b ~ U[0,1]^3, radius r_b ~ U[0.05, 0.2] (Gaussian standard
  deviation), peak p_b ~ U[0.5, 2];
  rho(x) = sum_b p_b exp(-|x - c_b|^2 / (2 r_b^2)) at voxel centres, in fp64,
  evaluated as the product of its three per-axis factors, stored as fp32;
* value noise (optional): lattice frequencies 4, 8, 16 with values U[-1, 1]
  on the (f+1)^3 lattice points i/f, trilinear between them, octave amplitudes
  1, 1/2, 1/4 divided by 1.75; rho <- max(0, rho * (1 + amp * n(x)));
* motion (optional): velocities v_b ~ U[-0.002, 0.002]^3 per frame, centres
  move linearly and reflect at the cube walls;
* obstacle (optional): voxels whose centre lies within ``radius`` of
  ``centre`` are set to zero.

Voxel (i, j, k) of an [nz][ny][nx] array (x fastest) has centre
((i + 1/2)/nx, (j + 1/2)/ny, (k + 1/2)/nz) in the unit cube.

Nothing here implements the rendering method.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace

import numpy as np

from .rng import substream

ORTHOGRAPHIC = 0
PERSPECTIVE = 1


@dataclass
class Blobs:
    centres: np.ndarray  # [n, 3] (x, y, z)
    radii: np.ndarray  # [n]
    peaks: np.ndarray  # [n]
    velocities: np.ndarray  # [n, 3] per frame


def draw_blobs(n_blobs: int, seed: int) -> Blobs:
    s = substream(seed, "blobs")
    u = s.uniform(5 * n_blobs).reshape(n_blobs, 5)
    v = substream(seed, "velocity").uniform(3 * n_blobs).reshape(n_blobs, 3)
    return Blobs(
        centres=u[:, :3].copy(),
        radii=0.05 + 0.15 * u[:, 3],
        peaks=0.5 + 1.5 * u[:, 4],
        velocities=(2.0 * v - 1.0) * 0.002,
    )


def blob_centres_at(blobs: Blobs, frame: int) -> np.ndarray:
    """Centres after ``frame`` steps of linear motion reflected at the walls."""
    p = blobs.centres + blobs.velocities * float(frame)
    p = np.mod(p, 2.0)
    return np.where(p > 1.0, 2.0 - p, p)


def _centres(n: int) -> np.ndarray:
    return (np.arange(n, dtype=np.float64) + 0.5) / n


def blob_field(shape, blobs: Blobs, frame: int = 0) -> np.ndarray:
    nz, ny, nx = shape
    xs, ys, zs = _centres(nx), _centres(ny), _centres(nz)
    cen = blob_centres_at(blobs, frame)
    rho = np.zeros((nz, ny, nx), dtype=np.float64)
    for b in range(len(blobs.radii)):
        inv = 1.0 / (2.0 * blobs.radii[b] ** 2)
        gx = np.exp(-((xs - cen[b, 0]) ** 2) * inv)
        gy = np.exp(-((ys - cen[b, 1]) ** 2) * inv)
        gz = np.exp(-((zs - cen[b, 2]) ** 2) * inv)
        rho += blobs.peaks[b] * (gz[:, None, None] * gy[None, :, None] * gx[None, None, :])
    return rho


def _lattice_weights(n: int, f: int) -> np.ndarray:
    """[n, f+1] linear-interpolation weights of voxel centres on lattice i/f."""
    g = _centres(n) * f
    i0 = np.minimum(np.floor(g).astype(np.int64), f - 1)
    fr = g - i0
    w = np.zeros((n, f + 1), dtype=np.float64)
    w[np.arange(n), i0] = 1.0 - fr
    w[np.arange(n), i0 + 1] += fr
    return w


def value_noise(shape, seed: int, freqs=(4, 8, 16), amps=(1.0, 0.5, 0.25)) -> np.ndarray:
    nz, ny, nx = shape
    s = substream(seed, "noise")
    out = np.zeros(shape, dtype=np.float64)
    for f, a in zip(freqs, amps):
        lat = 2.0 * s.uniform((f + 1) ** 3).reshape(f + 1, f + 1, f + 1) - 1.0  # [z][y][x]
        wz, wy, wx = _lattice_weights(nz, f), _lattice_weights(ny, f), _lattice_weights(nx, f)
        t = np.tensordot(wz, lat, axes=([1], [0]))  # [nz, f+1, f+1]
        t = np.tensordot(t, wy, axes=([1], [1]))  # [nz, f+1(x), ny]
        t = np.tensordot(t, wx, axes=([1], [1]))  # [nz, ny, nx]
        out += a * t
    return out / sum(amps)


def sphere_mask(shape, centre=(0.5, 0.5, 0.5), radius=0.15) -> np.ndarray:
    nz, ny, nx = shape
    xs, ys, zs = _centres(nx), _centres(ny), _centres(nz)
    d2 = ((zs - centre[2]) ** 2)[:, None, None] + ((ys - centre[1]) ** 2)[None, :, None] + (
        (xs - centre[0]) ** 2
    )[None, None, :]
    return d2 <= radius * radius


def make_volume(n, n_blobs: int, seed: int, noise_amp: float = 0.0, frame: int = 0,
                obstacle_radius: float | None = None) -> np.ndarray:
    """fp32 density grid [nz][ny][nx] (x fastest); ``n`` is an int or (nz, ny, nx)."""
    shape = (n, n, n) if isinstance(n, int) else tuple(n)
    blobs = draw_blobs(n_blobs, seed)
    rho = blob_field(shape, blobs, frame)
    if noise_amp:
        rho = np.maximum(0.0, rho * (1.0 + noise_amp * value_noise(shape, seed)))
    if obstacle_radius is not None:
        rho[sphere_mask(shape, radius=obstacle_radius)] = 0.0
    return np.ascontiguousarray(rho.astype(np.float32))


def light_direction(seed: int) -> np.ndarray:
    """A unit vector uniform on the sphere (direction toward the light)."""
    u = substream(seed, "light").uniform(2)
    z = 2.0 * u[0] - 1.0
    phi = 2.0 * math.pi * u[1]
    s = math.sqrt(max(0.0, 1.0 - z * z))
    return np.array([s * math.cos(phi), s * math.sin(phi), z])


def rotate_y(v, deg: float) -> np.ndarray:
    a = math.radians(deg)
    c, s = math.cos(a), math.sin(a)
    x, y, z = v
    return np.array([c * x + s * z, y, -s * x + c * z])


@dataclass
class Camera:
    projection: int
    eye: tuple
    target: tuple = (0.5, 0.5, 0.5)
    up: tuple = (0.0, 1.0, 0.0)
    fov_y_deg: float = 60.0
    ortho_half_extent: float = math.sqrt(3.0) / 2.0
    width: int = 64
    height: int = 64

    def resized(self, width: int, height: int) -> "Camera":
        return replace(self, width=width, height=height)


def ortho_camera(width=64, height=64, distance=2.5, half_extent=math.sqrt(3.0) / 2.0) -> Camera:
    return Camera(ORTHOGRAPHIC, (0.5 + distance, 0.5, 0.5), ortho_half_extent=half_extent,
                  width=width, height=height)


def perspective_camera(width=256, height=256, distance=2.5, fov_y_deg=60.0) -> Camera:
    return Camera(PERSPECTIVE, (0.5 + distance, 0.5, 0.5), fov_y_deg=fov_y_deg,
                  width=width, height=height)


def orbit_camera(frame: int, width=1024, height=1024, distance=2.5, deg_per_frame=1.5,
                 fov_y_deg=60.0) -> Camera:
    """Perspective camera orbiting the cube centre about the y axis."""
    off = rotate_y((distance, 0.0, 0.0), deg_per_frame * frame)
    eye = tuple(0.5 + off)
    return Camera(PERSPECTIVE, eye, fov_y_deg=fov_y_deg, width=width, height=height)


# ---------------------------------------------------------------- workloads
@dataclass
class Workload:
    """One seeded scene with its camera and march step (in voxels)."""
    name: str
    grid: int
    n_blobs: int
    noise_amp: float
    camera: Camera
    step_voxels: float
    levels: int
    base: int
    seed: int = 0
    light: np.ndarray = field(default=None)

    def volume(self, frame: int = 0, obstacle_radius=None) -> np.ndarray:
        return make_volume(self.grid, self.n_blobs, self.seed, self.noise_amp, frame, obstacle_radius)

    def light_dir(self) -> np.ndarray:
        return light_direction(self.seed) if self.light is None else self.light


def small_ortho(seed: int = 0) -> Workload:
    """32^3, 6 blobs, orthographic 64^2, step 2 voxels, 3-level base-16 U-Net."""
    return Workload("ortho32_64px", 32, 6, 0.0, ortho_camera(64, 64), 2.0, 3, 16, seed)


def headline(seed: int = 0, res: int = 256) -> Workload:
    """128^3, 24 blobs + noise 0.3, perspective 60 deg at 2.5, step 4, 4-level base-32."""
    return Workload(f"persp128_{res}px", 128, 24, 0.3, perspective_camera(res, res), 4.0, 4, 32, seed)


def dynamic(seed: int = 0) -> Workload:
    """256^3, 32 moving blobs + noise, sphere obstacle, orbit camera 1024^2, base-48."""
    return Workload("dynamic256_1024px", 256, 32, 0.3, orbit_camera(0), 4.0, 4, 48, seed)


def make_volume_torch(n: int, n_blobs: int, seed: int, noise_amp: float = 0.0, frame: int = 0,
                      obstacle_radius: float | None = None, device="cuda"):
    """The recipe of make_volume evaluated with torch in fp64 on `device`
    (same seeded draws; values agree with make_volume to fp64 rounding before
    the final fp32 cast).  For large serving-scale grids."""
    import torch

    blobs = draw_blobs(n_blobs, seed)
    c = torch.as_tensor(_centres(n), device=device)
    cen = blob_centres_at(blobs, frame)
    rho = torch.zeros((n, n, n), dtype=torch.float64, device=device)
    for b in range(len(blobs.radii)):
        inv = 1.0 / (2.0 * blobs.radii[b] ** 2)
        gx = torch.exp(-((c - cen[b, 0]) ** 2) * inv)
        gy = torch.exp(-((c - cen[b, 1]) ** 2) * inv)
        gz = torch.exp(-((c - cen[b, 2]) ** 2) * inv)
        rho += blobs.peaks[b] * (gz[:, None, None] * gy[None, :, None] * gx[None, None, :])
    if noise_amp:
        s = substream(seed, "noise")
        noise = torch.zeros_like(rho)
        for f, a in zip((4, 8, 16), (1.0, 0.5, 0.25)):
            lat = torch.as_tensor(2.0 * s.uniform((f + 1) ** 3).reshape(f + 1, f + 1, f + 1) - 1.0, device=device)
            w = torch.as_tensor(_lattice_weights(n, f), device=device)
            t = torch.tensordot(w, lat, dims=([1], [0]))  # [n, f+1 (y), f+1 (x)]
            t = torch.tensordot(t, w, dims=([1], [1]))  # [n, f+1 (x), n (y)]
            t = torch.tensordot(t, w, dims=([1], [1]))  # [n (z), n (y), n (x)]
            noise += a * t
        rho = torch.clamp(rho * (1.0 + noise_amp * noise / 1.75), min=0.0)
    if obstacle_radius is not None:
        rho[torch.as_tensor(sphere_mask((n, n, n), radius=obstacle_radius), device=device)] = 0.0
    return rho.to(torch.float32).contiguous()
