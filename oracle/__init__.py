"""FP64 CPU oracle of the neural six-way lightmaps hot path.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the GPU library or its binding.  The
arithmetic lives in ``oracle.c`` (plain fp64 loops); this module only
compiles it with gcc and marshals numpy arrays.

Parity status: every function here is pinned by CPU tests against closed
forms, invariants, brute force or library routines (torch CPU float64);
none is "parity unpinned".
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

CFLAGS = ["-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
          "-D_DEFAULT_SOURCE"]


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so next to it."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None
_D = C.POINTER(C.c_double)
_F = C.POINTER(C.c_float)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = C.CDLL(_LIB)
        L.orc_splitmix64.restype = C.c_uint64
        L.orc_splitmix64.argtypes = [C.c_uint64]
        L.orc_jitter.restype = C.c_double
        L.orc_jitter.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32]
        L.orc_sigma_vol.restype = C.c_double
        L.orc_sigma_vol.argtypes = [_F, C.c_int, C.c_int, C.c_int, C.c_double, _D]
        L.orc_march.restype = C.c_int
        L.orc_march.argtypes = [_F, C.c_int, C.c_int, C.c_int, C.c_double, _D, C.c_double, C.c_double, C.c_double,
                                C.c_int, C.c_uint64, C.c_uint32, C.c_int, _D, C.c_int, C.c_int, C.c_int, _D, _D,
                                C.POINTER(C.c_longlong)]
        L.orc_front_identity_gap.restype = C.c_double
        L.orc_front_identity_gap.argtypes = [_F, C.c_int, C.c_int, C.c_int, C.c_double, _D, C.c_double, C.c_int,
                                             C.c_uint64]
        L.orc_reference_lightmaps.restype = C.c_int
        L.orc_reference_lightmaps.argtypes = [_F, C.c_int, C.c_int, C.c_int, C.c_double, _D, C.c_double,
                                              C.c_double, _D]
        L.orc_srgb_encode.restype = C.c_double
        L.orc_srgb_encode.argtypes = [C.c_double]
        L.orc_srgb_decode.restype = C.c_double
        L.orc_srgb_decode.argtypes = [C.c_double]
        L.orc_composite.restype = C.c_int
        L.orc_composite.argtypes = [C.c_int, C.c_int, _D, _D, _D, _D, C.c_int, _D]
        L.orc_unet_param_count.restype = C.c_long
        L.orc_unet_param_count.argtypes = [C.c_int, C.c_int]
        L.orc_unet_forward.restype = C.c_int
        L.orc_unet_forward.argtypes = [C.c_int, C.c_int, _F, C.c_long, C.c_int, C.c_int, C.c_int, _D, _D, _D]
        L.orc_unet_loss_grad.restype = C.c_int
        L.orc_unet_loss_grad.argtypes = [C.c_int, C.c_int, _F, C.c_long, C.c_int, C.c_int, C.c_int, _D, _D, _D, _D]
        L.orc_unet_features.restype = C.c_int
        L.orc_unet_features.argtypes = [C.c_int, C.c_int, _F, C.c_long, C.c_int, C.c_int, C.c_int, _D, _D]
        L.orc_adapter_param_count.restype = C.c_long
        L.orc_adapter_param_count.argtypes = [C.c_int]
        L.orc_adapters_forward.restype = C.c_int
        L.orc_adapters_forward.argtypes = [C.c_int, _F, C.c_long, C.c_int, C.c_int, C.c_int, _D, _D, _D]
        L.orc_adapters_loss_grad.restype = C.c_int
        L.orc_adapters_loss_grad.argtypes = [C.c_int, C.c_int, _F, C.c_long, _F, C.c_long, C.c_int, C.c_int, C.c_int,
                                             _D, _D, _D, _D, _D]
        L.orc_adam.restype = None
        L.orc_adam.argtypes = [C.c_long, _D, _D, _D, _D, C.c_int, C.c_double, C.c_double, C.c_double, C.c_double]
        L.orc_num_threads.restype = C.c_int
        L.orc_shadow_map_sphere.restype = None
        L.orc_shadow_map_sphere.argtypes = [C.c_int, C.c_double, _D, _D, _D, C.c_double, _D]
        L.orc_shadow_visibility.restype = None
        L.orc_shadow_visibility.argtypes = [C.c_int, C.c_int, _D, _D, _D, C.c_int, C.c_double, _D, _D, C.c_double,
                                            _D, _D]
        L.orc_composite_shadowed.restype = C.c_int
        L.orc_composite_shadowed.argtypes = [C.c_int, C.c_int, _D, _D, _D, _D, C.c_int, _D, _D]
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(_D) if a is not None else None


def _fp(a):
    return a.ctypes.data_as(_F)


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def camera_array(cam) -> np.ndarray:
    """synth.scene.Camera -> the oracle's 16-double camera record."""
    return np.array([cam.projection, *cam.eye, *cam.target, *cam.up, cam.fov_y_deg, cam.ortho_half_extent,
                     cam.width, cam.height, 0.0, 0.0], dtype=np.float64)


def num_threads() -> int:
    return lib().orc_num_threads()


def splitmix64(state: int) -> int:
    return lib().orc_splitmix64(state)


def jitter(seed: int, frame: int, pixel: int) -> float:
    return lib().orc_jitter(seed, frame, pixel)


def sigma_at(volume, sigma_scale, p) -> float:
    v = _f32(volume)
    nz, ny, nx = v.shape
    return lib().orc_sigma_vol(_fp(v), nx, ny, nz, sigma_scale, _dp(_f64(p)))


def march(volume, sigma_scale, cam, step_voxels, depth_tau=0.1, ert_eps=1e-6, jitter=True, seed=0, frame=0,
          quadrature=0, light_w=(1.0, 1.0, 1.0), unit_radiance=False, stride=1, light_set=0):
    """Guiding map [H][W][3] = (L~, T, D), the depth margin [H][W] and
    (primary, secondary) sample counts.  With stride > 1 only pixels on that
    lattice are computed (others stay 0; margin +inf)."""
    v = _f32(volume)
    nz, ny, nx = v.shape
    g = np.zeros((cam.height, cam.width, 3), dtype=np.float64)
    m = np.full((cam.height, cam.width), np.inf, dtype=np.float64)
    cnt = (C.c_longlong * 2)()
    st = lib().orc_march(_fp(v), nx, ny, nz, sigma_scale, _dp(camera_array(cam)), step_voxels, depth_tau, ert_eps,
                         int(jitter), seed, frame, quadrature, _dp(_f64(light_w)), int(light_set), int(unit_radiance),
                         int(stride), _dp(g),
                         _dp(m), cnt)
    if st:
        raise ValueError(f"orc_march status {st}")
    return g, m, (cnt[0], cnt[1])


def front_identity_gap(volume, sigma_scale, cam, step_voxels, jitter=True, seed=0) -> float:
    v = _f32(volume)
    nz, ny, nx = v.shape
    return lib().orc_front_identity_gap(_fp(v), nx, ny, nz, sigma_scale, _dp(camera_array(cam)), step_voxels,
                                        int(jitter), seed)


def reference_lightmaps(volume, sigma_scale, cam, step_voxels=0.25, ert_eps=1e-6):
    """Six-way reference lightmaps [H][W][6] (+X,-X,+Y,-Y,+Z,-Z), linear."""
    v = _f32(volume)
    nz, ny, nx = v.shape
    out = np.zeros((cam.height, cam.width, 6), dtype=np.float64)
    st = lib().orc_reference_lightmaps(_fp(v), nx, ny, nz, sigma_scale, _dp(camera_array(cam)), step_voxels,
                                       ert_eps, _dp(out))
    if st:
        raise ValueError(f"orc_reference_lightmaps status {st}")
    return out


def srgb_encode(x):
    f = np.vectorize(lib().orc_srgb_encode, otypes=[np.float64])
    return f(np.asarray(x, dtype=np.float64))


def srgb_decode(x):
    f = np.vectorize(lib().orc_srgb_decode, otypes=[np.float64])
    return f(np.asarray(x, dtype=np.float64))


def composite(lightmaps, guide, cam, lights):
    """lights: iterable of (dir xyz, rgb) -> rgba [H][W][4]."""
    lm = _f64(lightmaps)
    H, W = lm.shape[:2]
    la = _f64(np.array([[*d, *c] for d, c in lights]).reshape(-1, 6))
    out = np.zeros((H, W, 4), dtype=np.float64)
    st = lib().orc_composite(H, W, _dp(lm), _dp(_f64(guide)), _dp(camera_array(cam)), _dp(la), la.shape[0],
                             _dp(out))
    if st:
        raise ValueError(f"orc_composite status {st}")
    return out


def shadow_map_sphere(size, half_extent, origin, light, centre, radius):
    """[S][S] occluder depths of a sphere seen from a directional light."""
    out = np.zeros((size, size), dtype=np.float64)
    lib().orc_shadow_map_sphere(size, half_extent, _dp(_f64(origin)), _dp(_f64(light)), _dp(_f64(centre)), radius,
                                _dp(out))
    return out


def shadow_visibility(guide, cam, light, depth, half_extent, origin, bias, with_margin=False):
    """[H][W] visibility in {0, 1} (and, with_margin, the decision margin)."""
    g = _f64(guide)
    H, W = g.shape[:2]
    d = _f64(depth)
    out = np.zeros((H, W), dtype=np.float64)
    mg = np.zeros((H, W), dtype=np.float64)
    lib().orc_shadow_visibility(H, W, _dp(g), _dp(camera_array(cam)), _dp(_f64(light)), d.shape[0], half_extent,
                                _dp(_f64(origin)), _dp(d), bias, _dp(out), _dp(mg))
    return (out, mg) if with_margin else out


def composite_shadowed(lightmaps, guide, cam, lights, vis):
    """orc_composite with light k's term multiplied by vis[k] ([n][H][W])."""
    lm = _f64(lightmaps)
    H, W = lm.shape[:2]
    la = _f64(np.array([[*d, *c] for d, c in lights]).reshape(-1, 6))
    out = np.zeros((H, W, 4), dtype=np.float64)
    st = lib().orc_composite_shadowed(H, W, _dp(lm), _dp(_f64(guide)), _dp(camera_array(cam)), _dp(la), la.shape[0],
                                      _dp(_f64(vis)), _dp(out))
    if st:
        raise ValueError(f"orc_composite_shadowed status {st}")
    return out


def unet_param_count(levels, base) -> int:
    return lib().orc_unet_param_count(levels, base)


def unet_forward(params, levels, base, guide):
    """guide [B][H][W][3] (or [H][W][3]) -> (lightmaps, logits), same leading shape."""
    g = _f64(guide)
    squeeze = g.ndim == 3
    if squeeze:
        g = g[None]
    B, H, W, _ = g.shape
    p = _f32(params)
    lm = np.zeros((B, H, W, 6), dtype=np.float64)
    lo = np.zeros((B, H, W, 6), dtype=np.float64)
    st = lib().orc_unet_forward(levels, base, _fp(p), p.size, B, H, W, _dp(g), _dp(lm), _dp(lo))
    if st:
        raise ValueError(f"orc_unet_forward status {st}")
    return (lm[0], lo[0]) if squeeze else (lm, lo)


def unet_features(params, levels, base, guide):
    """guide [B][H][W][3] (or [H][W][3]) -> decoder features [.., base] (the head's input)."""
    g = _f64(guide)
    squeeze = g.ndim == 3
    if squeeze:
        g = g[None]
    B, H, W, _ = g.shape
    p = _f32(params)
    out = np.zeros((B, H, W, base), dtype=np.float64)
    st = lib().orc_unet_features(levels, base, _fp(p), p.size, B, H, W, _dp(g), _dp(out))
    if st:
        raise ValueError(f"orc_unet_features status {st}")
    return out[0] if squeeze else out


def adapter_param_count(c) -> int:
    return lib().orc_adapter_param_count(c)


def adapters_forward(params, c, feat):
    """Four NAFBlock channel adapters: feat [B][H][W][c] (or [H][W][c]) ->
    (lightmaps [.., 6], extra [.., 2] = alpha, emissive)."""
    f = _f64(feat)
    squeeze = f.ndim == 3
    if squeeze:
        f = f[None]
    B, H, W, _ = f.shape
    p = _f32(params)
    lm = np.zeros((B, H, W, 6), dtype=np.float64)
    ex = np.zeros((B, H, W, 2), dtype=np.float64)
    st = lib().orc_adapters_forward(c, _fp(p), p.size, B, H, W, _dp(f), _dp(lm), _dp(ex))
    if st:
        raise ValueError(f"orc_adapters_forward status {st}")
    return (lm[0], ex[0]) if squeeze else (lm, ex)


def adapters_loss_grad(params, levels, base, ad_params, guide, target):
    """The network with the four adapters in place of its head: (loss,
    gradient of the trunk's parameters (head entries 0), gradient of the
    adapters' parameters)."""
    g = _f64(guide)
    t = _f64(target)
    if g.ndim == 3:
        g, t = g[None], t[None]
    B, H, W, _ = g.shape
    p = _f32(params)
    a = _f32(ad_params)
    grad = np.zeros(p.size, dtype=np.float64)
    grad_ad = np.zeros(a.size, dtype=np.float64)
    loss = np.zeros(1, dtype=np.float64)
    st = lib().orc_adapters_loss_grad(levels, base, _fp(p), p.size, _fp(a), a.size, B, H, W, _dp(g), _dp(t),
                                      _dp(loss), _dp(grad), _dp(grad_ad))
    if st:
        raise ValueError(f"orc_adapters_loss_grad status {st}")
    return float(loss[0]), grad, grad_ad


def unet_loss_grad(params, levels, base, guide, target):
    g = _f64(guide)
    t = _f64(target)
    if g.ndim == 3:
        g, t = g[None], t[None]
    B, H, W, _ = g.shape
    p = _f32(params)
    grad = np.zeros(p.size, dtype=np.float64)
    loss = np.zeros(1, dtype=np.float64)
    st = lib().orc_unet_loss_grad(levels, base, _fp(p), p.size, B, H, W, _dp(g), _dp(t), _dp(loss), _dp(grad))
    if st:
        raise ValueError(f"orc_unet_loss_grad status {st}")
    return float(loss[0]), grad


def adam(params, grad, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step on fp64 copies; returns (params, m, v)."""
    p, m2, v2 = _f64(params).copy(), _f64(m).copy(), _f64(v).copy()
    lib().orc_adam(p.size, _dp(p), _dp(_f64(grad)), _dp(m2), _dp(v2), t, lr, b1, b2, eps)
    return p, m2, v2
