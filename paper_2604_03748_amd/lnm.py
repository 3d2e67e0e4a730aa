"""ctypes binding of liblnm (include/lnm.h).

Argument marshalling only: every step of the path runs in the library's HIP
kernels.  PyTorch supplies device memory and the current stream.  If the
library is missing this module raises; there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import functools
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "liblnm.so")

LNM_OK, LNM_ERR_ARG, LNM_ERR_SHAPE, LNM_ERR_OOM, LNM_ERR_DEVICE, LNM_ERR_UNSUPPORTED = range(6)
FP32, BF16, FP8_E4M3 = 0, 1, 2
ORTHOGRAPHIC, PERSPECTIVE = 0, 1
QUAD_ALPHA, QUAD_RIEMANN = 0, 1
LIGHTS_TOP_BOTTOM, LIGHTS_LEFT_RIGHT = 0, 1
ORDER_AUTO, ORDER_BANDS, ORDER_Z, ORDER_CELLS = 0, 1, 2, 3

EXPORTS = [
    "lnm_abi_struct_size", "lnm_version", "lnm_ctx_create", "lnm_ctx_destroy", "lnm_last_error",
    "lnm_march_workspace_bytes", "lnm_march", "lnm_march_batch_workspace_bytes", "lnm_march_batch",
    "lnm_reference_lightmaps", "lnm_net_param_count",
    "lnm_net_device_bytes", "lnm_net_create", "lnm_net_destroy", "lnm_workspace_bytes", "lnm_infer", "lnm_frame",
    "lnm_composite", "lnm_profile_enable", "lnm_profile_read", "lnm_trainer_state_bytes", "lnm_frame_workspace_bytes",
    "lnm_train_workspace_bytes", "lnm_trainer_create", "lnm_trainer_destroy", "lnm_train_grad", "lnm_train_step",
    "lnm_trainer_read_params", "lnm_trainer_save", "lnm_trainer_load", "lnm_trainer_infer", "lnm_calibrate_amax",
    "lnm_shadow_map_sphere", "lnm_composite_shadowed", "lnm_bricks_bytes", "lnm_make_bricks",
    "lnm_adapters_param_count", "lnm_adapters_device_bytes", "lnm_adapters_create", "lnm_adapters_destroy",
    "lnm_adapters_workspace_bytes", "lnm_infer_adapters", "lnm_frame_static", "lnm_composite_batch",
    "lnm_trainer_adapters_state_bytes", "lnm_trainer_attach_adapters", "lnm_trainer_workspace_bytes",
    "lnm_trainer_read_adapters", "lnm_trainer_adapter_grad",
]
STATIC_SCRATCH_BYTES = 128 << 20  # LNM_STATIC_SCRATCH_BYTES
K_MARCH, K_CONV, K_HEAD, K_COMPOSITE, K_REFERENCE, K_ADAPTERS = range(6)


class LnmError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"liblnm status {status}: {msg}")
        self.status = status


class Volume(C.Structure):
    _fields_ = [("density", C.c_void_p), ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("sigma_scale", C.c_float), ("bricks", C.c_void_p)]


class Camera(C.Structure):
    _fields_ = [("projection", C.c_int32), ("eye", C.c_float * 3), ("target", C.c_float * 3), ("up", C.c_float * 3),
                ("fov_y_deg", C.c_float), ("ortho_half_extent", C.c_float), ("width", C.c_int32),
                ("height", C.c_int32)]


class MarchParams(C.Structure):
    _fields_ = [("step_voxels", C.c_float), ("depth_tau", C.c_float), ("ert_eps", C.c_float),
                ("jitter_on", C.c_int32), ("jitter_seed", C.c_uint64), ("frame", C.c_uint32),
                ("quadrature", C.c_int32), ("light_w", C.c_float * 3), ("light_set", C.c_int32),
                ("work_order", C.c_int32)]


class Light(C.Structure):
    _fields_ = [("dir", C.c_float * 3), ("rgb", C.c_float * 3)]


class ShadowFrame(C.Structure):
    _fields_ = [("origin", C.c_float * 3), ("half_extent", C.c_float), ("size", C.c_int32), ("bias", C.c_float)]


def make_shadow_frame(origin, half_extent, size, bias) -> ShadowFrame:
    return ShadowFrame((C.c_float * 3)(*[float(x) for x in origin]), float(half_extent), int(size), float(bias))


_lib = None


def lib():
    """Load liblnm.so; raises if it has not been built.

    torch is imported first: the library and torch's ROCm build both need
    the HIP runtime libamdhip64.so.7, and the process must end up with
    torch's copy (the one torch's device memory and streams belong to).
    Loading the library first would bind the runtime from the library's own
    search path, and torch would then find no GPU."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        import torch  # noqa: F401  (binds torch's HIP runtime before the library's)

        L = C.CDLL(LIB_PATH)
        vp, i32, sz = C.c_void_p, C.c_int32, C.c_size_t
        L.lnm_abi_struct_size.restype = sz
        L.lnm_abi_struct_size.argtypes = [i32]
        L.lnm_version.restype = C.c_char_p
        L.lnm_last_error.restype = C.c_char_p
        L.lnm_ctx_create.restype = i32
        L.lnm_ctx_create.argtypes = [i32, C.POINTER(vp)]
        L.lnm_ctx_destroy.argtypes = [vp]
        L.lnm_march_workspace_bytes.restype = sz
        L.lnm_march_workspace_bytes.argtypes = [C.POINTER(Volume), C.POINTER(Camera), C.POINTER(MarchParams)]
        L.lnm_frame_workspace_bytes.restype = sz
        L.lnm_frame_workspace_bytes.argtypes = [vp, C.POINTER(Volume), C.POINTER(Camera), C.POINTER(MarchParams)]
        L.lnm_march.restype = i32
        L.lnm_march.argtypes = [vp, C.POINTER(Volume), C.POINTER(Camera), C.POINTER(MarchParams), vp, vp, sz, vp]
        L.lnm_march_batch_workspace_bytes.restype = sz
        L.lnm_march_batch_workspace_bytes.argtypes = [i32, C.POINTER(Volume), C.POINTER(Camera),
                                                      C.POINTER(MarchParams)]
        L.lnm_march_batch.restype = i32
        L.lnm_march_batch.argtypes = [vp, i32, C.POINTER(Volume), C.POINTER(Camera), C.POINTER(MarchParams),
                                      C.POINTER(vp), vp, sz, vp]
        L.lnm_reference_lightmaps.restype = i32
        L.lnm_reference_lightmaps.argtypes = [vp, C.POINTER(Volume), C.POINTER(Camera), C.c_float, C.c_float, i32,
                                              vp, vp]
        L.lnm_net_param_count.restype = sz
        L.lnm_net_param_count.argtypes = [i32, i32]
        L.lnm_net_device_bytes.restype = sz
        L.lnm_net_device_bytes.argtypes = [i32, i32, i32]
        L.lnm_net_create.restype = i32
        L.lnm_net_create.argtypes = [vp, i32, i32, i32, vp, sz, vp, vp, sz, vp, C.POINTER(vp)]
        L.lnm_net_destroy.argtypes = [vp]
        L.lnm_workspace_bytes.restype = sz
        L.lnm_workspace_bytes.argtypes = [vp, i32, i32, i32]
        L.lnm_infer.restype = i32
        L.lnm_infer.argtypes = [vp, vp, i32, i32, i32, vp, vp, vp, vp, sz, vp]
        L.lnm_frame.restype = i32
        L.lnm_frame.argtypes = [vp, vp, C.POINTER(Volume), C.POINTER(Camera), C.POINTER(MarchParams),
                                C.POINTER(Light), i32, vp, vp, vp, vp, sz, vp]
        L.lnm_frame_static.restype = i32
        L.lnm_frame_static.argtypes = [vp, vp, C.POINTER(Volume), C.POINTER(Camera), C.POINTER(MarchParams),
                                       C.POINTER(Light), i32, vp, vp, vp, vp]
        L.lnm_composite_batch.restype = i32
        L.lnm_composite_batch.argtypes = [vp, i32, C.POINTER(Camera), C.POINTER(Light), C.POINTER(i32), i32, i32, vp,
                                          vp, vp, vp]
        L.lnm_composite.restype = i32
        L.lnm_composite.argtypes = [vp, C.POINTER(Camera), C.POINTER(Light), i32, i32, i32, i32, vp, vp, vp, vp]
        L.lnm_shadow_map_sphere.restype = i32
        L.lnm_shadow_map_sphere.argtypes = [vp, C.POINTER(ShadowFrame), C.POINTER(C.c_float), C.POINTER(C.c_float),
                                            C.c_float, vp, vp]
        L.lnm_composite_shadowed.restype = i32
        L.lnm_composite_shadowed.argtypes = [vp, C.POINTER(Camera), C.POINTER(Light), i32, C.POINTER(ShadowFrame),
                                             C.POINTER(vp), i32, i32, i32, vp, vp, vp, vp, vp]
        L.lnm_adapters_param_count.restype = sz
        L.lnm_adapters_param_count.argtypes = [i32]
        L.lnm_adapters_device_bytes.restype = sz
        L.lnm_adapters_device_bytes.argtypes = [i32]
        L.lnm_adapters_create.restype = i32
        L.lnm_adapters_create.argtypes = [vp, vp, vp, sz, vp, sz, vp, C.POINTER(vp)]
        L.lnm_adapters_destroy.argtypes = [vp]
        L.lnm_adapters_workspace_bytes.restype = sz
        L.lnm_adapters_workspace_bytes.argtypes = [vp, i32, i32, i32]
        L.lnm_infer_adapters.restype = i32
        L.lnm_infer_adapters.argtypes = [vp, vp, i32, i32, i32, vp, vp, vp, vp, sz, vp]
        L.lnm_bricks_bytes.restype = sz
        L.lnm_bricks_bytes.argtypes = [i32, i32, i32]
        L.lnm_make_bricks.restype = i32
        L.lnm_make_bricks.argtypes = [vp, C.POINTER(Volume), vp, sz, vp]
        L.lnm_calibrate_amax.restype = i32
        L.lnm_calibrate_amax.argtypes = [vp, vp, i32, i32, i32, vp, vp, i32, vp, sz, vp]
        L.lnm_profile_enable.restype = i32
        L.lnm_profile_enable.argtypes = [vp, i32]
        L.lnm_profile_read.restype = i32
        L.lnm_profile_read.argtypes = [vp, i32, C.POINTER(i32), C.POINTER(C.c_double)]
        _lib = L
    return _lib


def check(status: int):
    if status != LNM_OK:
        raise LnmError(status, lib().lnm_last_error().decode())


# ------------------------------------------------------------------ marshalling
def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _on_stream(fn):
    """Run a binding method with `stream` (when given) as torch's current
    stream, so every tensor the method allocates for the call (outputs,
    workspaces) belongs to the stream its kernels run on and the caching
    allocator never hands that memory to other work while they use it."""
    @functools.wraps(fn)
    def wrapper(*args, **kw):
        stream = kw.get("stream")
        if stream is None:
            return fn(*args, **kw)
        import torch

        with torch.cuda.stream(stream):
            return fn(*args, **kw)

    return wrapper


def _stream(stream=None):
    import torch

    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _need(t, shape, name):
    import torch

    if not isinstance(t, torch.Tensor) or t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous float32 CUDA tensor")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")


def make_camera(cam) -> Camera:
    """From any object with the fields of lnm_camera (e.g. synth.scene.Camera)."""
    c = Camera()
    c.projection = int(cam.projection)
    c.eye[:] = [float(v) for v in cam.eye]
    c.target[:] = [float(v) for v in cam.target]
    c.up[:] = [float(v) for v in cam.up]
    c.fov_y_deg = float(cam.fov_y_deg)
    c.ortho_half_extent = float(cam.ortho_half_extent)
    c.width = int(cam.width)
    c.height = int(cam.height)
    return c


def make_params(step_voxels, depth_tau=0.1, ert_eps=1e-6, jitter=True, seed=0, frame=0, quadrature=QUAD_ALPHA,
                light_w=(1.0, 1.0, 1.0), light_set=0, work_order=0) -> MarchParams:
    p = MarchParams()
    p.step_voxels = step_voxels
    p.depth_tau = depth_tau
    p.ert_eps = ert_eps
    p.jitter_on = int(bool(jitter))
    p.jitter_seed = int(seed) & (2**64 - 1)
    p.frame = int(frame)
    p.quadrature = int(quadrature)
    p.light_w[:] = [float(v) for v in light_w]
    p.light_set = int(light_set)
    p.work_order = int(work_order)
    return p


def make_volume(density, sigma_scale, bricks=None) -> Volume:
    """bricks: optional device tensor from Context.make_bricks(density)."""
    import torch

    if not isinstance(density, torch.Tensor) or density.dtype != torch.float32 or not density.is_cuda \
            or density.dim() != 3 or not density.is_contiguous():
        raise TypeError("density must be a contiguous 3-D float32 CUDA tensor [nz][ny][nx]")
    v = Volume()
    v.density = density.data_ptr()
    v.nz, v.ny, v.nx = (int(s) for s in density.shape)
    v.sigma_scale = float(sigma_scale)
    if bricks is not None:
        need = int(lib().lnm_bricks_bytes(v.nx, v.ny, v.nz))
        if not isinstance(bricks, torch.Tensor) or not bricks.is_cuda or not bricks.is_contiguous() \
                or bricks.numel() * bricks.element_size() < need:
            raise ValueError(f"bricks must be a contiguous CUDA tensor of at least {need} bytes")
        v.bricks = bricks.data_ptr()
    return v


def make_lights(lights):
    lights = list(lights or [])
    arr = (Light * max(1, len(lights)))()
    for k, (d, rgb) in enumerate(lights):
        arr[k].dir[:] = [float(v) for v in d]
        arr[k].rgb[:] = [float(v) for v in rgb]
    return arr, len(lights)


# ------------------------------------------------------------------ objects
class Context:
    def __init__(self, device: int = 0):
        h = C.c_void_p()
        check(lib().lnm_ctx_create(device, C.byref(h)))
        self.handle = h
        self.device = device

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.lnm_ctx_destroy(self.handle)
            self.handle = None

    # -- per-launch timing
    def profile(self, on: bool):
        check(lib().lnm_profile_enable(self.handle, int(bool(on))))

    def profile_read(self, kind: int):
        """(launches, total milliseconds) recorded for one kernel kind."""
        n, ms = C.c_int32(), C.c_double()
        check(lib().lnm_profile_read(self.handle, kind, C.byref(n), C.byref(ms)))
        return n.value, ms.value

    # -- march
    @_on_stream
    def make_bricks(self, density, out=None, stream=None):
        """Bricked copy of a density grid for repeated marches (lnm_make_bricks)."""
        import torch

        vol = make_volume(density, 1.0)
        n = int(lib().lnm_bricks_bytes(vol.nx, vol.ny, vol.nz))
        if out is None:
            out = torch.empty(n // 4, dtype=torch.float32, device=density.device)
        check(lib().lnm_make_bricks(self.handle, C.byref(vol), _ptr(out), out.numel() * out.element_size(),
                                    _stream(stream)))
        return out

    def march_workspace_bytes(self, density, sigma_scale, cam, params: MarchParams, bricks=None) -> int:
        vol = make_volume(density, sigma_scale, bricks)
        c = make_camera(cam)
        return int(lib().lnm_march_workspace_bytes(C.byref(vol), C.byref(c), C.byref(params)))

    @_on_stream
    def march(self, density, sigma_scale, cam, params: MarchParams, out=None, workspace=None, stream=None,
              bricks=None):
        import torch

        vol = make_volume(density, sigma_scale, bricks)
        c = make_camera(cam)
        if out is None:
            out = torch.empty((c.height, c.width, 3), dtype=torch.float32, device=density.device)
        _need(out, (c.height, c.width, 3), "guide")
        if workspace is None:
            n = int(lib().lnm_march_workspace_bytes(C.byref(vol), C.byref(c), C.byref(params)))
            workspace = torch.empty(max(n, 1), dtype=torch.uint8, device=density.device)
        check(lib().lnm_march(self.handle, C.byref(vol), C.byref(c), C.byref(params), _ptr(out), _ptr(workspace),
                              workspace.numel(), _stream(stream)))
        return out

    @_on_stream
    def march_batch(self, densities, sigma_scales, cams, params, outs=None, workspace=None, stream=None,
                    bricks=None):
        """n guiding maps in one call (lnm_march_batch): lists of grids,
        extinction scales, cameras, march parameters (and optional bricks),
        each march with its own sizes; returns the list of guides."""
        import torch

        n = len(densities)
        if not (len(sigma_scales) == len(cams) == len(params) == n) or n == 0:
            raise ValueError("densities, sigma_scales, cams and params must be non-empty lists of one length")
        bricks = bricks if bricks is not None else [None] * n
        vols = (Volume * n)(*[make_volume(d, ss, b) for d, ss, b in zip(densities, sigma_scales, bricks)])
        camv = (Camera * n)(*[make_camera(c) for c in cams])
        prmv = (MarchParams * n)(*params)
        if outs is None:
            outs = [torch.empty((c.height, c.width, 3), dtype=torch.float32, device=d.device)
                    for c, d in zip(camv, densities)]
        for o, c in zip(outs, camv):
            _need(o, (c.height, c.width, 3), "guide")
        if workspace is None:
            nb = int(lib().lnm_march_batch_workspace_bytes(n, vols, camv, prmv))
            workspace = torch.empty(max(nb, 1), dtype=torch.uint8, device=densities[0].device)
        ptrs = (C.c_void_p * n)(*[o.data_ptr() for o in outs])
        check(lib().lnm_march_batch(self.handle, n, vols, camv, prmv, ptrs, _ptr(workspace), workspace.numel(),
                                    _stream(stream)))
        return outs

    @_on_stream
    def reference_lightmaps(self, density, sigma_scale, cam, step_voxels=0.25, ert_eps=1e-6, srgb=False, out=None,
                            stream=None):
        import torch

        vol = make_volume(density, sigma_scale)
        c = make_camera(cam)
        if out is None:
            out = torch.empty((c.height, c.width, 6), dtype=torch.float32, device=density.device)
        _need(out, (c.height, c.width, 6), "lightmaps")
        check(lib().lnm_reference_lightmaps(self.handle, C.byref(vol), C.byref(c), step_voxels, ert_eps, int(srgb),
                                            _ptr(out), _stream(stream)))
        return out

    @_on_stream
    def composite(self, cam, lights, lightmaps, guide, out=None, stream=None):
        import torch

        c = make_camera(cam)
        B = lightmaps.shape[0] if lightmaps.dim() == 4 else 1
        H, W = c.height, c.width
        if out is None:
            out = torch.empty(tuple(lightmaps.shape[:-1]) + (4,), dtype=torch.float32, device=lightmaps.device)
        arr, n = make_lights(lights)
        check(lib().lnm_composite(self.handle, C.byref(c), arr, n, B, H, W, _ptr(lightmaps), _ptr(guide), _ptr(out),
                                  _stream(stream)))
        return out

    @_on_stream
    def composite_batch(self, cams, lights, lightmaps, guides, out=None, stream=None):
        """lnm_composite_batch: image b of lightmaps [B][H][W][6] / guides
        [B][H][W][3] shaded with cams[b] and its own list lights[b]."""
        import torch

        B, H, W = lightmaps.shape[0], lightmaps.shape[1], lightmaps.shape[2]
        _need(lightmaps, (B, H, W, 6), "lightmaps")
        _need(guides, (B, H, W, 3), "guides")
        if out is None:
            out = torch.empty((B, H, W, 4), dtype=torch.float32, device=lightmaps.device)
        _need(out, (B, H, W, 4), "out")
        if len(cams) != B or len(lights) != B:
            raise ValueError("one camera and one light list per image")
        ca = (Camera * B)(*[make_camera(c) for c in cams])
        flat = [l for ls in lights for l in ls]
        arr, _ = make_lights(flat)
        start = (C.c_int32 * (B + 1))()
        for b in range(B):
            start[b + 1] = start[b] + len(lights[b])
        check(lib().lnm_composite_batch(self.handle, B, ca, arr, start, H, W, _ptr(lightmaps), _ptr(guides), _ptr(out),
                                        _stream(stream)))
        return out

    @_on_stream
    def shadow_map_sphere(self, frame: ShadowFrame, light_dir, centre, radius, out=None, stream=None):
        """[size][size] obstacle depths of a sphere seen from a directional light."""
        import torch

        S = frame.size
        if out is None:
            out = torch.empty((S, S), dtype=torch.float32, device="cuda")
        _need(out, (S, S), "depth")
        f3 = C.c_float * 3
        check(lib().lnm_shadow_map_sphere(self.handle, C.byref(frame), f3(*map(float, light_dir)),
                                          f3(*map(float, centre)), float(radius), _ptr(out), _stream(stream)))
        return out

    @_on_stream
    def composite_shadowed(self, cam, lights, frame: ShadowFrame, depth_maps, lightmaps, guide, out=None, vis=None,
                           stream=None):
        """Six-way shading with light k's term masked by the visibility of each
        pixel's smoke surface in depth_maps[k] (a tensor, or None = unshadowed)."""
        import torch

        c = make_camera(cam)
        B = lightmaps.shape[0] if lightmaps.dim() == 4 else 1
        H, W = c.height, c.width
        if out is None:
            out = torch.empty(tuple(lightmaps.shape[:-1]) + (4,), dtype=torch.float32, device=lightmaps.device)
        arr, n = make_lights(lights)
        if len(depth_maps) != n:
            raise ValueError("one depth map (or None) per light")
        for d in depth_maps:
            if d is not None:
                _need(d, (frame.size, frame.size), "depth map")
        ptrs = (C.c_void_p * max(n, 1))(*[None if d is None else d.data_ptr() for d in depth_maps])
        check(lib().lnm_composite_shadowed(self.handle, C.byref(c), arr, n, C.byref(frame), ptrs, B, H, W,
                                           _ptr(lightmaps), _ptr(guide), _ptr(out), _ptr(vis), _stream(stream)))
        return out


def param_count(levels: int, base: int) -> int:
    return int(lib().lnm_net_param_count(levels, base))


class Net:
    """Packed U-Net weights in a torch-owned device buffer."""

    def __init__(self, ctx: Context, levels: int, base: int, params, precision: int = FP32, act_scales=None,
                 device=None, stream=None):
        import torch

        self.ctx, self.levels, self.base, self.precision = ctx, levels, base, precision
        p = np.ascontiguousarray(params, dtype=np.float32)
        nbytes = int(lib().lnm_net_device_bytes(levels, base, precision))
        if nbytes == 0:
            raise LnmError(LNM_ERR_UNSUPPORTED, f"no packed layout for levels={levels} base={base} "
                                                f"precision={precision}")
        dev = device if device is not None else torch.device("cuda", ctx.device)
        self.buf = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        sc = None if act_scales is None else np.ascontiguousarray(act_scales, dtype=np.float32)
        h = C.c_void_p()
        check(lib().lnm_net_create(ctx.handle, levels, base, precision, p.ctypes.data_as(C.c_void_p), p.size,
                                   None if sc is None else sc.ctypes.data_as(C.c_void_p), _ptr(self.buf), nbytes,
                                   _stream(stream), C.byref(h)))
        self.handle = h

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.lnm_net_destroy(self.handle)
            self.handle = None

    def workspace_bytes(self, batch, H, W) -> int:
        return int(lib().lnm_workspace_bytes(self.handle, batch, H, W))

    @_on_stream
    def calibrate_amax(self, guide, stream=None) -> np.ndarray:
        """Per-convolution maximum |output| of this (fp32) net on guide [B][H][W][3]."""
        g = guide if guide.dim() == 4 else guide.unsqueeze(0)
        B, H, W, _ = g.shape
        _need(g, (B, H, W, 3), "guide")
        n = 4 * self.levels - 2
        out = np.zeros(n, dtype=np.float32)
        ws = self.workspace(B, H, W)
        check(lib().lnm_calibrate_amax(self.ctx.handle, self.handle, B, H, W, _ptr(g), out.ctypes.data_as(C.c_void_p),
                                       n, _ptr(ws), ws.numel(), _stream(stream)))
        return out

    def workspace(self, batch, H, W):
        import torch

        return torch.empty(max(1, self.workspace_bytes(batch, H, W)), dtype=torch.uint8, device=self.buf.device)

    @_on_stream
    def infer(self, guide, out=None, logits=None, workspace=None, stream=None):
        import torch

        g = guide if guide.dim() == 4 else guide.unsqueeze(0)
        B, H, W, _ = g.shape
        _need(g, (B, H, W, 3), "guide")
        if out is None:
            out = torch.empty((B, H, W, 6), dtype=torch.float32, device=g.device)
        if workspace is None:
            workspace = self.workspace(B, H, W)
        check(lib().lnm_infer(self.ctx.handle, self.handle, B, H, W, _ptr(g), _ptr(out), _ptr(logits),
                              _ptr(workspace), workspace.numel(), _stream(stream)))
        return out if guide.dim() == 4 else out[0]

    def frame_workspace(self, density, sigma_scale, cam, params: MarchParams, bricks=None):
        import torch

        vol = make_volume(density, sigma_scale, bricks)
        c = make_camera(cam)
        n = int(lib().lnm_frame_workspace_bytes(self.handle, C.byref(vol), C.byref(c), C.byref(params)))
        if n == 0:
            raise LnmError(LNM_ERR_SHAPE, "no frame workspace for these arguments")
        return torch.empty(n, dtype=torch.uint8, device=density.device)

    @_on_stream
    def frame(self, density, sigma_scale, cam, params: MarchParams, lights=(), guide=None, lightmaps=None, rgba=None,
              workspace=None, stream=None, shade=True, bricks=None):
        import torch

        vol = make_volume(density, sigma_scale, bricks)
        c = make_camera(cam)
        H, W = c.height, c.width
        dev = density.device
        guide = guide if guide is not None else torch.empty((H, W, 3), dtype=torch.float32, device=dev)
        lightmaps = lightmaps if lightmaps is not None else torch.empty((H, W, 6), dtype=torch.float32, device=dev)
        if shade and rgba is None:
            rgba = torch.empty((H, W, 4), dtype=torch.float32, device=dev)
        if workspace is None:
            workspace = self.frame_workspace(density, sigma_scale, cam, params, bricks)
        arr, n = make_lights(lights)
        check(lib().lnm_frame(self.ctx.handle, self.handle, C.byref(vol), C.byref(c), C.byref(params), arr, n,
                              _ptr(guide), _ptr(lightmaps), _ptr(rgba) if shade else None, _ptr(workspace),
                              workspace.numel(), _stream(stream)))
        return guide, lightmaps, rgba

    def frame_static(self, density, sigma_scale, cam, params: MarchParams, guide, lightmaps, lights=(), rgba=None,
                     stream=None, bricks=None):
        """lnm_frame_static: the frame in the library's static workspace.
        The caller provides the output tensors (nothing is allocated here)."""
        vol = make_volume(density, sigma_scale, bricks)
        c = make_camera(cam)
        _need(guide, (c.height, c.width, 3), "guide")
        _need(lightmaps, (c.height, c.width, 6), "lightmaps")
        if rgba is not None:
            _need(rgba, (c.height, c.width, 4), "rgba")
        arr, n = make_lights(lights)
        check(lib().lnm_frame_static(self.ctx.handle, self.handle, C.byref(vol), C.byref(c), C.byref(params), arr, n,
                                     _ptr(guide), _ptr(lightmaps), _ptr(rgba), _stream(stream)))
        return guide, lightmaps, rgba


# ------------------------------------------------------------------ training
def _train_sigs(L):
    vp, i32, sz, f = C.c_void_p, C.c_int32, C.c_size_t, C.c_float
    L.lnm_trainer_state_bytes.restype = sz
    L.lnm_trainer_state_bytes.argtypes = [i32, i32]
    L.lnm_train_workspace_bytes.restype = sz
    L.lnm_train_workspace_bytes.argtypes = [i32, i32, i32, i32, i32]
    L.lnm_trainer_create.restype = i32
    L.lnm_trainer_create.argtypes = [vp, i32, i32, vp, sz, vp, sz, vp, C.POINTER(vp)]
    L.lnm_trainer_destroy.argtypes = [vp]
    L.lnm_train_grad.restype = i32
    L.lnm_train_grad.argtypes = [vp, vp, i32, i32, i32, vp, vp, vp, vp, vp, sz, vp]
    L.lnm_train_step.restype = i32
    L.lnm_train_step.argtypes = [vp, vp, i32, i32, i32, vp, vp, f, f, f, f, vp, vp, sz, vp]
    L.lnm_trainer_read_params.restype = i32
    L.lnm_trainer_read_params.argtypes = [vp, vp, sz, vp]
    L.lnm_trainer_save.restype = i32
    L.lnm_trainer_save.argtypes = [vp, vp, vp, C.POINTER(i32), sz, vp]
    L.lnm_trainer_load.restype = i32
    L.lnm_trainer_load.argtypes = [vp, vp, vp, vp, i32, sz, vp]
    L.lnm_trainer_infer.restype = i32
    L.lnm_trainer_infer.argtypes = [vp, vp, i32, i32, i32, vp, vp, vp, sz, vp]
    L.lnm_trainer_adapters_state_bytes.restype = sz
    L.lnm_trainer_adapters_state_bytes.argtypes = [i32]
    L.lnm_trainer_attach_adapters.restype = i32
    L.lnm_trainer_attach_adapters.argtypes = [vp, vp, sz, vp, sz, vp]
    L.lnm_trainer_workspace_bytes.restype = sz
    L.lnm_trainer_workspace_bytes.argtypes = [vp, i32, i32, i32]
    L.lnm_trainer_read_adapters.restype = i32
    L.lnm_trainer_read_adapters.argtypes = [vp, vp, sz, vp]
    L.lnm_trainer_adapter_grad.restype = i32
    L.lnm_trainer_adapter_grad.argtypes = [vp, vp, sz, vp]


class Trainer:
    """fp32 U-Net trained on the GPU by the library's forward/backward kernels."""

    def __init__(self, ctx: Context, levels: int, base: int, params, stream=None):
        import torch

        L = lib()
        if not hasattr(L, "_train_sigs_done"):
            _train_sigs(L)
            L._train_sigs_done = True
        self.ctx, self.levels, self.base = ctx, levels, base
        p = np.ascontiguousarray(params, dtype=np.float32)
        self.n_params = p.size
        nbytes = int(L.lnm_trainer_state_bytes(levels, base))
        if nbytes == 0:
            raise LnmError(LNM_ERR_SHAPE, f"no trainer for levels={levels} base={base}")
        self.state = torch.empty(nbytes, dtype=torch.uint8, device=torch.device("cuda", ctx.device))
        h = C.c_void_p()
        check(L.lnm_trainer_create(ctx.handle, levels, base, p.ctypes.data_as(C.c_void_p), p.size, _ptr(self.state),
                                   nbytes, _stream(stream), C.byref(h)))
        self.handle = h
        self._ws = {}
        self.n_adapter_params = 0

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.lnm_trainer_destroy(self.handle)
            self.handle = None

    def attach_adapters(self, adapter_params, stream=None):
        """Train the four channel adapters with the network in place of its
        plain head (before the first step)."""
        import torch

        a = np.ascontiguousarray(adapter_params, dtype=np.float32)
        nbytes = int(lib().lnm_trainer_adapters_state_bytes(self.base))
        if nbytes == 0:
            raise LnmError(LNM_ERR_UNSUPPORTED, f"no adapters for base {self.base}")
        self.ad_state = torch.empty(nbytes, dtype=torch.uint8, device=self.state.device)
        check(lib().lnm_trainer_attach_adapters(self.handle, a.ctypes.data_as(C.c_void_p), a.size,
                                                _ptr(self.ad_state), nbytes, _stream(stream)))
        self.n_adapter_params = a.size
        self._ws = {}

    def adapter_params(self, stream=None) -> np.ndarray:
        out = np.empty(self.n_adapter_params, dtype=np.float32)
        check(lib().lnm_trainer_read_adapters(self.handle, out.ctypes.data_as(C.c_void_p), out.size,
                                              _stream(stream)))
        return out

    @_on_stream
    def adapter_grad(self, stream=None):
        """The adapters' gradient of the last grad / step call (device tensor)."""
        import torch

        g = torch.empty(self.n_adapter_params, dtype=torch.float32, device=self.state.device)
        check(lib().lnm_trainer_adapter_grad(self.handle, _ptr(g), g.numel(), _stream(stream)))
        return g

    def workspace(self, B, H, W):
        import torch

        key = (B, H, W)
        if key not in self._ws:
            n = int(lib().lnm_trainer_workspace_bytes(self.handle, B, H, W))
            self._ws[key] = torch.empty(max(n, 1), dtype=torch.uint8, device=self.state.device)
        return self._ws[key]

    @_on_stream
    def grad(self, guide, target, stream=None):
        """(loss tensor [1], gradient tensor [n_params]) for one batch."""
        import torch

        B, H, W, _ = guide.shape
        _need(guide, (B, H, W, 3), "guide")
        _need(target, (B, H, W, 6), "target")
        loss = torch.empty(1, dtype=torch.float32, device=guide.device)
        g = torch.empty(self.n_params, dtype=torch.float32, device=guide.device)
        ws = self.workspace(B, H, W)
        check(lib().lnm_train_grad(self.ctx.handle, self.handle, B, H, W, _ptr(guide), _ptr(target), _ptr(loss),
                                   _ptr(g), _ptr(ws), ws.numel(), _stream(stream)))
        return loss, g

    @_on_stream
    def step(self, guide, target, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, loss=None, stream=None):
        import torch

        B, H, W, _ = guide.shape
        _need(guide, (B, H, W, 3), "guide")
        _need(target, (B, H, W, 6), "target")
        if loss is None:
            loss = torch.empty(1, dtype=torch.float32, device=guide.device)
        ws = self.workspace(B, H, W)
        check(lib().lnm_train_step(self.ctx.handle, self.handle, B, H, W, _ptr(guide), _ptr(target), lr, beta1,
                                   beta2, eps, _ptr(loss), _ptr(ws), ws.numel(), _stream(stream)))
        return loss

    def params(self, stream=None) -> np.ndarray:
        out = np.empty(self.n_params, dtype=np.float32)
        check(lib().lnm_trainer_read_params(self.handle, out.ctypes.data_as(C.c_void_p), out.size, _stream(stream)))
        return out

    def save(self, stream=None) -> dict:
        m = np.empty(self.n_params, dtype=np.float32)
        v = np.empty(self.n_params, dtype=np.float32)
        st = C.c_int32()
        check(lib().lnm_trainer_save(self.handle, m.ctypes.data_as(C.c_void_p), v.ctypes.data_as(C.c_void_p),
                                     C.byref(st), self.n_params, _stream(stream)))
        return {"params": self.params(stream), "m": m, "v": v, "step": st.value, "levels": self.levels,
                "base": self.base}

    def load(self, ck: dict, stream=None):
        p = np.ascontiguousarray(ck["params"], dtype=np.float32)
        m = np.ascontiguousarray(ck["m"], dtype=np.float32)
        v = np.ascontiguousarray(ck["v"], dtype=np.float32)
        check(lib().lnm_trainer_load(self.handle, p.ctypes.data_as(C.c_void_p), m.ctypes.data_as(C.c_void_p),
                                     v.ctypes.data_as(C.c_void_p), int(ck["step"]), self.n_params, _stream(stream)))

    @_on_stream
    def infer(self, guide, out=None, stream=None):
        import torch

        B, H, W, _ = guide.shape
        if out is None:
            out = torch.empty((B, H, W, 6), dtype=torch.float32, device=guide.device)
        ws = self.workspace(B, H, W)
        check(lib().lnm_trainer_infer(self.ctx.handle, self.handle, B, H, W, _ptr(guide), _ptr(out), _ptr(ws),
                                      ws.numel(), _stream(stream)))
        return out


def save_checkpoint(path, ck: dict):
    np.savez(path, **{k: np.asarray(v) for k, v in ck.items()})


def load_checkpoint(path) -> dict:
    with np.load(path, allow_pickle=False) as z:
        return {k: z[k] if z[k].ndim else z[k].item() for k in z.files}


class Adapters:
    """Four NAFBlock channel adapters bound to a Net (lnm_adapters_*)."""

    def __init__(self, net: Net, params, stream=None):
        import torch

        self.net, self.ctx = net, net.ctx
        p = np.ascontiguousarray(params, dtype=np.float32)
        nbytes = int(lib().lnm_adapters_device_bytes(net.base))
        if nbytes == 0:
            raise LnmError(LNM_ERR_UNSUPPORTED, f"no adapters for base width {net.base}")
        self.buf = torch.empty(nbytes, dtype=torch.uint8, device=net.buf.device)
        h = C.c_void_p()
        check(lib().lnm_adapters_create(self.ctx.handle, net.handle, p.ctypes.data_as(C.c_void_p), p.size,
                                        _ptr(self.buf), nbytes, _stream(stream), C.byref(h)))
        self.handle = h

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.lnm_adapters_destroy(self.handle)
            self.handle = None

    def workspace(self, batch, H, W):
        import torch

        n = int(lib().lnm_adapters_workspace_bytes(self.handle, batch, H, W))
        if n == 0:
            raise LnmError(LNM_ERR_SHAPE, "no adapter workspace for these sizes")
        return torch.empty(n, dtype=torch.uint8, device=self.buf.device)

    @_on_stream
    def infer(self, guide, out=None, extra=None, with_extra=True, workspace=None, stream=None):
        """guide [B][H][W][3] -> (lightmaps [B][H][W][6], extra [B][H][W][2] or None)."""
        import torch

        g = guide if guide.dim() == 4 else guide.unsqueeze(0)
        B, H, W, _ = g.shape
        _need(g, (B, H, W, 3), "guide")
        if out is None:
            out = torch.empty((B, H, W, 6), dtype=torch.float32, device=g.device)
        if with_extra and extra is None:
            extra = torch.empty((B, H, W, 2), dtype=torch.float32, device=g.device)
        if workspace is None:
            workspace = self.workspace(B, H, W)
        check(lib().lnm_infer_adapters(self.ctx.handle, self.handle, B, H, W, _ptr(g), _ptr(out),
                                       _ptr(extra) if with_extra else None, _ptr(workspace), workspace.numel(),
                                       _stream(stream)))
        if guide.dim() == 4:
            return out, extra
        return out[0], (extra[0] if extra is not None else None)
