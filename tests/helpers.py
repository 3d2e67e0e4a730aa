"""Shared helpers for the GPU parity tests: device setup, tolerance checks."""
from __future__ import annotations

import sys

import numpy as np

# Tolerances of the fp32 march against the fp64 oracle.  Relative 1e-5 on
# L~ and T; absolute floors from early termination: a ray cut where its
# transmittance fell below eps leaves out at most 3 eps of L~ (three unit
# lights) and eps of T.
MARCH_REL = 1e-5
ERT_EPS = 1e-6
FLOOR_L = 3 * ERT_EPS
FLOOR_T = ERT_EPS
# D is a threshold crossing: pixels whose deciding sample is within this
# fraction of tau_D of the threshold may legitimately differ by a step.  An
# fp32 sample position is off by about |eye| 2^-24 (1.5e-7 world units at
# distance 2.5); times the steepest density gradient of the synthetic fields
# (sigma_scale 8 x peak 2 over radius 0.05, plus the noise octaves) that moves
# sigma by up to about 3e-5 = 3e-4 tau_D, so the margin is 1e-3 tau_D.  At
# most 0.5% of a map's pixels may be flagged (measured 0 to 0.3%).
D_MARGIN = 1e-3

# fp32 network against fp64: max |d lightmap| and |d logit| / max(1, |logit|).
NET_ABS = 1e-4


def log(msg: str):
    sys.stdout.write(msg + "\n")
    sys.stdout.flush()


def device():
    import torch

    assert torch.cuda.is_available(), "GPU test run without a GPU"
    return torch.device("cuda", 0)


def to_dev(a, dtype=None):
    import torch

    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32), device=device())


def to_host(t) -> np.ndarray:
    import torch

    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def fp32_ray_allowance(orc, vol, ss, cam, step, eps=1e-5, **kw):
    """Per-pixel error allowance for representing each ray in fp32.

    An fp32 ray is exact only to about one unit in the last place of its
    coordinates, delta = 2^-23 (|eye|_inf + 2).  The oracle measures how much
    L~ and T move when the whole camera is shifted by eps along each world
    axis; the allowance is 2 * (that sensitivity) * delta.  It is negligible
    for most pixels and large only for rays that graze the face of the grid's
    support box, where sigma ramps from zero over half a voxel."""
    from dataclasses import replace

    g0, _, _ = orc.march(vol, ss, cam, step, **kw)
    sens = np.zeros(g0.shape[:2] + (2,))
    for a in range(3):
        for sgn in (-1.0, 1.0):
            e = list(cam.eye)
            t = list(cam.target)
            e[a] += sgn * eps
            t[a] += sgn * eps
            gp, _, _ = orc.march(vol, ss, replace(cam, eye=tuple(e), target=tuple(t)), step, **kw)
            sens = np.maximum(sens, np.abs(gp[..., :2] - g0[..., :2]) / eps)
    delta = 2.0**-23 * (max(abs(float(x)) for x in cam.eye) + 2.0)
    return 2.0 * sens * delta


def check_march(g_gpu, g_ref, margin, depth_tau, step_world, what="", allow=None):
    """Assert parity of a guiding map; returns the error summary.

    allow: optional [H][W][2] fp32 ray-representation allowance for (L~, T)."""
    dL = np.abs(g_gpu[..., 0] - g_ref[..., 0])
    dT = np.abs(g_gpu[..., 1] - g_ref[..., 1])
    tolL = MARCH_REL * np.abs(g_ref[..., 0]) + FLOOR_L
    tolT = MARCH_REL * np.abs(g_ref[..., 1]) + FLOOR_T
    n_cond = 0
    if allow is not None:
        n_cond = int(((allow[..., 0] > tolL) | (allow[..., 1] > tolT)).sum())
        tolL = tolL + allow[..., 0]
        tolT = tolT + allow[..., 1]
    okL = dL <= tolL
    okT = dT <= tolT
    flagged = margin < D_MARGIN * max(depth_tau, 1e-30)
    dD = np.abs(g_gpu[..., 2] - g_ref[..., 2])
    okD = (dD <= 1e-6 * np.abs(g_ref[..., 2]) + 1e-7) | flagged
    rel_ok = (dL <= MARCH_REL * np.abs(g_ref[..., 0]) + FLOOR_L) & (dT <= MARCH_REL * np.abs(g_ref[..., 1]) + FLOOR_T)
    needed = int((~rel_ok & okL & okT).sum())  # passed only thanks to the fp32 ray allowance
    summary = dict(max_dL=float(dL.max()), max_dT=float(dT.max()), bad_L=int((~okL).sum()), bad_T=int((~okT).sum()),
                   bad_D=int((~okD).sum()), flagged=int(flagged.sum()), pixels=int(dL.size),
                   ill_conditioned=n_cond, needed_allowance=needed, within_1e5_rel=int(rel_ok.sum()))
    log(f"march parity {what}: {summary}")
    assert okL.all(), (what, summary, np.argwhere(~okL)[:5])
    assert okT.all(), (what, summary, np.argwhere(~okT)[:5])
    assert okD.all(), (what, summary, np.argwhere(~okD)[:5])
    assert flagged.mean() <= 0.005, summary
    assert needed <= 0.01 * dL.size, summary
    return summary


def check_net(lm_gpu, lm_ref, lo_gpu=None, lo_ref=None, what=""):
    d = np.abs(lm_gpu - lm_ref)
    s = dict(max_abs_lightmap=float(d.max()), mean_abs=float(d.mean()))
    if lo_gpu is not None:
        dz = np.abs(lo_gpu - lo_ref) / np.maximum(1.0, np.abs(lo_ref))
        s["max_rel_logit"] = float(dz.max())
    log(f"net parity {what}: {s}")
    assert s["max_abs_lightmap"] <= NET_ABS, s
    if lo_gpu is not None:
        assert s["max_rel_logit"] <= NET_ABS, s
    return s
