"""Benchmark of the neural six-way lightmaps hot path on one MI355X.

One step = one frame of the whole path through lnm_frame: brick relayout and
guiding-map march of a 128^3 smoke grid (24 blobs + value noise) seen by a
60-degree perspective camera at 256x256 with a 4-voxel step, the 4-level
base-32 U-Net, and six-way shading for one light.  Inputs (grid, weights,
buffers) are resident in HBM before the timed region.  The frame is timed
with the fp32 network (`value`) and the bf16 and fp8 networks (`modes`).
Per-kernel durations come from HIP events the library records on its stream
in a second pass over the same frames; `roofline` is the 3x3 conv layers'
(the dominant kernel) algorithmic FLOP rate against the dtype's MFMA peak,
with HBM traffic from the committed rocprofv3 counter summary when it
matches the current conv sources.

Further sections (each can be skipped): per-channel error of the three
precisions against the fp64 oracle on the 512x512 guiding map of the same
volume and camera (the precision configuration); the channel-adapter network;
the dynamic 256^3 / 1024^2 bf16 scene with its obstacle shadowing; the
continuous-batching server (64 instances, Poisson arrivals, HBM budget); the
oracle's CPU frame rate (`cpu_baseline`).
Prints one JSON line.

Usage: python bench.py [--steps K] [--warmup W] [--dtype fp32|bf16|fp8] [--only]
       [--no-cpu-baseline] [--no-serve] [--no-dynamic] [--no-precision] [--no-adapters]
       [--no-two-streams]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT =os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "lightmap frames/s at 128³ grid/256² view, FP32 vs BF16; served p50/p99 latency"
# published dense matrix peaks of MI355X (TFLOP/s) and HBM bandwidth (GB/s)
PEAK_TFLOPS = {"fp32": 157.3, "bf16": 2500.0, "fp8": 5000.0}
HBM_PEAK_GBS = 8000.0


def log(msg):
    sys.stderr.write(msg + "\n")
    sys.stderr.flush()


def cpu_baseline(wl, params, light, seconds):
    """Time the fp64 oracle on whole frames of the same workload."""
    import oracle

    vol = wl.volume()
    n, t_total = 0, 0.0
    while True:
        t0 = time.perf_counter()
        g, _, _ = oracle.march(vol, 8.0, wl.camera, wl.step_voxels, seed=0, frame=n)
        lm, _ = oracle.unet_forward(params, wl.levels, wl.base, g)
        oracle.composite(lm, g, wl.camera, [light])
        t_total += time.perf_counter() - t0
        n += 1
        log(f"cpu oracle frame {n}: {t_total / n:.2f} s/frame")
        if t_total >= seconds or n >= 64:
            break
    out = {"value": round(n / t_total, 4), "unit": "frames/s", "cores": oracle.num_threads(), "kind": "oracle",
           "sample": f"{n} whole frame(s) (march + U-Net + shading) of the same 128^3 / 256x256 workload in fp64, "
                     f"{t_total:.1f} s"}
    # the oracle on the other configurations, once each: the small
    # configuration's whole frame (32^3, 64x64 orthographic, 3-level base-16)
    # and the precision configuration's network alone (512x512, 4-level base 32)
    from synth.scene import headline, small_ortho
    from synth.weights import he_normal_params

    sm = small_ortho()
    sp = he_normal_params(sm.levels, sm.base, seed=0)
    t0 = time.perf_counter()
    g, _, _ = oracle.march(sm.volume(), 8.0, sm.camera, sm.step_voxels, seed=0)
    lm, _ = oracle.unet_forward(sp, sm.levels, sm.base, g)
    oracle.composite(lm, g, sm.camera, [light])
    t_small = time.perf_counter() - t0
    c3 = headline(res=512)
    g3 = np.random.default_rng(0).random((512, 512, 3))
    t0 = time.perf_counter()
    oracle.unet_forward(params, c3.levels, c3.base, g3)
    t_net = time.perf_counter() - t0
    log(f"cpu oracle: {sm.name} frame {t_small:.3f} s, 512x512 network {t_net:.2f} s")
    out["other_configs"] = {f"{sm.name}_frame_s": round(t_small, 4), "persp128_512px_network_s": round(t_net, 3)}
    return out


def measure(lnm, ctx, net, dens, wl, light, steps, warmup, stream):
    import torch

    H, W = wl.camera.height, wl.camera.width
    dev = dens.device
    guide = torch.empty((H, W, 3), dtype=torch.float32, device=dev)
    lm = torch.empty((H, W, 6), dtype=torch.float32, device=dev)
    rgba = torch.empty((H, W, 4), dtype=torch.float32, device=dev)
    prm = lnm.make_params(wl.step_voxels, seed=0)
    ws = net.frame_workspace(dens, 8.0, wl.camera, prm)

    def step(i):
        prm.frame = i
        net.frame(dens, 8.0, wl.camera, prm, lights=[light], guide=guide, lightmaps=lm, rgba=rgba, workspace=ws,
                  stream=stream)

    for i in range(warmup):
        step(i)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        step(i)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    # per-kernel durations: HIP events the library records around each launch
    nprof = max(20, min(steps, 200))
    ctx.profile(True)
    for i in range(nprof):
        step(i)
    torch.cuda.synchronize()
    stage = {}
    # lnm_frame shades in the head launch, so "head_composite" covers both
    for name, k in (("march", lnm.K_MARCH), ("conv3x3", lnm.K_CONV), ("head_composite", lnm.K_HEAD)):
        n, ms = ctx.profile_read(k)
        stage[name] = {"launches_per_frame": n / nprof, "us_per_frame": 1e3 * ms / nprof,
                       "us_per_launch": 1e3 * ms / max(n, 1)}
    ctx.profile(False)
    return {"fps": steps / elapsed, "ms_per_step": 1e3 * elapsed / steps, "stage": stage}


def measure_two_streams(lnm, net, dens, wl, light, steps, warmup):
    """The same frames issued alternately on two HIP streams (default
    priority), each with its own buffers, so one frame's march can overlap
    the previous frame's network: whole-job throughput of K complete frames."""
    import torch

    H, W = wl.camera.height, wl.camera.width
    dev = dens.device
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    prms = [lnm.make_params(wl.step_voxels, seed=0) for _ in range(2)]
    bufs = []
    for q in range(2):
        bufs.append(dict(guide=torch.empty((H, W, 3), dtype=torch.float32, device=dev),
                         lightmaps=torch.empty((H, W, 6), dtype=torch.float32, device=dev),
                         rgba=torch.empty((H, W, 4), dtype=torch.float32, device=dev),
                         workspace=net.frame_workspace(dens, 8.0, wl.camera, prms[q])))
    torch.cuda.synchronize()

    def step(i):
        q = i & 1
        prms[q].frame = i
        net.frame(dens, 8.0, wl.camera, prms[q], lights=[light], stream=streams[q], **bufs[q])

    for i in range(warmup):
        step(i)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        step(i)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    return {"fps": steps / elapsed, "ms_per_frame_amortised": 1e3 * elapsed / steps}


def served(lnm, ctx, params, seconds, warmup_s, rate_hz=2000.0, budget_gb=64.0, n_instances=64, seed=7,
           hold_ms=0.0):
    """Continuous-batching server: n_instances smoke instances (grids
    {64,96,128,192,256}^3, views {128,256,512}^2, own seeded blobs + noise and
    light), Poisson arrivals at rate_hz, bf16 network, HBM budget (resident
    grids and brick copies included), batches held up to hold_ms."""
    import torch

    from paper_2604_03748_amd.serve import Backend, Instance, Scheduler, poisson_requests
    from synth.rng import substream
    from synth.scene import light_direction, make_volume_torch

    grids, views = (64, 96, 128, 192, 256), (128, 256, 512)
    pick = substream(seed, "instances").uniform(2 * n_instances).reshape(n_instances, 2)
    insts = {}
    for k in range(n_instances):
        n = grids[int(pick[k, 0] * len(grids))]
        res = views[int(pick[k, 1] * len(views))]
        insts[k] = Instance(k, make_volume_torch(n, 24, 1000 + k, 0.3, device="cuda"), res,
                            start_deg=(37.0 * k) % 360.0, seed=1000 + k,
                            light=(tuple(light_direction(1000 + k)), (1.0, 1.0, 1.0)))
    for inst in insts.values():  # the grids are static: brick them once, like keeping them resident
        inst.prepare(ctx)
    torch.cuda.synchronize()
    net = lnm.Net(ctx, 4, 32, params, precision=lnm.BF16)
    be = Backend(ctx, net, n_streams=4)
    budget = int(budget_gb * 2**30)
    if warmup_s > 0:
        Scheduler(be, insts, budget, max_batch=16, hold_s=hold_ms * 1e-3).run(
            poisson_requests(n_instances, rate_hz, warmup_s, seed + 1))
    reqs = poisson_requests(n_instances, rate_hz, seconds, seed)
    sch = Scheduler(be, insts, budget, max_batch=16, hold_s=hold_ms * 1e-3)
    st = sch.run(reqs)
    # the completed frames' network work against the bf16 matrix peak
    from synth.weights import unet_flops

    fl = sum(unet_flops(4, 32, 1, insts[r.instance].res, insts[r.instance].res) for r in sch.done)
    st["net_tflops"] = fl / st["wall_s"] / 1e12 if st["wall_s"] > 0 else 0.0
    st["net_frac_of_bf16_peak"] = st["net_tflops"] / PEAK_TFLOPS["bf16"]
    st.update({"offered_rate_fps": rate_hz, "instances": n_instances, "duration_s": seconds,
               "grids": sorted({v.density.shape[0] for v in insts.values()}), "views": list(views),
               "dtype": "bf16", "budget_gb": budget_gb})
    return st


def dynamic_scene(lnm, ctx, frames, warmup=3):
    """256^3 grid of 32 moving blobs + noise with a sphere obstacle (r 0.15),
    camera orbiting 1.5 deg/frame, light rotating 0.5 deg/frame, 1024^2 view,
    step 4 voxels, 4-level base-48 bf16 network.  Method time (march + U-Net +
    shading) is measured with HIP events on the stream, and the obstacle
    shadowing of the same frame (sphere depth map + shadowed shading) beside
    it; regenerating the density each frame is timed separately and not
    counted.  A few more frames with per-launch events give the stage split."""
    import torch

    from synth.scene import dynamic, light_direction, make_volume_torch, orbit_camera, rotate_y
    from synth.weights import he_normal_params

    wl = dynamic()
    params = he_normal_params(wl.levels, wl.base, seed=0)
    net = lnm.Net(ctx, wl.levels, wl.base, params, precision=lnm.BF16)
    stream = torch.cuda.current_stream()
    light0 = light_direction(0)
    cam0 = orbit_camera(0)
    prm = lnm.make_params(wl.step_voxels, seed=0)
    dens = make_volume_torch(256, 32, 0, 0.3, frame=0, obstacle_radius=0.15)
    ws = net.frame_workspace(dens, 8.0, cam0, prm)
    H = W = 1024
    guide = torch.empty((H, W, 3), dtype=torch.float32, device="cuda")
    lm = torch.empty((H, W, 6), dtype=torch.float32, device="cuda")
    rgba = torch.empty((H, W, 4), dtype=torch.float32, device="cuda")
    # obstacle shadowing (Section 4.5): the sphere's depth map seen from the
    # light (1024^2 texels over the cube) and the shading with each pixel's
    # smoke surface tested against it, after the frame
    centre, radius = (0.5, 0.5, 0.5), 0.15
    sf = lnm.make_shadow_frame(centre, 0.9, 1024, 2.0 / 256)
    dmap = torch.empty((1024, 1024), dtype=torch.float32, device="cuda")
    rgba_s = torch.empty_like(rgba)
    gen_ms, frame_ms, shadow_ms = [], [], []
    for f in range(warmup + frames):
        e0, e1, e2, e3 = (torch.cuda.Event(enable_timing=True) for _ in range(4))
        e0.record(stream)
        dens = make_volume_torch(256, 32, 0, 0.3, frame=f, obstacle_radius=radius)
        e1.record(stream)
        prm.frame = f
        cam = orbit_camera(f)
        light = (tuple(rotate_y(light0, 0.5 * f)), (1.0, 1.0, 1.0))
        net.frame(dens, 8.0, cam, prm, lights=[light], guide=guide, lightmaps=lm, rgba=rgba,
                  workspace=ws, stream=stream)
        e2.record(stream)
        ctx.shadow_map_sphere(sf, light[0], centre, radius, out=dmap, stream=stream)
        ctx.composite_shadowed(cam, [light], sf, [dmap], lm, guide, out=rgba_s, stream=stream)
        e3.record(stream)
        e3.synchronize()
        if f >= warmup:
            gen_ms.append(e0.elapsed_time(e1))
            frame_ms.append(e1.elapsed_time(e2))
            shadow_ms.append(e2.elapsed_time(e3))
    # stage split of the same frames: HIP events the library records around each launch
    nprof = 5
    ctx.profile(True)
    for f in range(nprof):
        prm.frame = f
        net.frame(dens, 8.0, orbit_camera(f), prm, lights=[(tuple(rotate_y(light0, 0.5 * f)), (1.0, 1.0, 1.0))],
                  guide=guide, lightmaps=lm, rgba=rgba, workspace=ws, stream=stream)
    torch.cuda.synchronize()
    stages = {}
    for name, k in (("march", lnm.K_MARCH), ("conv3x3", lnm.K_CONV), ("head_composite", lnm.K_HEAD)):
        stages[name] = round(ctx.profile_read(k)[1] / nprof, 4)
    ctx.profile(False)
    fm = np.array(frame_ms)
    from synth.weights import unet_flops

    conv_fl = unet_flops(wl.levels, wl.base, 1, H, W) - 2.0 * H * W * 6 * wl.base  # 3x3 layers only
    conv_tf = conv_fl / (stages["conv3x3"] * 1e-3) / 1e12
    prim, sec = DYNAMIC_SAMPLES
    return {"workload": "dynamic256_1024px", "frames": frames, "dtype": "bf16", "stages_ms_per_frame": stages,
            "conv_roofline": {"bound": "mfma", "achieved": round(conv_tf, 2), "peak": PEAK_TFLOPS["bf16"],
                              "unit": "TFLOP/s", "frac": round(conv_tf / PEAK_TFLOPS["bf16"], 4),
                              "flops_per_frame": round(conv_fl)},
            "march_g_samples_per_s": round((prim + sec) / (stages["march"] * 1e-3) / 1e9, 2),
            "method_frames_per_s": round(1e3 / fm.mean(), 2), "latency_ms_p50": round(float(np.median(fm)), 4),
            "latency_ms_p99": round(float(np.percentile(fm, 99)), 4),
            "shadow_ms_mean": round(float(np.mean(shadow_ms)), 4),
            "with_shadows_frames_per_s": round(1e3 / (fm.mean() + float(np.mean(shadow_ms))), 2),
            "density_regen_ms_mean": round(float(np.mean(gen_ms)), 4)}


def adapters_mode(lnm, ctx, wl, params, dens, steps, warmup):
    """The network with the four NAFBlock channel adapters in place of the
    plain head (fp32), on the headline guiding map: U-Net trunk + adapters per
    frame, and the adapters' own time from HIP events around their kernels
    (their 1x1 convolutions on the fp32 matrix cores: priced against that
    peak)."""
    import torch

    from synth.weights import adapter_flops, adapter_params

    net = lnm.Net(ctx, wl.levels, wl.base, params)
    ad = lnm.Adapters(net, adapter_params(wl.base, seed=0))
    g = ctx.march(dens, 8.0, wl.camera, lnm.make_params(wl.step_voxels, seed=0))[None]
    H, W = wl.camera.height, wl.camera.width
    lm = torch.empty((1, H, W, 6), dtype=torch.float32, device=dens.device)
    ex = torch.empty((1, H, W, 2), dtype=torch.float32, device=dens.device)
    ws = ad.workspace(1, H, W)
    for _ in range(warmup):
        ad.infer(g, out=lm, extra=ex, workspace=ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ad.infer(g, out=lm, extra=ex, workspace=ws)
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / steps
    ctx.profile(True)
    for _ in range(steps):
        ad.infer(g, out=lm, extra=ex, workspace=ws)
    torch.cuda.synchronize()
    n, tot = ctx.profile_read(lnm.K_ADAPTERS)
    ctx.profile(False)
    us = 1e3 * tot / max(n, 1)
    fl = adapter_flops(wl.base, 1, H, W)
    return {"workload": "persp128_256px", "net": f"L{wl.levels} base {wl.base} fp32 + 4 NAFBlock adapters",
            "ms_per_frame_net_plus_adapters": round(ms, 4), "adapters_us": round(us, 2),
            "adapters_flops": fl, "adapters_tflops": round(fl / (us * 1e-6) / 1e12, 3),
            "peak_fp32_mfma_tflops": PEAK_TFLOPS["fp32"],
            "frac_of_fp32_peak": round(fl / (us * 1e-6) / 1e12 / PEAK_TFLOPS["fp32"], 4)}


TRAINED_WEIGHTS = os.path.join(ROOT, "tests", "golden", "trained_L4b32.npy")


def precision_report(lnm, ctx, wl, params, dens, weights="He-normal seed 0 (untrained)"):
    """Max / mean abs error per lightmap channel of fp32, bf16 and fp8
    against the fp64 oracle, on one frame's guiding map of workload wl; fp8
    activation maxima calibrated on four other scenes of the same recipe."""
    import numpy as np
    import torch

    import oracle
    from synth.scene import headline

    prm = lnm.make_params(wl.step_voxels, seed=0)
    g = ctx.march(dens, 8.0, wl.camera, prm)
    gh = g.cpu().numpy().astype(np.float64)
    ref, _ = oracle.unet_forward(params, wl.levels, wl.base, gh)
    n32 = lnm.Net(ctx, wl.levels, wl.base, params)
    H = wl.camera.height
    calib = [ctx.march(torch.as_tensor(headline(seed=s, res=H).volume(), device=dens.device), 8.0, wl.camera,
                       lnm.make_params(wl.step_voxels, seed=s)) for s in (1, 2, 3, 4)]
    amax = np.max([n32.calibrate_amax(c) for c in calib], axis=0)
    nets = {"fp32": n32, "bf16": lnm.Net(ctx, wl.levels, wl.base, params, precision=lnm.BF16),
            "fp8": lnm.Net(ctx, wl.levels, wl.base, params, precision=lnm.FP8_E4M3, act_scales=amax)}
    out = {}
    for k, net in nets.items():
        lm = net.infer(g)
        torch.cuda.synchronize()
        d = np.abs(lm.cpu().numpy().astype(np.float64) - ref).reshape(-1, 6)
        out[k] = {"max_abs": [round(float(x), 6) for x in d.max(axis=0)],
                  "mean_abs": [round(float(x), 7) for x in d.mean(axis=0)]}
    out["weights"] = weights
    out["workload"] = wl.name
    return out, amax


# the conv kernels, their tiling / split-K choice (conv_layer_tiling in
# plan.hip) and the head epilogue; the march kernels and their work order
# and buffers (plan.hip)
CONV_SOURCES = ("paper_2604_03748_amd/csrc/conv.hip", "paper_2604_03748_amd/csrc/conv_bf16.hip",
                "paper_2604_03748_amd/csrc/conv_fp8.hip", "paper_2604_03748_amd/csrc/head.h",
                "paper_2604_03748_amd/csrc/first_layer.h", "paper_2604_03748_amd/csrc/plan.hip")
MARCH_SOURCES = ("paper_2604_03748_amd/csrc/march.hip", "paper_2604_03748_amd/csrc/ray.h",
                 "paper_2604_03748_amd/csrc/plan.hip")


def source_hash(sources=CONV_SOURCES) -> str:
    """sha256[:16] of the sources' code: comments and blank space removed, so
    that an edit of the documentation alone keeps a profile of the same
    kernels valid."""
    import hashlib
    import re

    h = hashlib.sha256()
    for rel in sources:
        with open(os.path.join(ROOT, rel), encoding="utf-8") as f:
            text = f.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def conv_source_hash() -> str:
    return source_hash(CONV_SOURCES)


# Samples of one frame's march (primary + light-march samples, the geometric
# count with early termination as the method takes it), from the oracle's
# counters for frame 0 of each workload: the per-unit figure of the march's
# rate.  persp128: 270,662 + 8,304,019 at 256x256, 1,082,304 + 33,217,091
# at 512x512.
MARCH_SAMPLES = {"persp128_256px": (270662, 8304019), "persp128_512px": (1082304, 33217091)}
# dynamic256_1024px, frame 0 (the blobs move, so later frames differ a little)
DYNAMIC_SAMPLES = (8463809, 521045931)
# A CU issues at most one wave64 VALU instruction per clock (four SIMDs, each
# taking four clocks per wave64 instruction): 256 CUs x 2.4 GHz.
VALU_PEAK_INSTS = 256 * 2.4e9


def profile_blob(name, sources):
    """The json block of a committed profile summary, or None when there is
    none or the kernel sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    try:
        blob = json.loads(open(path).read().split("```json", 1)[1].split("```", 1)[0])
    except (IndexError, ValueError):
        return None
    return blob if blob.get("source_hash") == source_hash(sources) else None


def march_traffic():
    """HBM bytes of one headline march (relayout + march kernels) from the
    committed rocprofv3 counter summary, or None when there is none or the
    march sources changed since it was taken."""
    blob = profile_blob("march_persp128_256px_traffic.md", MARCH_SOURCES)
    return blob.get("bytes_per_march") if blob else None


def march_roofline(lnm, wl, stage, relayout_us=None):
    """The march against its binding bound, the VALU issue rate: VALU
    instructions per march (committed rocprofv3 counters, SQ_INSTS_VALU) over
    the measured march time, against one wave64 instruction per CU per clock.
    Beside it: samples per second (oracle sample counts of the frame), the
    algorithmic HBM bytes (grid read once, guiding map written once) and the
    measured HBM traffic against the 8 TB/s peak, and the brick relayout (a
    plain copy: grid read, bricks written) against the same peak."""
    n = wl.grid
    H, W = wl.camera.height, wl.camera.width
    us = stage["march"]["us_per_frame"]
    prim, sec = MARCH_SAMPLES[wl.name]
    algorithmic = 4 * n ** 3 + 12 * H * W
    headline = wl.name == "persp128_256px"  # the workload the committed counters were taken on
    t = march_traffic() if headline else None
    blob = profile_blob("march_persp128_256px_counters.md", MARCH_SOURCES) if headline else None
    insts = blob.get("valu_insts_per_march") if blob else None
    out = {"bound": "alu", "unit": "G VALU instr/s", "peak": round(VALU_PEAK_INSTS / 1e9, 1),
           "achieved": round(insts / (us * 1e-6) / 1e9, 2) if insts else None,
           "frac": round(insts / (us * 1e-6) / VALU_PEAK_INSTS, 4) if insts else None,
           "valu_insts_per_march": insts, "us_per_frame": round(us, 2),
           "samples": prim + sec, "g_samples_per_s": round((prim + sec) / (us * 1e-6) / 1e9, 2),
           "hbm": {"algorithmic_bytes": algorithmic, "achieved_gbs": round(algorithmic / (us * 1e-6) / 1e9, 1),
                   "peak_gbs": HBM_PEAK_GBS, "frac": round(algorithmic / (us * 1e-6) / 1e9 / HBM_PEAK_GBS, 5),
                   "traffic": t, "traffic_gbs": round(t / (us * 1e-6) / 1e9, 1) if t else None}}
    if relayout_us:
        bricks = int(lnm.lib().lnm_bricks_bytes(n, n, n))
        b = 4 * n ** 3 + bricks
        out["relayout"] = {"bound": "hbm", "bytes": b, "us": round(relayout_us, 3),
                           "achieved_gbs": round(b / (relayout_us * 1e-6) / 1e9, 1), "peak_gbs": HBM_PEAK_GBS,
                           "frac": round(b / (relayout_us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)}
    return out


def relayout_time(lnm, ctx, dens, reps=50):
    """Mean duration of the brick relayout of the grid (lnm_make_bricks: grid
    read, bricks written), HIP events on the stream it runs on."""
    import torch

    out = ctx.make_bricks(dens)
    for _ in range(5):
        ctx.make_bricks(dens, out=out)
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(reps):
        ctx.make_bricks(dens, out=out)
    e1.record(st)
    e1.synchronize()
    return 1e3 * e0.elapsed_time(e1) / reps


def measured_traffic(dtype):
    """HBM bytes per conv launch from the committed rocprofv3 counter summary
    (FETCH_SIZE + WRITE_SIZE, scaled by a plain copy of known size), or None
    when there is none or the conv sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"conv3x3_{dtype}_persp128_256px_traffic.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    try:
        blob = json.loads(text.split("```json", 1)[1].split("```", 1)[0])
    except (IndexError, ValueError):
        return None
    if blob.get("source_hash") != conv_source_hash():
        return None
    return blob.get("bytes_per_launch")


def conv_roofline(wl, stage, dtype):
    from synth.weights import unet_flops

    H, W = wl.camera.height, wl.camera.width
    conv_flops = unet_flops(wl.levels, wl.base, 1, H, W) - 2.0 * H * W * 6 * wl.base  # 3x3 layers only
    # the 3x3 layers' algorithmic FLOPs over their time per frame; the
    # launches are counted as made (fp32 and bf16 run the first two layers
    # as one)
    n_conv = stage["conv3x3"]["launches_per_frame"]
    us = stage["conv3x3"]["us_per_frame"] / n_conv
    per_launch = conv_flops / n_conv
    achieved = per_launch / (us * 1e-6) / 1e12
    kern = {"fp32": "conv3x3_f32 (v_mfma_f32_16x16x4_f32)", "bf16": "conv3x3_bf16 (v_mfma_f32_16x16x32_bf16)",
            "fp8": "conv3x3_fp8 (v_mfma_f32_16x16x32_fp8_fp8)"}[dtype]
    return {"bound": "mfma", "achieved": round(achieved, 3), "peak": PEAK_TFLOPS[dtype], "unit": "TFLOP/s",
            "frac": round(achieved / PEAK_TFLOPS[dtype], 5), "traffic": measured_traffic(dtype), "kernel": kern,
            "flops_per_launch": round(per_launch), "us_per_launch": round(us, 3),
            "launches_per_frame": round(n_conv, 3)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--dtype", default="fp32", choices=["fp32", "bf16", "fp8"])
    ap.add_argument("--only", action="store_true", help="time only --dtype")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serve", action="store_true", help="skip the served (continuous batching) mode")
    ap.add_argument("--no-precision", action="store_true", help="skip the per-channel error report")
    ap.add_argument("--serve-seconds", type=float, default=10.0,
                    help="arrival window of the main served run (the serving configuration's 10 s)")
    ap.add_argument("--no-dynamic", action="store_true", help="skip the dynamic-scene mode")
    ap.add_argument("--no-adapters", action="store_true", help="skip the channel-adapter mode")
    ap.add_argument("--no-two-streams", action="store_true", help="skip the two-stream throughput pass")
    ap.add_argument("--no-c3", action="store_true", help="skip the 512x512 frame timing")
    ap.add_argument("--dynamic-frames", type=int, default=240)
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="CPU time of the oracle sample")
    ap.add_argument("--copy-mb", type=int, default=0,
                    help="first run one plain device copy of this many MiB (reference for HBM counters)")
    ap.add_argument("--source-hash", action="store_true", help="print the conv and march sources' hashes and exit")
    args = ap.parse_args()
    if args.source_hash:
        print(conv_source_hash(), source_hash(MARCH_SOURCES))
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported: frames and smoke instances are "
              f"independent, so the path shards by frame or instance with no exchange", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2604_03748_amd import lnm
    from synth.scene import headline, light_direction
    from synth.weights import he_normal_params

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda", 0)
    wl = headline()
    params = he_normal_params(wl.levels, wl.base, seed=0)
    light = (tuple(light_direction(0)), (1.0, 1.0, 1.0))
    ctx = lnm.Context(0)
    dens = torch.as_tensor(wl.volume(), device=dev)
    stream = torch.cuda.current_stream()
    if args.copy_mb > 0:
        # one elementwise kernel reading and writing copy_mb MiB each
        a = torch.empty(args.copy_mb * 2**18, dtype=torch.float32, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        torch.mul(a, 1.0, out=b)
        torch.cuda.synchronize()
        del a, b
    prec = {"fp32": lnm.FP32, "bf16": lnm.BF16, "fp8": lnm.FP8_E4M3}
    order = [args.dtype] + ([] if args.only else [d for d in ("fp32", "bf16", "fp8") if d != args.dtype])
    # fp8 activation scales: maxima of the fp32 network over 4 jittered frames
    n32 = lnm.Net(ctx, wl.levels, wl.base, params)
    calib = [ctx.march(dens, 8.0, wl.camera, lnm.make_params(wl.step_voxels, seed=0, frame=1000 + f))
             for f in range(4)]
    amax = np.max([n32.calibrate_amax(c) for c in calib], axis=0)
    del n32
    res = {}
    for dt in order:
        net = lnm.Net(ctx, wl.levels, wl.base, params, precision=prec[dt],
                      act_scales=amax if dt == "fp8" else None)
        r = measure(lnm, ctx, net, dens, wl, light, args.steps, args.warmup, stream)
        r["roofline"] = conv_roofline(wl, r["stage"], dt)
        if not args.no_two_streams:
            r["two_streams"] = measure_two_streams(lnm, net, dens, wl, light, args.steps, args.warmup)
        res[dt] = r
        stages = ", ".join("%s: %.1f us" % (k, v["us_per_frame"]) for k, v in r["stage"].items())
        two = f" ({r['two_streams']['fps']:.1f} on two streams)" if "two_streams" in r else ""
        log(f"{dt}: {r['ms_per_step']:.4f} ms/frame, {r['fps']:.1f} frames/s{two}, stages {stages}")
        del net

    main_r = res[args.dtype]
    H, W = wl.camera.height, wl.camera.width
    out = {
        "metric": METRIC,
        "value": round(main_r["fps"], 2),
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(main_r["ms_per_step"], 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic (seeded blob+noise smoke grid, He-normal weights)",
        "config": {"workload": "persp128_256px", "grid": 128, "blobs": 24, "noise_amp": 0.3, "view": [H, W],
                   "camera": "perspective 60deg at 2.5", "step_voxels": wl.step_voxels, "unet_levels": wl.levels,
                   "unet_base": wl.base, "batch": 1, "lights": 1},
        "roofline": main_r["roofline"],
        "march_roofline": march_roofline(lnm, wl, main_r["stage"], relayout_time(lnm, ctx, dens)),
        "stages_us_per_frame": {k: round(v["us_per_frame"], 2) for k, v in main_r["stage"].items()},
        "frames_per_s_two_streams": round(main_r["two_streams"]["fps"], 2) if "two_streams" in main_r else None,
        "modes": {dt: {"value": round(r["fps"], 2), "ms_per_step": round(r["ms_per_step"], 5),
                       "frames_per_s_two_streams": round(r["two_streams"]["fps"], 2) if "two_streams" in r else None,
                       "roofline": r["roofline"],
                       "stages_us_per_frame": {k: round(v["us_per_frame"], 2) for k, v in r["stage"].items()}}
                  for dt, r in res.items() if dt != args.dtype},
    }
    if not args.no_c3:
        # the precision configuration's frame: the same volume and camera at
        # 512x512, each precision
        wl3 = headline(res=512)
        c3 = {}
        for dt in ("fp32", "bf16", "fp8"):
            net = lnm.Net(ctx, wl3.levels, wl3.base, params, precision=prec[dt],
                          act_scales=amax if dt == "fp8" else None)
            steps3 = max(20, args.steps // 4)
            r = measure(lnm, ctx, net, dens, wl3, light, steps3, max(5, args.warmup // 4), stream)
            del net
            c3[dt] = {"value": round(r["fps"], 2), "ms_per_step": round(r["ms_per_step"], 5),
                      "roofline": conv_roofline(wl3, r["stage"], dt),
                      "stages_us_per_frame": {k: round(v["us_per_frame"], 2) for k, v in r["stage"].items()}}
            if dt == "fp32":
                c3[dt]["march_roofline"] = march_roofline(lnm, wl3, r["stage"])
            log(f"512x512 {dt}: {r['ms_per_step']:.4f} ms/frame, {r['fps']:.1f} frames/s")
        out["persp128_512px"] = c3
    if not args.no_precision:
        # the precision configuration: the same volume and camera, 512x512,
        # the configured network with trained weights (and untrained, as
        # information)
        wl3 = headline(res=512)
        if os.path.exists(TRAINED_WEIGHTS):
            out["precision_error_vs_fp64_oracle"], _ = precision_report(
                lnm, ctx, wl3, np.load(TRAINED_WEIGHTS), dens,
                weights="trained by the oracle (tests/golden/trained_L4b32.npy)")
        out["precision_error_untrained_vs_fp64_oracle"], _ = precision_report(lnm, ctx, wl3, params, dens)
        log(f"precision: {out.get('precision_error_vs_fp64_oracle')}")
    if not args.no_adapters:
        out["adapters"] = adapters_mode(lnm, ctx, wl, params, dens, max(20, args.steps // 4), 5)
        log(f"adapters: {out['adapters']}")
    if not args.no_dynamic:
        out["dynamic"] = dynamic_scene(lnm, ctx, args.dynamic_frames)
        log(f"dynamic: {out['dynamic']}")
    if not args.no_serve:
        def rounded(st):
            return {k: (round(v, 4) if isinstance(v, float) else v) for k, v in st.items()}

        # the configured load (2000 frames/s offered, 64 GB) with batches held
        # up to 2 ms while the device is busy; then the same load launched
        # without holding, half that load, the configured load under a 6 GB
        # budget (resident grids and bricks included) so admission binds, and
        # 8000 frames/s offered for 3 s, beyond what the server keeps up
        # with: its throughput there is the server's capacity
        out["served"] = rounded(served(lnm, ctx, params, args.serve_seconds, warmup_s=1.0, hold_ms=2.0))
        log(f"served: {out['served']}")
        other_s = min(args.serve_seconds, 5.0)
        out["served_other_loads"] = [
            rounded(served(lnm, ctx, params, other_s, warmup_s=1.0, hold_ms=0.0)),
            rounded(served(lnm, ctx, params, other_s, warmup_s=1.0, rate_hz=1000.0, hold_ms=2.0)),
            rounded(served(lnm, ctx, params, other_s, warmup_s=1.0, budget_gb=6.0, hold_ms=2.0)),
            rounded(served(lnm, ctx, params, min(other_s, 3.0), warmup_s=1.0, rate_hz=8000.0, hold_ms=2.0)),
        ]
        log(f"served at other loads: {out['served_other_loads']}")
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl, params, light, args.cpu_seconds)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
