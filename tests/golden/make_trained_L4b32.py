"""Train the configured 4-level base-32 U-Net on the CPU with the fp64 oracle
and store its weights as a test fixture (tests/golden/trained_L4b32.npy).

The precision forms are judged on a trained network (untrained He-normal
weights drive the sigmoid into regimes a trained one does not visit), and an
input of the comparison against the oracle must not come from the GPU path:
so these weights depend on nothing but the oracle and the seeded inputs.

Data: 128^3 grids of 24 blobs + 3-octave noise (the headline scene recipe,
seeds 3000 + i), each seen by perspective cameras at distance 2.5 from
random directions, rendered at 64x64.  One view in three frames the whole
volume (60 degree field of view); the others are zoomed windows (16.43 and
8.25 degrees, aimed at a point within 0.25 of the centre) whose pixels
subtend what a 256x256 or a 512x512 view's pixels do, so the network sees
the image statistics of the configured view sizes.  Inputs are the oracle's
guiding maps (step 4 voxels, jitter on); targets its fine-step reference
lightmaps (0.5 voxel, Section 5 references replaced by the deterministic
single-scatter march) encoded in sRGB (the loss is in sRGB space, Section 4.4).
Training: Adam (Section 5: lr 1e-3), batch 4, a fixed number of steps, all in
the oracle (fp64 arithmetic on fp32-rounded weights).

Usage:
  python tests/golden/make_trained_L4b32.py [--steps N] [--checkpoint PATH]
With --checkpoint the dataset and the optimiser state are saved there every
50 steps, and a later run with the same path resumes from them.
"""
import argparse
import math
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from synth.rng import substream  # noqa: E402
from synth.scene import Camera, PERSPECTIVE, make_volume  # noqa: E402
from synth.weights import he_normal_params  # noqa: E402

LEVELS, BASE, RES, GRID = 4, 32, 64, 128
N_SCENES, VIEWS_PER_SCENE = 48, 3
FOVS = (60.0, 16.43, 8.25)
OUT = os.path.join(HERE, "trained_L4b32.npy")


def view(seed: int, k: int) -> Camera:
    u = substream(seed * 16 + k, "train-view").uniform(6)
    az, el = 2 * math.pi * u[0], 0.6 * (u[1] - 0.5)
    fov = FOVS[k % len(FOVS)]
    tgt = np.array([0.5, 0.5, 0.5])
    if fov < 60.0:
        tgt = tgt + 0.5 * (u[2:5] - 0.5)
    eye = tgt + 2.5 * np.array([math.cos(el) * math.cos(az), math.sin(el), math.cos(el) * math.sin(az)])
    return Camera(PERSPECTIVE, tuple(eye), target=tuple(tgt), fov_y_deg=fov, width=RES, height=RES)


def dataset():
    gs, ts = [], []
    for i in range(N_SCENES):
        s = 3000 + i
        vol = make_volume(GRID, 24, s, noise_amp=0.3)
        for k in range(VIEWS_PER_SCENE):
            cam = view(s, k)
            g, _, _ = oracle.march(vol, 8.0, cam, 4.0, seed=s, frame=k)
            ref = oracle.reference_lightmaps(vol, 8.0, cam, 0.5)
            gs.append(g)
            ts.append(oracle.srgb_encode(ref))
        print(f"scene {i + 1}/{N_SCENES}", flush=True)
    return np.stack(gs), np.stack(ts)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--batch", type=int, default=4)
    ap.add_argument("--checkpoint", default=None)
    a = ap.parse_args()

    ck = a.checkpoint
    if ck and os.path.exists(ck + ".data.npz"):
        d = np.load(ck + ".data.npz")
        G, T = d["G"], d["T"]
    else:
        G, T = dataset()
        if ck:
            np.savez(ck + ".data.npz", G=G, T=T)
    p = he_normal_params(LEVELS, BASE, seed=0).astype(np.float64)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    t0 = 0
    if ck and os.path.exists(ck + ".state.npz"):
        s = np.load(ck + ".state.npz")
        p, m, v, t0 = s["p"], s["m"], s["v"], int(s["t"])
    rng = np.random.default_rng(0)
    for t in range(1, t0 + 1):  # replay the batch draws of the steps already taken
        rng.choice(len(G), a.batch, replace=False)
    for t in range(t0 + 1, a.steps + 1):
        idx = rng.choice(len(G), a.batch, replace=False)
        loss, grad = oracle.unet_loss_grad(p.astype(np.float32), LEVELS, BASE, G[idx], T[idx])
        p, m, v = oracle.adam(p, grad, m, v, t, lr=1e-3)
        if t % 25 == 0 or t == 1:
            print(f"step {t}: loss {loss:.5f}", flush=True)
        if ck and t % 50 == 0:
            np.savez(ck + ".state.npz", p=p, m=m, v=v, t=t)
    np.save(OUT, p.astype(np.float32))
    print("wrote", OUT)


if __name__ == "__main__":
    main()
