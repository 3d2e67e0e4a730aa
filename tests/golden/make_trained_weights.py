"""Train the small 3-level base-16 U-Net on the CPU with the fp64 oracle and
store its weights as a test fixture (tests/golden/trained_L3b16.npy).

Data: seeded 32^3 six-blob scenes seen from random orbit cameras at 32x32;
inputs are the oracle's guiding maps (step 2 voxels, jitter on), targets the
oracle's fine-step reference lightmaps (0.5 voxel) encoded in sRGB.  Training:
Adam, lr 1e-3, batch 4, fixed number of steps, all in the oracle (fp64), so
the weights depend on nothing but the oracle and the seeded inputs.

Usage: python tests/golden/make_trained_weights.py
"""
import math
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from synth.rng import substream  # noqa: E402
from synth.scene import Camera, ORTHOGRAPHIC, PERSPECTIVE, make_volume  # noqa: E402
from synth.weights import he_normal_params  # noqa: E402

LEVELS, BASE, RES, N = 3, 16, 32, 32
OUT = os.path.join(HERE, "trained_L3b16.npy")


def scene(seed):
    vol = make_volume(N, 6, seed)
    u = substream(seed, "view").uniform(3)
    az, el = 2 * math.pi * u[0], 0.5 * (u[1] - 0.5)
    eye = (0.5 + 2.5 * math.cos(el) * math.cos(az), 0.5 + 2.5 * math.sin(el), 0.5 + 2.5 * math.cos(el) * math.sin(az))
    proj = PERSPECTIVE if u[2] < 0.5 else ORTHOGRAPHIC
    return vol, Camera(proj, eye, fov_y_deg=40.0, ortho_half_extent=0.8, width=RES, height=RES)


def dataset(seeds):
    gs, ts = [], []
    for s in seeds:
        vol, cam = scene(s)
        g, _, _ = oracle.march(vol, 8.0, cam, 2.0, seed=s)
        ref = oracle.reference_lightmaps(vol, 8.0, cam, 0.5)
        gs.append(g)
        ts.append(oracle.srgb_encode(ref))
    return np.stack(gs), np.stack(ts)


def main(steps=300, batch=4):
    G, T = dataset(range(500, 564))
    p = he_normal_params(LEVELS, BASE, seed=0).astype(np.float64)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    rng = np.random.default_rng(0)
    for t in range(1, steps + 1):
        idx = rng.choice(len(G), batch, replace=False)
        loss, grad = oracle.unet_loss_grad(p.astype(np.float32), LEVELS, BASE, G[idx], T[idx])
        p, m, v = oracle.adam(p, grad, m, v, t, lr=1e-3)
        if t % 50 == 0 or t == 1:
            print(f"step {t}: loss {loss:.5f}", flush=True)
    np.save(OUT, p.astype(np.float32))
    print("wrote", OUT)


if __name__ == "__main__":
    main()
