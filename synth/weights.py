"""Seeded U-Net parameters (He-normal) in the flat parameter-file order.

The paper names a modified U-Net (Section 4.3) without sizes; the sizes used
here are: L levels of widths C_l = base * 2^l; two 3x3 convolutions per
encoder level, the bottleneck and each decoder level; the first decoder
convolution of level l reads concat(skip_l, up(level l+1)) = 3 C_l channels;
a 1x1 head C_0 -> 6.

Flat order: enc0a, enc0b, enc1a, ..., bottleneck a/b, dec(L-2)a, dec(L-2)b,
..., dec0a, dec0b, head.  Each layer stores W as [C_out][C_in][k][k] followed
by b as [C_out], fp32 little-endian.

W ~ N(0, 2 / (C_in k^2)) drawn in that order from one SplitMix64 stream
(Box-Muller); biases are zero, or U[-0.1, 0.1] from a second stream when
``bias='uniform'`` (used by parity tests so a fused bias is exercised).
"""
from __future__ import annotations

import numpy as np

from .rng import substream

N_OUT = 6
N_IN = 3


def unet_layers(levels: int, base: int):
    """[(name, c_in, c_out, k)] in parameter-file order."""
    w = [base << l for l in range(levels)]
    layers = []
    c_in = N_IN
    for l in range(levels - 1):
        layers.append((f"enc{l}a", c_in, w[l], 3))
        layers.append((f"enc{l}b", w[l], w[l], 3))
        c_in = w[l]
    l = levels - 1
    layers.append((f"bot{l}a", c_in, w[l], 3))
    layers.append((f"bot{l}b", w[l], w[l], 3))
    for l in range(levels - 2, -1, -1):
        layers.append((f"dec{l}a", w[l] + w[l + 1], w[l], 3))
        layers.append((f"dec{l}b", w[l], w[l], 3))
    layers.append(("head", w[0], N_OUT, 1))
    return layers


def n_params(levels: int, base: int) -> int:
    return sum(co * ci * k * k + co for _, ci, co, k in unet_layers(levels, base))


def he_normal_params(levels: int, base: int, seed: int = 0, bias: str = "zero") -> np.ndarray:
    layers = unet_layers(levels, base)
    ws = substream(seed, "weights")
    bs = substream(seed, "bias")
    parts = []
    for _, ci, co, k in layers:
        nw = co * ci * k * k
        parts.append(ws.normal(nw) * np.sqrt(2.0 / (ci * k * k)))
        if bias == "zero":
            parts.append(np.zeros(co))
        elif bias == "uniform":
            parts.append(0.2 * bs.uniform(co) - 0.1)
        else:
            raise ValueError(bias)
    return np.ascontiguousarray(np.concatenate(parts).astype(np.float32))


def flops_per_pixel_table(levels: int, base: int):
    """[(name, M_scale, N, K)]: GEMM shape per layer, M = pixels / 4^level."""
    out = []
    for name, ci, co, k in unet_layers(levels, base):
        lvl = int(name[3]) if name[:3] in ("enc", "bot", "dec") else 0
        out.append((name, 4 ** lvl, co, ci * k * k))
    return out


def unet_flops(levels: int, base: int, batch: int, h: int, w: int) -> float:
    """Algorithmic FLOPs (2 per multiply-add) of one forward pass."""
    total = 0.0
    for _, div, n, k in flops_per_pixel_table(levels, base):
        total += 2.0 * batch * (h * w / div) * n * k
    return total


# ---------------------------------------------------------- channel adapters
ADAPTER_GROUPS = ("front/back", "left/right", "up/down", "alpha/emissive")


def adapter_tensors(c: int):
    """[(name, shape, fan_in or None)] of one adapter (NAFBlock of width c +
    1x1 head to 2 channels) in parameter-file order; fan_in None marks
    layer-norm weights/biases, the residual scales and biases."""
    return [("ln1_w", (c,), None), ("ln1_b", (c,), None),
            ("conv1_w", (2 * c, c), c), ("conv1_b", (2 * c,), None),
            ("dw_w", (2 * c, 3, 3), 9), ("dw_b", (2 * c,), None),
            ("sca_w", (c, c), c), ("sca_b", (c,), None),
            ("conv3_w", (c, c), c), ("conv3_b", (c,), None),
            ("beta", (c,), None),
            ("ln2_w", (c,), None), ("ln2_b", (c,), None),
            ("conv4_w", (2 * c, c), c), ("conv4_b", (2 * c,), None),
            ("conv5_w", (c, c), c), ("conv5_b", (c,), None),
            ("gamma", (c,), None),
            ("head_w", (2, c), c), ("head_b", (2,), None)]


def adapter_param_count(c: int) -> int:
    return 4 * sum(int(np.prod(s)) for _, s, _ in adapter_tensors(c))


def adapter_params(c: int, seed: int = 0, init: str = "random") -> np.ndarray:
    """Parameters of the four adapters (group order of ADAPTER_GROUPS).

    init='identity': conv weights He-normal, biases 0, layer norms (1, 0) and
    beta = gamma = 0, so each NAFBlock starts as the identity (its published
    initialisation).  init='random' (parity tests): layer-norm weights
    U[0.8, 1.2], biases U[-0.1, 0.1], beta and gamma U[-0.5, 0.5], so every
    term of the block is exercised."""
    ws = substream(seed, "adapter_weights")
    us = substream(seed, "adapter_other")
    parts = []
    for _ in range(4):
        for name, shape, fan_in in adapter_tensors(c):
            n = int(np.prod(shape))
            if fan_in is not None:
                parts.append(ws.normal(n) * np.sqrt(2.0 / fan_in))
            elif init == "identity":
                parts.append(np.ones(n) if name in ("ln1_w", "ln2_w") else np.zeros(n))
            elif init == "random":
                u = us.uniform(n)
                if name in ("ln1_w", "ln2_w"):
                    parts.append(0.8 + 0.4 * u)
                elif name in ("beta", "gamma"):
                    parts.append(u - 0.5)
                else:
                    parts.append(0.2 * u - 0.1)
            else:
                raise ValueError(init)
    return np.ascontiguousarray(np.concatenate(parts).astype(np.float32))


def adapter_flops(c: int, batch: int, h: int, w: int) -> float:
    """Algorithmic FLOPs of the four adapters (2 per multiply-add of the
    1x1 and depthwise convolutions and the head)."""
    per_px = 2 * c * c + 18 * c + c * c + 2 * c * c + c * c + 2 * c  # conv1, dw, conv3, conv4, conv5, head
    return 2.0 * 4 * batch * h * w * per_px
