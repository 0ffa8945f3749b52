"""CPU oracle of the learned per-patch threshold predictor -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the CPU-baseline leg of the benchmark
may import this module; the GPU library never calls it and shares no code
with it.

The paper tunes its threshold constant by hand for an error target (Section
2.2 and the threshold studies of Section 3.2); the learned part replaces the
single global constant by one threshold per patch, chosen from a small set
of candidates by a network that predicts, from the patch's coarse
coefficients, the error each candidate would cause.

Network (plain definition, float64 here; the GPU stores the weights in
bfloat16 and accumulates in float32):

  input  raw[B, 36, 8, 8] the patch features: channels 0..8 every field's
                          coefficients at the 8 x 8 owned positions of stride
                          8; channel 9 + 3 f + l - 1 the energy (sum of
                          squares) of field f's coefficients of level l
                          (l = 1, 2, 3, the finer of the two per-dimension
                          levels) in each 8 x 8 block of owned positions
  map    x[B, 12, 8, 8]   asinh(c / 1e-4) of the 9 coefficient channels, and
                          asinh(sqrt(sum over fields of the level-l energy) / 1e-4)
  conv1  3x3, pad 1, 12 -> 32 channels, bias, ReLU
  conv2  3x3, pad 1, 32 -> 32, bias, ReLU
  conv3  3x3, pad 1, stride 2, 32 -> 32 (output 4 x 4), bias, ReLU
  pool   mean over the 4 x 4 positions -> [B, 32]
  head   linear 32 -> K, bias: predicted log10 of the patch's squared error
         for each of the K candidate thresholds

Loss: mean squared difference to the targets.  Parameters:
3,488 + 9,248 + 9,248 + 33 K (22,380 for K = 12).

Gradients are written out by hand (the chain rule through each layer) and
pinned in the tests against central finite differences of the loss.
"""
from __future__ import annotations

import numpy as np

C_FIELDS = 9
C_RAW = 4 * C_FIELDS
C_IN = C_FIELDS + 3
C_HID = 32
SIDE = 8
FEATURE_SCALE = 1e-4


def bf16_round(x: np.ndarray) -> np.ndarray:
    """Round float32 values to the nearest bfloat16 (ties to even), as float32."""
    a = np.ascontiguousarray(x, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    r = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
    out = r.astype(np.uint32).view(np.float32)
    return np.where(np.isnan(a), a, out).astype(np.float32)


def param_shapes(k: int):
    return {
        "w1": (C_HID, C_IN, 3, 3), "b1": (C_HID,),
        "w2": (C_HID, C_HID, 3, 3), "b2": (C_HID,),
        "w3": (C_HID, C_HID, 3, 3), "b3": (C_HID,),
        "wh": (k, C_HID), "bh": (k,),
    }


def init_params(k: int, seed: int = 0) -> dict:
    """He-uniform weights, zero biases (float64)."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, shp in param_shapes(k).items():
        if name.startswith("b"):
            p[name] = np.zeros(shp)
        else:
            fan_in = int(np.prod(shp[1:]))
            lim = np.sqrt(6.0 / fan_in)
            p[name] = rng.uniform(-lim, lim, size=shp)
    return p


def conv3x3(x: np.ndarray, w: np.ndarray, b: np.ndarray, stride: int = 1) -> np.ndarray:
    """y[n, o, i, j] = b[o] + sum_{c, di, dj} w[o, c, di, dj] x[n, c, s i + di - 1, s j + dj - 1] (zero padding)."""
    n, c, h, wd = x.shape
    xp = np.pad(x, ((0, 0), (0, 0), (1, 1), (1, 1)))
    ho, wo = (h - 1) // stride + 1, (wd - 1) // stride + 1
    y = np.zeros((n, w.shape[0], ho, wo))
    for di in range(3):
        for dj in range(3):
            patch = xp[:, :, di:di + stride * (ho - 1) + 1:stride, dj:dj + stride * (wo - 1) + 1:stride]
            y += np.einsum("nchw,oc->nohw", patch, w[:, :, di, dj])
    return y + b[None, :, None, None]


def conv3x3_backward(x, w, gy, stride: int = 1):
    """Gradients ``(gx, gw, gb)`` of :func:`conv3x3` for the output gradient ``gy``."""
    n, c, h, wd = x.shape
    ho, wo = gy.shape[2], gy.shape[3]
    xp = np.pad(x, ((0, 0), (0, 0), (1, 1), (1, 1)))
    gxp = np.zeros_like(xp)
    gw = np.zeros_like(w)
    for di in range(3):
        for dj in range(3):
            sl = (slice(None), slice(None), slice(di, di + stride * (ho - 1) + 1, stride),
                  slice(dj, dj + stride * (wo - 1) + 1, stride))
            gw[:, :, di, dj] = np.einsum("nohw,nchw->oc", gy, xp[sl])
            gxp[sl] += np.einsum("nohw,oc->nchw", gy, w[:, :, di, dj])
    gb = gy.sum(axis=(0, 2, 3))
    return gxp[:, :, 1:-1, 1:-1], gw, gb


def forward(p: dict, x: np.ndarray):
    """Predictions ``[B, K]`` and the cache of intermediate values."""
    a1 = conv3x3(x, p["w1"], p["b1"])
    h1 = np.maximum(a1, 0.0)
    a2 = conv3x3(h1, p["w2"], p["b2"])
    h2 = np.maximum(a2, 0.0)
    a3 = conv3x3(h2, p["w3"], p["b3"], stride=2)
    h3 = np.maximum(a3, 0.0)
    g = h3.mean(axis=(2, 3))
    y = g @ p["wh"].T + p["bh"]
    return y, (x, a1, h1, a2, h2, a3, h3, g)


def loss_and_grads(p: dict, x: np.ndarray, t: np.ndarray):
    """Mean squared error over all ``B * K`` outputs and its gradients."""
    y, (x, a1, h1, a2, h2, a3, h3, g) = forward(p, x)
    bsz, k = y.shape
    d = y - t
    loss = float(np.mean(d * d))
    gy = 2.0 * d / (bsz * k)
    grads = {"wh": gy.T @ g, "bh": gy.sum(axis=0)}
    gg = gy @ p["wh"]
    gh3 = np.broadcast_to(gg[:, :, None, None] / (h3.shape[2] * h3.shape[3]), h3.shape)
    ga3 = gh3 * (a3 > 0)
    gh2, grads["w3"], grads["b3"] = conv3x3_backward(h2, p["w3"], ga3, stride=2)
    ga2 = gh2 * (a2 > 0)
    gh1, grads["w2"], grads["b2"] = conv3x3_backward(h1, p["w2"], ga2)
    ga1 = gh1 * (a1 > 0)
    _, grads["w1"], grads["b1"] = conv3x3_backward(x, p["w1"], ga1)
    return loss, grads


def adam_step(p: dict, m: dict, v: dict, grads: dict, step: int, lr: float = 1e-3,
              beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
    """One Adam update (Kingma and Ba) of the float64 master weights, in place."""
    for name in p:
        m[name] = beta1 * m[name] + (1 - beta1) * grads[name]
        v[name] = beta2 * v[name] + (1 - beta2) * grads[name] ** 2
        mh = m[name] / (1 - beta1 ** step)
        vh = v[name] / (1 - beta2 ** step)
        p[name] = p[name] - lr * mh / (np.sqrt(vh) + eps)


def coefficient_levels(s: int, levels: int) -> np.ndarray:
    """Level of each coefficient of an ``s x s`` tile: the finer of its two
    per-dimension levels (1 = finest); a sample index counts as coarser than
    any level, so pure samples get a level above ``levels``."""
    lev = np.full(s, levels + 1, dtype=np.int64)
    for i in range(s):
        if i % (1 << levels):
            lev[i] = 1 + (i & -i).bit_length() - 1
    return np.minimum(lev[:, None], lev[None, :])


def raw_features(coef: np.ndarray, levels: int) -> np.ndarray:
    """The patch features of coefficient tiles ``[B, 9, s, s]`` (64 x 64
    patches): the stride-8 coefficients and, per field, the energy of the
    level 1, 2 and 3 coefficients of every 8 x 8 block, ``[B, 36, 8, 8]``."""
    c = np.asarray(coef, dtype=np.float64)
    b, m = c.shape[0], c.shape[1]
    out = np.zeros((b, 4 * m, SIDE, SIDE))
    out[:, :m] = c[:, :, 0:SIDE * 8:8, 0:SIDE * 8:8]
    lev = coefficient_levels(c.shape[-1], levels)[:SIDE * 8, :SIDE * 8]
    sq = c[:, :, :SIDE * 8, :SIDE * 8] ** 2
    for f in range(m):
        for lv in (1, 2, 3):
            e = np.where(lev == lv, sq[:, f], 0.0)
            out[:, m + 3 * f + lv - 1] = e.reshape(b, SIDE, 8, SIDE, 8).sum(axis=(2, 4))
    return out


def input_map(raw: np.ndarray) -> np.ndarray:
    """The network's input map of raw features ``[B, 36, 8, 8]`` -> ``[B, 12, 8, 8]``."""
    r = np.asarray(raw, dtype=np.float64)
    m = C_FIELDS
    x = np.empty((r.shape[0], C_IN, SIDE, SIDE))
    x[:, :m] = np.arcsinh(r[:, :m] / FEATURE_SCALE)
    for lv in range(3):
        e = sum(r[:, m + 3 * f + lv] for f in range(m))
        x[:, m + lv] = np.arcsinh(np.sqrt(e) / FEATURE_SCALE)
    return x


def features(coef: np.ndarray, levels: int = 5) -> np.ndarray:
    """Network input of coefficient tiles ``[B, 9, s, s]`` (the input map of their raw features)."""
    return input_map(raw_features(coef, levels))


def choose_thresholds(pred: np.ndarray, candidates, budget_log10: np.ndarray, fallback: float) -> np.ndarray:
    """Per patch, the largest candidate whose predicted log10 squared error is
    within the patch's budget; the fixed threshold where none is."""
    cand = np.asarray(candidates, dtype=np.float64)
    ok = pred <= budget_log10[:, None]
    out = np.full(pred.shape[0], fallback, dtype=np.float64)
    for q in range(pred.shape[0]):
        idx = np.flatnonzero(ok[q])
        if idx.size:
            out[q] = cand[idx].max()
    return out
