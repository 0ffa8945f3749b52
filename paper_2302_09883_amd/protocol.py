"""The paper's own measurement protocol on the transport test, run on the GPU.

Section 3.2 (transport simulation, compression, methodology and results):
a 128 x 128 grid split into four 64 x 64 patches (65 x 65 folded BL5/3
tiles), the upwind finite-volume scheme with speed (0.9, 0.9) and CFL 0.45,
a compression-decompression cycle between every two steps, and

* the compression ratio at every step (the paper's Fig. 4, CSR curve),
* the compression ratio averaged over the run against the threshold
  {0, 0.0025, 0.005, 0.01, 0.02, 0.04} and the compression level (Fig. 5),
* the L2 error of equation "L2_error" (cell area times the sum of squared
  differences, no square root) against the exact solution at t = 0.5 (Fig. 6),

for every threshold rule of Section 2.2 (constant, accumulation, capped).
Two ratios are reported: the library's own store (values + u16 index list or
bitmask + offset table) and the CSR equivalent the paper measured (per tile
matrix: 4-byte column indices, S + 1 row pointers, the values).

Readings (the paper does not state them): the domain is the periodic square
[-1, 1)^2 with the Gaussian at its centre, values at the cell centres, the
computation in float64; with dt = CFL h / max(alpha, beta), t = 0.5 takes
n / 2 steps.  The paper's levels 5 and 6 need more than the BL5/3 level cap
(J - 1 = 5 for 64-cell patches) allows, so the sweep stops at level 5.

Everything runs through the C ABI of ``liblbmz``; this module only loops
over the sweep and does the bookkeeping on the host.
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np

N = 128
PATCH = 64
VEL = (0.9, 0.9)
CFL = 0.45
T_END = 0.5
LO, HI = -1.0, 1.0
LEVELS = (1, 2, 3, 4, 5)
THRESHOLDS = (0.0, 0.0025, 0.005, 0.01, 0.02, 0.04)
RULES = ("constant", "accum", "capped")


def steps_to(t_end: float = T_END, n: int = N) -> int:
    """Number of steps of dt = CFL h / max(|alpha|, |beta|) that reach t_end."""
    h = (HI - LO) / n
    dt = CFL * h / max(abs(VEL[0]), abs(VEL[1]))
    k = t_end / dt
    if abs(k - round(k)) > 1e-9:
        raise ValueError("t_end is not a whole number of steps")
    return int(round(k))


def csr_bytes(table: np.ndarray, s: int, value_bytes: int) -> int:
    """Bytes of the same coefficients as one CSR matrix per (patch, field)
    tile: ``nnz`` values and 4-byte column indices plus ``s + 1`` 4-byte row
    pointers."""
    nnz = (table[..., 1].astype(np.int64) & 0x7FFFFFFF)
    return int(nnz.sum()) * (value_bytes + 4) + table[..., 1].size * 4 * (s + 1)


def l2_paper(sim: np.ndarray, exact: np.ndarray) -> float:
    """Equation "L2_error": cell area times the sum of squared differences."""
    h = (HI - LO) / sim.shape[-1]
    return float(h * h * np.sum((sim - exact) ** 2))


def run_point(level: int, thr: float, rule: str, n: int = N, dtype: str = "f64", keep_series: bool = True):
    """One sweep point: the whole run, with the ratios after every step."""
    from synth import transport_gaussian

    from .lbmz import Context

    steps = steps_to(T_END, n)
    f0 = transport_gaussian(n, 0.0, VEL, LO, HI)
    exact = transport_gaussian(n, T_END, VEL, LO, HI)
    vb = 8 if dtype == "f64" else 4
    ctx = Context(n, scheme="fv_upwind", dtype=dtype, p=PATCH, wavelet="bl53", levels=level, eps=thr,
                  rule=rule, vel=VEL, cfl=CFL)
    try:
        ctx.set_field(0, f0.astype(np.float64 if dtype == "f64" else np.float32))
        dense = n * n * vb
        ratio, ratio_csr, nnz = [], [], []
        for _ in range(steps):
            ctx.step(1)
            st = ctx.stats()
            table, _ = ctx.store()
            ratio.append(st["ratio"])
            ratio_csr.append(dense / csr_bytes(table, ctx.s, vb))
            nnz.append(int(st["nnz_total"]))
        sim = ctx.fields()[0].astype(np.float64)
        tot = ctx.stats()["totals"][0]
    finally:
        ctx.close()
    out = {
        "level": level, "threshold": thr, "rule": rule, "steps": steps,
        "ratio_mean": float(np.mean(ratio)), "ratio_final": float(ratio[-1]),
        "csr_ratio_mean": float(np.mean(ratio_csr)), "csr_ratio_final": float(ratio_csr[-1]),
        "l2_exact": l2_paper(sim, exact), "total": float(tot),
    }
    if keep_series:
        out["ratio_series"] = ratio
        out["csr_ratio_series"] = ratio_csr
        out["nnz_series"] = nnz
    out["_field"] = sim
    return out


def sweep(levels=LEVELS, thresholds=THRESHOLDS, rules=RULES, n: int = N, dtype: str = "f64"):
    """The full grid of points, plus the uncompressed run's error for context."""
    from .lbmz import Context
    from synth import transport_gaussian

    steps = steps_to(T_END, n)
    ref = Context(n, scheme="fv_upwind", dtype=dtype, reference=True, vel=VEL, cfl=CFL)
    try:
        ref.set_field(0, transport_gaussian(n, 0.0, VEL, LO, HI))
        ref.step(steps)
        plain = ref.fields()[0].astype(np.float64)
    finally:
        ref.close()
    exact = transport_gaussian(n, T_END, VEL, LO, HI)
    points = []
    for rule in rules:
        for level in levels:
            for thr in thresholds:
                p = run_point(level, thr, rule, n, dtype, keep_series=False)
                sim = p.pop("_field")
                p["rel_l2_vs_plain"] = float(np.linalg.norm(sim - plain) / np.linalg.norm(plain))
                points.append(p)
    return {"grid": n, "patch": PATCH, "steps": steps, "dtype": dtype, "l2_exact_uncompressed": l2_paper(plain, exact),
            "points": points}


def main(argv=None):
    ap = argparse.ArgumentParser(description="paper-protocol sweep on the transport test (GPU)")
    ap.add_argument("--dtype", default="f64", choices=("f64", "f32"))
    ap.add_argument("--json", default=None, help="write the full result here")
    args = ap.parse_args(argv)
    t0 = time.perf_counter()
    res = sweep(dtype=args.dtype)
    res["seconds"] = time.perf_counter() - t0
    if args.json:
        with open(args.json, "w") as fh:
            json.dump(res, fh, indent=1)
    print(f"transport {res['grid']}^2, {res['steps']} steps to t = {T_END}, {res['dtype']}; "
          f"L2 (paper) of the uncompressed run vs exact: {res['l2_exact_uncompressed']:.4e}")
    for rule in RULES:
        print(f"\nrule {rule}: mean ratio own store / CSR equivalent; L2 vs exact at t = {T_END}")
        print("level " + "".join(f"  thr={t:<7g}" + " " * 14 for t in THRESHOLDS))
        for level in LEVELS:
            row = [p for p in res["points"] if p["rule"] == rule and p["level"] == level]
            cells = "".join(f"  {p['ratio_mean']:7.1f} / {p['csr_ratio_mean']:6.1f}  {p['l2_exact']:.2e}" for p in row)
            print(f"{level:5d}" + cells)
    print(f"\n{res['seconds']:.1f} s")
    return 0


if __name__ == "__main__":
    sys.exit(main())
