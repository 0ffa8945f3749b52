"""Measurement of the 3-D D3Q19 patch loop.

Workload (default): 768^3 periodic grid, 32^3 patches (13,824), folded BL5/3
with L = 3, capped threshold eps = 1e-4, tau = 0.55, a Taylor--Green vortex
plus seeded jets (``synth.taylor_green_jets_3d``).  Reports MLUPS including
decompression and compression (HIP-event time of the step launches and wall
clock), the compression ratio, the error against the uncompressed D3Q19 run
of the same number of steps, the drift of the conserved totals, and the
roofline figures of the step kernel.

    python -m paper_2302_09883_amd.d3q19 [--n 768] [--steps 200] [--eps 1e-4]
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0
# MI355X's published FP32 vector peak (packed FP32), and the rate without
# packed-FP32 instructions, which this build does not emit
VALU_PEAK_TFLOPS = 157.3
VALU_PEAK_NONPACKED_TFLOPS = 256 * 64 * 2 * 2.4e9 / 1e12
C = np.array([(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1), (1, 1, 0),
              (-1, -1, 0), (1, -1, 0), (-1, 1, 0), (1, 0, 1), (-1, 0, -1), (1, 0, -1), (-1, 0, 1), (0, 1, 1),
              (0, -1, -1), (0, 1, -1), (0, -1, 1)], dtype=np.float64)


def line_flops(s: int, levels: int) -> int:
    """FP32 flops of one multi-level folded BL5/3 pass over a line of s nodes
    (3 per predicted detail, 4 per updated interior sample)."""
    tot = 0
    for lev in range(1, levels + 1):
        m = (s - 1) >> lev
        tot += 3 * m + 4 * (m - 1)
    return tot


def flops_per_patch3(p: int, levels: int) -> int:
    """Algorithmic FP32 flops of one patch step: three 3-D transforms (inverse,
    forward, re-inverse) of 19 populations, each 3 directions x s^2 lines, plus
    the collision of every tile node (57 flops of moments and velocity, 10 per
    population for the equilibrium and the relaxation: 247)."""
    s = p + 1
    return 3 * 19 * 3 * s * s * line_flops(s, levels) + 247 * s ** 3


def halo_bytes3(npatch: int, p: int) -> int:
    """Halo floats written (and read) per step: six faces of five populations
    and twelve edge lines of one population per patch."""
    s = p + 1
    return npatch * (6 * 5 * s * s + 12 * s) * 4


def _say(msg: str):
    print("[d3q19]", msg, file=sys.stderr, flush=True)


def _error_on_device(ctx, ref, nfields: int = 19):
    import torch
    n = ctx.n
    a = torch.empty((n, n, n), dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    sd = sr = 0.0
    mx = 0.0
    for f in range(nfields):
        ctx.decompress_field(f, out=a)
        ref.decompress_field(f, out=b)
        d = (a.double() - b.double())
        sd += float((d * d).sum())
        sr += float((b.double() ** 2).sum())
        mx = max(mx, float(d.abs().max()))
    return float(np.sqrt(sd / sr)), mx, (1.0 / n) ** 3 * sd


def run(n: int = 768, p: int = 32, levels: int = 3, eps: float = 1e-4, tau: float = 0.55, steps: int = 200,
        warmup: int = 5, seed: int = 0, reference: bool = True, copy_calibration: bool = False) -> dict:
    import torch

    if copy_calibration:
        # three plain 256 MiB device copies: the reference kernel of known
        # traffic for scaling the memory counters of a profiled run
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    from paper_2302_09883_amd import Context
    from synth import taylor_green_jets_3d

    t_setup = time.perf_counter()
    macro = taylor_green_jets_3d(n, seed=seed, dtype=np.float32)
    ctx = Context(n, scheme="d3q19_bgk", dtype="f32", p=p, wavelet="bl53", levels=levels, eps=eps, tau=tau)
    ctx.set_macroscopic(*macro)
    t_setup = time.perf_counter() - t_setup
    _say(f"set-up done in {t_setup:.1f} s")
    ctx.step(warmup)
    s0 = ctx.stats()
    t0_tot = ctx.totals()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.step(steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    s1 = ctx.stats()
    t1_tot = ctx.totals()
    ev_ms = s1["ms_last_call"]
    npatch = (n // p) ** 3
    store_avg = 0.5 * (s0["store_bytes"] + s1["store_bytes"])
    bytes_launch = 2.0 * store_avg + 2.0 * halo_bytes3(npatch, p)
    flops_launch = float(flops_per_patch3(p, levels)) * npatch
    k_ms = ev_ms / steps
    out = {
        "workload": f"D3Q19 BGK {n}^3, {p}^3 patches, BL5/3 L={levels}, eps={eps}, tau={tau}, "
                    "Taylor-Green + jets",
        "steps": steps, "warmup": warmup,
        "mlups": n ** 3 * steps / wall / 1e6,
        "mlups_events": n ** 3 * steps / (ev_ms * 1e-3) / 1e6,
        "kernel_ms_avg": k_ms,
        "ratio": s1["ratio"],
        "store_bytes": s1["store_bytes"],
        "rho_nz": s1["nnz_total"] / (npatch * 19 * (p + 1) ** 3),
        "regrows": s1["regrows"],
        "mass_drift": float(t1_tot.sum() / t0_tot.sum() - 1.0),
        "momentum_drift": float(np.max(np.abs(t1_tot @ C - t0_tot @ C)) / t0_tot.sum()),
        "setup_s": t_setup,
        "roofline": {
            "bytes_per_launch": bytes_launch,
            "flops_per_launch": flops_launch,
            "hbm_gbs": bytes_launch / (k_ms * 1e-3) / 1e9,
            "hbm_frac": bytes_launch / (k_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "tflops": flops_launch / (k_ms * 1e-3) / 1e12,
            "alu_frac": flops_launch / (k_ms * 1e-3) / 1e12 / VALU_PEAK_TFLOPS,
            "alu_frac_nonpacked": flops_launch / (k_ms * 1e-3) / 1e12 / VALU_PEAK_NONPACKED_TFLOPS,
        },
    }
    _say(f"{steps} timed steps: {k_ms:.3f} ms per step")
    if reference:
        ref = Context(n, scheme="d3q19_bgk", dtype="f32", tau=tau, reference=True)
        ref.set_macroscopic(*macro)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ref.step(warmup + steps)
        torch.cuda.synchronize()
        out["reference_mlups"] = n ** 3 * (warmup + steps) / (time.perf_counter() - t0) / 1e6
        rel, linf, paper = _error_on_device(ctx, ref)
        out.update({"rel_l2": rel, "linf": linf, "paper_l2": paper})
        ref.close()
    ctx.close()
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--n", type=int, default=768)
    ap.add_argument("--p", type=int, default=32)
    ap.add_argument("--levels", type=int, default=3)
    ap.add_argument("--eps", type=float, default=1e-4)
    ap.add_argument("--tau", type=float, default=0.55)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-reference", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run plain 256 MiB device copies (the reference kernel for counter scaling)")
    a = ap.parse_args()
    res = run(a.n, a.p, a.levels, a.eps, a.tau, a.steps, a.warmup, a.seed, not a.no_reference, a.copy_calibration)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
