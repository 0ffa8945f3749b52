"""Execution modes and patch shapes of the step on the hot-path workloads (GPU).

For each workload the autotuner of the library times the four modes -- one
workgroup per patch or a persistent work-queue kernel, plain launches or HIP
graph chunks -- on the real state (the modes compute identical records) and
keeps the fastest.  Workloads: the 256^2 upwind-transport run (64 patches of
32^2, Haar, 4 levels, float64: launch-bound) and the 2048^2 D2Q9 run (1024
patches of 64^2, BL5/3, 5 levels, float32).
"""
from __future__ import annotations

import argparse
import json
import sys

import numpy as np


def measure(steps_per_variant: int = 10):
    from synth import fv_gaussians_and_step, shear_layer_macroscopic

    from .lbmz import Context

    out = {}
    c = Context(256, scheme="fv_upwind", dtype="f64", p=32, wavelet="haar", levels=4, eps=1e-4)
    c.set_field(0, fv_gaussians_and_step(256, seed=0))
    ms = c.autotune(steps_per_variant)
    out["transport_256_f64"] = {"ms_per_step": [float(v) for v in ms], "chosen": c.execution()}
    c.close()
    n = 2048
    c = Context(n, scheme="d2q9_bgk", dtype="f32", p=64, wavelet="bl53", levels=5, eps=1e-4, tau=0.6)
    rho, ux, uy = shear_layer_macroscopic(n, seed=0)
    c.set_macroscopic(*(a.astype(np.float32) for a in (rho, ux, uy)))
    ms = c.autotune(steps_per_variant)
    out["d2q9_2048_f32"] = {"ms_per_step": [float(v) for v in ms], "chosen": c.execution()}
    c.close()
    return out


# Patch shapes of the D2Q9 workload the shape tuner compares: patch side and
# its level count (the folded BL5/3 cap J - 1, so that each shape compresses
# as deeply as it can).
SHAPES = ((64, 5), (32, 4))


def tune_patch_shape(n: int = 2048, eps: float = 1e-4, steps: int = 60, tune_steps: int = 3, shapes=SHAPES,
                     tol: float = 0.25, seed: int = 0):
    """Patch-shape tuner of the D2Q9 workload: for every patch shape, the
    library's mode autotuner runs first (8 x ``tune_steps`` steps), then
    ``steps`` steps are timed (HIP events) and the state is compared with the
    uncompressed run of the same length.  Shapes are compared at equal error:
    the tuner keeps the fastest shape whose relative L2 error is within
    ``1 + tol`` of the smallest error of the shapes (a shape that is faster
    only because it compresses more loosely does not win).  Returns the
    measurements and the choice."""
    import torch

    from synth import shear_layer_macroscopic

    from .lbmz import Context

    rho, ux, uy = shear_layer_macroscopic(n, seed=seed)
    macro = [a.astype(np.float32) for a in (rho, ux, uy)]
    total = 8 * tune_steps + steps
    ref = Context(n, scheme="d2q9_bgk", dtype="f32", tau=0.6, reference=True)
    ref.set_macroscopic(*macro)
    ref.step(total)
    truth = torch.empty((9, n, n), dtype=torch.float32, device="cuda")
    for f in range(9):
        ref.decompress_field(f, out=truth[f])
    ref.close()
    got = torch.empty_like(truth)
    out = []
    for p, levels in shapes:
        c = Context(n, scheme="d2q9_bgk", dtype="f32", p=p, wavelet="bl53", levels=levels, eps=eps, tau=0.6)
        c.set_macroscopic(*macro)
        ms = c.autotune(tune_steps)
        mode = c.execution()
        c.step(steps)
        st = c.stats()
        for f in range(9):
            c.decompress_field(f, out=got[f])
        rel = float(((got.double() - truth.double()) ** 2).sum().sqrt() / (truth.double() ** 2).sum().sqrt())
        out.append({"patch": p, "levels": levels, "mlups_events": n * n * steps / (st["ms_last_call"] * 1e-3) / 1e6,
                    "ratio": st["ratio"], "rel_l2": rel, "persistent": mode[0], "graph": mode[1],
                    "autotune_ms_per_step": [round(float(v), 5) for v in ms]})
        c.close()
    best_err = min(r["rel_l2"] for r in out)
    ok = [r for r in out if r["rel_l2"] <= (1.0 + tol) * best_err]
    chosen = max(ok, key=lambda r: r["mlups_events"])
    return {"eps": eps, "steps": steps, "tolerance": tol, "shapes": out,
            "chosen": {"patch": chosen["patch"], "levels": chosen["levels"], "persistent": chosen["persistent"],
                       "graph": chosen["graph"]}}


def main(argv=None):
    ap = argparse.ArgumentParser(description="execution modes of the step (GPU)")
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--shapes", action="store_true", help="also run the patch-shape tuner on the D2Q9 workload")
    args = ap.parse_args(argv)
    if args.shapes:
        tuned = tune_patch_shape()
        for r in tuned["shapes"]:
            print(f"patch {r['patch']:3d} L={r['levels']}: {r['mlups_events']:9.0f} MLUPS  ratio {r['ratio']:7.1f}  "
                  f"rel_l2 {r['rel_l2']:.3e}  persistent={r['persistent']} graph={r['graph']}")
        print("chosen", tuned["chosen"])
    res = measure(args.steps)
    names = ("plain", "graph", "persistent", "persistent+graph")
    for w, r in res.items():
        cells = "  ".join(f"{nm} {1e3 * v:8.2f} us" for nm, v in zip(names, r["ms_per_step"]))
        print(f"{w:20s} {cells}   chosen persistent={r['chosen'][0]} graph={r['chosen'][1]}")
    print(json.dumps(res))
    return 0


if __name__ == "__main__":
    sys.exit(main())
