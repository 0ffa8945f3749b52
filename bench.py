#!/usr/bin/env python
"""Benchmark of the compressed patch loop on one MI355X.

Workload (the lattice-Boltzmann configuration): D2Q9 BGK, tau = 0.6, float32
populations, 2048 x 2048 periodic grid, 64 x 64 patches (1024 patches of
65 x 65 shared-border tiles), folded BL5/3 wavelet with 5 levels, capped
threshold, eps swept over {1e-5, 1e-4, 1e-3, 3e-3, 1e-2}; initial state:
double shear layer at equilibrium (seed 0).  A "step" is one time step of the
whole hot path over all patches: one launch of the fused patch kernel.

Every sweep point times ``--steps`` steps after the warm-up and then runs on
to the workload's length of 1000 steps (counted from the initial state), where
its error against the uncompressed run of the same length is taken.  The two
largest thresholds are there to bracket the 1e-3 error target when the flow
allows it; on this smooth flow every threshold from 1e-3 up drops every detail
coefficient, the error saturates below 1e-3 and the largest ratio is
reported with a note.

Printed: one JSON line with MLUPS at the primary eps (1e-4) including the
decompression and recompression, the sweep's compression ratios and errors,
the compression ratio at fixed relative L2 errors, a roofline object for the
fused kernel, the HBM-bound operating points (eps = 0) and the CPU oracle's
throughput on a bounded sample (one core and all available cores).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

N = 2048
P = 64
LEVELS = 5
TAU = 0.6
SEED = 0
PRIMARY_EPS = 1e-4
TARGET_REL_L2 = (1e-3, 5e-4)   # the learned-part error budget, and one inside the swept range

ERROR_STEPS = 1000              # the workload's length: errors are taken after this many steps
DEFAULT_EPS = (1e-5, 1e-4, 1e-3, 3e-3, 1e-2)

HBM_PEAK_GBS = 8000.0
# MI355X's published FP32 vector peak (packed FP32: 256 CUs x 64 lanes x 2
# FMA x 2 flops x 2.4 GHz), and the rate without packed-FP32 instructions,
# which this build does not emit (256 x 64 x 2 x 2.4 GHz).
VALU_PEAK_TFLOPS = 157.3
VALU_PEAK_NONPACKED_TFLOPS = 256 * 64 * 2 * 2.4e9 / 1e12


def line_flops(s: int, levels: int) -> int:
    """FP32 flops of one multi-level folded BL5/3 pass over a line of s = 2^J + 1 nodes.

    Per level with m details: predict = add + fused multiply-add (3 flops) per
    detail, update = two fused multiply-adds (4 flops) per interior sample.
    """
    tot = 0
    for lev in range(1, levels + 1):
        m = (s - 1) >> lev
        tot += 3 * m + 4 * (m - 1)
    return tot


def flops_per_patch(p: int = P, levels: int = LEVELS, nfields: int = 9) -> int:
    """Algorithmic FP32 flops of one patch step: the inverse (S2) and forward
    (S5) 2-D transforms of every field; for the export (S8) the column half of
    the re-inverse, the two edge values of every row of the 6 populations that
    cross the x faces (7 flops per level: an update of two fused multiply-adds
    and a predict of an add and a fused multiply-add) and the full inverse of
    the 6 exported rows; plus the D2Q9 collision of every node (126 flops: 18
    for the moments, 9 for the velocity, 99 for the nine equilibria and
    relaxations)."""
    s = p + 1
    lf = line_flops(s, levels)
    transforms = 2 * nfields * 2 * s * lf + nfields * s * lf
    export = 6 * s * 7 * levels + 6 * lf
    return transforms + export + 126 * s * s


def halo_bytes(npatch: int) -> int:
    """Halo strips written (and read) per step: 4 sides x 3 populations x 65 nodes x 4 B per patch."""
    return npatch * 4 * 3 * (P + 1) * 4


KERNEL_SOURCES = ["paper_2302_09883_amd/csrc/lbmz_patch_kernel.h", "paper_2302_09883_amd/csrc/lbmz_internal.h",
                  "paper_2302_09883_amd/csrc/lbmz_inst_f32_lbm.hip"]
TRAFFIC_FILE = "profiles/traffic_patch_step_d2q9_2048_eps1e-4.txt"


def kernel_source_digest() -> str:
    """First 16 hex digits of the SHA-256 of the kernel sources' code: line
    comments, trailing blanks and empty lines are dropped, so that a change of
    comments alone does not mark measured counters as stale."""
    import hashlib
    import re
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), encoding="utf-8") as fh:
            for line in fh:
                code = re.sub(r"//.*$", "", line).rstrip()
                if code:
                    h.update(code.encode("utf-8") + b"\n")
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per step-kernel launch from the committed counter summary.

    The summary holds FETCH_SIZE + WRITE_SIZE of the step kernel, scaled by what
    the same counters read for a plain copy of known size, and the digest of the
    kernel sources it was taken on; None when the kernel has changed since.
    """
    path = os.path.join(ROOT, TRAFFIC_FILE)
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as fh:
        for ln in fh:
            parts = ln.split()
            if len(parts) >= 2 and not ln.startswith("#"):
                kv[parts[0]] = parts[1]
    if kv.get("source_digest") != kernel_source_digest():
        return None
    return int(float(kv["bytes_per_launch"]))


TUNE_STEPS = 3   # steps per autotuner variant (8 x this many steps before the warm-up)


def bytes_model(rho_nz: float, npatch: int, p: int = P) -> float:
    """Algorithmic HBM bytes of one step at stored density ``rho_nz``: each
    record read once and written once (values plus the u16 index list, 6 B per
    kept coefficient, below density 1/16, else the values plus the bitmask,
    4 rho + 1/8 B per coefficient), the halo strips written and read, the
    offset table read and written."""
    s = p + 1
    per_coef = 6.0 * rho_nz if rho_nz < 1.0 / 16 else 4.0 * rho_nz + 0.125
    records = npatch * 9 * s * s * per_coef
    return 2.0 * records + 2.0 * halo_bytes(npatch) + 2.0 * npatch * 9 * 8


def run_point(eps: float, steps: int, warmup: int, macro, ref_state, error_steps: int, autotune: bool = True):
    import torch

    from paper_2302_09883_amd import Context

    ctx = Context(N, scheme="d2q9_bgk", dtype="f32", p=P, wavelet="bl53", levels=LEVELS, eps=eps, tau=TAU)
    ctx.set_macroscopic(*macro)
    tune_ms = None
    if autotune:
        tune_ms = [round(float(v), 5) for v in ctx.autotune(TUNE_STEPS)]
    mode = ctx.execution()
    ctx.step(warmup)
    s0 = ctx.stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.step(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    s1 = ctx.stats()
    wall = t1 - t0
    ev_ms = s1["ms_last_call"]
    npatch = (N // P) ** 2
    ncoef = npatch * 9 * (P + 1) ** 2
    rho1 = s1["nnz_total"] / ncoef
    # measured bytes: both stores as they are (start and end of the timed steps)
    store_avg = 0.5 * (s0["store_bytes"] + s1["store_bytes"])
    bytes_launch = 2.0 * store_avg + 2.0 * halo_bytes(npatch)
    ctx.step(max(0, error_steps - s1["steps"]))
    s2 = ctx.stats()
    state = ctx.fields()
    d = state.astype(np.float64) - ref_state
    rel = float(np.linalg.norm(d) / np.linalg.norm(ref_state))
    linf = float(np.max(np.abs(d)))
    paper_l2 = float((1.0 / N) ** 2 * np.sum(d * d))
    out = {
        "eps": eps,
        "mlups": N * N * steps / wall / 1e6,
        "mlups_events": N * N * steps / (ev_ms * 1e-3) / 1e6,
        "ms_per_step": wall * 1e3 / steps,
        "kernel_ms_avg": ev_ms / steps,
        "ratio": s1["ratio"],
        "ratio_at_error_step": s2["ratio"],
        "store_bytes": s1["store_bytes"],
        "rho_nz": rho1,
        "error_steps": s2["steps"],
        "rel_l2": rel,
        "linf": linf,
        "paper_l2": paper_l2,
        "bytes_per_launch": bytes_launch,
        "bytes_model": bytes_model(rho1, npatch),
        "regrows": s2["regrows"],
        "execution": {"persistent": mode[0], "graph": mode[1], "autotune_ms_per_step": tune_ms},
        "mass_drift": (sum(s2["totals"])) / (sum(s0["totals"])) - 1.0,
    }
    ctx.close()
    return out


def reference_state(macro, total_steps: int):
    import torch

    from paper_2302_09883_amd import Context

    ref = Context(N, scheme="d2q9_bgk", dtype="f32", reference=True, tau=TAU)
    ref.set_macroscopic(*macro)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ref.step(total_steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st = ref.fields().astype(np.float64)
    mlups = N * N * total_steps / (t1 - t0) / 1e6
    ref.close()
    return st, mlups


def cr_at_error(points, target):
    """Compression ratio at a relative L2 error.

    Log-log interpolation between the two swept thresholds whose errors
    bracket ``target``.  When every swept threshold stays below the target the
    answer is the largest swept ratio (at the largest thresholds every detail
    coefficient is dropped and the ratio saturates); when none does, None.
    """
    pts = sorted((p["rel_l2"], p["ratio"], p["eps"]) for p in points if p["rel_l2"] > 0)
    for (e0, c0, k0), (e1, c1, k1) in zip(pts, pts[1:]):
        if e0 <= target <= e1 and e1 > e0:
            w = (math.log(target) - math.log(e0)) / (math.log(e1) - math.log(e0))
            return {"target_rel_l2": target, "ratio": round(math.exp(math.log(c0) + w * (math.log(c1) - math.log(c0))), 2),
                    "bracket_eps": [k0, k1]}
    if pts and all(e <= target for e, _, _ in pts):
        best = max(pts, key=lambda t: t[1])
        return {"target_rel_l2": target, "ratio": round(best[1], 2), "bracket_eps": None,
                "note": f"every swept eps meets the target; largest ratio at eps={best[2]} "
                        f"(rel_l2 {best[0]:.3g})"}
    return {"target_rel_l2": target, "ratio": None, "bracket_eps": None,
            "note": "no swept eps meets the target"}


def _sig(v, digits=6):
    return float(f"{v:.{digits}g}") if isinstance(v, float) else v


def _cpu_info():
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    return {"nproc": os.cpu_count(), "available": avail, "model": model}


# -- the oracle on several cores: a harness around it, parallel over patches --
# Workers hold the oracle run object and views of shared arrays; a step is
# (1) every worker rebuilds its patches' tiles (inverse transform), (2) the
# parent gathers the ghost rings of all tiles (the oracle's gather, serial),
# (3) every worker advances its patches (stencil, forward transform,
# threshold, record encoding).  The oracle itself is unchanged.
_CPU = {}


def _cpu_init(spec, n, eps):
    from multiprocessing import shared_memory

    from oracle import lbmz_oracle as O
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except Exception:   # noqa: BLE001 - elementwise NumPy is single-threaded anyway
        pass
    g = O.Geometry(n, P, O.BL53, LEVELS)
    _CPU["run"] = O.CompressedRun(g, O.Scheme("d2q9_bgk", tau=TAU), eps, O.RULE_CAPPED, np.float32)
    _CPU["O"] = O
    for key, (name, shape) in spec.items():
        shm = shared_memory.SharedMemory(name=name)
        _CPU[key] = (shm, np.ndarray(shape, dtype=np.float32, buffer=shm.buf))


def _cpu_rebuild(span):
    lo, hi = span
    _CPU["lossy"][1][lo:hi] = _CPU["run"].decompress_tiles(_CPU["coef"][1][lo:hi])


def _cpu_advance(span):
    lo, hi = span
    run, O = _CPU["run"], _CPU["O"]
    c = run.compress_tiles(run.scheme.update(_CPU["padded"][1][lo:hi]).astype(np.float32))
    _CPU["coef"][1][lo:hi] = c
    for q in range(c.shape[0]):
        for f in range(9):
            O.encode_record(c[q, f])


def cpu_baseline(steps: int = 3, workers: int | None = None, n: int = N):
    """The oracle (float32 NumPy) on a bounded sample, on one core and on all
    available cores (at most 16).

    Sample: ``steps`` consecutive steps of the patch loop on the whole
    workload (state compressed from the same initial condition): inverse
    transform of every patch, ghost gathering, stencil, forward transform,
    threshold and record encoding.  Throughput in MLUPS over the owned cells.
    Must run before the GPU is initialised (the multi-core leg forks).
    """
    import multiprocessing as mp
    from multiprocessing import shared_memory

    from oracle import lbmz_oracle as O
    from synth import shear_layer_macroscopic

    rho, ux, uy = shear_layer_macroscopic(n, seed=SEED)
    grid = O.d2q9_equilibrium(rho, ux, uy).astype(np.float32)
    g = O.Geometry(n, P, O.BL53, LEVELS)
    run = O.CompressedRun(g, O.Scheme("d2q9_bgk", tau=TAU), PRIMARY_EPS, O.RULE_CAPPED, np.float32)
    coef0 = run.compress_tiles(O.extract_tiles(grid, g))
    cells = g.npatch * P * P * steps

    # one core: the oracle's own loop
    coef = coef0
    t0 = time.perf_counter()
    for _ in range(steps):
        padded = O.gather_ghosts(run.decompress_tiles(coef), g)
        coef = run.compress_tiles(run.scheme.update(padded).astype(np.float32))
        for q in range(g.npatch):
            for f in range(9):
                O.encode_record(coef[q, f])
    t1 = time.perf_counter() - t0
    info = _cpu_info()
    nw = workers or min(16, info["available"])

    # all cores: the harness above
    shapes = {"coef": coef0.shape, "lossy": coef0.shape, "padded": (g.npatch, 9, g.s + 2, g.s + 2)}
    shms = {k: shared_memory.SharedMemory(create=True, size=int(np.prod(v)) * 4) for k, v in shapes.items()}
    try:
        arr = {k: np.ndarray(shapes[k], dtype=np.float32, buffer=shms[k].buf) for k in shapes}
        arr["coef"][...] = coef0
        spec = {k: (shms[k].name, shapes[k]) for k in shapes}
        bounds = np.linspace(0, g.npatch, 4 * nw + 1).astype(int)
        spans = [(int(a), int(b)) for a, b in zip(bounds, bounds[1:]) if b > a]
        with mp.get_context("fork").Pool(nw, initializer=_cpu_init, initargs=(spec, n, PRIMARY_EPS)) as pool:
            pool.map(_cpu_rebuild, spans[:nw])            # warm the workers
            arr["coef"][...] = coef0
            t0 = time.perf_counter()
            for _ in range(steps):
                pool.map(_cpu_rebuild, spans)
                arr["padded"][...] = O.gather_ghosts(arr["lossy"], g)
                pool.map(_cpu_advance, spans)
            tn = time.perf_counter() - t0
        same = bool(np.array_equal(arr["coef"], coef))
        del arr
    finally:
        for shm in shms.values():
            shm.close()
            shm.unlink()
    return {"value": round(cells / tn / 1e6, 3), "unit": "MLUPS", "cores": nw, "kind": "oracle",
            "sample": f"{steps} consecutive steps of the whole {n}^2 D2Q9 workload ({g.npatch} patches of 64x64 cells) "
                      f"at eps={PRIMARY_EPS}, float32 NumPy oracle, patches split over {nw} worker processes "
                      f"(ghost gathering serial), {tn:.1f} s; the same steps on one core: {t1:.1f} s",
            "one_core": {"value": round(cells / t1 / 1e6, 3), "unit": "MLUPS", "cores": 1},
            "identical_results": same,
            "cpu": info}


def copy_calibration():
    """Three plain device copies of 256 MiB: the kernel of known traffic that
    the HBM byte counters are scaled by."""
    import torch

    src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst


def hbm_point(n: int, steps: int, warmup: int = 5):
    """The operating point bound by HBM bytes: eps = 0 keeps every coefficient
    (bitmask records, stored density ~0.96).  Plain launches, no error run.
    Bytes per launch from the byte model at the measured end-state density."""
    from paper_2302_09883_amd import Context
    from synth import shear_layer_macroscopic

    macro = [a.astype(np.float32) for a in shear_layer_macroscopic(n, seed=SEED)]
    ctx = Context(n, scheme="d2q9_bgk", dtype="f32", p=P, wavelet="bl53", levels=LEVELS, eps=0.0, tau=TAU)
    ctx.set_macroscopic(*macro)
    ctx.step(warmup)
    ctx.step(steps)
    s1 = ctx.stats()
    k_ms = s1["ms_last_call"] / steps
    npatch = (n // P) ** 2
    rho = s1["nnz_total"] / (npatch * 9 * (P + 1) ** 2)
    b = bytes_model(rho, npatch)
    gbs = b / (k_ms * 1e-3) / 1e9
    ctx.close()
    return {"grid": n, "eps": 0.0, "steps": steps, "kernel_ms_avg": _sig(k_ms),
            "mlups": _sig(n * n / (k_ms * 1e-3) / 1e6), "rho_nz": _sig(rho), "bytes_per_launch": round(b),
            "bytes_of_stores": round(2.0 * s1["store_bytes"] + 2.0 * halo_bytes(npatch)),
            "hbm_gbs": _sig(gbs), "hbm_frac": _sig(gbs / HBM_PEAK_GBS),
            "alu_frac": _sig(flops_per_patch() * npatch / (k_ms * 1e-3) / 1e12 / VALU_PEAK_TFLOPS)}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--eps", type=float, nargs="*", default=list(DEFAULT_EPS),
                    help="threshold sweep (eps=1e-4 is always run: it is the headline point)")
    ap.add_argument("--error-steps", type=int, default=ERROR_STEPS,
                    help="steps from the initial state after which errors are taken (at least the timed ones)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="time one workgroup per patch with plain launches instead of the autotuned mode")
    ap.add_argument("--cpu-steps", type=int, default=3)
    ap.add_argument("--no-hbm-points", action="store_true",
                    help="skip the eps=0 runs at 2048^2 and 4096^2 (the HBM-bound operating points)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 256 MiB device copy (the reference kernel for counter scaling)")
    ap.add_argument("--hbm-point", type=int, default=0, metavar="N",
                    help="profiling aid: run only the eps=0 operating point on an N x N grid for --steps steps "
                         "and print its figures (no bench line)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the compressed patch loop runs on a single MI355X "
              "(multi-GPU sharding is a design note only); run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    if args.hbm_point:
        import torch

        torch.cuda.set_device(0)
        if args.copy_calibration:
            copy_calibration()
        print(json.dumps(hbm_point(args.hbm_point, args.steps, args.warmup)), flush=True)
        return

    # the CPU leg first: its worker processes are forked before the GPU is touched
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(args.cpu_steps)

    import torch

    from synth import shear_layer_macroscopic

    torch.cuda.set_device(0)
    rho, ux, uy = shear_layer_macroscopic(N, seed=SEED)
    macro = tuple(a.astype(np.float32) for a in (rho, ux, uy))
    pre = (8 * TUNE_STEPS if not args.no_autotune else 0) + args.warmup
    total = max(args.error_steps, pre + args.steps)
    ref_state, ref_mlups = reference_state(macro, total)

    eps_list = list(dict.fromkeys(args.eps + [PRIMARY_EPS]))
    points = [run_point(e, args.steps, args.warmup, macro, ref_state, total, not args.no_autotune)
              for e in sorted(eps_list)]
    prim = next(p for p in points if p["eps"] == PRIMARY_EPS)

    npatch = (N // P) ** 2
    ksec = prim["kernel_ms_avg"] * 1e-3
    hbm_gbs = prim["bytes_per_launch"] / ksec / 1e9
    flops_launch = flops_per_patch() * npatch
    tflops = flops_launch / ksec / 1e12
    hbm_frac = hbm_gbs / HBM_PEAK_GBS
    alu_frac = tflops / VALU_PEAK_TFLOPS
    alu = {"achieved": round(tflops, 3), "peak": VALU_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": round(alu_frac, 4),
           "peak_nonpacked": round(VALU_PEAK_NONPACKED_TFLOPS, 1),
           "frac_nonpacked": round(tflops / VALU_PEAK_NONPACKED_TFLOPS, 4)}
    hbm = {"achieved": round(hbm_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(hbm_frac, 4)}
    if alu_frac >= hbm_frac:
        roof = {"bound": "alu", **alu, "traffic": None, "hbm": hbm}
    else:
        roof = {"bound": "hbm", **hbm, "traffic": None, "alu": alu}
    roof["traffic"] = measured_traffic()
    roof["kernel"] = "patch_step_kernel<float, 64, BL53, D2Q9>"
    roof["flops_per_launch"] = flops_launch
    roof["flops_per_lup"] = round(flops_launch / (N * N), 1)
    roof["bytes_per_launch"] = round(prim["bytes_per_launch"])

    shape = None
    if not args.no_autotune:
        from paper_2302_09883_amd.execution import tune_patch_shape
        shape = tune_patch_shape(N, PRIMARY_EPS)
        print(f"[bench] patch-shape tuner: {shape['chosen']}", file=sys.stderr, flush=True)

    if args.copy_calibration:
        copy_calibration()

    hbm_points = None
    if not args.no_hbm_points:
        hbm_points = [hbm_point(N, 200), hbm_point(2 * N, 100)]

    line = {
        "metric": "MLUPS incl. compress/decompress + compression ratio at fixed L2 error",
        "value": round(prim["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(prim["ms_per_step"], 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "D2Q9 BGK tau=0.6, 2048x2048 periodic, 64x64 patches, folded BL5/3 L=5, "
                               "capped threshold, double shear layer",
                   "grid": N, "patch": P, "levels": LEVELS, "eps": PRIMARY_EPS, "parallelism": "single GPU",
                   "execution": dict(prim["execution"], patch_shape=shape)},
        "compression_ratio": round(prim["ratio"], 2),
        "rel_l2_vs_uncompressed": prim["rel_l2"],
        "error_steps": total,
        "cr_at_fixed_l2": [cr_at_error(points, t) for t in TARGET_REL_L2],
        "sweep": [{k: _sig(v) for k, v in p.items()} for p in points],
        "uncompressed_mlups": round(ref_mlups, 1),
        "roofline": roof,
        "hbm_bound_points": hbm_points,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
