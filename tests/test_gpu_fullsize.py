"""GPU parity at the benchmark's full size (2048^2 D2Q9, 64^2 patches, BL5/3 L = 5).

The library runs the same kernel and launch configuration as ``bench.py``.  The
oracle cannot step the whole grid quickly, so it recomputes one step of a
sample of patches from the GPU's own compressed state (their neighbours give
the ghost ring) and the test compares the sampled records; global properties
(store accounting, conservation) are checked on the whole grid.
"""
import sys

import numpy as np
import pytest

from oracle import lbmz_oracle as O
from synth import shear_layer_macroscopic

from gpu_helpers import make_ctx, require_gpu, torch  # noqa: F401

pytestmark = pytest.mark.gpu

N, P, L = 2048, 64, 5
SAMPLE = [0, 31, 32 * 5 + 7, 32 * 16 + 16, 32 * 31, 1023]   # corners, interior, wrap-around


def _say(*args):
    print("[case]", *args, flush=True)
    sys.stdout.flush()


@pytest.fixture(autouse=True)
def _gpu():
    require_gpu()


def _neighbourhood(q, npx):
    px, py = q % npx, q // npx
    return sorted({((px + dx) % npx) + npx * ((py + dy) % npx) for dx in (-1, 0, 1) for dy in (-1, 0, 1)})


@pytest.mark.parametrize("eps", [1e-4, 0.0])
def test_sampled_patches_one_step_at_full_size(eps):
    _say("full size sampled", eps)
    from gpu_helpers import decode_records
    ctx = make_ctx(N, "d2q9_bgk", "f32", P, "bl53", L, eps)
    rho, ux, uy = shear_layer_macroscopic(N, seed=0)
    ctx.set_macroscopic(*(a.astype(np.float32) for a in (rho, ux, uy)))
    ctx.step(10)
    table, pool = ctx.store()
    g = O.Geometry(N, P, O.BL53, L)
    npx = g.npx
    need = sorted({r for q in SAMPLE for r in _neighbourhood(q, npx)})
    coef = np.zeros((g.npatch, 9, g.s, g.s), dtype=np.float32)
    coef[need] = decode_records(table[need], pool, g.s, np.float32)
    run = O.CompressedRun(g, O.Scheme("d2q9_bgk", tau=0.6), eps, O.RULE_CAPPED, np.float32)
    lossy = np.zeros_like(coef)
    lossy[need] = run.decompress_tiles(coef[need])
    padded = O.gather_ghosts(lossy, g)[SAMPLE]
    want = run.compress_tiles(run.scheme.update(padded).astype(np.float32))

    ctx.step(1)
    t2, p2 = ctx.store()
    got = decode_records(t2[SAMPLE], p2, g.s, np.float32)
    u = np.finfo(np.float32).eps
    scale = float(np.max(np.abs(lossy[SAMPLE])))
    delta = 1e-5 * scale   # the stated float32 bar, 1e-5 of the field scale
    thr = np.broadcast_to(run.thr, want.shape)
    kg, kw = got != 0, want != 0
    flip = kg != kw
    near = np.abs(np.abs(np.where(kg, got, want)) - thr) <= delta
    assert np.all(near[flip]), int(flip.sum())
    both = kg & kw
    assert np.max(np.abs(got[both] - want[both]), initial=0.0) <= delta
    # the records' counts and encodings are those of the decoded coefficients
    for i, q in enumerate(SAMPLE):
        for f in range(9):
            nnz = int(np.count_nonzero(got[i, f]))
            is_mask = O.record_layout(nnz, g.s * g.s, 4)[0]
            assert int(t2[q, f, 1]) == nnz | (O.MASK_BIT if is_mask else 0)


def test_store_accounting_and_conservation_at_full_size():
    _say("full size accounting")
    ctx = make_ctx(N, "d2q9_bgk", "f32", P, "bl53", L, 1e-4)
    rho, ux, uy = shear_layer_macroscopic(N, seed=0)
    ctx.set_macroscopic(*(a.astype(np.float32) for a in (rho, ux, uy)))
    t0 = np.array(ctx.stats()["totals"])
    ctx.step(50)
    st = ctx.stats()
    table, pool = ctx.store()
    nnz = table[..., 1] & (O.MASK_BIT - 1)
    rec = sum(O.record_layout(int(k), 65 * 65, 4)[3] for k in nnz.reshape(-1))
    assert st["store_bytes"] == rec + table.size * 4
    assert len(pool) == rec                       # bump allocation leaves no gaps
    assert st["nnz_total"] == int(nnz.sum())
    t1 = np.array(st["totals"])
    assert abs(t1.sum() - t0.sum()) <= 2e-6 * abs(t0.sum())
    c = O.D2Q9_C
    for ax in (0, 1):
        assert abs((c[:, ax] * t1).sum() - (c[:, ax] * t0).sum()) <= 2e-6 * abs(t0.sum())
