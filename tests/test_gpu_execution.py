"""Execution modes of the step: persistent work-queue kernel, HIP graph chunks, autotuner.

Every mode must compute the same records as one workgroup per patch with
plain launches: the decoded coefficient tiles are compared bit for bit after
step counts that cover whole graph chunks, partial chunks and repeated calls
with host work in between (graph replays), including a pool overflow that is
absorbed by a regrow in the middle of a chunk.
"""
import sys

import numpy as np
import pytest

from synth import shear_layer_macroscopic, fv_gaussians_and_step

from gpu_helpers import make_ctx, require_gpu, torch  # noqa: F401

pytestmark = pytest.mark.gpu

MODES = [(False, False), (True, False), (False, True), (True, True)]


def _say(*args):
    print("[case]", *args, flush=True)
    sys.stdout.flush()


@pytest.fixture(autouse=True)
def _gpu():
    require_gpu()


def _lbm(n=256, eps=1e-4, p=64, levels=5, **kw):
    ctx = make_ctx(n, "d2q9_bgk", "f32", p, "bl53", levels, eps, **kw)
    rho, ux, uy = shear_layer_macroscopic(n, seed=2)
    ctx.set_macroscopic(*(a.astype(np.float32) for a in (rho, ux, uy)))
    return ctx


def _tiles(ctx):
    from gpu_helpers import decode_records
    table, pool = ctx.store()
    return decode_records(table, pool, ctx.s, ctx.np_dtype), table


def _same(a, b):
    ta, tba = _tiles(a)
    tb, tbb = _tiles(b)
    assert np.array_equal(ta.view(np.uint32), tb.view(np.uint32))
    assert np.array_equal(tba[..., 1], tbb[..., 1])          # counts and encodings (placement may differ)
    sa, sb = a.stats(), b.stats()
    assert sa["totals"] == sb["totals"] and sa["store_bytes"] == sb["store_bytes"]


@pytest.mark.parametrize("persistent,graph", MODES[1:])
def test_modes_match_plain_launches(persistent, graph):
    _say("mode", persistent, graph)
    base = _lbm()
    other = _lbm()
    other.set_execution(persistent, graph)
    assert other.execution() == (persistent, graph)
    for n in (13, 6, 1, 12, 7):          # whole and partial chunks, repeated calls
        base.step(n)
        other.step(n)
        _same(base, other)
        _ = other.stats()                # host work between graph replays


@pytest.mark.parametrize("persistent,graph", MODES[1:])
def test_modes_absorb_a_pool_overflow(persistent, graph):
    _say("mode overflow", persistent, graph)
    base = _lbm(eps=0.0, pool_capacity=4096)
    other = _lbm(eps=0.0, pool_capacity=4096)
    other.set_execution(persistent, graph)
    base.step(14)
    other.step(14)
    assert other.stats()["regrows"] >= 1
    _same(base, other)


def test_persistent_on_a_small_grid_and_fv():
    _say("persistent small fv")
    from paper_2302_09883_amd import Context
    f0 = fv_gaussians_and_step(256, seed=1)
    runs = []
    for persistent, graph in ((False, False), (True, True)):
        c = Context(256, scheme="fv_upwind", dtype="f64", p=32, wavelet="haar", levels=4, eps=1e-4)
        c.set_execution(persistent, graph)
        c.set_field(0, f0)
        c.step(25)
        runs.append(c)
    _same(runs[0], runs[1])


def test_autotune_keeps_the_trajectory():
    _say("autotune")
    spv = 3
    tuned = _lbm()
    ms = tuned.autotune(spv)
    assert ms.shape == (4,) and np.all(ms > 0)
    assert tuned.execution() in [(bool(p), bool(g)) for p, g in MODES]
    base = _lbm()
    base.step(8 * spv)
    _same(base, tuned)
    tuned.step(9)
    base.step(9)
    _same(base, tuned)
    print("[case] autotune ms/step (plain, graph, persistent, both):", ms.tolist(), "chose", tuned.execution())


def test_patch_shape_tuner_compares_at_equal_error():
    """The patch-shape tuner measures every compiled shape of the D2Q9
    workload (speed, ratio, error against the uncompressed run of the same
    length) and keeps the fastest one whose error is within its tolerance of
    the smallest error."""
    from paper_2302_09883_amd.execution import SHAPES, tune_patch_shape
    print("[case] patch-shape tuner", flush=True)
    res = tune_patch_shape(n=256, eps=1e-4, steps=10, tune_steps=1)
    assert [(r["patch"], r["levels"]) for r in res["shapes"]] == list(SHAPES)
    for r in res["shapes"]:
        assert r["mlups_events"] > 0 and r["ratio"] > 1 and 0 < r["rel_l2"] < 1e-2
    best = min(r["rel_l2"] for r in res["shapes"])
    ok = [r for r in res["shapes"] if r["rel_l2"] <= (1 + res["tolerance"]) * best]
    fastest = max(ok, key=lambda r: r["mlups_events"])
    assert (res["chosen"]["patch"], res["chosen"]["levels"]) == (fastest["patch"], fastest["levels"])


@pytest.mark.parametrize("persistent,graph", MODES[1:])
def test_modes_match_plain_launches_with_per_patch_controls(persistent, graph):
    """The step-kernel variant with per-patch thresholds, level counts and the
    network-input export, in every execution mode, against plain launches; the
    controls are switched off and on again between calls (the graph chunks are
    rebuilt for the other variant)."""
    _say("mode with per-patch controls", persistent, graph)
    rng = np.random.default_rng(31)
    base = _lbm()
    other = _lbm()
    other.set_execution(persistent, graph)
    npatch = (256 // 64) ** 2
    eps = 10.0 ** rng.uniform(-5, -3, npatch)
    lev = rng.integers(2, 6, npatch)
    for c in (base, other):
        c.set_patch_eps(eps)
        c.set_patch_levels(lev)
        c.enable_features(True)
    for n in (7, 6):
        base.step(n)
        other.step(n)
        _same(base, other)
        assert np.array_equal(base.features(), other.features())
    for c in (base, other):          # back to the uniform variant, then controls again
        c.set_patch_eps(None)
        c.set_patch_levels(None)
        c.enable_features(False)
    base.step(6)
    other.step(6)
    _same(base, other)
    for c in (base, other):
        c.set_patch_eps(eps)
    base.step(7)
    other.step(7)
    _same(base, other)
