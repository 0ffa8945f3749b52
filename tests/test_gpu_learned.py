"""GPU parity of the learned-threshold path.

* The network's HIP forward pass, gradients and Adam step against the
  oracle (same bfloat16-rounded weights; float32 accumulation vs float64).
* Per-patch thresholds: one step from a common state against the oracle with
  the same per-patch threshold tables.
* The exported network inputs are the stored coefficients at stride 8.
* A small end-to-end run (data, training, controlled run, fixed sweep) that
  reports what the trained network gains over the fixed threshold.
"""
import sys

import numpy as np
import pytest

from oracle import lbmz_learned as NL
from oracle import lbmz_oracle as O
from synth import shear_with_vortices

from gpu_helpers import make_ctx, require_gpu, torch  # noqa: F401

pytestmark = pytest.mark.gpu


def _say(*args):
    print("[case]", *args, flush=True)
    sys.stdout.flush()


@pytest.fixture(autouse=True)
def _gpu():
    require_gpu()


def _oracle_params(flat, k):
    p, off = {}, 0
    for name, shp in NL.param_shapes(k).items():
        size = int(np.prod(shp))
        p[name] = NL.bf16_round(flat[off:off + size]).astype(np.float64).reshape(shp)
        off += size
    assert off == flat.size
    return p


def _inputs(b, seed):
    """Raw patch features [b, 36, 8, 8]: coefficients, then non-negative energies."""
    rng = np.random.default_rng(seed)
    x = (rng.standard_normal((b, 36, 8, 8)) * 10.0 ** rng.uniform(-6, -1, (b, 36, 8, 8))).astype(np.float32)
    x[rng.random(x.shape) < 0.3] = 0
    x[:, 9:] = x[:, 9:] ** 2
    return x


def _oracle_x(x):
    return NL.input_map(x.astype(np.float64))


@pytest.mark.parametrize("k", [3, 12])
def test_forward_matches_oracle(k):
    from paper_2302_09883_amd import Net
    from paper_2302_09883_amd.learned import init_params
    _say("net forward", k)
    net = Net(k)
    flat = init_params(k, seed=3)
    flat[-k:] = np.linspace(-1, 1, k)            # non-zero head biases
    net.set_params(flat)
    x = _inputs(40, seed=4)
    got = net.forward(x)
    want, _ = NL.forward(_oracle_params(flat, k), _oracle_x(x))
    assert np.max(np.abs(got - want)) <= 1e-4 * (1 + np.max(np.abs(want)))
    assert np.allclose(net.params(), flat)        # the master copy is what was set


def test_gradients_match_oracle():
    from paper_2302_09883_amd import Net
    from paper_2302_09883_amd.learned import init_params
    _say("net gradients")
    k = 6
    net = Net(k)
    flat = init_params(k, seed=5)
    rng = np.random.default_rng(6)
    flat = (flat + 0.02 * rng.standard_normal(flat.size)).astype(np.float32)   # every ReLU branch
    net.set_params(flat)
    x = _inputs(37, seed=7)                        # not a multiple of the samples per workgroup
    t = rng.standard_normal((37, k)).astype(np.float32)
    g, loss = net.gradients(x, t)
    p = _oracle_params(flat, k)
    wl, wg = NL.loss_and_grads(p, _oracle_x(x), t.astype(np.float64))
    assert abs(loss - wl) <= 1e-4 * abs(wl)
    off = 0
    for name, shp in NL.param_shapes(k).items():
        size = int(np.prod(shp))
        a = g[off:off + size]
        b = wg[name].reshape(-1)
        off += size
        # per parameter, relative to the tensor's largest gradient (float32
        # accumulation against float64; a ReLU whose input sits within
        # rounding of 0 may switch, which moves a few entries by ~1e-4)
        err = float(np.max(np.abs(a - b)) / np.max(np.abs(b)))
        print(f"[grad] {name}: max |gpu - oracle| / max |oracle| = {err:.2e}", flush=True)
        assert err <= 1e-3, name


def test_adam_step_matches_oracle():
    from paper_2302_09883_amd import Net
    from paper_2302_09883_amd.learned import init_params
    _say("net adam")
    k = 4
    net = Net(k)
    flat = init_params(k, seed=8)
    net.set_params(flat)
    x = _inputs(32, seed=9)
    t = np.random.default_rng(10).standard_normal((32, k)).astype(np.float32)
    g, _ = net.gradients(x, t)
    net.train_step(x, t, lr=1e-3)
    got = net.params()
    p = {"w": flat.astype(np.float64)}
    m = {"w": np.zeros(flat.size)}
    v = {"w": np.zeros(flat.size)}
    NL.adam_step(p, m, v, {"w": g.astype(np.float64)}, step=1, lr=1e-3)
    assert np.max(np.abs(got - p["w"])) <= 1e-6


def test_training_reduces_the_loss_on_the_gpu():
    from paper_2302_09883_amd import Net
    from paper_2302_09883_amd.learned import init_params
    _say("net training")
    k = 2
    x = _inputs(256, seed=11)
    ox = _oracle_x(x)
    t = np.stack([ox.std(axis=(1, 2, 3)), ox[:, 0].mean(axis=(1, 2))], axis=1).astype(np.float32)
    net = Net(k)
    net.set_params(init_params(k, seed=12))
    l0 = net.gradients(x, t)[1]
    for _ in range(80):
        net.train_step(x, t, lr=3e-3)
    l1 = net.gradients(x, t)[1]
    assert l1 < 0.3 * l0


def _macro(n, seed):
    rho, ux, uy = shear_with_vortices(n, seed=seed)
    return [a.astype(np.float32) for a in (rho, ux, uy)]


def test_per_patch_thresholds_one_step_from_common_state():
    from gpu_helpers import decode_records
    _say("per-patch eps")
    n, p, levels = 256, 64, 5
    rng = np.random.default_rng(13)
    eps = 10.0 ** rng.uniform(-5, -2.5, (n // p) ** 2)
    ctx = make_ctx(n, "d2q9_bgk", "f32", p, "bl53", levels, 1e-4)
    ctx.set_patch_eps(eps)
    g = O.Geometry(n, p, O.BL53, levels)
    twin = O.CompressedRun(g, O.Scheme("d2q9_bgk", tau=0.6), 1e-4, O.RULE_CAPPED, np.float32)
    twin.set_patch_eps(eps)
    rho, ux, uy = shear_with_vortices(n, seed=14)
    twin.set_grid(O.d2q9_equilibrium(rho, ux, uy).astype(np.float32))
    twin.step(2)
    table, pool = O.encode_store(twin.coef)
    ctx.put_store(table, pool)
    ctx.step(1)
    twin.step(1)
    t2, p2 = ctx.store()
    got = decode_records(t2, p2, g.s, np.float32)
    want = twin.coef
    u = np.finfo(np.float32).eps
    delta = 1e-5 * float(np.max(np.abs(twin.grid())))
    flip = (got != 0) != (want != 0)
    near = np.abs(np.abs(np.where(got != 0, got, want)) - twin.thr) <= delta
    assert np.all(near[flip]), int(flip.sum())
    assert np.max(np.abs(np.where(flip, 0.0, got - want))) <= delta
    # the thresholds really differ per patch: more kept coefficients where eps is small
    kept = (got != 0).reshape(got.shape[0], -1).sum(axis=1)
    assert np.corrcoef(np.log(eps), kept)[0, 1] < 0
    ctx.set_patch_eps(None)


def _patch_controls(npatch, levels, seed):
    rng = np.random.default_rng(seed)
    return 10.0 ** rng.uniform(-5, -2.5, npatch), rng.integers(levels - 2, levels + 1, npatch)


def test_per_patch_thresholds_and_levels_one_step_from_common_state():
    """Per-patch threshold constants and level counts, one step from a common
    state, against the oracle with the same controls (shared bordering lines
    at the smaller threshold of their tiles)."""
    from gpu_helpers import decode_records
    _say("per-patch eps and levels, one step")
    n, p, levels = 256, 64, 5
    g = O.Geometry(n, p, O.BL53, levels)
    eps, lev = _patch_controls(g.npatch, levels, 21)
    ctx = make_ctx(n, "d2q9_bgk", "f32", p, "bl53", levels, 1e-4)
    ctx.set_patch_eps(eps)
    ctx.set_patch_levels(lev)
    twin = O.CompressedRun(g, O.Scheme("d2q9_bgk", tau=0.6), 1e-4, O.RULE_CAPPED, np.float32)
    twin.set_patch_eps(eps)
    twin.set_patch_levels(lev)
    rho, ux, uy = shear_with_vortices(n, seed=22)
    twin.set_grid(O.d2q9_equilibrium(rho, ux, uy).astype(np.float32))
    twin.step(2)
    table, pool = O.encode_store(twin.coef)
    ctx.put_store(table, pool)
    ctx.step(1)
    twin.step(1)
    t2, p2 = ctx.store()
    got = decode_records(t2, p2, g.s, np.float32)
    want = twin.coef
    delta = 1e-5 * float(np.max(np.abs(twin.grid())))
    flip = (got != 0) != (want != 0)
    near = np.abs(np.abs(np.where(got != 0, got, want)) - twin.thr) <= delta
    assert np.all(near[flip]), int(flip.sum())
    assert np.max(np.abs(np.where(flip, 0.0, got - want))) <= delta
    # smaller level counts keep more coefficients
    kept = (got != 0).reshape(got.shape[0], -1).sum(axis=1)
    assert np.corrcoef(lev + np.log10(eps), kept)[0, 1] < 0


def test_per_patch_controls_keep_shared_faces_and_totals():
    """Many steps with mixed per-patch thresholds and level counts: the tiles
    sharing a bordering line reconstruct it identically (decoded GPU store),
    and mass and momentum stay constant to float32 round-off."""
    from gpu_helpers import decode_records
    _say("per-patch controls, faces and totals")
    n, p, levels = 256, 64, 5
    g = O.Geometry(n, p, O.BL53, levels)
    eps, lev = _patch_controls(g.npatch, levels, 31)
    ctx = make_ctx(n, "d2q9_bgk", "f32", p, "bl53", levels, 1e-4)
    ctx.set_patch_eps(eps)
    ctx.set_patch_levels(lev)
    ctx.set_macroscopic(*_macro(n, 32))
    t0 = np.array(ctx.stats()["totals"])
    ctx.step(60)
    t1 = np.array(ctx.stats()["totals"])
    c = O.D2Q9_C
    for w in (np.ones(9), c[:, 0], c[:, 1]):
        assert abs((w * t1).sum() - (w * t0).sum()) <= 2e-6 * t0.sum()
    table, pool = ctx.store()
    lossy = O.inverse_2d(decode_records(table, pool, g.s, np.float32).astype(np.float64), levels, O.BL53)
    for q in range(g.npatch):
        px, py = q % g.npx, q // g.npx
        right = (px + 1) % g.npx + g.npx * py
        up = px + g.npx * ((py + 1) % g.npx)
        assert np.max(np.abs(lossy[q][:, :, p] - lossy[right][:, :, 0])) <= 1e-12
        assert np.max(np.abs(lossy[q][:, p, :] - lossy[up][:, 0, :])) <= 1e-12


def test_features_are_the_stored_coefficients_and_level_energies():
    """The exported features: the stored coefficients at stride 8 (any eps),
    and at eps = 0 (nothing zeroed, so the coefficients before the threshold
    are the stored ones) the level 1-3 energies of every block, against the
    oracle's features of the decoded store."""
    from gpu_helpers import decode_records
    _say("features")
    n = 256
    for eps in (1e-4, 0.0):
        ctx = make_ctx(n, "d2q9_bgk", "f32", 64, "bl53", 5, eps)
        ctx.enable_features(True)
        ctx.set_macroscopic(*_macro(n, 15))
        ctx.step(3)
        feats = ctx.features()
        table, pool = ctx.store()
        coef = decode_records(table, pool, 65, np.float32)
        assert np.array_equal(feats[:, :9], coef[:, :, 0:64:8, 0:64:8])
        if eps == 0.0:
            want = NL.raw_features(coef, 5)[:, 9:]
            got = feats[:, 9:].astype(np.float64)
            assert np.all(np.abs(got - want) <= 1e-5 * want + 1e-30), float(np.max(np.abs(got - want) / (want + 1e-30)))


def test_end_to_end_small():
    """Data, training, the fixed sweep and a judged controlled run on a small
    grid.  Every window of the controlled run is kept only if it adds no more
    error than the fixed threshold's window from the same state and its store
    is no larger, so the run must not lose to the fixed threshold: error at
    most the fixed run's (plus the divergence of later windows, 2 %), ratio at
    least the fixed run's, and a gain >= 1 at equal error against the fixed
    sweep (where that error lies inside the sweep)."""
    from paper_2302_09883_amd import learned as LRN
    _say("learned end to end")
    res = LRN.evaluate(n_train=256, train_seeds=(1, 2), times=(40, 80), n_eval=256, eval_seed=50, steps=150,
                       epochs=8, fixed=(3e-5,))
    assert res["samples"] == 2 * 2 * 16
    assert len(res["fixed"]) == len(LRN.EPS)
    r = res["runs"][0]
    L = r["learned"]
    print("[case] learned small:", L, "fixed", r["fixed_rel_l2"], r["fixed_ratio"], "gain", r["gain"], flush=True)
    assert np.isfinite(L["rel_l2"]) and L["ratio_mean"] > 1
    assert L["rel_l2"] <= 1.02 * r["fixed_rel_l2"]
    assert L["ratio_mean"] >= r["fixed_ratio"]
    if r["gain"] is not None:
        assert r["gain"] >= 1.0 - 1e-9          # (a run equal to the fixed one gives 1 up to rounding)
