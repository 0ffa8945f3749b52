"""GPU parity of the 3-D D3Q19 patch loop (persistent step kernel with
per-workgroup scratch, halo planes and lines, flat-order records).

* Set-up and decompression reproduce the oracle's equilibrium state.
* At eps = 0 the compressed loop equals the uncompressed reference kernel and
  the oracle's plain scheme.
* Records written from given coefficients are byte-identical to the oracle's.
* One step from a common state matches the oracle's step (keep / drop flips
  only at round-off distance from a threshold).
* Several steps at eps > 0 stay close to the oracle, conserve mass and
  momentum, and absorb a pool overflow with the same result.
"""
import sys

import numpy as np
import pytest

from oracle import lbmz_oracle3d as O3
from synth import taylor_green_jets_3d

from gpu_helpers import require_gpu, torch  # noqa: F401

pytestmark = pytest.mark.gpu

TAU = 0.55


def _say(*args):
    print("[case]", *args, flush=True)
    sys.stdout.flush()


@pytest.fixture(autouse=True)
def _gpu():
    require_gpu()


def _ctx(n, p, levels, eps, reference=False, **kw):
    from paper_2302_09883_amd import Context
    return Context(n, scheme="d3q19_bgk", dtype="f32", p=p, wavelet="bl53", levels=levels, eps=eps, tau=TAU,
                   reference=reference, **kw)


def _macro(n, seed):
    return taylor_green_jets_3d(n, seed=seed, n_jets=3, dtype=np.float32)


def _oracle_state(n, seed, dtype=np.float64):
    rho, ux, uy, uz = (a.astype(np.float64) for a in _macro(n, seed))
    return O3.d3q19_equilibrium(rho, ux, uy, uz).astype(dtype)


def _tiles(ctx):
    from gpu_helpers import decode_records3
    table, pool = ctx.store()
    return decode_records3(table, pool, ctx.s), table, pool


@pytest.mark.parametrize("n,p,levels", [(32, 16, 3), (64, 32, 3), (32, 16, 0), (32, 16, 1)])
def test_setup_and_decompression(n, p, levels):
    _say("3d setup", n, p, levels)
    ctx = _ctx(n, p, levels, 0.0)
    ctx.set_macroscopic(*_macro(n, 1))
    got = ctx.fields()
    want = _oracle_state(n, 1)
    assert got.shape == (19, n, n, n)
    assert np.max(np.abs(got - want)) <= 2e-6 * np.max(np.abs(want))
    t = ctx.totals()
    assert np.allclose(t, want.sum(axis=(1, 2, 3)), rtol=2e-6)


@pytest.mark.parametrize("n,p,levels", [(48, 16, 3), (64, 32, 3)])
def test_eps0_equals_reference_and_oracle(n, p, levels):
    _say("3d eps0", n, p, levels)
    steps = 6
    ref = _ctx(n, p, levels, 0.0, reference=True)
    ref.set_macroscopic(*_macro(n, 2))
    cmp = _ctx(n, p, levels, 0.0)
    cmp.set_macroscopic(*_macro(n, 2))
    ref.step(steps)
    cmp.step(steps)
    a, b = ref.fields(), cmp.fields()
    f = _oracle_state(n, 2)
    for _ in range(steps):
        f = O3.dense_step3(f, TAU)
    rel = np.linalg.norm(b - f) / np.linalg.norm(f)
    assert rel <= 1e-5, rel
    assert np.linalg.norm(a - f) / np.linalg.norm(f) <= 1e-5
    assert np.max(np.abs(a - b)) <= 1e-5 * np.max(np.abs(f))


@pytest.mark.parametrize("n,p,density", [(32, 16, 0.002), (32, 16, 0.3), (64, 32, 0.045)])
def test_records_from_given_coefficients_are_the_oracles(n, p, density):
    """Byte-exact records; at P = 32 and density 0.045 every index list holds
    about 1,100 - 2,200 entries, beyond the first workgroup-wide batch of the
    expansion's list loads, so the prefetched entries and the tail loop of the
    scatter are both exercised (the records are decompressed and compared)."""
    _say("3d records", n, p, density)
    levels, eps = 3, 1e-3
    g = O3.Geometry3(n, p, levels)
    rng = np.random.default_rng(5)
    coef = (rng.standard_normal((g.npatch, 19, g.s, g.s, g.s)) * 1e-2).astype(np.float32)
    coef[rng.random(coef.shape) >= density] = 0
    coef[:, :, ::8, ::8, ::8] = 0.05          # samples (never thresholded)
    ctx = _ctx(n, p, levels, eps)
    ctx.set_coefficients(coef)
    twin = O3.CompressedRun3(g, TAU, eps, dtype=np.float32)
    twin.set_coefficients(coef)
    got, table, pool = _tiles(ctx)
    assert np.array_equal(got, twin.coef)
    want_table, _ = twin.store()
    assert np.array_equal(table[..., 1], want_table[..., 1])
    for q in range(g.npatch):
        for f in range(19):
            rec = O3.encode_record3(twin.coef[q, f])
            off = int(table[q, f, 0]) * 16
            assert pool[off:off + len(rec)] == rec, (q, f)
    st = ctx.stats()
    assert st["store_bytes"] == twin.store_bytes()
    assert st["mask_records"] + st["list_records"] == g.npatch * 19
    if density < 0.01:
        assert st["list_records"] > 0
    elif p == 32:
        nnz = table[..., 1] & (O3.MASK_BIT - 1)
        assert st["list_records"] == g.npatch * 19
        assert 1024 < int(nnz.min()) and int(nnz.max()) < 2248
        # the expansion of those lists: decompressed fields against the oracle's
        want = twin.grid()
        got_f = ctx.fields()
        assert np.max(np.abs(got_f - want)) <= 2e-6 * np.max(np.abs(want))
    else:
        assert st["mask_records"] > 0


@pytest.mark.parametrize("n,p,levels,eps", [(48, 16, 3, 1e-4), (64, 32, 3, 1e-4), (32, 16, 2, 1e-3),
                                             (32, 16, 1, 1e-3)])
def test_one_step_from_common_state(n, p, levels, eps):
    _say("3d one step", n, p, levels, eps)
    g = O3.Geometry3(n, p, levels)
    twin = O3.CompressedRun3(g, TAU, eps, dtype=np.float32)
    twin.set_grid(_oracle_state(n, 3, np.float32))
    twin.step(1)
    table, pool = twin.store()
    ctx = _ctx(n, p, levels, eps)
    ctx.put_store(table, pool)
    ctx.step(1)
    twin.step(1)
    got, _, _ = _tiles(ctx)
    want = twin.coef
    u = np.finfo(np.float32).eps
    delta = 1e-5 * float(np.max(np.abs(want)))
    flip = (got != 0) != (want != 0)
    near = np.abs(np.abs(np.where(got != 0, got, want)) - twin.thr) <= delta
    assert np.all(near[flip]), int(flip.sum())
    assert np.max(np.abs(np.where(flip, 0.0, got - want))) <= delta
    assert flip.sum() <= 1e-4 * flip.size
    assert 0 < np.count_nonzero(got) < got.size


def _rest_with_bump(n, amp, width):
    """Fluid at rest (rho = 1, u = 0) but for a density bump of the given width
    around one point, cut off at three widths: tiles beyond are constant, so
    their records keep coarse samples only."""
    z, y, x = np.meshgrid(*(np.arange(n, dtype=np.float64),) * 3, indexing="ij")
    c = n / 4 + 0.5
    r2 = ((x - c) ** 2 + (y - c) ** 2 + (z - c) ** 2) / width ** 2
    rho = 1.0 + amp * np.exp(-r2) * (r2 < 9.0)
    zero = np.zeros_like(rho)
    return O3.d3q19_equilibrium(rho, zero, zero, zero).astype(np.float32)


def _samples_only(tile, levels):
    m = (1 << levels) - 1
    z, y, x = np.nonzero(tile)
    return bool(np.all(((x | y | z) & m) == 0))


@pytest.mark.parametrize("n,p,levels,eps", [(64, 16, 3, 1e-4), (64, 16, 2, 1e-4), (32, 16, 3, 0.5), (64, 32, 3, 1e-4),
                                             (64, 32, 2, 1e-4)])
def test_step_records_of_samples_only_tiles(n, p, levels, eps):
    """One step from a state whose records hold coarse samples only in most
    tiles (constant fluid at rest; at eps = 0.5 every detail of every tile is
    dropped and the samples differ from node to node), beside tiles with
    details: every record the step writes is byte for byte the encoding of its
    own tile, and the tiles match the oracle's step."""
    _say("3d samples-only step", n, p, levels, eps)
    g = O3.Geometry3(n, p, levels)
    twin = O3.CompressedRun3(g, TAU, eps, dtype=np.float32)
    twin.set_grid(_rest_with_bump(n, 0.02, n / 12 if eps < 0.1 else n / 3))
    table0, pool0 = twin.store()
    ctx = _ctx(n, p, levels, eps)
    ctx.put_store(table0, pool0)
    ctx.step(1)
    twin.step(1)
    got, table, pool = _tiles(ctx)
    for q in range(g.npatch):
        for f in range(19):
            rec = O3.encode_record3(got[q, f])
            off = int(table[q, f, 0]) * 16
            assert pool[off:off + len(rec)] == rec, (q, f)
            assert int(table[q, f, 1]) & (O3.MASK_BIT - 1) == np.count_nonzero(got[q, f])
    only = np.array([[_samples_only(got[q, f], levels) for f in range(19)] for q in range(g.npatch)])
    if eps < 0.1:
        assert 0 < only.sum() < only.size, int(only.sum())
    else:
        assert only.all()
        assert all(len(np.unique(got[q, f][got[q, f] != 0])) > 1 for q in range(g.npatch) for f in range(19))
    want = twin.coef
    delta = 1e-5 * float(np.max(np.abs(want)))
    flip = (got != 0) != (want != 0)
    near = np.abs(np.abs(np.where(got != 0, got, want)) - twin.thr) <= delta
    assert np.all(near[flip]), int(flip.sum())
    assert np.max(np.abs(np.where(flip, 0.0, got - want))) <= delta


def test_multi_step_close_to_oracle_and_conserving():
    _say("3d multi step")
    n, p, levels, eps, steps = 48, 16, 3, 1e-4, 8
    g = O3.Geometry3(n, p, levels)
    twin = O3.CompressedRun3(g, TAU, eps)
    twin.set_grid(_oracle_state(n, 4))
    ctx = _ctx(n, p, levels, eps)
    ctx.set_macroscopic(*_macro(n, 4))
    t0 = ctx.totals()
    ctx.step(steps)
    twin.step(steps)
    a, b = ctx.fields(), twin.grid()
    rel = np.linalg.norm(a - b) / np.linalg.norm(b)
    assert rel <= 1e-4, rel
    # kept coefficients (the float64 twin's ratio would count 8-byte values)
    assert abs(ctx.stats()["nnz_total"] / twin.nnz().sum() - 1) <= 0.01
    t1 = ctx.totals()
    c = O3.D3Q19_C.astype(np.float64)
    assert abs(t1.sum() - t0.sum()) <= 2e-6 * abs(t0.sum())
    assert np.allclose(t1 @ c, t0 @ c, atol=2e-6 * abs(t0.sum()))
    assert np.allclose(t1, twin.field_totals(), rtol=1e-5)


def test_pool_overflow_is_absorbed():
    _say("3d overflow")
    n, p, levels, eps = 32, 16, 3, 1e-5
    base = _ctx(n, p, levels, eps)
    small = _ctx(n, p, levels, eps, pool_capacity=4096)
    for c in (base, small):
        c.set_macroscopic(*_macro(n, 5))
        c.step(5)
    assert small.stats()["regrows"] >= 1
    a, _, _ = _tiles(base)
    b, _, _ = _tiles(small)
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32))
    assert base.stats()["store_bytes"] == small.stats()["store_bytes"]


def test_graph_mode_gives_the_same_records():
    _say("3d graph")
    n, p, levels, eps = 32, 16, 3, 1e-4
    a = _ctx(n, p, levels, eps)
    b = _ctx(n, p, levels, eps)
    b.set_execution(False, True)
    for c in (a, b):
        c.set_macroscopic(*_macro(n, 6))
        c.step(13)
    ta, _, _ = _tiles(a)
    tb, _, _ = _tiles(b)
    assert np.array_equal(ta.view(np.uint32), tb.view(np.uint32))


def test_invalid_3d_configurations_are_rejected():
    from paper_2302_09883_amd import LbmzError
    with pytest.raises(LbmzError):
        _ctx(32, 8, 2, 1e-4)          # 8^3 patches: no kernel
    with pytest.raises(LbmzError):
        _ctx(48, 16, 4, 1e-4)         # L = J: no update step, no conservation
    with pytest.raises(LbmzError):
        _ctx(40, 16, 3, 1e-4)         # n not a multiple of p
    ctx = _ctx(32, 16, 3, 1e-4)
    with pytest.raises(LbmzError):
        ctx.set_patch_eps(np.full(8, 1e-4))


def test_full_size_sampled_patches():
    """768^3, 32^3 patches, L = 3 (the measured workload, same launch): one GPU
    step of sampled patches against the oracle's step of the same patches,
    computed from the GPU's own store (the neighbours' records decoded and
    rebuilt on the host)."""
    _say("3d full size sampled")
    n, p, levels, eps = 768, 32, 3, 1e-4
    g = O3.Geometry3(n, p, levels)
    ctx = _ctx(n, p, levels, eps)
    macro = taylor_green_jets_3d(n, seed=0, dtype=np.float32)
    ctx.set_macroscopic(*macro)
    del macro
    ctx.step(2)
    table, pool = ctx.store()
    thr = O3.threshold_table3(g.s, levels, eps, "capped", np.float32)
    cache = {}

    def lossy(k):
        if k not in cache:
            c = np.stack([O3.decode_record3(pool, int(table[k, f, 0]), int(table[k, f, 1]), g.s, np.float32)
                          for f in range(19)])
            cache[k] = O3.inverse_3d(c, levels)
        return cache[k]

    npx = g.npx
    samples = [0, g.npatch - 1, (npx // 2) + npx * (npx // 3) + npx * npx * (npx - 2)]
    want = {}
    for q in samples:
        padded = O3.gather_ghosts3_one(lossy, g, q)
        new = O3.d3q19_bgk_update(padded, TAU).astype(np.float32)
        want[q] = O3.hard_threshold(O3.forward_3d(new, levels), thr)
    ctx.step(1)
    table2, pool2 = ctx.store()
    u = np.finfo(np.float32).eps
    for q in samples:
        got = np.stack([O3.decode_record3(pool2, int(table2[q, f, 0]), int(table2[q, f, 1]), g.s, np.float32)
                        for f in range(19)])
        w = want[q]
        delta = 1e-5 * float(np.max(np.abs(w)))
        flip = (got != 0) != (w != 0)
        near = np.abs(np.abs(np.where(got != 0, got, w)) - thr) <= delta
        assert np.all(near[flip]), (q, int(flip.sum()))
        assert np.max(np.abs(np.where(flip, 0.0, got - w))) <= delta, q
        assert 0 < np.count_nonzero(got) < got.size
    assert ctx.stats()["regrows"] == 0


def test_single_patch_grid_is_its_own_neighbour():
    """n = p: every halo plane and line comes from the patch itself (periodic)."""
    _say("3d single patch")
    n, p, levels, eps = 16, 16, 3, 1e-3
    g = O3.Geometry3(n, p, levels)
    twin = O3.CompressedRun3(g, TAU, eps, dtype=np.float32)
    twin.set_grid(_oracle_state(n, 7, np.float32))
    table, pool = twin.store()
    ctx = _ctx(n, p, levels, eps)
    ctx.put_store(table, pool)
    ctx.step(1)
    twin.step(1)
    got, _, _ = _tiles(ctx)
    want = twin.coef
    delta = 256 * np.finfo(np.float32).eps * float(np.max(np.abs(want)))
    flip = (got != 0) != (want != 0)
    near = np.abs(np.abs(np.where(got != 0, got, want)) - twin.thr) <= delta
    assert np.all(near[flip])
    assert np.max(np.abs(np.where(flip, 0.0, got - want))) <= delta


def test_set_field_per_population():
    _say("3d set_field")
    n, p, levels = 32, 16, 2
    f0 = _oracle_state(n, 8, np.float32)
    ctx = _ctx(n, p, levels, 0.0)
    for i in range(19):
        ctx.set_field(i, f0[i])
    got = ctx.fields()
    assert np.max(np.abs(got - f0)) <= 2e-6 * np.max(np.abs(f0))
    ctx.step(2)
    ref = f0.astype(np.float64)
    for _ in range(2):
        ref = O3.dense_step3(ref, TAU)
    assert np.linalg.norm(ctx.fields() - ref) / np.linalg.norm(ref) <= 1e-5
