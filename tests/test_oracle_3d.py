"""Pins of the 3-D oracle (D3Q19 BGK, tensor 3-D transform, 3-D thresholds,
records, ghost layer) against the lattice's moment identities, closed forms,
brute force and the 2-D oracle's already pinned parts."""
import itertools
import math

import numpy as np
import pytest

from oracle import lbmz_oracle as O
from oracle import lbmz_oracle3d as O3
from synth import taylor_green_jets_3d


# -- D3Q19 lattice --------------------------------------------------------------

def test_lattice_moments_are_isotropic():
    """Textbook moment identities of the D3Q19 set: sum w = 1, odd moments
    vanish, second moment = delta / 3, fourth moment = (dd + dd + dd) / 9."""
    c = O3.D3Q19_C.astype(np.float64)
    w = O3.D3Q19_W
    assert len({tuple(v) for v in O3.D3Q19_C}) == 19
    assert np.isclose(w.sum(), 1.0)
    assert np.allclose(w @ c, 0.0)
    d = np.eye(3)
    assert np.allclose(np.einsum("i,ia,ib->ab", w, c, c), d / 3.0)
    assert np.allclose(np.einsum("i,ia,ib,ic->abc", w, c, c, c), 0.0)
    m4 = np.einsum("i,ia,ib,ic,id->abcd", w, c, c, c, c)
    want = (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d) + np.einsum("ad,bc->abcd", d, d)) / 9.0
    assert np.allclose(m4, want)
    # every velocity has its opposite; no corner (three non-zero components) velocities
    assert all(tuple(-v) in {tuple(u) for u in O3.D3Q19_C} for v in O3.D3Q19_C)
    assert np.abs(O3.D3Q19_C).sum(axis=1).max() == 2


def test_equilibrium_moments():
    rng = np.random.default_rng(0)
    rho = 1.0 + 0.1 * rng.random((2, 3, 4))
    u = 0.05 * rng.standard_normal((3, 2, 3, 4))
    feq = O3.d3q19_equilibrium(rho, *u)
    r, ux, uy, uz = O3.d3q19_moments(feq)
    assert np.allclose(r, rho, rtol=1e-14)
    assert np.allclose(np.stack([ux, uy, uz]), u, atol=1e-15)
    c = O3.D3Q19_C.astype(np.float64)
    pi = np.einsum("i...,ia,ib->ab...", feq, c, c)
    want = rho * (np.eye(3)[:, :, None, None, None] / 3.0 + u[:, None] * u[None, :])
    assert np.allclose(pi, want, atol=1e-14)


def test_collision_conserves_mass_and_momentum_and_fixes_equilibrium():
    rng = np.random.default_rng(1)
    f = 0.05 * (1.0 + 0.3 * rng.random((19, 3, 3, 3)))
    post = O3.d3q19_collide(f, 0.7)
    a, b = O3.d3q19_moments(f), O3.d3q19_moments(post)
    assert np.allclose(a[0], b[0], rtol=1e-14)
    for k in range(1, 4):
        assert np.allclose(a[0] * a[k], b[0] * b[k], atol=1e-15)
    feq = O3.d3q19_equilibrium(a[0], a[1], a[2], a[3])
    assert np.allclose(O3.d3q19_collide(feq, 0.7), feq, atol=1e-16)


def test_streaming_is_a_periodic_roll():
    rng = np.random.default_rng(2)
    g = rng.random((19, 5, 6, 7))
    fin = O3.d3q19_stream(O3.periodic_pad3(g))
    for i in range(19):
        cx, cy, cz = (int(v) for v in O3.D3Q19_C[i])
        assert np.array_equal(fin[i], np.roll(g[i], shift=(cz, cy, cx), axis=(0, 1, 2)))


def test_shear_wave_decays_at_the_bgk_viscosity():
    """u_x(y) = U sin(k y) decays as exp(-nu k^2 t), nu = (tau - 1/2) / 3 (lattice units)."""
    n, tau, steps, amp = 64, 0.8, 150, 1e-3
    y = np.arange(n, dtype=np.float64)
    k = 2.0 * math.pi / n
    ux = np.broadcast_to(amp * np.sin(k * y)[None, :, None], (2, n, 2)).copy()
    z = np.zeros_like(ux)
    f = O3.d3q19_equilibrium(np.ones_like(ux), ux, z, z)
    for _ in range(steps):
        f = O3.dense_step3(f, tau)
    _, u, _, _ = O3.d3q19_moments(f)
    got = float(np.sum(u[0, :, 0] * np.sin(k * y)) / np.sum(np.sin(k * y) ** 2))
    nu = (tau - 0.5) / 3.0
    assert abs(got / (amp * math.exp(-nu * k * k * steps)) - 1.0) < 2e-3


# -- transform and threshold ------------------------------------------------------

@pytest.mark.parametrize("s,levels", [(9, 2), (17, 3)])
def test_transform_is_the_tensor_product_of_1d_transforms(s, levels):
    rng = np.random.default_rng(3)
    a, b, c = (rng.standard_normal(s) for _ in range(3))
    tile = c[:, None, None] * b[None, :, None] * a[None, None, :]
    ta, tb, tc = (O.forward_1d(v, levels, O.BL53) for v in (a, b, c))
    want = tc[:, None, None] * tb[None, :, None] * ta[None, None, :]
    got = O3.forward_3d(tile, levels)
    assert np.allclose(got, want, atol=1e-13)
    assert np.allclose(O3.inverse_3d(got, levels), tile, atol=1e-13)


def test_transform_round_trip_and_direction_symmetry():
    rng = np.random.default_rng(4)
    t = rng.standard_normal((2, 17, 17, 17))
    c = O3.forward_3d(t, 3)
    assert np.allclose(O3.inverse_3d(c, 3), t, atol=1e-12)
    # the three directions commute: transposing the tile transposes the coefficients
    assert np.allclose(O3.forward_3d(np.swapaxes(t, -1, -3), 3), np.swapaxes(c, -1, -3), atol=1e-12)


@pytest.mark.parametrize("levels", [1, 2, 3])
def test_trapezoid_mass_equals_coarse_sample_mass(levels):
    """Equation "conservation" per dimension: the trapezoid mass of the tile is
    8^L times the trapezoid mass of the coarse samples, whatever the details."""
    rng = np.random.default_rng(5)
    s = 17
    t = rng.standard_normal((s, s, s))
    c = O3.forward_3d(t, levels)
    g = O3.Geometry3(16, 16, levels)
    mass = float((t * O3.tile_weights3(g)).sum())
    st = 1 << levels
    samp = c[::st, ::st, ::st]
    w1 = np.ones(samp.shape[0])
    w1[0] = w1[-1] = 0.5
    cmass = float((samp * w1[:, None, None] * w1[None, :, None] * w1[None, None, :]).sum())
    assert abs(mass - 8 ** levels * cmass) < 1e-11 * np.abs(t).sum()
    # zeroing every detail keeps that mass
    only = np.zeros_like(c)
    only[::st, ::st, ::st] = samp
    rec = O3.inverse_3d(only, levels)
    assert abs(float((rec * O3.tile_weights3(g)).sum()) - mass) < 1e-11 * np.abs(t).sum()


@pytest.mark.parametrize("rule", [O.RULE_CAPPED, O.RULE_CONSTANT, O.RULE_ACCUM])
def test_threshold_table_by_brute_force(rule):
    s, levels, eps = 17, 3, 1e-3
    thr = O3.threshold_table3(s, levels, eps, rule, np.float64)

    def rank(i):
        if i % (1 << levels) == 0:
            return None
        lev = 1
        while i % 2 == 0:
            i //= 2
            lev += 1
        return levels - lev

    for z, y, x in itertools.product(range(s), repeat=3):
        rs = [rank(v) for v in (x, y, z)]
        if all(r is None for r in rs):
            assert thr[z, y, x] == 0.0
            continue
        rr = [0 if r is None else r for r in rs]
        r = {O.RULE_CAPPED: max(rr), O.RULE_CONSTANT: 0, O.RULE_ACCUM: sum(rr)}[rule]
        assert thr[z, y, x] == eps * 2.0 ** r
    # a plane at a sample index in z reduces to the 2-D table (pinned separately)
    assert np.array_equal(thr[0], O.threshold_table(s, levels, eps, rule, np.float64))
    assert np.count_nonzero(thr == 0) == ((s - 1) // 8 + 1) ** 3


# -- records ---------------------------------------------------------------------

@pytest.mark.parametrize("density", [0.0, 0.01, 0.2, 1.0])
def test_records_round_trip_and_brute_force_layout(density):
    rng = np.random.default_rng(6)
    s = 17
    tile = rng.standard_normal((s, s, s)).astype(np.float32)
    tile[rng.random(tile.shape) >= density] = 0
    rec = O3.encode_record3(tile)
    nnz = int(np.count_nonzero(tile))
    w = (s ** 3 + 63) // 64
    is_mask = 2 * nnz >= 8 * w
    assert len(rec) == O3.record_layout3(nnz, s ** 3, 4)[3]
    vals = np.frombuffer(rec, dtype="<f4", count=nnz)
    flat = tile.reshape(-1)
    assert np.array_equal(vals, flat[flat != 0])
    vb = (4 * nnz + 7) // 8 * 8
    if is_mask:
        words = np.frombuffer(rec, dtype="<u8", count=w, offset=vb)
        for k in range(s ** 3):
            assert ((int(words[k // 64]) >> (k % 64)) & 1) == (flat[k] != 0)
    else:
        idx = np.frombuffer(rec, dtype="<u2", count=nnz, offset=vb)
        assert np.array_equal(idx, np.flatnonzero(flat))
    word = nnz | (O.MASK_BIT if is_mask else 0)
    assert np.array_equal(O3.decode_record3(rec, 0, word, s, np.float32), tile)


# -- the patch loop ------------------------------------------------------------------

def _state(n, seed=0, dtype=np.float64):
    rho, ux, uy, uz = taylor_green_jets_3d(n, seed=seed, n_jets=2, dtype=np.float64)
    return O3.d3q19_equilibrium(rho, ux, uy, uz).astype(dtype)


def test_ghost_layer_matches_the_periodic_grid():
    g = O3.Geometry3(24, 8, 2)
    rng = np.random.default_rng(7)
    grid = rng.standard_normal((2, 24, 24, 24))
    tiles = O3.extract_tiles3(grid, g)
    pad = O3.gather_ghosts3(tiles, g)
    full = np.pad(grid, ((0, 0), (1, 1), (1, 1), (1, 1)), mode="wrap")
    big = np.pad(grid, ((0, 0), (1, 2), (1, 2), (1, 2)), mode="wrap")   # nodes -1 .. n + 1
    for q in range(g.npatch):
        px, py, pz = g.patch_coords(q)
        want = big[:, pz * 8:pz * 8 + 11, py * 8:py * 8 + 11, px * 8:px * 8 + 11]
        assert np.array_equal(pad[q], want)
    assert np.array_equal(O3.assemble_grid3(tiles, g), grid)
    assert full.shape[-1] == 26


def test_patch_loop_equals_whole_grid_protocol():
    g = O3.Geometry3(24, 8, 2)
    a = O3.CompressedRun3(g, tau=0.55, eps=1e-4)
    b = O3.CompressedRun3(g, tau=0.55, eps=1e-4)
    f0 = _state(24, seed=1)
    a.set_grid(f0)
    b.set_grid(f0)
    for _ in range(3):
        a.step(1)
        O3.whole_grid_step3(b)
        assert np.array_equal(a.coef, b.coef)
    assert 0 < a.nnz().sum() < a.coef.size


def test_eps_zero_equals_the_uncompressed_scheme():
    g = O3.Geometry3(32, 16, 3)
    run = O3.CompressedRun3(g, tau=0.55, eps=0.0)
    f = _state(32, seed=2)
    run.set_grid(f)
    for _ in range(4):
        f = O3.dense_step3(f, 0.55)
    run.step(4)
    assert np.max(np.abs(run.grid() - f)) < 1e-13


def test_mass_and_momentum_are_conserved_at_eps_above_zero():
    g = O3.Geometry3(32, 16, 3)
    run = O3.CompressedRun3(g, tau=0.55, eps=1e-3)
    run.set_grid(_state(32, seed=3))
    t0 = run.field_totals()
    c = O3.D3Q19_C.astype(np.float64)
    run.step(3)
    t1 = run.field_totals()
    assert abs(t1.sum() - t0.sum()) < 1e-12 * abs(t0.sum())
    assert np.allclose(t1 @ c, t0 @ c, atol=1e-12 * abs(t0.sum()))
    assert run.ratio() > 2.0


def test_shared_faces_agree_between_neighbours():
    g = O3.Geometry3(32, 16, 3)
    run = O3.CompressedRun3(g, tau=0.55, eps=1e-3)
    run.set_grid(_state(32, seed=4))
    run.step(2)
    lossy = run.decompress_tiles()
    for q in range(g.npatch):
        px, py, pz = g.patch_coords(q)
        nxq = (px + 1) % g.npx + g.npx * py + g.npx ** 2 * pz
        assert np.array_equal(lossy[q, :, :, :, -1], lossy[nxq, :, :, :, 0])
        nzq = px + g.npx * py + g.npx ** 2 * ((pz + 1) % g.npx)
        assert np.array_equal(lossy[q, :, -1], lossy[nzq, :, 0])
