"""Pins of the oracle's patch loop (Sections 3.1.1 and 3.1.3, Introduction).

* the patch loop with ghosts from the neighbours' lossy tiles equals the
  paper's whole-grid protocol (decompress all, step, recompress) bit for bit;
* shared bordering nodes stay bit-identical in the tiles that share them;
* a zero threshold nullifies nothing (Section 3.1.3), so the compressed run
  tracks the uncompressed scheme to round-off;
* the global total is conserved by the lossy method (Section 3.1.1);
* the order in which patches are processed does not matter.
"""
import numpy as np
import pytest

from oracle import lbmz_oracle as O
from synth import fv_gaussians_and_step, random_signal, shear_layer_macroscopic

CASES = [
    ("fv_upwind", O.HAAR, 64, 16, 3, 1e-3),
    ("fv_upwind", O.BL53, 64, 16, 3, 1e-3),
    ("d2q9_bgk", O.BL53, 64, 16, 3, 1e-4),
    ("d2q9_bgk", O.HAAR, 32, 8, 2, 1e-4),
]


def _initial(kind, n, seed=0):
    if kind == "fv_upwind":
        return fv_gaussians_and_step(n, seed=seed, step_side=n // 4)[None]
    rho, ux, uy = shear_layer_macroscopic(n, seed=seed, kappa=20.0)
    return O.d2q9_equilibrium(rho, ux, uy)


def _scheme(kind):
    return O.Scheme(kind, vel=(1.0, 0.5), cfl=0.5, tau=0.6)


def test_gather_ghosts_matches_periodic_padding():
    for wavelet in (O.BL53, O.HAAR):
        g = O.Geometry(32, 8, wavelet, 2)
        grid = random_signal((2, 32, 32), seed=1)
        tiles = O.extract_tiles(grid, g)
        padded = O.gather_ghosts(tiles, g)
        big = np.pad(grid, ((0, 0), (1, 1), (1, 1)), mode="wrap")
        for py in range(g.npx):
            for px in range(g.npx):
                want = big[:, py * 8:py * 8 + g.s + 2, px * 8:px * 8 + g.s + 2] if wavelet == O.HAAR \
                    else np.pad(grid, ((0, 0), (1, 2), (1, 2)), mode="wrap")[
                        :, py * 8:py * 8 + g.s + 2, px * 8:px * 8 + g.s + 2]
                assert np.array_equal(padded[px + g.npx * py], want)


@pytest.mark.parametrize("kind,wavelet,n,p,L,eps", CASES)
def test_patch_loop_equals_whole_grid_protocol(kind, wavelet, n, p, L, eps):
    g = O.Geometry(n, p, wavelet, L)
    a = O.CompressedRun(g, _scheme(kind), eps)
    b = O.CompressedRun(g, _scheme(kind), eps)
    init = _initial(kind, n)
    a.set_grid(init)
    b.set_grid(init)
    for _ in range(4):
        a.step()
        O.whole_grid_step(b)
        assert np.array_equal(a.coef, b.coef)
    assert np.count_nonzero(a.coef) < a.coef.size      # the threshold did act


@pytest.mark.parametrize("kind,wavelet,n,p,L,eps", CASES)
def test_shared_nodes_stay_identical(kind, wavelet, n, p, L, eps):
    if wavelet != O.BL53:
        pytest.skip("Haar tiles do not overlap")
    g = O.Geometry(n, p, wavelet, L)
    run = O.CompressedRun(g, _scheme(kind), eps)
    run.set_grid(_initial(kind, n))
    run.step(3)
    lossy = run.decompress_tiles()
    for py in range(g.npx):
        for px in range(g.npx):
            q = px + g.npx * py
            right = ((px + 1) % g.npx) + g.npx * py
            up = px + g.npx * ((py + 1) % g.npx)
            assert np.array_equal(lossy[q][:, :, p], lossy[right][:, :, 0])
            assert np.array_equal(lossy[q][:, p, :], lossy[up][:, 0, :])


@pytest.mark.parametrize("kind,wavelet,n,p,L,eps", CASES)
def test_zero_threshold_tracks_uncompressed_scheme(kind, wavelet, n, p, L, eps):
    g = O.Geometry(n, p, wavelet, L)
    run = O.CompressedRun(g, _scheme(kind), 0.0)
    init = _initial(kind, n)
    run.set_grid(init)
    ref = init.copy()
    for _ in range(5):
        run.step()
        ref = O.dense_step(ref, _scheme(kind))
    assert np.max(np.abs(run.grid() - ref)) <= 1e-13 * np.max(np.abs(ref))


@pytest.mark.parametrize("kind,wavelet,n,p,L,eps", CASES)
def test_global_total_conserved_with_threshold(kind, wavelet, n, p, L, eps):
    g = O.Geometry(n, p, wavelet, L)
    run = O.CompressedRun(g, _scheme(kind), 30 * eps)
    init = _initial(kind, n)
    run.set_grid(init)
    t0 = run.field_totals()
    for _ in range(4):
        run.step()
    t1 = run.field_totals()
    scale = np.abs(init).sum()
    # total over all fields (LBM collision exchanges mass between populations)
    assert abs(t1.sum() - t0.sum()) <= 1e-13 * scale
    if kind == "d2q9_bgk":
        c = O.D2Q9_C
        for a in (0, 1):
            assert abs((c[:, a] * t1).sum() - (c[:, a] * t0).sum()) <= 1e-13 * scale
    # and the trapezoid totals equal the unique-node sums of the global grid
    assert abs(run.grid().astype(np.float64).sum() - t1.sum()) <= 1e-13 * scale


def test_patch_order_does_not_matter():
    kind, wavelet, n, p, L, eps = CASES[2]
    g = O.Geometry(n, p, wavelet, L)
    run = O.CompressedRun(g, _scheme(kind), eps)
    run.set_grid(_initial(kind, n))
    lossy = run.decompress_tiles()
    padded = O.gather_ghosts(lossy, g)
    rng = np.random.default_rng(11)
    coef = np.empty_like(run.coef)
    for q in rng.permutation(g.npatch):
        coef[q] = run.compress_tiles(run.scheme.update(padded[q:q + 1]))[0]
    run.step()
    assert np.array_equal(coef, run.coef)


# ---------------------------------------------------------------- per-patch controls

def _controls(g, seed=0):
    """Mixed per-patch threshold constants and threshold level counts."""
    rng = np.random.default_rng(seed)
    eps = 10.0 ** rng.uniform(-5, -3, g.npatch)
    lev = rng.integers(max(g.levels - 2, 0), g.levels + 1, size=g.npatch)
    return eps, lev


@pytest.mark.parametrize("kind,wavelet,n,p,L,eps", CASES)
def test_uniform_controls_change_nothing(kind, wavelet, n, p, L, eps):
    g = O.Geometry(n, p, wavelet, L)
    a = O.CompressedRun(g, _scheme(kind), eps)
    b = O.CompressedRun(g, _scheme(kind), eps)
    b.set_patch_eps(np.full(g.npatch, eps))
    b.set_patch_levels(np.full(g.npatch, L))
    init = _initial(kind, n)
    a.set_grid(init)
    b.set_grid(init)
    for _ in range(3):
        a.step()
        b.step()
    assert np.array_equal(a.coef, b.coef)


@pytest.mark.parametrize("kind,wavelet,n,p,L,eps", CASES)
def test_mixed_controls_keep_shared_faces_and_the_protocol(kind, wavelet, n, p, L, eps):
    # per-patch constants and level counts: the shared bordering lines take the
    # smaller threshold of their two tiles, so both tiles reconstruct the same
    # values there, the patch loop still equals the whole-grid protocol bit for
    # bit, and the global total is conserved
    g = O.Geometry(n, p, wavelet, L)
    e, lev = _controls(g, seed=n + p)
    runs = []
    for _ in range(2):
        r = O.CompressedRun(g, _scheme(kind), eps)
        r.set_patch_eps(e)
        r.set_patch_levels(lev)
        r.set_grid(_initial(kind, n))
        runs.append(r)
    a, b = runs
    m0 = a.field_totals()
    for _ in range(4):
        a.step()
        O.whole_grid_step(b)
        assert np.array_equal(a.coef, b.coef)
    m1 = a.field_totals()
    if kind == "d2q9_bgk":          # mass and momentum of the populations
        c = O.D2Q9_C
        m0 = np.array([m0.sum(), (c[:, 0] * m0).sum(), (c[:, 1] * m0).sum()])
        m1 = np.array([m1.sum(), (c[:, 0] * m1).sum(), (c[:, 1] * m1).sum()])
    assert np.all(np.abs(m1 - m0) <= 1e-13 * np.abs(m0).sum())
    if wavelet == O.BL53:
        lossy = a.decompress_tiles()
        for py in range(g.npx):
            for px in range(g.npx):
                q = px + g.npx * py
                right = ((px + 1) % g.npx) + g.npx * py
                up = px + g.npx * ((py + 1) % g.npx)
                assert np.array_equal(lossy[q][:, :, p], lossy[right][:, :, 0])
                assert np.array_equal(lossy[q][:, p, :], lossy[up][:, 0, :])


def test_face_thresholds_are_the_smaller_of_the_two_tiles():
    g = O.Geometry(64, 16, O.BL53, 3)
    r = O.CompressedRun(g, _scheme("d2q9_bgk"), 1e-4)
    e, lev = _controls(g, seed=5)
    r.set_patch_eps(e)
    r.set_patch_levels(lev)
    base = [O.threshold_table(g.s, int(lev[q]), float(e[q]), O.RULE_CAPPED, np.float64) for q in range(g.npatch)]
    q, right, up = 5, 6, 9                                    # px = 1, py = 1 on the 4 x 4 patch grid
    thr = r.thr[:, 0]
    assert np.array_equal(thr[q][1:-1, 1:-1], base[q][1:-1, 1:-1])      # interior: the patch's own table
    assert np.array_equal(thr[q][:, 16], np.minimum(base[q][:, 16], base[right][:, 0]))
    assert np.array_equal(thr[q][16, :], np.minimum(base[q][16, :], base[up][0, :]))
    assert np.array_equal(thr[q][:, 16], thr[right][:, 0])               # one threshold per shared entry
    assert thr[q][0, 0] == 0 and thr[q][16, 16] == 0                      # corners are samples


def test_level_count_semantics():
    # L_q = 0 zeroes nothing; a smaller level count thresholds fewer levels,
    # with ranks counted from the coarsest thresholded one
    s, L, eps = 17, 3, 1e-3
    t0 = O.threshold_table(s, 0, eps, O.RULE_CAPPED, np.float64)
    assert np.all(t0 == 0)
    t3 = O.threshold_table(s, 3, eps, O.RULE_CAPPED, np.float64)
    t2 = O.threshold_table(s, 2, eps, O.RULE_CAPPED, np.float64)
    assert t3[0, 1] == eps * 4 and t2[0, 1] == eps * 2          # finest detail: rank L_q - 1
    assert t3[0, 4] == eps * 1 and t2[0, 4] == 0                # level 3 kept like a sample at L_q = 2
    assert np.all(t2 <= t3)


def test_smaller_level_counts_keep_more_coefficients():
    kind, wavelet, n, p, L, eps = CASES[2]
    g = O.Geometry(n, p, wavelet, L)
    kept = []
    for lv in (L, L - 1, L - 2, 0):
        r = O.CompressedRun(g, _scheme(kind), eps)
        r.set_patch_levels(np.full(g.npatch, lv))
        r.set_grid(_initial(kind, n))
        kept.append(int(r.nnz().sum()))
    assert kept[0] < kept[1] < kept[2] < kept[3]
    assert kept[3] == int(np.count_nonzero(r.coef))
