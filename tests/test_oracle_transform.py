"""Pins of the oracle's wavelet transforms against what the paper and mathematics fix.

* the printed 9x9 matrices A and A^-1 of one folded BL5/3 level (Section 2.1.2);
* exact cancellation of linear signals ("filters out linear polynomials");
* the mass-conservation identity (equation "conservation"), and its failure
  one level beyond the cap, which is why the API caps bl53 at J - 1 levels;
* perfect reconstruction (the transform is bijective, Section 2.1.1);
* Haar: mean and weighted-energy identities in closed form.
"""
import numpy as np
import pytest

from oracle import lbmz_oracle as O
from synth import random_signal


def _matrix(level_fn, n):
    m = np.zeros((n, n))
    for i in range(n):
        e = np.zeros(n)
        e[i] = 1.0
        m[:, i] = level_fn(e)
    return m


def test_bl53_matrix_matches_printed_A(golden):
    rows = [list(map(float, ln.split())) for ln in golden("bl53_matrix_j3.txt")]
    a8 = np.array(rows[:9])
    ainv8 = np.array(rows[9:18])
    assert np.array_equal(8.0 * _matrix(O.bl53_forward_level, 9), a8)
    assert np.array_equal(8.0 * _matrix(O.bl53_inverse_level, 9), ainv8)
    # and the two printed matrices are inverse to each other
    assert np.array_equal(a8 @ ainv8, 64.0 * np.eye(9))


@pytest.mark.parametrize("j", [2, 3, 4, 5, 6, 7])
def test_bl53_kills_linear_signals(j):
    n = (1 << j) + 1
    i = np.arange(n, dtype=np.float64)
    u = 3.0 - 5.0 * i                      # dyadic-exact linear ramp
    for L in range(1, j):
        v = O.forward_1d(u, L, O.BL53)
        lev = O.index_levels(n, L)
        assert np.all(v[lev > 0] == 0.0), (j, L)


def _trapezoid_mass(u):
    w = np.ones(u.shape[-1])
    w[0] = w[-1] = 0.5
    return float((u * w).sum())


@pytest.mark.parametrize("j", [2, 3, 4, 5, 6, 7])
def test_bl53_mass_conserved_under_any_detail_zeroing(j):
    n = (1 << j) + 1
    rng = np.random.default_rng(j)
    for L in range(1, j):
        for trial in range(20):
            u = rng.standard_normal(n)
            v = O.forward_1d(u, L, O.BL53)
            lev = O.index_levels(n, L)
            drop = (lev > 0) & (rng.uniform(size=n) < rng.uniform())
            v2 = v.copy()
            v2[drop] = 0.0
            u2 = O.inverse_1d(v2, L, O.BL53)
            scale = np.abs(u).sum()
            assert abs(_trapezoid_mass(u2) - _trapezoid_mass(u)) <= 1e-13 * scale
            # the samples alone carry the mass: coarse trapezoid times 2^L
            lev_s = v[::1 << L]
            assert abs((1 << L) * _trapezoid_mass(lev_s) - _trapezoid_mass(u)) <= 1e-13 * scale


@pytest.mark.parametrize("j", [2, 3, 4, 5])
def test_bl53_one_level_past_the_cap_breaks_conservation(j):
    # With L = J the last level acts on 3 samples and has no update step,
    # so zeroing its detail moves mass: the reason L <= J - 1 is enforced.
    n = (1 << j) + 1
    rng = np.random.default_rng(100 + j)
    u = rng.standard_normal(n)
    v = O.forward_1d(u, j, O.BL53)
    v[n // 2] = 0.0                          # the single coarsest detail
    u2 = O.inverse_1d(v, j, O.BL53)
    assert abs(_trapezoid_mass(u2) - _trapezoid_mass(u)) > 1e-3


@pytest.mark.parametrize("wavelet,p", [(O.BL53, 8), (O.BL53, 64), (O.HAAR, 8), (O.HAAR, 32)])
def test_perfect_reconstruction_2d(wavelet, p):
    s = p + 1 if wavelet == O.BL53 else p
    j = p.bit_length() - 1
    cap = j - 1 if wavelet == O.BL53 else j
    for dtype, tol in [(np.float64, 1e-13), (np.float32, 3e-6)]:
        u = random_signal((3, s, s), seed=p, dtype=dtype)
        for L in range(0, cap + 1):
            c = O.forward_2d(u, L, wavelet)
            r = O.inverse_2d(c, L, wavelet)
            assert r.dtype == dtype
            assert np.max(np.abs(r - u)) <= tol * np.max(np.abs(u)), (L, dtype)


def test_2d_transform_is_rows_then_columns():
    # A tensor transform of a separable signal is the outer product of the 1-D ones.
    rng = np.random.default_rng(7)
    a = rng.standard_normal(33)
    b = rng.standard_normal(33)
    u = np.outer(b, a)                        # u[y, x] = b[y] a[x]
    c = O.forward_2d(u, 3, O.BL53)
    expect = np.outer(O.forward_1d(b, 3, O.BL53), O.forward_1d(a, 3, O.BL53))
    assert np.allclose(c, expect, rtol=0, atol=1e-13)


def test_index_levels_brute_force():
    # Independent derivation: the level-lev details are the odd points of the
    # sub-lattice of stride 2^(lev-1), for lev = 1 .. L; everything else is a sample.
    for s, L in [(65, 5), (65, 1), (32, 4), (129, 6), (16, 4)]:
        expect = np.zeros(s, dtype=np.int64)
        for lev in range(1, L + 1):
            st = 1 << (lev - 1)
            pts = list(range(0, s, st))
            for k, pos in enumerate(pts):
                if k % 2 == 1:
                    expect[pos] = lev
        assert np.array_equal(O.index_levels(s, L), expect), (s, L)


@pytest.mark.parametrize("L", [1, 2, 3, 4, 5])
def test_haar_mean_and_weighted_energy(L):
    p = 32
    u = random_signal((p, p), seed=L)
    c = O.forward_2d(u, L, O.HAAR)
    lev = O.index_levels(p, L)
    # 1-D weights: 2^L for a sample, 2^(lev-2) for a level-lev detail
    w1 = np.where(lev == 0, float(1 << L), 2.0 ** (lev - 2))
    w = w1[:, None] * w1[None, :]
    assert abs((u * u).sum() - (w * c * c).sum()) <= 1e-12 * (u * u).sum()
    samples = c[::1 << L, ::1 << L]
    assert abs(u.sum() - (1 << (2 * L)) * samples.sum()) <= 1e-12 * np.abs(u).sum()


def test_haar_one_level_is_pairwise_mean_and_difference():
    u = np.array([1.0, 3.0, -2.0, 6.0])
    v = O.forward_1d(u, 1, O.HAAR)
    assert np.array_equal(v, [2.0, 2.0, 2.0, 8.0])
