"""Host logic of the learned threshold controller (CPU)."""
import numpy as np

from paper_2302_09883_amd import learned as Lr


def _preds(npatch, seed):
    """Predicted log10 errors and bytes of the K candidates: within each
    threshold level count, the error rises and the bytes fall with eps."""
    rng = np.random.default_rng(seed)
    e = np.empty((npatch, Lr.K))
    b = np.empty((npatch, Lr.K))
    for k, (eps, lev) in enumerate(Lr.CANDIDATES):
        e[:, k] = np.log10(eps) * 2 - 0.5 * (5 - lev) + rng.normal(0, 0.2, npatch)
        b[:, k] = 4.0 - 0.4 * np.log10(eps / 1e-5) + 0.15 * (5 - lev) + rng.normal(0, 0.05, npatch)
    return e, b


def test_candidates_and_fixed_index():
    assert Lr.K == len(Lr.EPS) * len(Lr.LEVS)
    for eps in Lr.EPS:
        assert Lr.CANDIDATES[Lr.candidate_index(eps)] == (eps, Lr.LEVELS)


def test_hull_is_convex_and_decreasing():
    rng = np.random.default_rng(3)
    for _ in range(50):
        e = rng.normal(size=Lr.K)
        b = rng.normal(size=Lr.K)
        ch = Lr._hull(e, b)
        assert ch[0] == min(range(Lr.K), key=lambda k: (b[k], e[k]))
        for i in range(1, len(ch)):
            assert b[ch[i]] > b[ch[i - 1]] and e[ch[i]] < e[ch[i - 1]]
        slopes = [(e[ch[i]] - e[ch[i - 1]]) / (b[ch[i]] - b[ch[i - 1]]) for i in range(1, len(ch))]
        assert all(s0 <= s1 + 1e-12 for s0, s1 in zip(slopes, slopes[1:]))   # convex: slopes rise
        # no candidate lies below the chain
        for k in range(Lr.K):
            for i in range(1, len(ch)):
                k0, k1 = ch[i - 1], ch[i]
                if b[k0] < b[k] < b[k1]:
                    line = e[k0] + (e[k1] - e[k0]) * (b[k] - b[k0]) / (b[k1] - b[k0])
                    assert e[k] >= line - 1e-12


def test_allocation_keeps_the_predicted_error_within_the_fallback_budget():
    e, b = _preds(40, 0)
    fb = Lr.candidate_index(1e-4)
    idx = Lr.allocate(e, b, None, fb)
    pe = np.power(10.0, e)
    assert np.sum(pe[np.arange(40), idx]) <= np.sum(pe[:, fb]) * (1 + 1e-12)
    # and it spends fewer predicted bytes than the fixed candidate where the hull allows
    pb = np.power(10.0, b)
    assert np.sum(pb[np.arange(40), idx]) <= np.sum(pb[:, fb])


def test_non_finite_rows_fall_back_and_do_not_move_the_others():
    e, b = _preds(30, 1)
    fb = Lr.candidate_index(1e-4)
    clean = Lr.allocate(e, b, None, fb)
    e2 = np.vstack([e[:10], np.full((1, Lr.K), np.nan), e[10:20], np.full((1, Lr.K), np.inf), e[20:]])
    b2 = np.vstack([b[:10], b[:1], b[10:20], b[:1], b[20:]])
    got = Lr.allocate(e2, b2, None, fb)
    assert got[10] == fb and got[21] == fb
    assert np.array_equal(np.delete(got, [10, 21]), clean)
    b3 = b2.copy()
    b3[5, 3] = np.nan
    got3 = Lr.allocate(e2, b3, None, fb)
    assert got3[5] == fb


def test_ratio_at_error_interpolates_in_log_log():
    sweep = [{"eps": 1e-5, "rel_l2": 1e-4, "ratio_mean": 100.0}, {"eps": 1e-4, "rel_l2": 1e-2, "ratio_mean": 400.0}]
    assert abs(Lr.ratio_at_error(sweep, 1e-3) - 200.0) < 1e-9
    assert Lr.ratio_at_error(sweep, 1e-1) is None
