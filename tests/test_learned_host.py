"""Host logic of the learned threshold controller (CPU)."""
import numpy as np

from paper_2302_09883_amd import learned as Lr


def _preds(npatch, seed):
    rng = np.random.default_rng(seed)
    # error falls and bytes rise towards the smaller candidates (index 0)
    e = np.sort(rng.uniform(-12, -6, size=(npatch, Lr.K)), axis=1)
    b = np.sort(rng.uniform(2, 5, size=(npatch, Lr.K)), axis=1)[:, ::-1]
    return e, b


def test_allocation_keeps_the_predicted_error_within_the_fallback_budget():
    e, b = _preds(40, 0)
    fb = 2
    idx = Lr.allocate(e, b, None, fb)
    pe = np.power(10.0, e)
    assert np.sum(pe[np.arange(40), idx]) <= np.sum(pe[:, fb]) * (1 + 1e-12)


def test_non_finite_rows_fall_back_and_do_not_move_the_others():
    e, b = _preds(30, 1)
    fb = 2
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
