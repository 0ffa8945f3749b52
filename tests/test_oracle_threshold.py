"""Pins of thresholding and compaction in the oracle.

* the worked example of Section 2.1.2 (481 non-null coefficients out of 16641
  with the constant rule at 0.2, 6 levels, 129 x 129), which also pins the 2-D
  decomposition order (rows then columns), the detail classification and the
  count of exact zeros;
* masses equal before and after thresholding, even with all details dropped;
* structural properties of the three rules of Section 2.2;
* the record encoding against a brute-force ``np.flatnonzero``.
"""
import numpy as np
import pytest

from oracle import lbmz_oracle as O
from synth import random_coefficient_tiles, worked_example_field


def _golden_kv(golden):
    return dict(ln.split() for ln in golden("worked_example.txt"))


def test_worked_example_481_nonzeros(golden):
    kv = _golden_kv(golden)
    n, L, thr = int(kv["grid"]), int(kv["levels"]), float(kv["threshold"])
    f = worked_example_field(n)
    c = O.forward_2d(f, L, O.BL53)
    t = O.threshold_table(n, L, thr, O.RULE_CONSTANT, np.float64)
    ct = O.hard_threshold(c, t)
    assert ct.size == int(kv["total"])
    assert np.count_nonzero(ct) == int(kv["nonzero"])
    # the same count in single precision
    c32 = O.forward_2d(f.astype(np.float32), L, O.BL53)
    t32 = O.threshold_table(n, L, thr, O.RULE_CONSTANT, np.float32)
    assert np.count_nonzero(O.hard_threshold(c32, t32)) == int(kv["nonzero"])


def test_worked_example_mass_conserved(golden):
    kv = _golden_kv(golden)
    n, L, thr = int(kv["grid"]), int(kv["levels"]), float(kv["threshold"])
    f = worked_example_field(n)
    w = np.ones(n)
    w[0] = w[-1] = 0.5
    w2 = w[:, None] * w[None, :]
    c = O.forward_2d(f, L, O.BL53)
    for t in (O.threshold_table(n, L, thr, O.RULE_CONSTANT, np.float64),
              O.threshold_table(n, L, np.inf, O.RULE_CONSTANT, np.float64)):
        r = O.inverse_2d(O.hard_threshold(c, t), L, O.BL53)
        assert abs((r * w2).sum() - (f * w2).sum()) <= 1e-12 * np.abs(f).sum()


def test_rules_coincide_with_one_level():
    for rule in (O.RULE_CAPPED, O.RULE_ACCUM):
        assert np.array_equal(O.threshold_table(65, 1, 1e-3, rule, np.float64),
                              O.threshold_table(65, 1, 1e-3, O.RULE_CONSTANT, np.float64))


def test_rule_ordering_and_coarsest_value():
    s, L, eps = 65, 5, 1e-4
    con = O.threshold_table(s, L, eps, O.RULE_CONSTANT, np.float64)
    cap = O.threshold_table(s, L, eps, O.RULE_CAPPED, np.float64)
    acc = O.threshold_table(s, L, eps, O.RULE_ACCUM, np.float64)
    assert np.all(con <= cap) and np.all(cap <= acc)
    lev = O.index_levels(s, L)
    # samples are never thresholded
    samp = (lev[:, None] == 0) & (lev[None, :] == 0)
    assert np.all(con[samp] == 0) and np.all(cap[samp] == 0) and np.all(acc[samp] == 0)
    # the coarsest detail (level L in x, sample in y) gets exactly eps
    x = 1 << (L - 1)
    assert cap[0, x] == eps and acc[0, x] == eps
    # the finest detail in both dims gets eps 2^(L-1) (capped) and eps 2^(2L-2) (accumulated)
    assert cap[1, 1] == eps * 2 ** (L - 1)
    assert acc[1, 1] == eps * 2 ** (2 * L - 2)


def test_threshold_is_strict_and_samples_survive():
    s, L = 9, 2
    c = np.full((s, s), 0.5)
    t = O.threshold_table(s, L, 0.5, O.RULE_CONSTANT, np.float64)
    out = O.hard_threshold(c, t)
    assert np.array_equal(out, c)                   # |c| == thr is kept
    t2 = O.threshold_table(s, L, 0.75, O.RULE_CONSTANT, np.float64)
    out2 = O.hard_threshold(c, t2)
    lev = O.index_levels(s, L)
    samp = (lev[:, None] == 0) & (lev[None, :] == 0)
    assert np.all(out2[samp] == 0.5) and np.all(out2[~samp] == 0)


def test_record_order_is_a_core_then_rim_permutation():
    for s in (9, 17, 65, 8, 32):
        order = O.record_order(s)
        assert np.array_equal(np.sort(order), np.arange(s * s))
        p = s - 1 if s % 2 else s
        # brute force: the owned block row by row comes first
        k = 0
        for y in range(p):
            for x in range(p):
                assert order[k] == y * s + x
                k += 1
        if p != s:
            assert list(order[k:k + p]) == [y * s + p for y in range(p)]
            assert list(order[k + p:k + 2 * p]) == [p * s + x for x in range(p)]
            assert order[-1] == p * s + p


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_record_roundtrip_and_brute_force(dtype):
    tiles = random_coefficient_tiles((6, 65, 65), seed=3, dtype=dtype, zero_frac=0.3)
    # vary density across the encoding switch (2 nnz < 8 W  <=>  nnz < 4 W = 268)
    tiles[1] = 0
    tiles[2] = 0
    tiles[2].reshape(-1)[[0, 64, 65, 4224]] = 1.5
    tiles[3] = 0
    tiles[3].reshape(-1)[:267] = 2.0
    tiles[4] = 0
    tiles[4].reshape(-1)[:268] = -3.0
    tiles[5].reshape(-1)[17] = np.nan
    order = O.record_order(65)
    for t in tiles:
        rec = O.encode_record(t)
        seq = t.reshape(-1)[order]
        nnz = int(np.count_nonzero(seq != 0))
        is_mask, vb, mb, rb = O.record_layout(nnz, seq.size, np.dtype(dtype).itemsize)
        assert len(rec) == rb and rb % 16 == 0
        assert is_mask == (nnz >= 268)
        word = nnz | (O.MASK_BIT if is_mask else 0)
        back = O.decode_record(rec, 0, word, 65, dtype)
        assert np.array_equal(back, np.where(t == 0, 0, t).astype(dtype), equal_nan=True)
        keep = np.flatnonzero(seq != 0)             # brute force
        vals = np.frombuffer(rec, dtype=dtype, count=nnz)
        assert np.array_equal(vals, seq[keep], equal_nan=True)
        if is_mask:
            words = np.frombuffer(rec, dtype="<u8", count=(seq.size + 63) // 64, offset=vb)
            bits = np.unpackbits(words.view(np.uint8), bitorder="little")[:seq.size]
            assert np.array_equal(np.flatnonzero(bits), keep)
        else:
            idx = np.frombuffer(rec, dtype="<u2", count=nnz, offset=vb)
            assert np.array_equal(idx, keep)
        assert all(b == 0 for b in rec[nnz * np.dtype(dtype).itemsize:vb])


def test_negative_zero_is_not_stored():
    t = np.zeros((65, 65), dtype=np.float32)
    t[0, 5] = -0.0
    t[0, 6] = 1.0
    rec = O.encode_record(t)
    assert len(rec) == 16                            # one value + one u16 index, padded
    assert np.frombuffer(rec, dtype="<u2", count=1, offset=8)[0] == 6


def test_store_placement_is_serial_prefix():
    tiles = random_coefficient_tiles((4, 2, 33, 33), seed=9, dtype=np.float64, zero_frac=0.9)
    table, pool = O.encode_store(tiles)
    off = 0
    for q in range(4):
        for f in range(2):
            assert table[q, f, 0] * 16 == off
            nnz = int(table[q, f, 1]) & (O.MASK_BIT - 1)
            off += O.record_layout(nnz, 33 * 33, 8)[3]
    assert off == len(pool)
    assert np.array_equal(O.decode_store(table, pool, 33, np.float64), tiles)
    assert O.store_bytes(table, 33, 8) == len(pool) + table.size * 4


def _encode_in_order(tile, order):
    """Record bytes of a tile under an arbitrary node order (test-side re-encoding)."""
    seq = tile.reshape(-1)[order]
    keep = np.flatnonzero(seq != 0)
    nnz = keep.size
    is_mask, vb, mb, rb = O.record_layout(nnz, seq.size, tile.dtype.itemsize)
    return nnz, is_mask, rb, {int(order[k]): seq[k] for k in keep}


@pytest.mark.parametrize("s", [65, 33, 17, 32])
def test_record_contents_do_not_depend_on_the_order(s):
    """The in-record order is a bijection of the tile's nodes (the CSR role of
    Section 2.3.1 fixes no order inside a subgrid): the kept set, the values,
    nnz, the encoding tag and the record size are the same under the record
    order and under plain row-major order, and both round-trip the tile."""
    tiles = random_coefficient_tiles((4, s, s), seed=s + 1, dtype=np.float64, zero_frac=0.5)
    tiles[1][np.abs(tiles[1]) < np.quantile(np.abs(tiles[1]), 0.97)] = 0
    rowmajor = np.arange(s * s)
    for t in tiles:
        a = _encode_in_order(t, O.record_order(s))
        b = _encode_in_order(t, rowmajor)
        assert a[:3] == b[:3]
        assert a[3].keys() == b[3].keys() == set(np.flatnonzero(t.reshape(-1)).tolist())
        assert all(a[3][k] == b[3][k] for k in a[3])
        rec = O.encode_record(t)
        word = a[0] | (O.MASK_BIT if a[1] else 0)
        assert len(rec) == a[2]
        assert np.array_equal(O.decode_record(rec, 0, word, s, np.float64), t)
