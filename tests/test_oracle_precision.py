"""Pins of the reduced-precision storage oracle (samples exact, details quantised).

The quantisers are checked against the formats' definitions and independent
library routines; the records against brute force; the conservation claim
against the identity of equation "conservation".
"""
import struct

import numpy as np
import pytest

from oracle import lbmz_oracle as O
from oracle import lbmz_precision as Q


# ---------------------------------------------------------------- E4M3 format

def test_e4m3_code_values_from_the_format_definition():
    assert Q.e4m3_value(0x00) == 0.0
    assert Q.e4m3_value(0x01) == 2.0 ** -9          # smallest subnormal
    assert Q.e4m3_value(0x07) == 7 * 2.0 ** -9      # largest subnormal
    assert Q.e4m3_value(0x08) == 2.0 ** -6          # smallest normal
    assert Q.e4m3_value(0x38) == 1.0
    assert Q.e4m3_value(0x3C) == 1.5
    assert Q.e4m3_value(0x7E) == 448.0              # largest finite
    assert np.isnan(Q.e4m3_value(0x7F)) and np.isnan(Q.e4m3_value(0xFF))
    assert Q.e4m3_value(0xB8) == -1.0
    vals = [Q.e4m3_value(c) for c in range(0x7F)]
    assert all(a < b for a, b in zip(vals, vals[1:]))   # codes ordered by value
    assert len(set(vals)) == 127


def test_e4m3_roundtrip_of_every_finite_code():
    codes = np.array([c for c in range(256) if (c & 0x7F) != 0x7F], dtype=np.uint8)
    back = Q.e4m3_encode(Q.e4m3_decode(codes))
    assert np.array_equal(back, codes)


def test_e4m3_round_to_nearest_ties_to_even():
    cases = {1.0625: 0x38,            # halfway 1.0 / 1.125 -> even mantissa 0
             1.1875: 0x3A,            # halfway 1.125 / 1.25 -> even mantissa 2
             2.0 ** -10: 0x00,        # halfway 0 / 2^-9 -> code 0
             3 * 2.0 ** -10: 0x02,    # halfway 2^-9 / 2^-8 -> code 2
             432.0: 0x7E,             # halfway 416 / 448 -> code 0x7E (even)
             -0.0: 0x80,
             -1.0625: 0xB8}
    for x, want in cases.items():
        assert int(Q.e4m3_encode(np.array([x]))[0]) == want, x


def test_e4m3_nearest_by_brute_force():
    rng = np.random.default_rng(7)
    x = np.concatenate([rng.uniform(-448, 448, 3000), rng.uniform(-0.02, 0.02, 3000),
                        rng.standard_normal(3000)])
    got = Q.e4m3_decode(Q.e4m3_encode(x))
    table = np.array([Q.e4m3_value(c) for c in range(0x7F)])
    table = np.concatenate([-table[::-1], table])
    best = np.min(np.abs(x[:, None] - table[None, :]), axis=1)
    assert np.array_equal(np.abs(x - got), best)
    # error bounds of the format: relative 2^-4 when normal, absolute 2^-10 when subnormal
    a = np.abs(x)
    normal = a >= 2.0 ** -6
    assert np.all(np.abs(x - got)[normal] <= 2.0 ** -4 * a[normal])
    assert np.all(np.abs(x - got)[~normal] <= 2.0 ** -10)


# ---------------------------------------------------------------- binary16

def test_f16_matches_the_struct_half_float_packing():
    rng = np.random.default_rng(8)
    x = np.concatenate([rng.standard_normal(2000) * 1e3, rng.uniform(-1e-6, 1e-6, 500)]).astype(np.float32)
    ours = Q.quantize(x, "f16").view(np.uint16)
    lib = np.array([struct.unpack("<H", struct.pack("<e", float(v)))[0] for v in x], dtype=np.uint16)
    assert np.array_equal(ours, lib)


# ---------------------------------------------------------------- scales

FIXED = ("f16", "e4m3")


@pytest.mark.parametrize("fmt", FIXED)
def test_pow2_scale_is_the_tightest_power_of_two(fmt):
    rng = np.random.default_rng(9)
    for m in np.concatenate([rng.uniform(1e-9, 1e6, 500), [448.0, 65504.0, 1.0, 2.0 ** -30]]):
        s = float(Q.pow2_scale(m, fmt))
        assert np.log2(s) == int(np.log2(s))
        assert m <= Q.FMT_MAX[fmt] * s and m > Q.FMT_MAX[fmt] * s / 2


# ---------------------------------------------------------------- records

def _tile(s, L, seed, zero_frac):
    rng = np.random.default_rng(seed)
    t = (rng.standard_normal((s, s)) * np.exp(rng.uniform(-8, 2, (s, s)))).astype(np.float32)
    t[rng.random((s, s)) < zero_frac] = 0
    return t


def _thr(s, L, eps=1e-3, rule="capped"):
    return O.threshold_table(s, L, eps, rule, np.float32)


@pytest.mark.parametrize("fmt", Q.FORMATS)
@pytest.mark.parametrize("s,L", [(65, 5), (65, 2), (33, 4), (64, 6), (16, 3)])
@pytest.mark.parametrize("zero_frac", [0.0, 0.9, 0.995, 1.0])
def test_record_roundtrip_and_layout(fmt, s, L, zero_frac):
    t = _tile(s, L, seed=s + L, zero_frac=zero_frac)
    thr = _thr(s, L) if fmt == "e4m3b" else None
    buf, ndet, is_mask = Q.encode_record_q(t, L, fmt, thr)
    back = Q.decode_record_q(buf, 0, ndet | (O.MASK_BIT if is_mask else 0), s, L, fmt)
    deq, scales, occ = Q.quantize_tile(t, L, fmt, thr)
    assert np.array_equal(back.view(np.uint32), deq.view(np.uint32))
    eff = Q.effective_format(t, L, fmt, thr)
    if fmt == "e4m3b":
        assert bool(occ & Q.OCC_E4M3_BIT) == (eff == "e4m3")
        occ &= ~Q.OCC_E4M3_BIT
        # the e4m3b record reads back as the record of its effective format
        assert np.array_equal(deq.view(np.uint32), Q.quantize_tile(t, L, eff)[0].view(np.uint32))
    # brute force: kept details in record order, samples untouched, sizes
    sb = Q.subband_table(s, L)
    order = O.record_order(s)
    det = [(k, p) for k, p in enumerate(order) if sb.reshape(-1)[p] != 0 and t.reshape(-1)[p] != 0]
    assert ndet == len(det)
    samples = sb == 0
    assert np.array_equal(back[samples], t[samples])
    assert occ == sum(1 << b for b in set(sb[(sb != 0) & (t != 0)].tolist()))
    assert len(buf) % 16 == 0
    nsamp = len(Q.sample_positions(s, L)[0])
    assert len(buf) == Q.record_layout_q(ndet, len(scales), s * s, nsamp, eff)[4]
    if not is_mask and ndet:
        *_, vb, _ = Q.record_layout_q(ndet, len(scales), s * s, nsamp, eff)
        idx = np.frombuffer(buf, dtype="<u2", count=ndet, offset=vb)
        assert idx.tolist() == [k for k, _ in det]


@pytest.mark.parametrize("fmt", FIXED)
def test_quantisation_error_bounds(fmt):
    t = _tile(65, 5, seed=3, zero_frac=0.2)
    deq, scales, _ = Q.quantize_tile(t, 5, fmt)
    sb = Q.subband_table(65, 5)
    for b, sc in scales.items():
        sel = (sb == b) & (t != 0)
        err = np.abs(deq[sel].astype(np.float64) - t[sel])
        if fmt == "f16":
            # binary16 keeps 11 significant bits above 2^-14 of the scaled value
            bound = 2.0 ** -11 * np.abs(t[sel]) + 2.0 ** -25 * float(sc)
        else:
            bound = 2.0 ** -4 * np.abs(t[sel]) + 2.0 ** -10 * float(sc)
        assert np.all(err <= bound)


@pytest.mark.parametrize("fmt", Q.FORMATS)
def test_mass_unchanged_by_quantisation(fmt):
    # equation "conservation": the trapezoid mass of a reconstructed tile
    # depends on its samples only, which are stored exactly
    rng = np.random.default_rng(4)
    tile = rng.uniform(0.5, 1.5, (65, 65))
    coef = O.forward_2d(tile, 5, O.BL53).astype(np.float32)
    # e4m3b: a threshold table of zeros (eps = 0) makes the record binary16
    deq, _, _ = Q.quantize_tile(coef, 5, fmt, _thr(65, 5, 0.0) if fmt == "e4m3b" else None)
    assert not np.array_equal(deq, coef)
    w = np.ones(65)
    w[0] = w[-1] = 0.5
    wt = w[:, None] * w[None, :]
    m0 = float(np.sum(wt * O.inverse_2d(coef.astype(np.float64), 5, O.BL53)))
    m1 = float(np.sum(wt * O.inverse_2d(deq.astype(np.float64), 5, O.BL53)))
    assert abs(m1 - m0) <= 1e-12 * abs(m0)


def test_store_roundtrip():
    rng = np.random.default_rng(5)
    coef = rng.standard_normal((3, 2, 33, 33)).astype(np.float32)
    coef[rng.random(coef.shape) < 0.97] = 0
    thr = _thr(33, 4, 0.3)
    for fmt in Q.FORMATS:
        th = thr if fmt == "e4m3b" else None
        table, pool = Q.encode_store_q(coef, 4, fmt, th)
        back = Q.decode_store_q(table, pool, 33, 4, fmt)
        assert np.array_equal(back, Q.quantize_tiles(coef, 4, fmt, th))
        assert Q.store_bytes_q(coef, 4, fmt, th) == len(pool) + table.size * 4


# ---------------------------------------------------------------- e4m3b choice

def _bounded_tiles(seed, n=40):
    """Thresholded tiles whose kept details span [thr, 30 thr] per subband."""
    rng = np.random.default_rng(seed)
    s, L = 33, 4
    thr = _thr(s, L, 1e-3)
    tiles = []
    for _ in range(n):
        top = rng.choice([2.0, 6.0, 7.9, 12.0, 30.0])
        t = (thr * rng.uniform(1.0, top, (s, s)) * rng.choice([-1.0, 1.0], (s, s))).astype(np.float32)
        t[rng.random((s, s)) < rng.uniform(0.3, 0.98)] = 0
        samples = Q.subband_table(s, L) == 0
        t[samples] = rng.uniform(0.5, 1.5, int(samples.sum())).astype(np.float32)
        tiles.append(t)
    return tiles, thr, L


def test_e4m3b_records_keep_the_quantisation_within_half_the_threshold():
    # brute force over every kept detail of every record that the rule stores
    # in E4M3: its read-back error is at most half its threshold
    tiles, thr, L = _bounded_tiles(21)
    sb = Q.subband_table(33, L)
    chosen = {"e4m3": 0, "f16": 0}
    for t in tiles:
        eff = Q.effective_format(t, L, "e4m3b", thr)
        chosen[eff] += 1
        deq = Q.quantize_tile(t, L, "e4m3b", thr)[0]
        if eff == "e4m3":
            det = (sb != 0) & (t != 0)
            err = np.abs(deq[det].astype(np.float64) - t[det].astype(np.float64))
            assert np.all(err <= 0.5 * thr[det].astype(np.float64))
    assert chosen["e4m3"] > 0 and chosen["f16"] > 0


def test_e4m3b_choice_at_the_edge_of_the_bound():
    # one kept detail in the finest subband of a capped L = 4 tile: E4M3 up to
    # 8 thr (2^-4 * 8 thr = thr / 2), binary16 just above
    s, L = 33, 4
    thr = _thr(s, L, 1e-3)
    t = np.zeros((s, s), dtype=np.float32)
    t[0, 0] = 1.0
    y, x = 1, 1                              # finest level in both dimensions
    for mult, want in ((1.0, "e4m3"), (8.0, "e4m3"), (float(np.nextafter(np.float32(8.0), np.float32(9.0))), "f16"),
                       (100.0, "f16")):
        t[y, x] = np.float32(thr[y, x] * np.float32(mult))
        assert Q.effective_format(t, L, "e4m3b", thr) == want, mult
    # eps = 0: zero thresholds, any kept detail needs binary16; no detail at all: E4M3
    t[y, x] = 1e-3
    assert Q.effective_format(t, L, "e4m3b", _thr(s, L, 0.0)) == "f16"
    t[y, x] = 0.0
    assert Q.effective_format(t, L, "e4m3b", _thr(s, L, 0.0)) == "e4m3"


def test_e4m3b_store_lies_between_the_fixed_formats():
    tiles, thr, L = _bounded_tiles(22, n=24)
    coef = np.stack(tiles).reshape(6, 4, 33, 33)
    b8 = Q.store_bytes_q(coef, L, "e4m3", thr)
    b16 = Q.store_bytes_q(coef, L, "f16", thr)
    bb = Q.store_bytes_q(coef, L, "e4m3b", thr)
    assert b8 < bb < b16
