"""The tests' vectorised store readers against the oracle's encoders (CPU).

The GPU parity tests decode what the library wrote with the readers of
``gpu_helpers``; these checks tie those readers to the oracle's record
encoders on seeded tiles of both encodings, every value format and 2-D / 3-D
tiles, so that a decoding mistake cannot hide a kernel mistake.
"""
import numpy as np
import pytest

from oracle import lbmz_oracle as O
from oracle import lbmz_oracle3d as O3
from oracle import lbmz_precision as Q
from synth import random_coefficient_tiles

gh = pytest.importorskip("gpu_helpers")


def _mixed_tiles(shape, seed, dtype):
    t = random_coefficient_tiles(shape, seed=seed, dtype=dtype, zero_frac=0.3)
    flat = t.reshape(shape[0], shape[1], -1)
    rng = np.random.default_rng(seed)
    # a spread of densities across the index-list / bitmask switch
    for q in range(shape[0]):
        for f in range(shape[1]):
            keep = rng.uniform(0.0, 0.25 if (q + f) % 2 else 1.0)
            flat[q, f, rng.uniform(size=flat.shape[2]) > keep] = 0
    return t


@pytest.mark.parametrize("s,dtype", [(65, np.float32), (33, np.float64), (32, np.float64), (17, np.float32)])
def test_reader_matches_oracle_encoder(s, dtype):
    tiles = _mixed_tiles((3, 4, s, s), seed=s, dtype=dtype)
    table, pool = O.encode_store(tiles)
    assert any(int(w) & O.MASK_BIT for w in table[..., 1].ravel())
    assert any(not int(w) & O.MASK_BIT for w in table[..., 1].ravel())
    got = gh.decode_records(table, pool, s, dtype)
    assert np.array_equal(got, O.decode_store(table, pool, s, dtype))


@pytest.mark.parametrize("fmt", ["f16", "e4m3", "e4m3b"])
def test_narrow_reader_matches_oracle_encoder(fmt):
    levels = 5
    tiles = _mixed_tiles((2, 3, 65, 65), seed=7, dtype=np.float32) * np.float32(1e-2)
    thr = None
    if fmt == "e4m3b":
        # per-tile thresholds: every other tile gets a large one, so both record formats occur
        thr = np.stack([O.threshold_table(65, levels, e, "capped", np.float32)
                        for e in (1e-9, 1.0)] * 3).reshape(2, 3, 65, 65)
    table, pool = Q.encode_store_q(tiles, levels, fmt, thr)
    if fmt == "e4m3b":
        occ = [int(np.frombuffer(pool, dtype="<u8", count=1, offset=16 * int(o))[0]) for o in table[..., 0].ravel()]
        assert any(o >> 63 for o in occ) and any(not o >> 63 for o in occ)
    got = gh.decode_records(table, pool, 65, np.float32, values=fmt, levels=levels)
    want = Q.decode_store_q(table, pool, 65, levels, fmt)
    assert np.array_equal(got, want)


def test_3d_reader_matches_oracle_encoder():
    s = 17
    tiles = _mixed_tiles((2, 19, s, s * s), seed=5, dtype=np.float32).reshape(2, 19, s, s, s)
    table, pool = O3.encode_store3(tiles)
    got = gh.decode_records3(table, pool, s)
    assert np.array_equal(got, O3.decode_store3(table, pool, s, np.float32))
