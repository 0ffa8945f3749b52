"""CPU oracle of reduced-precision coefficient storage -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the CPU-baseline leg of the benchmark
may import this module; the GPU library never calls it and shares no code or
table with it.

The stencil arithmetic stays in float32; what changes is how the surviving
coefficients of a tile are stored.  The paper asks for the global mass to be
conserved whatever the compression does (equation "conservation" and
Section 3.1.1): by that identity the trapezoid mass of a reconstructed tile is
4^L times the coarse trapezoid mass of its samples, whatever the details are.
So the samples are stored exactly (float32) and only the details are
quantised -- no mass-correction step is needed, the defect is zero.

Narrow value formats:

* ``"f16"``: IEEE binary16, round to nearest, ties to even (NumPy's float16
  conversion of a float32 value, one rounding);
* ``"e4m3"``: the 8-bit OCP E4M3 (FN) format -- 1 sign bit, 4 exponent bits
  with bias 7, 3 mantissa bits, subnormals for exponent 0, no infinities,
  code 0x7F / 0xFF is NaN, largest finite magnitude 448.  Written below from
  that definition (the value of every code), rounding to the nearest value,
  ties to the even code.

* ``"e4m3b"``: E4M3 where it is error-bounded, binary16 elsewhere, chosen per
  record.  A kept detail c read back from E4M3 with scale 2**k is off by at
  most max(2**-4 |c|, 2**(k - 10)) (half a unit of the 3-bit mantissa in the
  normal range, half the subnormal spacing 2**-9 below it).  A record is
  stored in E4M3 when, for every subband holding a kept detail, that bound
  at the subband's largest kept magnitude m_b and E4M3 scale 2**k_b is at
  most half the subband's threshold (:data:`E4M3B_FRACTION` x thr_b): the
  quantisation then adds less than half of the error the threshold already
  accepts for a dropped detail.  Otherwise the whole record is binary16 (as
  is every record at eps = 0, where the threshold is zero).  Bit 63 of OCC
  is set for an E4M3 record.  The threshold of a subband is the one the
  thresholding used (one value per subband for every rule).

Per-subband scales: a detail at tile position (y, x) belongs to subband
``(cy, cx)``, the per-dimension classes (0 for a sample index, else the
detail level, 1 = finest) of the thresholding; its index is
``b = cy * (L + 1) + cx``.  For every subband of a record that holds a kept
detail, the scale is the power of two ``2**k`` with the smallest integer
``k`` such that ``max |c| <= FMT_MAX * 2**k`` (FMT_MAX = 65504 for f16, 448 for
e4m3), raised to ``k = -126`` if smaller (a normal float32); a detail is stored as ``Q(c / 2**k)`` and read back as
``Q(c / 2**k) * 2**k`` (both scalings exact).

Record of one (patch, field) tile in a narrow format (little-endian):

  u64 OCC, bit b set when subband b holds a kept detail;
  one float32 scale per set bit of OCC, in increasing b;  zero pad to 8;
  float32 samples, every sample position of the tile (kept or zero) in
    row-major order of the sample grid: slot ``(y >> L) * SC + (x >> L)``
    with ``SC`` samples per side;  zero pad to 8;
  the kept details' narrow values, in record order;  zero pad to 8;
  then, as in the float32 record, either the u16 record indices of the kept
    details or (when ``2 * ndet >= 8 * W``) W u64 mask words with a bit per
    record index (sample positions never set);  zero pad to 16.
Offset-table entry: u32 offset in 16-byte units, u32 ``ndet`` with bit 31 set
for a bitmask.  A detail is "kept" by the threshold decision, before
quantisation (its stored value may read back as zero).
"""
from __future__ import annotations

import numpy as np

from .lbmz_oracle import MASK_BIT, index_levels, record_order, _align

FORMATS = ("f16", "e4m3", "e4m3b")
FMT_MAX = {"f16": 65504.0, "e4m3": 448.0}
FMT_BYTES = {"f16": 2, "e4m3": 1}
E4M3B_FRACTION = 0.5          # E4M3 rounding bound allowed, as a fraction of the subband threshold
OCC_E4M3_BIT = 1 << 63        # "e4m3b" records: OCC bit of an E4M3 record


# ---------------------------------------------------------------------------
# E4M3 (OCP 8-bit float, FN variant), from the format definition
# ---------------------------------------------------------------------------

def e4m3_value(code: int) -> float:
    """Value of one E4M3 code (NaN for 0x7F and 0xFF)."""
    code = int(code) & 0xFF
    sign = -1.0 if code & 0x80 else 1.0
    e = (code >> 3) & 0xF
    m = code & 0x7
    if e == 0xF and m == 0x7:
        return float("nan")
    if e == 0:
        return sign * m * 2.0 ** -9            # subnormal: m/8 * 2^(1-7)
    return sign * (1.0 + m / 8.0) * 2.0 ** (e - 7)


_E4M3_POS = np.array([e4m3_value(c) for c in range(0x7F)], dtype=np.float64)   # codes 0 .. 0x7E


def e4m3_encode(x) -> np.ndarray:
    """Nearest E4M3 code of each value (ties to the even code); |x| <= 448 required."""
    x = np.asarray(x, dtype=np.float64)
    a = np.abs(x)
    if np.any(~np.isfinite(a)) or np.any(a > 448.0):
        raise ValueError("e4m3_encode needs finite values of magnitude <= 448")
    # neighbours in the sorted table of non-negative values
    hi = np.searchsorted(_E4M3_POS, a, side="left")          # first value >= a
    hi = np.minimum(hi, _E4M3_POS.size - 1)
    lo = np.maximum(hi - 1, 0)
    dlo = a - _E4M3_POS[lo]
    dhi = _E4M3_POS[hi] - a
    pick_hi = (dhi < dlo) | ((dhi == dlo) & (hi % 2 == 0))
    code = np.where(pick_hi, hi, lo)
    code = np.where(a == _E4M3_POS[hi], hi, code)
    sign = np.signbit(x).astype(np.int64) << 7
    return (code | sign).astype(np.uint8)


def e4m3_decode(code) -> np.ndarray:
    c = np.asarray(code, dtype=np.int64) & 0xFF
    mag = _E4M3_POS[np.minimum(c & 0x7F, 0x7E)]
    return np.where(c & 0x80, -mag, mag)


# ---------------------------------------------------------------------------
# Quantisers of one value stream (float32 in, float32 out)
# ---------------------------------------------------------------------------

def quantize(x: np.ndarray, fmt: str) -> np.ndarray:
    """Stored codes of float32 values already divided by their scale."""
    x = np.asarray(x, dtype=np.float32)
    if fmt == "f16":
        return x.astype(np.float16)
    if fmt == "e4m3":
        return e4m3_encode(x.astype(np.float64))
    raise ValueError(fmt)


def dequantize(q: np.ndarray, fmt: str) -> np.ndarray:
    if fmt == "f16":
        return np.asarray(q, dtype=np.float16).astype(np.float32)
    if fmt == "e4m3":
        return e4m3_decode(q).astype(np.float32)
    raise ValueError(fmt)


def pow2_scale(maxabs: float, fmt: str) -> np.float32:
    """Smallest power of two ``2**k`` with ``maxabs <= FMT_MAX * 2**k``, with
    ``k >= -126`` so that the scale is a normal float32 (1 for 0)."""
    m = float(maxabs)
    if m == 0.0:
        return np.float32(1.0)
    fmax = FMT_MAX[fmt]
    k = int(np.floor(np.log2(m / fmax)))
    while m > fmax * 2.0 ** k:
        k += 1
    while m <= fmax * 2.0 ** (k - 1):
        k -= 1
    return np.float32(2.0 ** max(k, -126))


# ---------------------------------------------------------------------------
# Subbands and samples of a tile
# ---------------------------------------------------------------------------

def index_classes(s: int, levels: int) -> np.ndarray:
    """Per index of one dimension: 0 for a sample index, else its detail level (1 = finest)."""
    return index_levels(s, levels)


def subband_table(s: int, levels: int) -> np.ndarray:
    """Subband index ``cy * (L + 1) + cx`` of every tile position ``[s, s]`` (0 = samples)."""
    c = index_classes(s, levels)
    return c[:, None] * (levels + 1) + c[None, :]


def sample_positions(s: int, levels: int):
    """Tile positions (y, x) of the samples, in slot order, and samples per side."""
    step = 1 << levels
    idx = [i for i in range(s) if i % step == 0]
    return [(y, x) for y in idx for x in idx], len(idx)


def e4m3_bound_holds(tile: np.ndarray, levels: int, thr: np.ndarray) -> bool:
    """The "e4m3b" choice for one thresholded float32 tile with its threshold
    table ``thr`` ([s, s], float32): True when every occupied subband's E4M3
    rounding bound is at most E4M3B_FRACTION times its threshold."""
    t = np.asarray(tile, dtype=np.float32)
    s = t.shape[-1]
    sb = subband_table(s, levels)
    th = np.broadcast_to(np.asarray(thr, dtype=np.float32), t.shape)
    for b in range(1, (levels + 1) ** 2):
        sel = (sb == b) & (t != 0)
        if not np.any(sel):
            continue
        m = float(np.max(np.abs(t[sel])))
        k = int(np.log2(float(pow2_scale(m, "e4m3"))))
        bound = max(m * 2.0 ** -4, 2.0 ** (k - 10))
        thr_b = float(th[sb == b][0])
        if not bound <= E4M3B_FRACTION * thr_b:
            return False
    return True


def effective_format(tile: np.ndarray, levels: int, fmt: str, thr=None) -> str:
    """The code format a record of this tile uses: ``fmt`` itself, or for
    ``"e4m3b"`` "e4m3" or "f16" by :func:`e4m3_bound_holds` (``thr`` needed)."""
    if fmt != "e4m3b":
        return fmt
    if thr is None:
        raise ValueError("the e4m3b format needs the threshold table")
    return "e4m3" if e4m3_bound_holds(tile, levels, thr) else "f16"


def quantize_tile(tile: np.ndarray, levels: int, fmt: str, thr=None):
    """Stored representation of one thresholded float32 tile.

    Returns ``(deq, scales, occ)``: the tile as read back (samples unchanged,
    kept details quantised with their subband scale), the per-subband scales
    (index b -> float32, only for occupied subbands) and the occupancy mask
    (with OCC_E4M3_BIT for an E4M3 "e4m3b" record).
    """
    t = np.asarray(tile, dtype=np.float32)
    s = t.shape[-1]
    eff = effective_format(t, levels, fmt, thr)
    sb = subband_table(s, levels)
    out = t.copy()
    scales = {}
    occ = 0
    for b in range(1, (levels + 1) ** 2):
        sel = (sb == b) & (t != 0)
        if not np.any(sel):
            continue
        sc = pow2_scale(float(np.max(np.abs(t[sel]))), eff)
        scales[b] = sc
        occ |= 1 << b
        q = quantize(t[sel] / sc, eff)
        out[sel] = dequantize(q, eff) * sc
    if fmt == "e4m3b" and eff == "e4m3":
        occ |= OCC_E4M3_BIT
    return out, scales, occ


def _tile_thresholds(thr, shape):
    """Per-tile threshold tables for tiles of ``shape`` = [..., s, s] (None kept)."""
    if thr is None:
        return None
    t = np.broadcast_to(np.asarray(thr, dtype=np.float32), shape)
    return t.reshape(-1, shape[-2], shape[-1])


def quantize_tiles(coef: np.ndarray, levels: int, fmt: str, thr=None) -> np.ndarray:
    """:func:`quantize_tile` applied to every tile of ``[..., s, s]``; ``thr``
    broadcasts against the tiles (the "e4m3b" choice needs it)."""
    c = np.asarray(coef, dtype=np.float32)
    flat = c.reshape(-1, c.shape[-2], c.shape[-1])
    th = _tile_thresholds(thr, c.shape)
    out = np.empty_like(flat)
    for i in range(flat.shape[0]):
        out[i] = quantize_tile(flat[i], levels, fmt, None if th is None else th[i])[0]
    return out.reshape(c.shape)


# ---------------------------------------------------------------------------
# Records in a narrow format
# ---------------------------------------------------------------------------

def record_layout_q(ndet: int, nocc: int, ncoef: int, nsamp: int, fmt: str):
    """``(is_mask, scales_end, samples_end, values_end, record_bytes)`` in bytes."""
    w = (ncoef + 63) // 64
    is_mask = not (2 * ndet < 8 * w)
    hb = _align(8 + 4 * nocc, 8)
    sb = hb + _align(4 * nsamp, 8)
    vb = sb + _align(FMT_BYTES[fmt] * ndet, 8)
    mb = 8 * w if is_mask else 2 * ndet
    return is_mask, hb, sb, vb, _align(vb + mb, 16)


def encode_record_q(tile: np.ndarray, levels: int, fmt: str, thr=None):
    """``(bytes, ndet, is_mask)`` of one thresholded float32 tile (``thr``: its
    threshold table, needed by "e4m3b")."""
    t = np.asarray(tile, dtype=np.float32)
    s = t.shape[-1]
    ncoef = s * s
    sb = subband_table(s, levels)
    _, scales, occ = quantize_tile(t, levels, fmt, thr)
    fmt = effective_format(t, levels, fmt, thr)
    order = record_order(s)
    flat = t.reshape(-1)
    sbf = sb.reshape(-1)
    det_k = [k for k, pos in enumerate(order) if sbf[pos] != 0 and flat[pos] != 0]
    ndet = len(det_k)
    spos, _ = sample_positions(s, levels)
    is_mask, hb, sbe, vb, rb = record_layout_q(ndet, len(scales), ncoef, len(spos), fmt)
    buf = bytearray(rb)
    buf[0:8] = np.array([occ], dtype="<u8").tobytes()
    sc_list = [scales[b] for b in sorted(scales)]
    buf[8:8 + 4 * len(sc_list)] = np.array(sc_list, dtype="<f4").tobytes()
    buf[hb:hb + 4 * len(spos)] = np.array([t[y, x] for (y, x) in spos], dtype="<f4").tobytes()
    if ndet:
        pos = order[det_k]
        vals = flat[pos]
        scl = np.array([scales[int(sbf[p])] for p in pos], dtype=np.float32)
        q = quantize(vals / scl, fmt)
        raw = q.astype("<f2").tobytes() if fmt == "f16" else q.astype(np.uint8).tobytes()
        buf[sbe:sbe + len(raw)] = raw
    if is_mask:
        w = (ncoef + 63) // 64
        words = np.zeros(w, dtype="<u8")
        for k in det_k:
            words[k // 64] |= np.uint64(1) << np.uint64(k % 64)
        buf[vb:vb + 8 * w] = words.tobytes()
    else:
        buf[vb:vb + 2 * ndet] = np.array(det_k, dtype="<u2").tobytes()
    return bytes(buf), ndet, is_mask


def decode_record_q(buf: bytes, off16: int, word: int, s: int, levels: int, fmt: str) -> np.ndarray:
    """Inverse of :func:`encode_record_q`: the tile as read back, float32 ``[s, s]``."""
    ncoef = s * s
    ndet = word & (MASK_BIT - 1)
    is_mask = bool(word & MASK_BIT)
    base = 16 * off16
    occ = int(np.frombuffer(buf, dtype="<u8", count=1, offset=base)[0])
    if fmt == "e4m3b":
        fmt = "e4m3" if occ & OCC_E4M3_BIT else "f16"
        occ &= ~OCC_E4M3_BIT
    bands = [b for b in range(64) if (occ >> b) & 1]
    scl = np.frombuffer(buf, dtype="<f4", count=len(bands), offset=base + 8)
    scale_of = {b: np.float32(v) for b, v in zip(bands, scl)}
    spos, _ = sample_positions(s, levels)
    _, hb, sbe, vb, _ = record_layout_q(ndet, len(bands), ncoef, len(spos), fmt)
    out = np.zeros((s, s), dtype=np.float32)
    samp = np.frombuffer(buf, dtype="<f4", count=len(spos), offset=base + hb)
    for (y, x), v in zip(spos, samp):
        out[y, x] = v
    if ndet == 0:
        return out
    if fmt == "f16":
        q = np.frombuffer(buf, dtype="<f2", count=ndet, offset=base + sbe)
    else:
        q = np.frombuffer(buf, dtype=np.uint8, count=ndet, offset=base + sbe)
    if is_mask:
        w = (ncoef + 63) // 64
        words = np.frombuffer(buf, dtype="<u8", count=w, offset=base + vb)
        ks = [k for k in range(ncoef) if (int(words[k // 64]) >> (k % 64)) & 1]
    else:
        ks = np.frombuffer(buf, dtype="<u2", count=ndet, offset=base + vb).astype(np.int64).tolist()
    order = record_order(s)
    sb = subband_table(s, levels).reshape(-1)
    deq = dequantize(q, fmt)
    flat = out.reshape(-1)
    for k, v in zip(ks, deq):
        p = order[k]
        flat[p] = np.float32(v * scale_of[int(sb[p])])
    return out


def encode_store_q(coef: np.ndarray, levels: int, fmt: str, thr=None):
    """Offset table and pool of ``[npatch, m, s, s]`` thresholded float32 tiles
    (serial placement); ``thr`` broadcasts against the tiles ("e4m3b")."""
    npatch, m = coef.shape[0], coef.shape[1]
    th = _tile_thresholds(thr, coef.shape)
    table = np.zeros((npatch, m, 2), dtype=np.uint32)
    parts = []
    off = 0
    for q in range(npatch):
        for f in range(m):
            rec, ndet, is_mask = encode_record_q(coef[q, f], levels, fmt,
                                                 None if th is None else th[q * m + f])
            table[q, f, 0] = off // 16
            table[q, f, 1] = ndet | (MASK_BIT if is_mask else 0)
            parts.append(rec)
            off += len(rec)
    return table, b"".join(parts)


def decode_store_q(table: np.ndarray, pool: bytes, s: int, levels: int, fmt: str) -> np.ndarray:
    npatch, m = table.shape[:2]
    out = np.zeros((npatch, m, s, s), dtype=np.float32)
    for q in range(npatch):
        for f in range(m):
            out[q, f] = decode_record_q(pool, int(table[q, f, 0]), int(table[q, f, 1]), s, levels, fmt)
    return out


def store_bytes_q(coef: np.ndarray, levels: int, fmt: str, thr=None) -> int:
    """Bytes of the narrow store of thresholded tiles: all records plus the
    offset table ("e4m3b" needs the kept values and ``thr``)."""
    npatch, m, s = coef.shape[0], coef.shape[1], coef.shape[-1]
    th = _tile_thresholds(thr, coef.shape)
    sb = subband_table(s, levels)
    nsamp = len(sample_positions(s, levels)[0])
    tot = 0
    for q in range(npatch):
        for f in range(m):
            t = coef[q, f]
            det = (sb != 0) & (t != 0)
            nocc = len(set(sb[det].tolist()))
            eff = effective_format(t, levels, fmt, None if th is None else th[q * m + f])
            tot += record_layout_q(int(det.sum()), nocc, s * s, nsamp, eff)[4]
    return tot + npatch * m * 8
