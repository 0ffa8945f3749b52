"""Shared helpers of the GPU parity tests (imports the oracle; test-only)."""
import numpy as np
import pytest

from oracle import lbmz_oracle as O

torch = pytest.importorskip("torch")


def require_gpu():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")


def make_ctx(n, scheme, dtype, p, wavelet, levels, eps, rule="capped", **kw):
    from paper_2302_09883_amd import Context
    return Context(n, scheme=scheme, dtype=dtype, p=p, wavelet=wavelet, levels=levels, eps=eps, rule=rule,
                   vel=kw.pop("vel", (1.0, 0.5)), cfl=kw.pop("cfl", 0.5), tau=kw.pop("tau", 0.6), **kw)


def oracle_twin(ctx, dtype=None):
    """Oracle run with the same geometry, scheme and threshold as a context."""
    g = O.Geometry(ctx.n, ctx.p, ctx.wavelet, ctx.levels)
    sch = O.Scheme(ctx.scheme, vel=(1.0, 0.5), cfl=0.5, tau=0.6)
    dt = dtype if dtype is not None else ctx.np_dtype
    return O.CompressedRun(g, sch, ctx.eps, ctx.rule, dt)


def gpu_coefficients(ctx):
    """The context's stored coefficient tiles, decoded on the host."""
    table, pool = ctx.store()
    return decode_records(table, pool, ctx.s, ctx.np_dtype), table, pool


def records_of(table, pool, q, f, ctx):
    """Bytes of one record, using the same size rule as the oracle."""
    nnz = int(table[q, f, 1]) & (O.MASK_BIT - 1)
    rb = O.record_layout(nnz, ctx.s * ctx.s, np.dtype(ctx.np_dtype).itemsize)[3]
    off = int(table[q, f, 0]) * 16
    return pool[off:off + rb]


def borderline(c, thr, delta):
    """Coefficients whose keep / drop decision is within rounding of the threshold."""
    return np.abs(np.abs(c) - thr) <= delta


# ---------------------------------------------------------------------------
# Host readers of the store layouts declared in include/lbmz.h.  They read what
# the library wrote so that tests can compare it with the oracle; vectorised
# over a whole store (the oracle's own record decoder walks bits one by one).
# ---------------------------------------------------------------------------

def store_record_order(s: int) -> np.ndarray:
    """Flat tile indices (y * s + x) in the record order of include/lbmz.h
    (owned block row by row, then the shared column, row and corner)."""
    p = s - 1 if s % 2 == 1 else s
    yy, xx = np.meshgrid(np.arange(p), np.arange(p), indexing="ij")
    parts = [(yy * s + xx).reshape(-1)]
    if p != s:
        parts += [np.arange(p) * s + p, p * s + np.arange(p), np.array([p * s + p])]
    return np.concatenate(parts).astype(np.int64)


def _e4m3_values(codes: np.ndarray) -> np.ndarray:
    c = codes.astype(np.int64)
    e = (c >> 3) & 15
    m = (c & 7).astype(np.float64)
    mag = np.where(e == 0, m * 2.0 ** -9, (1.0 + m / 8.0) * np.exp2(e - 7.0))
    return np.where(c & 0x80, -mag, mag).astype(np.float32)


def _decode_narrow(table, pool, s, values, levels):
    npatch, nf = table.shape[:2]
    nc = s * s
    w = (nc + 63) // 64
    order = store_record_order(s)
    step = 1 << levels
    sc = (s - 1) // step + 1
    ns = sc * sc
    cls = np.array([0 if i % step == 0 else (i & -i).bit_length() for i in range(s)])
    band = (cls[:, None] * (levels + 1) + cls[None, :]).reshape(-1)[order]
    buf = np.frombuffer(pool, dtype=np.uint8)
    out = np.zeros((npatch, nf, s, s), dtype=np.float32)
    for q in range(npatch):
        for f in range(nf):
            off = int(table[q, f, 0]) * 16
            word = int(table[q, f, 1])
            ndet = word & (O.MASK_BIT - 1)
            occ = int(buf[off:off + 8].view("<u8")[0])
            fmt = values
            if values == "e4m3b":   # bit 63: an E4M3 record, else binary16
                fmt = "e4m3" if (occ >> 63) & 1 else "f16"
                occ &= (1 << 63) - 1
            by = 2 if fmt == "f16" else 1
            bands = [b for b in range(64) if (occ >> b) & 1]
            scale = dict(zip(bands, buf[off + 8:off + 8 + 4 * len(bands)].view("<f4")))
            hb = (8 + 4 * len(bands) + 7) // 8 * 8
            sb = hb + (4 * ns + 7) // 8 * 8
            vb = sb + (by * ndet + 7) // 8 * 8
            samp = buf[off + hb:off + hb + 4 * ns].view("<f4").reshape(sc, sc)
            out[q, f, ::step, ::step] = samp
            if ndet == 0:
                continue
            raw = buf[off + sb:off + sb + by * ndet]
            vals = raw.view("<f2").astype(np.float32) if fmt == "f16" else _e4m3_values(raw)
            if word & O.MASK_BIT:
                bits = np.unpackbits(buf[off + vb:off + vb + 8 * w], bitorder="little")[:nc].astype(bool)
                ks = np.flatnonzero(bits)
            else:
                ks = buf[off + vb:off + vb + 2 * ndet].view("<u2").astype(np.int64)
            sc_of = np.array([scale[int(b)] for b in band[ks]], dtype=np.float32)
            flat = out[q, f].reshape(-1)
            flat[order[ks]] = vals * sc_of
    return out


def decode_records(table: np.ndarray, pool: bytes, s: int, dtype, values: str = "f32",
                   levels: int | None = None) -> np.ndarray:
    """Coefficient tiles ``[npatch, nfields, s, s]`` from a store (host-side reader).

    Reads the record layouts of include/lbmz.h; used to inspect what the
    library wrote.  The narrow value formats need the level count and give
    float32 tiles as read back (details times their subband scale).
    """
    if values != "f32":
        if levels is None:
            raise ValueError("narrow records need the level count")
        return _decode_narrow(table, pool, s, values, levels)
    dtype = np.dtype(dtype)
    npatch, nf = table.shape[:2]
    nc = s * s
    w = (nc + 63) // 64
    order = store_record_order(s)
    seq = np.zeros((npatch, nf, nc), dtype=dtype)
    buf = np.frombuffer(pool, dtype=np.uint8)
    for q in range(npatch):
        for f in range(nf):
            off = int(table[q, f, 0]) * 16
            word = int(table[q, f, 1])
            nnz = word & (O.MASK_BIT - 1)
            vb = (nnz * dtype.itemsize + 7) // 8 * 8
            vals = buf[off:off + nnz * dtype.itemsize].view(dtype)
            if word & O.MASK_BIT:
                words = buf[off + vb:off + vb + 8 * w].view("<u8")
                bits = np.unpackbits(words.view(np.uint8), bitorder="little")[:nc].astype(bool)
                seq[q, f, bits] = vals
            else:
                idx = buf[off + vb:off + vb + 2 * nnz].view("<u2").astype(np.int64)
                seq[q, f, idx] = vals
    out = np.zeros_like(seq)
    out[:, :, order] = seq
    return out.reshape(npatch, nf, s, s)


def decode_records3(table: np.ndarray, pool: bytes, s: int) -> np.ndarray:
    """Coefficient tiles ``float32 [npatch, nfields, s, s, s]`` of a 3-D store
    (record index k = x + s y + s^2 z; host-side reader of include/lbmz.h)."""
    npatch, nf = table.shape[:2]
    nc = s ** 3
    w = (nc + 63) // 64
    out = np.zeros((npatch, nf, nc), dtype=np.float32)
    buf = np.frombuffer(pool, dtype=np.uint8)
    for q in range(npatch):
        for f in range(nf):
            off = int(table[q, f, 0]) * 16
            word = int(table[q, f, 1])
            nnz = word & (O.MASK_BIT - 1)
            vb = (4 * nnz + 7) // 8 * 8
            vals = buf[off:off + 4 * nnz].view("<f4")
            if word & O.MASK_BIT:
                bits = np.unpackbits(buf[off + vb:off + vb + 8 * w], bitorder="little")[:nc].astype(bool)
                out[q, f, bits] = vals
            else:
                out[q, f, buf[off + vb:off + vb + 2 * nnz].view("<u2").astype(np.int64)] = vals
    return out.reshape(npatch, nf, s, s, s)
