"""CPU oracle of the 3-D DWT-compressed patch loop with a D3Q19 BGK scheme --
TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the CPU-baseline leg of the benchmark
may import this module.  The GPU library never calls it, and it shares no
code, table or constant with the GPU library.

The paper's subgrids are three-dimensional (Section 3.1.1: a cube of 2^J + 1
nodes per side with shared bordering values and a one-node ghost layer), and
its multi-dimensional transform is the tensor one (end of Section 2.1: the 1-D
transform on every line of one dimension, then of the next).  This module
extends the 2-D oracle to three dimensions:

* geometry: a periodic ``n^3`` grid cut into ``(n/p)^3`` patches; with the
  folded BL5/3 wavelet a tile holds the ``p + 1`` nodes ``p*k .. p*k + p`` per
  dimension, the last one shared with the next patch; patch
  ``(px, py, pz)`` has index ``px + npx*py + npx^2*pz``; arrays are
  ``[..., z, y, x]`` (x fastest);
* 3-D transform: all L levels along x on every x-line, then along y, then
  along z; the inverse runs z, y, x;
* threshold (Section 2.2) with a rank per dimension, ``r = L - lev``
  (0 = coarsest detail, a sample dimension counts 0): constant ``eps``,
  capped ``eps * 2**max(r)``, accumulation ``eps * 2**sum(r)``; a coefficient
  is a detail when it is a detail in at least one dimension, samples are
  never zeroed, a detail is zeroed when ``|c| < thr``;
* a textbook D3Q19 BGK lattice-Boltzmann step (the paper names LBM and cites
  the textbook scheme without writing one down): pull streaming
  ``f_i^in(x) = f*_i(x - c_i)``, then ``f*_i <- f_i^in - (f_i^in - f_i^eq)/tau``
  with ``f_i^eq = w_i rho (1 + 3 c.u + 4.5 (c.u)^2 - 1.5 u.u)``;
* records per (patch, field): the kept coefficients in ascending flat tile
  index ``t = x + s*y + s*s*z``, then a u16 index list or a bitmask of
  ``ceil(s^3/64)`` u64 words, whichever is smaller (the rule of the 2-D
  records);
* halo rule: ghost values at time n are the neighbours' lossy
  reconstructions at time n, which makes the patch loop equal to the paper's
  whole-grid protocol (Section 3.1.3).

Arithmetic follows the array dtype (float64 by default); NumPy rounds every
elementwise operation once and never fuses a multiply with an add.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from .lbmz_oracle import (BL53, MASK_BIT, RULE_ACCUM, RULE_CAPPED, RULE_CONSTANT, _align, forward_1d,
                          hard_threshold, index_levels, inverse_1d)

# ---------------------------------------------------------------------------
# D3Q19 lattice (textbook; velocity numbering fixed here)
# ---------------------------------------------------------------------------

D3Q19_C = np.array([
    (0, 0, 0),
    (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
    (1, 1, 0), (-1, -1, 0), (1, -1, 0), (-1, 1, 0),
    (1, 0, 1), (-1, 0, -1), (1, 0, -1), (-1, 0, 1),
    (0, 1, 1), (0, -1, -1), (0, 1, -1), (0, -1, 1),
], dtype=np.int64)
D3Q19_W = np.array([1.0 / 3.0] + [1.0 / 18.0] * 6 + [1.0 / 36.0] * 12)


def d3q19_equilibrium(rho, ux, uy, uz):
    """Equilibrium populations stacked on axis -4 (arrays ``[..., z, y, x]``)."""
    rho = np.asarray(rho)
    dt = rho.dtype
    usq = ux * ux + uy * uy + uz * uz
    out = []
    for i in range(19):
        cx, cy, cz = (int(v) for v in D3Q19_C[i])
        cu = cx * ux + cy * uy + cz * uz
        out.append(np.asarray(D3Q19_W[i], dtype=dt) * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * usq))
    return np.stack(out, axis=-4).astype(dt)


def d3q19_moments(f):
    """``(rho, ux, uy, uz)`` of populations stacked on axis -4."""
    rho = f.sum(axis=-4)
    j = [sum(int(D3Q19_C[i, a]) * f[..., i, :, :, :] for i in range(19)) for a in range(3)]
    return rho, j[0] / rho, j[1] / rho, j[2] / rho


def d3q19_stream(padded: np.ndarray) -> np.ndarray:
    """Pull streaming on ghost-padded populations ``[..., 19, d+2, h+2, w+2]``:
    ``f_i^in(x) = f*_i(x - c_i)`` on the interior nodes."""
    d, h, w = (padded.shape[k] - 2 for k in (-3, -2, -1))
    out = []
    for i in range(19):
        cx, cy, cz = (int(v) for v in D3Q19_C[i])
        out.append(padded[..., i, 1 - cz:1 - cz + d, 1 - cy:1 - cy + h, 1 - cx:1 - cx + w])
    return np.stack(out, axis=-4)


def d3q19_collide(fin: np.ndarray, tau: float) -> np.ndarray:
    """BGK relaxation towards the equilibrium of the moments of ``fin``."""
    rho, ux, uy, uz = d3q19_moments(fin)
    feq = d3q19_equilibrium(rho, ux, uy, uz)
    return fin - (fin - feq) / tau


def d3q19_bgk_update(padded: np.ndarray, tau: float) -> np.ndarray:
    """One D3Q19 BGK step (pull streaming, then collision) on padded populations."""
    return d3q19_collide(d3q19_stream(padded), tau)


def periodic_pad3(grid: np.ndarray) -> np.ndarray:
    """Global state ``[m, nz, ny, nx]`` with a one-node periodic ghost layer."""
    return np.pad(grid, ((0, 0), (1, 1), (1, 1), (1, 1)), mode="wrap")


def dense_step3(grid: np.ndarray, tau: float) -> np.ndarray:
    """One uncompressed D3Q19 BGK step on the periodic global grid."""
    return d3q19_bgk_update(periodic_pad3(grid), tau)


# ---------------------------------------------------------------------------
# Geometry (Section 3.1.1, three-dimensional subgrids)
# ---------------------------------------------------------------------------

@dataclass(frozen=True)
class Geometry3:
    """A periodic ``n^3`` grid cut into ``(n/p)^3`` cubic patches, folded BL5/3 tiles of ``p + 1`` nodes."""

    n: int
    p: int
    levels: int = 1

    @property
    def s(self) -> int:
        return self.p + 1

    @property
    def npx(self) -> int:
        return self.n // self.p

    @property
    def npatch(self) -> int:
        return self.npx ** 3

    def validate(self):
        j = int(round(math.log2(self.p)))
        if self.p < 4 or (1 << j) != self.p:
            raise ValueError("patch size must be a power of two >= 4")
        if self.n % self.p != 0:
            raise ValueError("grid size must be a multiple of the patch size")
        if not (0 <= self.levels <= j - 1):
            raise ValueError(f"levels must lie in [0, {j - 1}] on 2^{j} cells")
        return self

    def patch_coords(self, q: int):
        npx = self.npx
        return q % npx, (q // npx) % npx, q // (npx * npx)


def extract_tiles3(grid: np.ndarray, g: Geometry3) -> np.ndarray:
    """Cut a periodic global state ``[m, n, n, n]`` into tiles ``[npatch, m, s, s, s]``."""
    m = grid.shape[0]
    out = np.empty((g.npatch, m, g.s, g.s, g.s), dtype=grid.dtype)
    local = np.arange(g.s)
    for q in range(g.npatch):
        px, py, pz = g.patch_coords(q)
        xs = (px * g.p + local) % g.n
        ys = (py * g.p + local) % g.n
        zs = (pz * g.p + local) % g.n
        out[q] = grid[:, zs[:, None, None], ys[None, :, None], xs[None, None, :]]
    return out


def assemble_grid3(tiles: np.ndarray, g: Geometry3) -> np.ndarray:
    """Global state ``[m, n, n, n]`` from the owned nodes ``[0, p)^3`` of every tile."""
    m = tiles.shape[1]
    p = g.p
    out = np.empty((m, g.n, g.n, g.n), dtype=tiles.dtype)
    for q in range(g.npatch):
        px, py, pz = g.patch_coords(q)
        out[:, pz * p:(pz + 1) * p, py * p:(py + 1) * p, px * p:(px + 1) * p] = tiles[q, :, :p, :p, :p]
    return out


def gather_ghosts3_one(tile_of, g: Geometry3, q: int) -> np.ndarray:
    """Tile ``q`` with a one-node ghost layer, ``[m, s + 2, s + 2, s + 2]``.

    ``tile_of(k)`` gives tile ``k`` (``[m, s, s, s]``).  Along each dimension,
    ghost node ``-1`` is node ``p - 1`` of the lower neighbour and ghost node
    ``s`` is node ``1`` of the upper neighbour; nodes off the tile in two or
    three dimensions come from the edge and corner neighbours.  Every value is
    taken from the neighbours' tiles as given.
    """
    npx, p, s = g.npx, g.p, g.s
    coord = np.arange(-1, s + 1)
    off = np.where(coord < 0, -1, np.where(coord >= s, 1, 0))
    loc = coord - p * off
    px, py, pz = g.patch_coords(q)
    out = None
    for oz in (-1, 0, 1):
        for oy in (-1, 0, 1):
            for ox in (-1, 0, 1):
                k = (px + ox) % npx + npx * ((py + oy) % npx) + npx * npx * ((pz + oz) % npx)
                t = tile_of(k)
                if out is None:
                    out = np.empty((t.shape[0], s + 2, s + 2, s + 2), dtype=t.dtype)
                iz, iy, ix = (np.flatnonzero(off == o) for o in (oz, oy, ox))
                out[:, iz[:, None, None], iy[None, :, None], ix[None, None, :]] = \
                    t[:, loc[iz][:, None, None], loc[iy][None, :, None], loc[ix][None, None, :]]
    return out


def gather_ghosts3(tiles: np.ndarray, g: Geometry3) -> np.ndarray:
    """All tiles with their ghost layer, ``[npatch, m, s + 2, s + 2, s + 2]``."""
    return np.stack([gather_ghosts3_one(lambda k: tiles[k], g, q) for q in range(g.npatch)])


# ---------------------------------------------------------------------------
# 3-D tensor transform and threshold (Sections 2.1, 2.2)
# ---------------------------------------------------------------------------

def forward_3d(tile: np.ndarray, levels: int) -> np.ndarray:
    """Tensor transform of ``[..., s, s, s]`` tiles: every x-line, then y, then z."""
    v = forward_1d(tile, levels, BL53)
    v = np.swapaxes(forward_1d(np.swapaxes(v, -1, -2), levels, BL53), -1, -2)
    v = np.swapaxes(forward_1d(np.swapaxes(v, -1, -3), levels, BL53), -1, -3)
    return np.ascontiguousarray(v)


def inverse_3d(coef: np.ndarray, levels: int) -> np.ndarray:
    """Inverse of :func:`forward_3d`: z-lines, then y, then x."""
    u = np.swapaxes(inverse_1d(np.swapaxes(coef, -1, -3), levels, BL53), -1, -3)
    u = np.swapaxes(inverse_1d(np.swapaxes(u, -1, -2), levels, BL53), -1, -2)
    u = inverse_1d(u, levels, BL53)
    return np.ascontiguousarray(u)


def threshold_table3(s: int, levels: int, eps: float, rule: str, dtype) -> np.ndarray:
    """Threshold per coefficient of an ``s^3`` tile (0 for pure samples)."""
    lev = index_levels(s, levels)
    rank = np.where(lev > 0, levels - lev, 0)
    rz = rank[:, None, None]
    ry = rank[None, :, None]
    rx = rank[None, None, :]
    if rule == RULE_CONSTANT:
        r = np.zeros((s, s, s), dtype=np.int64)
    elif rule == RULE_CAPPED:
        r = np.maximum(np.maximum(rx, ry), rz)
    elif rule == RULE_ACCUM:
        r = rx + ry + rz
    else:
        raise ValueError(rule)
    thr = (np.asarray(eps, dtype=dtype) * (2.0 ** r)).astype(dtype)
    det = lev > 0
    detail = det[:, None, None] | det[None, :, None] | det[None, None, :]
    return np.where(detail, thr, np.zeros((), dtype=dtype)).astype(dtype)


# ---------------------------------------------------------------------------
# Records (the role of CSR, Section 2.3.1), flat tile order x fastest
# ---------------------------------------------------------------------------

def record_layout3(nnz: int, ncoef: int, esize: int):
    """``(is_mask, value_bytes_padded, meta_bytes, record_bytes)`` of one record."""
    w = (ncoef + 63) // 64
    is_mask = not (2 * nnz < 8 * w)
    vb = _align(nnz * esize, 8)
    mb = 8 * w if is_mask else 2 * nnz
    return is_mask, vb, mb, _align(vb + mb, 16)


def encode_record3(tile: np.ndarray) -> bytes:
    """Bytes of one record from a thresholded ``s^3`` tile."""
    seq = np.ascontiguousarray(tile).reshape(-1)
    keep = seq != 0
    idx = np.flatnonzero(keep)
    nnz = idx.size
    is_mask, vb, mb, rb = record_layout3(nnz, seq.size, seq.dtype.itemsize)
    buf = bytearray(rb)
    buf[0:nnz * seq.dtype.itemsize] = seq[idx].astype(seq.dtype.newbyteorder("<")).tobytes()
    if is_mask:
        w = (seq.size + 63) // 64
        bits = np.zeros(64 * w, dtype=np.uint8)
        bits[idx] = 1
        words = np.packbits(bits.reshape(w, 64)[:, ::-1], axis=1).view(">u8").reshape(-1)
        buf[vb:vb + mb] = words.astype("<u8").tobytes()
    else:
        buf[vb:vb + mb] = idx.astype("<u2").tobytes()
    return bytes(buf)


def decode_record3(buf: bytes, off16: int, word: int, s: int, dtype) -> np.ndarray:
    """Inverse of :func:`encode_record3` for the record at ``16 * off16``."""
    dtype = np.dtype(dtype)
    ncoef = s ** 3
    nnz = word & (MASK_BIT - 1)
    base = 16 * off16
    vb = _align(nnz * dtype.itemsize, 8)
    vals = np.frombuffer(buf, dtype=dtype.newbyteorder("<"), count=nnz, offset=base)
    if word & MASK_BIT:
        w = (ncoef + 63) // 64
        words = np.frombuffer(buf, dtype="<u8", count=w, offset=base + vb)
        bits = np.array([(int(words[k // 64]) >> (k % 64)) & 1 for k in range(ncoef)], dtype=bool)
        idx = np.flatnonzero(bits)
    else:
        idx = np.frombuffer(buf, dtype="<u2", count=nnz, offset=base + vb).astype(np.int64)
    out = np.zeros(ncoef, dtype=dtype)
    out[idx] = vals
    return out.reshape(s, s, s)


def encode_store3(coef: np.ndarray):
    """Offset table ``uint32 [npatch, m, 2]`` and pool bytes from ``[npatch, m, s, s, s]``."""
    npatch, m = coef.shape[:2]
    ncoef = coef.shape[2] ** 3
    table = np.zeros((npatch, m, 2), dtype=np.uint32)
    parts = []
    off = 0
    for q in range(npatch):
        for f in range(m):
            rec = encode_record3(coef[q, f])
            nnz = int(np.count_nonzero(coef[q, f]))
            is_mask = record_layout3(nnz, ncoef, coef.dtype.itemsize)[0]
            table[q, f, 0] = off // 16
            table[q, f, 1] = nnz | (MASK_BIT if is_mask else 0)
            parts.append(rec)
            off += len(rec)
    return table, b"".join(parts)


def decode_store3(table: np.ndarray, pool: bytes, s: int, dtype) -> np.ndarray:
    npatch, m = table.shape[:2]
    out = np.zeros((npatch, m, s, s, s), dtype=dtype)
    for q in range(npatch):
        for f in range(m):
            out[q, f] = decode_record3(pool, int(table[q, f, 0]), int(table[q, f, 1]), s, dtype)
    return out


def tile_weights3(g: Geometry3, dtype=np.float64) -> np.ndarray:
    """Trapezoid weights ``[s, s, s]``: 1/2 per shared bordering node and dimension."""
    w1 = np.ones(g.s, dtype=dtype)
    w1[0] = 0.5
    w1[-1] = 0.5
    return w1[:, None, None] * w1[None, :, None] * w1[None, None, :]


# ---------------------------------------------------------------------------
# The compressed method, patch at a time (Sections 3.1.1, 3.1.3)
# ---------------------------------------------------------------------------

class CompressedRun3:
    """State held as thresholded coefficient tiles ``[npatch, 19, s, s, s]``.

    ``step()`` is the patch loop: every patch is rebuilt by the inverse
    transform, completed with a ghost layer from the neighbours' rebuilt
    tiles, advanced by the D3Q19 BGK step, transformed forward,
    hard-thresholded and stored.
    """

    def __init__(self, g: Geometry3, tau: float, eps: float, rule: str = RULE_CAPPED, dtype=np.float64):
        self.g = g.validate()
        self.tau = tau
        self.eps = eps
        self.rule = rule
        self.dtype = np.dtype(dtype)
        self.thr = threshold_table3(g.s, g.levels, eps, rule, self.dtype)
        self.coef = None
        self.steps = 0

    def compress_tiles(self, tiles: np.ndarray) -> np.ndarray:
        c = forward_3d(tiles.astype(self.dtype), self.g.levels)
        return hard_threshold(c, self.thr)

    def decompress_tiles(self, coef: np.ndarray | None = None) -> np.ndarray:
        return inverse_3d(self.coef if coef is None else coef, self.g.levels)

    def set_grid(self, grid: np.ndarray):
        self.coef = self.compress_tiles(extract_tiles3(np.asarray(grid, dtype=self.dtype), self.g))
        self.steps = 0

    def set_coefficients(self, coef: np.ndarray, threshold: bool = True):
        c = np.asarray(coef, dtype=self.dtype)
        self.coef = hard_threshold(c, self.thr) if threshold else c.copy()

    def grid(self) -> np.ndarray:
        return assemble_grid3(self.decompress_tiles(), self.g)

    def step(self, n: int = 1):
        for _ in range(n):
            lossy = self.decompress_tiles()
            padded = gather_ghosts3(lossy, self.g)
            self.coef = self.compress_tiles(d3q19_bgk_update(padded, self.tau).astype(self.dtype))
            self.steps += 1

    def store(self):
        return encode_store3(self.coef)

    def nnz(self) -> np.ndarray:
        return np.count_nonzero(self.coef.reshape(self.coef.shape[0], self.coef.shape[1], -1), axis=-1)

    def store_bytes(self) -> int:
        ncoef = self.g.s ** 3
        tot = sum(record_layout3(int(v), ncoef, self.dtype.itemsize)[3] for v in self.nnz().reshape(-1))
        return tot + self.coef.shape[0] * self.coef.shape[1] * 8

    def dense_bytes(self) -> int:
        return self.g.n ** 3 * 19 * self.dtype.itemsize

    def ratio(self) -> float:
        return self.dense_bytes() / self.store_bytes()

    def field_totals(self) -> np.ndarray:
        """Per-population trapezoid-weighted sums of the lossy state, float64."""
        lossy = self.decompress_tiles().astype(np.float64)
        return (lossy * tile_weights3(self.g)).sum(axis=(0, 2, 3, 4))


def whole_grid_step3(run: CompressedRun3):
    """The paper's protocol (Section 3.1.3): decompress everything, step on the
    periodic global grid, cut into tiles again and recompress."""
    new_grid = dense_step3(run.grid(), run.tau).astype(run.dtype)
    run.coef = run.compress_tiles(extract_tiles3(new_grid, run.g))
    run.steps += 1
