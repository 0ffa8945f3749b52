"""CPU oracle of the DWT-compressed patch loop -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the CPU-baseline leg of the benchmark
may import this module.  The GPU library never calls it, and it shares no code,
table or constant with the GPU library.

It is a plain, slow, obviously-correct NumPy implementation of what the
method computes, written from Flint & Helluy, "Reducing the memory usage of
Lattice-Boltzmann schemes with a DWT-based compression" (arXiv 2302.09883):

* finite-volume scheme and its two-buffer time loop (Section 1, equation
  "vf_scheme"), with the upwind transport flux (Section 3.1.2, equation
  "upwind_trans");
* a textbook D2Q9 BGK lattice-Boltzmann step (the paper names LBM but never
  writes one down; this is the standard scheme it cites);
* the folded BL5/3 lifting wavelet on 2^j + 1 samples with fixed boundary
  samples and mass-conserving update weights (Section 2.1.2), repeated over
  the sample sub-lattice for L levels, and extended to 2-D by transforming
  every row and then every column (end of Section 2.1);
* a Haar lifting wavelet on 2^j samples (mean-preserving form), used by the
  transport workload;
* hard thresholding of the details only, with the constant, accumulation and
  capped rules of Section 2.2;
* a compaction of the surviving coefficients into per-(patch, field) records
  that plays the role of the CSR stage of Section 2.3.1;
* the subgrid decomposition with shared bordering values and a one-cell ghost
  ring (Section 3.1.1), and the compress/decompress cycle between steps
  (Section 3.1.3), run patch by patch (the Introduction's patch-at-a-time
  residency) and, for comparison, on the whole grid at once.

Floating-point arithmetic follows the array dtype: float64 by default, float32
when the caller wants decisions taken in the GPU kernel's precision.  NumPy
evaluates every elementwise operation with one IEEE round-to-nearest rounding
and never fuses a multiply with an add.  Vectorisation runs over independent
patches, fields and lines only; the order of operations inside each
coefficient's update is the one written in the formulas below.

Readings of passages the paper leaves open (all of them listed with their
reasons in the design notes of the repository):

* threshold rules: a detail of level ``lev`` (1 = finest) in an L-level
  transform has rank ``r = L - lev`` (0 = coarsest detail); capped threshold
  ``eps * 2**max(r_x, r_y)``, accumulation ``eps * 2**(r_x + r_y)``, constant
  ``eps``; a coefficient is a detail if it is a detail in at least one
  dimension, and a sample dimension contributes rank 0.  The direction of
  the rank is pinned by the paper's own comparison of the rules (capped
  keeps fewer coefficients than constant at the same error; the opposite
  direction fails it); the values of the capped and accumulation thresholds
  have no printed example (the paper shows them in figures only); the
  constant rule is pinned by the worked example of Section 2.1.2.
* a detail is zeroed when ``|c| < thr`` (strict).
* the bl53 transform keeps L <= J - 1 levels on a 2^J + 1 tile, the largest
  number for which the level update exists and conserves mass.
* Haar is not in the paper; its lifting form is ``d = b - a``,
  ``s = a + d / 2`` (pairwise mean), inverse ``a = s - d / 2``, ``b = a + d``.
* halo rule: ghost values at time n are the neighbours' lossy
  reconstructions at time n (the inverse transform of their stored
  coefficients), which makes the patch loop equal to the paper's whole-grid
  protocol.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

# ---------------------------------------------------------------------------
# Geometry (Section 3.1.1: subgrids with shared bordering values)
# ---------------------------------------------------------------------------

BL53 = "bl53"
HAAR = "haar"

RULE_CAPPED = "capped"
RULE_CONSTANT = "constant"
RULE_ACCUM = "accum"


@dataclass(frozen=True)
class Geometry:
    """A periodic ``n x n`` grid cut into ``(n/p)^2`` square patches of ``p`` cells.

    With the bl53 wavelet a patch's tile holds the ``p + 1`` nodes
    ``p*px .. p*px + p`` in each dimension: the last node is shared with the
    next patch, the logical-size convention of Section 3.1.1 that lets the
    trapezoid mass of every subgrid add up to the global mass.  With Haar the
    tile holds the ``p`` owned nodes only.  Patch ``(px, py)`` has index
    ``px + (n/p) * py``.
    """

    n: int
    p: int
    wavelet: str = BL53
    levels: int = 1

    @property
    def s(self) -> int:
        return self.p + 1 if self.wavelet == BL53 else self.p

    @property
    def npx(self) -> int:
        return self.n // self.p

    @property
    def npatch(self) -> int:
        return self.npx * self.npx

    def validate(self):
        j = int(round(math.log2(self.p)))
        if self.p < 2 or (1 << j) != self.p:
            raise ValueError("patch size must be a power of two >= 2")
        if self.n % self.p != 0:
            raise ValueError("grid size must be a multiple of the patch size")
        cap = j - 1 if self.wavelet == BL53 else j
        if not (1 <= self.levels <= cap) and self.levels != 0:
            raise ValueError(f"levels must lie in [0, {cap}] for {self.wavelet} on 2^{j} cells")
        return self


def extract_tiles(grid: np.ndarray, g: Geometry) -> np.ndarray:
    """Cut a periodic global state ``[m, n, n]`` into tiles ``[npatch, m, s, s]``."""
    m = grid.shape[0]
    out = np.empty((g.npatch, m, g.s, g.s), dtype=grid.dtype)
    local = np.arange(g.s)
    for py in range(g.npx):
        ys = (py * g.p + local) % g.n
        for px in range(g.npx):
            xs = (px * g.p + local) % g.n
            out[px + g.npx * py] = grid[:, ys[:, None], xs[None, :]]
    return out


def assemble_grid(tiles: np.ndarray, g: Geometry) -> np.ndarray:
    """Global state ``[m, n, n]`` from the owned nodes ``[0, p)^2`` of every tile."""
    m = tiles.shape[1]
    out = np.empty((m, g.n, g.n), dtype=tiles.dtype)
    for py in range(g.npx):
        for px in range(g.npx):
            out[:, py * g.p:(py + 1) * g.p, px * g.p:(px + 1) * g.p] = \
                tiles[px + g.npx * py, :, :g.p, :g.p]
    return out


def gather_ghosts(tiles: np.ndarray, g: Geometry) -> np.ndarray:
    """Tiles with a one-node ghost ring, ``[npatch, m, s + 2, s + 2]``.

    Ghost node ``-1`` of a tile is node ``p - 1`` of the lower neighbour and
    ghost node ``s`` is node ``s - p`` of the upper neighbour (node 1 with
    bl53, node 0 with Haar); corners come from the diagonal neighbours.
    These are exactly the copies of Fig. 3's synchronisation, taken from the
    neighbours' tiles as given (their lossy reconstructions in the method).
    """
    npx, p, s = g.npx, g.p, g.s
    m = tiles.shape[1]
    out = np.empty((g.npatch, m, s + 2, s + 2), dtype=tiles.dtype)
    # local ghost-ring coordinate -> (neighbour offset, local node in neighbour)
    coord = np.arange(-1, s + 1)
    off = np.where(coord < 0, -1, np.where(coord >= s, 1, 0))
    loc = coord - p * off
    for py in range(npx):
        for px in range(npx):
            q = px + npx * py
            nb_y = (py + off) % npx
            nb_x = (px + off) % npx
            nb = nb_x[None, :] + npx * nb_y[:, None]           # [s+2, s+2]
            out[q] = tiles[nb, :, loc[:, None], loc[None, :]].transpose(2, 0, 1)
    return out


# ---------------------------------------------------------------------------
# 1-D transforms (Section 2.1.2) -- in-place interleaved layout
# ---------------------------------------------------------------------------
#
# A level acts on the current sample sub-lattice (stride 2**(lev-1)); after it
# the even positions of that sub-lattice hold the coarser samples and the odd
# positions hold the details, so a level-``lev`` detail sits at an index
# congruent to 2**(lev-1) modulo 2**lev ("samples distributed evenly",
# Section 3.2.4), and the samples left after L levels are the indices that are
# multiples of 2**L.


def _bl53_alpha(m: int, dtype) -> np.ndarray:
    """Update weights alpha_k, k = 0 .. m-1 (m details at this level).

    1/2 at both ends of the detail range and 1/4 inside: the unique choice that
    satisfies the mass-conservation requirement (equation "conservation").
    """
    a = np.full(m, 0.25, dtype=dtype)
    a[0] = 0.5
    a[m - 1] = 0.5
    return a


def bl53_forward_level(u: np.ndarray) -> np.ndarray:
    """One folded BL5/3 level along the last axis on ``2m + 1`` samples.

    Predict: ``d_k = u_{2k+1} - (u_{2k} + u_{2k+2}) / 2``.  Boundary samples are
    kept (equation "boundary_values").  Update for ``0 < k < m``:
    ``s_k = (u_{2k} + alpha_{k-1} d_{k-1}) + alpha_k d_k``.
    """
    even = u[..., 0::2]
    odd = u[..., 1::2]
    m = odd.shape[-1]
    d = odd - (even[..., :-1] + even[..., 1:]) * 0.5
    s = even.copy()
    if m >= 2:
        al = _bl53_alpha(m, u.dtype)
        s[..., 1:m] = (even[..., 1:m] + al[:m - 1] * d[..., :m - 1]) + al[1:m] * d[..., 1:m]
    out = np.empty_like(u)
    out[..., 0::2] = s
    out[..., 1::2] = d
    return out


def bl53_inverse_level(v: np.ndarray) -> np.ndarray:
    """Inverse of :func:`bl53_forward_level` (the lifting steps undone in reverse).

    ``e_k = (s_k - alpha_{k-1} d_{k-1}) - alpha_k d_k`` for ``0 < k < m``,
    ``e_0 = s_0``, ``e_m = s_m``; then ``u_{2k+1} = d_k + (e_k + e_{k+1}) / 2``.
    """
    s = v[..., 0::2]
    d = v[..., 1::2]
    m = d.shape[-1]
    e = s.copy()
    if m >= 2:
        al = _bl53_alpha(m, v.dtype)
        e[..., 1:m] = (s[..., 1:m] - al[:m - 1] * d[..., :m - 1]) - al[1:m] * d[..., 1:m]
    out = np.empty_like(v)
    out[..., 0::2] = e
    out[..., 1::2] = d + (e[..., :-1] + e[..., 1:]) * 0.5
    return out


def haar_forward_level(u: np.ndarray) -> np.ndarray:
    """One Haar lifting level on ``2m`` samples: ``d = b - a``, ``s = a + d / 2``."""
    a = u[..., 0::2]
    b = u[..., 1::2]
    d = b - a
    s = a + d * 0.5
    out = np.empty_like(u)
    out[..., 0::2] = s
    out[..., 1::2] = d
    return out


def haar_inverse_level(v: np.ndarray) -> np.ndarray:
    """Inverse Haar lifting: ``a = s - d / 2``, ``b = a + d``."""
    s = v[..., 0::2]
    d = v[..., 1::2]
    a = s - d * 0.5
    b = a + d
    out = np.empty_like(v)
    out[..., 0::2] = a
    out[..., 1::2] = b
    return out


def forward_1d(u: np.ndarray, levels: int, wavelet: str) -> np.ndarray:
    """``levels`` forward levels along the last axis, finest first."""
    lvl = bl53_forward_level if wavelet == BL53 else haar_forward_level
    v = np.array(u, copy=True)
    for lev in range(1, levels + 1):
        st = 1 << (lev - 1)
        v[..., ::st] = lvl(v[..., ::st])
    return v


def inverse_1d(v: np.ndarray, levels: int, wavelet: str) -> np.ndarray:
    """Inverse of :func:`forward_1d`: coarsest level first."""
    lvl = bl53_inverse_level if wavelet == BL53 else haar_inverse_level
    u = np.array(v, copy=True)
    for lev in range(levels, 0, -1):
        st = 1 << (lev - 1)
        u[..., ::st] = lvl(u[..., ::st])
    return u


def forward_2d(tile: np.ndarray, levels: int, wavelet: str) -> np.ndarray:
    """2-D transform of ``[..., s, s]`` tiles: every row (x), then every column (y)."""
    v = forward_1d(tile, levels, wavelet)
    v = np.swapaxes(forward_1d(np.swapaxes(v, -1, -2), levels, wavelet), -1, -2)
    return np.ascontiguousarray(v)


def inverse_2d(coef: np.ndarray, levels: int, wavelet: str) -> np.ndarray:
    """Inverse of :func:`forward_2d`: columns first, then rows."""
    u = np.swapaxes(inverse_1d(np.swapaxes(coef, -1, -2), levels, wavelet), -1, -2)
    u = inverse_1d(u, levels, wavelet)
    return np.ascontiguousarray(u)


# ---------------------------------------------------------------------------
# Thresholding (Section 2.2)
# ---------------------------------------------------------------------------

def index_levels(s: int, levels: int) -> np.ndarray:
    """Per index of one dimension: 0 for a sample, else the detail level (1 = finest)."""
    lev = np.zeros(s, dtype=np.int64)
    for i in range(s):
        if i % (1 << levels) == 0:
            continue
        k, lv = i, 1
        while k % 2 == 0:
            k //= 2
            lv += 1
        lev[i] = lv
    return lev


def threshold_table(s: int, levels: int, eps: float, rule: str, dtype) -> np.ndarray:
    """Threshold per coefficient of an ``s x s`` tile, ``[s, s]`` in ``dtype``.

    Pure samples get 0 (never zeroed).  For a detail, each dimension's rank is
    ``levels - lev`` (0 for a sample dimension); the threshold is ``eps``
    (constant), ``eps * 2**max(rank)`` (capped) or ``eps * 2**sum(rank)``
    (accumulation), evaluated by exact power-of-two scaling of ``dtype(eps)``.
    """
    lev = index_levels(s, levels)
    rank = np.where(lev > 0, levels - lev, 0)
    ry = rank[:, None]
    rx = rank[None, :]
    if rule == RULE_CONSTANT:
        r = np.zeros((s, s), dtype=np.int64)
    elif rule == RULE_CAPPED:
        r = np.maximum(rx, ry)
    elif rule == RULE_ACCUM:
        r = rx + ry
    else:
        raise ValueError(rule)
    thr = (np.asarray(eps, dtype=dtype) * (2.0 ** r)).astype(dtype)
    detail = (lev[:, None] > 0) | (lev[None, :] > 0)
    return np.where(detail, thr, np.zeros((), dtype=dtype)).astype(dtype)


def hard_threshold(coef: np.ndarray, thr: np.ndarray) -> np.ndarray:
    """Zero every coefficient whose magnitude is strictly below its threshold."""
    out = np.array(coef, copy=True)
    out[np.abs(coef) < thr] = 0
    return out


# ---------------------------------------------------------------------------
# Compaction: per-(patch, field) records (the role of CSR, Section 2.3.1)
# ---------------------------------------------------------------------------
#
# Record order of the coefficients of one (patch, field) tile: the owned
# p x p block first, row by row (x fastest), then, for bl53 tiles (size
# p + 1), the shared bordering column x = p (y = 0 .. p-1), the shared row
# y = p (x = 0 .. p-1) and the shared corner (p, p).  For a Haar tile (size p)
# this is plain row-major order.  A coefficient's record index k is its
# position in this order.
#
# Record of one tile:
#   kept[k] = coefficient != 0 (negative zero counts as zero, NaN is kept);
#   values  = the kept coefficients in ascending k;
#   then, if 2*nnz < 8*W with W = ceil(s*s / 64): the u16 indices k (an index
#   list), otherwise W little-endian u64 words with bit (k % 64) of word
#   (k // 64) set for a kept coefficient (a bitmask);
#   layout: values, zero padding to a multiple of 8 bytes, the index list or
#   the mask words, zero padding to a multiple of 16 bytes.
# Offset table entry per (patch, field): u32 record offset in 16-byte units,
#   u32 nnz with bit 31 set when the record holds a bitmask.
# Pool placement in this oracle: records in (patch, field) order, each at the
#   exclusive prefix sum of the previous record sizes.

MASK_BIT = 1 << 31


def record_order(s: int) -> np.ndarray:
    """Flat tile indices (``y * s + x``) in record order for an ``s x s`` tile.

    ``s`` odd means a bl53 tile of ``p = s - 1`` owned cells plus the shared
    border; ``s`` even means a Haar tile of ``p = s`` cells.
    """
    p = s - 1 if s % 2 == 1 else s
    order = [y * s + x for y in range(p) for x in range(p)]
    if p != s:
        order += [y * s + p for y in range(p)]
        order += [p * s + x for x in range(p)]
        order += [p * s + p]
    return np.array(order, dtype=np.int64)


def _align(x: int, a: int) -> int:
    return (x + a - 1) // a * a


def record_layout(nnz: int, ncoef: int, esize: int):
    """Return ``(is_mask, value_bytes_padded, meta_bytes, record_bytes)``."""
    w = (ncoef + 63) // 64
    is_mask = not (2 * nnz < 8 * w)
    vb = _align(nnz * esize, 8)
    mb = 8 * w if is_mask else 2 * nnz
    return is_mask, vb, mb, _align(vb + mb, 16)


def encode_record(tile: np.ndarray) -> bytes:
    """Bytes of one record from a thresholded ``s x s`` tile (see layout above)."""
    s = tile.shape[-1]
    seq = np.ascontiguousarray(tile).reshape(-1)[record_order(s)]
    ncoef = seq.size
    keep = seq != 0
    idx = np.flatnonzero(keep)
    nnz = idx.size
    esize = seq.dtype.itemsize
    is_mask, vb, mb, rb = record_layout(nnz, ncoef, esize)
    buf = bytearray(rb)
    buf[0:nnz * esize] = seq[idx].astype(seq.dtype.newbyteorder("<")).tobytes()
    if is_mask:
        w = (ncoef + 63) // 64
        words = np.zeros(w, dtype="<u8")
        for k in idx:
            words[k // 64] |= np.uint64(1) << np.uint64(k % 64)
        buf[vb:vb + mb] = words.tobytes()
    else:
        buf[vb:vb + mb] = idx.astype("<u2").tobytes()
    return bytes(buf)


def decode_record(buf: bytes, off16: int, word: int, s: int, dtype) -> np.ndarray:
    """Inverse of :func:`encode_record` for the record at ``16 * off16``; ``s x s`` tile."""
    dtype = np.dtype(dtype)
    ncoef = s * s
    nnz = word & (MASK_BIT - 1)
    is_mask = bool(word & MASK_BIT)
    base = 16 * off16
    vb = _align(nnz * dtype.itemsize, 8)
    vals = np.frombuffer(buf, dtype=dtype.newbyteorder("<"), count=nnz, offset=base)
    if is_mask:
        w = (ncoef + 63) // 64
        words = np.frombuffer(buf, dtype="<u8", count=w, offset=base + vb)
        bits = [(int(words[k // 64]) >> (k % 64)) & 1 for k in range(ncoef)]
        idx = np.flatnonzero(np.array(bits, dtype=bool))
    else:
        idx = np.frombuffer(buf, dtype="<u2", count=nnz, offset=base + vb).astype(np.int64)
    seq = np.zeros(ncoef, dtype=dtype)
    seq[idx] = vals
    out = np.zeros(ncoef, dtype=dtype)
    out[record_order(s)] = seq
    return out.reshape(s, s)


def encode_store(coef: np.ndarray):
    """Offset table ``uint32 [npatch, m, 2]`` and pool bytes from ``[npatch, m, s, s]``."""
    npatch, m, s = coef.shape[0], coef.shape[1], coef.shape[2]
    table = np.zeros((npatch, m, 2), dtype=np.uint32)
    parts = []
    off = 0
    for q in range(npatch):
        for f in range(m):
            rec = encode_record(coef[q, f])
            nnz = int(np.count_nonzero(coef[q, f] != 0))
            is_mask = record_layout(nnz, s * s, coef.dtype.itemsize)[0]
            table[q, f, 0] = off // 16
            table[q, f, 1] = nnz | (MASK_BIT if is_mask else 0)
            parts.append(rec)
            off += len(rec)
    return table, b"".join(parts)


def decode_store(table: np.ndarray, pool: bytes, s: int, dtype) -> np.ndarray:
    """Coefficient tiles ``[npatch, m, s, s]`` from an offset table and a pool."""
    npatch, m = table.shape[:2]
    out = np.zeros((npatch, m, s, s), dtype=dtype)
    for q in range(npatch):
        for f in range(m):
            out[q, f] = decode_record(pool, int(table[q, f, 0]), int(table[q, f, 1]), s, dtype)
    return out


def store_bytes(table: np.ndarray, s: int, esize: int) -> int:
    """Bytes of the compressed store: all records plus the offset table."""
    tot = 0
    for word in table[..., 1].reshape(-1):
        nnz = int(word) & (MASK_BIT - 1)
        tot += record_layout(nnz, s * s, esize)[3]
    return tot + table.size * 4


# ---------------------------------------------------------------------------
# Schemes (Section 1; Section 3.1.2; textbook D2Q9 BGK)
# ---------------------------------------------------------------------------

# Outward normals N^0..N^3 (equation "directions"): +x, -x, +y, -y.
NORMALS = ((1, 0), (-1, 0), (0, 1), (0, -1))


def upwind_flux(wl, wr, vel, normal):
    """Upwind transport flux ``W_L max(a.N, 0) + W_R min(a.N, 0)`` (equation "upwind_trans")."""
    an = vel[0] * normal[0] + vel[1] * normal[1]
    return wl * max(an, 0.0) + wr * min(an, 0.0)


def fv_dt_over_h(vel, cfl: float) -> float:
    """``dt / h = CFL / v_max`` with ``v_max`` the largest speed component magnitude."""
    return cfl / max(abs(vel[0]), abs(vel[1]))


def fv_upwind_update(padded: np.ndarray, vel, cfl: float) -> np.ndarray:
    """One finite-volume step on ghost-padded arrays ``[..., h + 2, w + 2]``.

    Equation "vf_scheme" evaluated in the order of the transport-kernel listing:
    start from ``W``, then for each direction ``k = 0..3`` subtract
    ``dt/h * Q(W, W_{+N^k}, N^k)``.
    """
    r = fv_dt_over_h(vel, cfl)
    w = padded[..., 1:-1, 1:-1]
    out = np.array(w, copy=True)
    hh, ww = w.shape[-2], w.shape[-1]
    for (nx, ny) in NORMALS:
        nb = padded[..., 1 + ny:1 + ny + hh, 1 + nx:1 + nx + ww]
        out = out - r * upwind_flux(w, nb, vel, (nx, ny))
    return out


# Compressible Euler equations with the Rusanov (local Lax-Friedrichs) flux:
# the scheme of equation "vf_scheme" with m = 4 conserved fields
# W = (rho, rho u, rho v, E) and the physical flux
# F(W).N = (rho un, rho u un + p Nx, rho v un + p Ny, (E + p) un),
# un = u Nx + v Ny, p = (gamma - 1) (E - rho (u^2 + v^2) / 2).  The paper
# leaves the flux of a system to the scheme (it uses a Godunov flux for its
# shallow-water test); Rusanov is the first-order flux of the precision
# workload.  The time step is dt = CFL h / s_max with s_max a bound of
# |u| + c given with the scheme.

def euler_physical_flux(w: np.ndarray, normal, gamma: float):
    """``(F(W).N, un, c)`` for states ``w[4, ...]``."""
    nx, ny = normal
    rho, mx, my, e = w[0], w[1], w[2], w[3]
    u = mx / rho
    v = my / rho
    p = (gamma - 1.0) * (e - 0.5 * rho * (u * u + v * v))
    un = u * nx + v * ny
    c = np.sqrt(gamma * p / rho)
    f = np.stack([rho * un, mx * un + p * nx, my * un + p * ny, (e + p) * un])
    return f, un, c


def rusanov_flux(wl: np.ndarray, wr: np.ndarray, normal, gamma: float) -> np.ndarray:
    """``Q(W_L, W_R, N) = (F(W_L).N + F(W_R).N) / 2 - lambda (W_R - W_L) / 2`` with
    ``lambda = max(|un_L| + c_L, |un_R| + c_R)``."""
    fl, unl, cl = euler_physical_flux(wl, normal, gamma)
    fr, unr, cr = euler_physical_flux(wr, normal, gamma)
    lam = np.maximum(np.abs(unl) + cl, np.abs(unr) + cr)
    return 0.5 * (fl + fr) - 0.5 * lam * (wr - wl)


def euler_rusanov_update(padded: np.ndarray, dt_over_h: float, gamma: float) -> np.ndarray:
    """One step on a ghost-padded state ``[..., 4, h + 2, w + 2]`` (fields on
    the third axis from the end), in the order of the transport-kernel
    listing: start from ``W``, then for each direction ``k = 0..3`` subtract
    ``dt/h * Q(W, W_{+N^k}, N^k)``."""
    pf = np.moveaxis(padded, -3, 0)          # fields first
    w = pf[..., 1:-1, 1:-1]
    out = np.array(w, copy=True)
    hh, ww = w.shape[-2], w.shape[-1]
    for (nx, ny) in NORMALS:
        nb = pf[..., 1 + ny:1 + ny + hh, 1 + nx:1 + nx + ww]
        out = out - dt_over_h * rusanov_flux(w, nb, (nx, ny), gamma)
    return np.moveaxis(out, 0, -3)


def euler_conserved(rho, u, v, p, gamma: float) -> np.ndarray:
    """Conserved fields ``[4, ...]`` from primitive ones."""
    rho = np.asarray(rho, dtype=np.float64)
    e = np.asarray(p, dtype=np.float64) / (gamma - 1.0) + 0.5 * rho * (np.asarray(u) ** 2 + np.asarray(v) ** 2)
    return np.stack([rho, rho * u, rho * v, e])


# D2Q9 velocity set and weights (numbering 0: rest, 1-4: axes, 5-8: diagonals).
D2Q9_C = np.array([(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1),
                   (1, 1), (-1, 1), (-1, -1), (1, -1)], dtype=np.int64)
D2Q9_W = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4, dtype=np.float64)


def d2q9_equilibrium(rho, ux, uy):
    """``f_i^eq = w_i rho (1 + 3 c.u + 4.5 (c.u)^2 - 1.5 u.u)``, stacked on axis -3."""
    rho = np.asarray(rho)
    dt = rho.dtype
    usq = ux * ux + uy * uy
    out = []
    for i in range(9):
        cx, cy = int(D2Q9_C[i, 0]), int(D2Q9_C[i, 1])
        cu = cx * ux + cy * uy
        out.append(np.asarray(D2Q9_W[i], dtype=dt) * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * usq))
    return np.stack(out, axis=-3).astype(dt)


def d2q9_moments(f):
    """``(rho, ux, uy)`` of populations stacked on axis -3."""
    rho = f.sum(axis=-3)
    jx = sum(int(D2Q9_C[i, 0]) * f[..., i, :, :] for i in range(9))
    jy = sum(int(D2Q9_C[i, 1]) * f[..., i, :, :] for i in range(9))
    return rho, jx / rho, jy / rho


def d2q9_bgk_update(padded: np.ndarray, tau: float) -> np.ndarray:
    """One D2Q9 BGK step on ghost-padded post-collision populations.

    Pull streaming ``f_i^in(x) = f*_i(x - c_i)``, moments of ``f^in``, then
    ``f*_i <- f_i^in - (f_i^in - f_i^eq) / tau``.  Input ``[..., 9, h + 2, w + 2]``.
    """
    hh = padded.shape[-2] - 2
    ww = padded.shape[-1] - 2
    c = [(int(cx), int(cy)) for cx, cy in D2Q9_C]
    fin = np.stack([padded[..., i, 1 - c[i][1]:1 - c[i][1] + hh, 1 - c[i][0]:1 - c[i][0] + ww]
                    for i in range(9)], axis=-3)
    rho, ux, uy = d2q9_moments(fin)
    feq = d2q9_equilibrium(rho, ux, uy)
    return fin - (fin - feq) / tau


@dataclass(frozen=True)
class Scheme:
    kind: str                     # "fv_upwind", "d2q9_bgk" or "euler_rusanov"
    vel: tuple = (1.0, 0.5)       # FV: transport velocity; Euler: (s_max, -) bound of |u| + c
    cfl: float = 0.5
    tau: float = 0.6
    gamma: float = 1.4

    @property
    def nfields(self) -> int:
        return {"d2q9_bgk": 9, "euler_rusanov": 4}.get(self.kind, 1)

    def update(self, padded: np.ndarray) -> np.ndarray:
        if self.kind == "fv_upwind":
            return fv_upwind_update(padded, self.vel, self.cfl)
        if self.kind == "d2q9_bgk":
            return d2q9_bgk_update(padded, self.tau)
        if self.kind == "euler_rusanov":
            return euler_rusanov_update(padded, self.cfl / self.vel[0], self.gamma)
        raise ValueError(self.kind)


def periodic_pad(grid: np.ndarray) -> np.ndarray:
    """Global state ``[m, n, n]`` with a one-cell periodic ghost ring."""
    return np.pad(grid, ((0, 0), (1, 1), (1, 1)), mode="wrap")


def dense_step(grid: np.ndarray, scheme: Scheme) -> np.ndarray:
    """One uncompressed step of the scheme on the periodic global grid."""
    return scheme.update(periodic_pad(grid))


# ---------------------------------------------------------------------------
# The compressed method (Sections 3.1.1 and 3.1.3, patch at a time)
# ---------------------------------------------------------------------------

def tile_weights(g: Geometry, dtype=np.float64) -> np.ndarray:
    """Trapezoid weights ``[s, s]``: 1/2 per shared bordering node (bl53), else 1."""
    w1 = np.ones(g.s, dtype=dtype)
    if g.wavelet == BL53:
        w1[0] = 0.5
        w1[-1] = 0.5
    return w1[:, None] * w1[None, :]


class CompressedRun:
    """State held as thresholded coefficient tiles ``[npatch, m, s, s]``.

    ``step()`` is the patch loop: every patch is rebuilt from its coefficients
    by the inverse transform, completed with a ghost ring taken from the
    neighbours' rebuilt tiles, advanced by the scheme, transformed forward,
    hard-thresholded, and stored.  All inputs of a step are time-n data, so
    the patch order is irrelevant (the loop is written over all patches at once).
    """

    def __init__(self, g: Geometry, scheme: Scheme, eps: float, rule: str = RULE_CAPPED,
                 dtype=np.float64, values: str = "f32"):
        self.g = g.validate()
        self.scheme = scheme
        self.eps = eps
        self.rule = rule
        self.dtype = np.dtype(dtype)
        self.values = values
        if values != "f32" and self.dtype != np.float32:
            raise ValueError("narrow value formats store float32 coefficients")
        self.eps_patch = None     # per-patch threshold constants, or None for eps
        self.levels_patch = None  # per-patch level counts, or None for g.levels
        self.thr = threshold_table(g.s, g.levels, eps, rule, self.dtype)
        self.coef = None
        self.kept = None          # threshold decisions of the stored coefficients
        self.steps = 0

    # -- per-patch threshold controls -------------------------------------------
    def _rebuild_thresholds(self):
        """Threshold tables: one per patch when its constant or level count is its own.

        Patch q's table is that of its constant eps_q and its threshold level
        count L_q (Section 2.2 with L_q in place of L: the L_q finest detail
        levels may be zeroed, ranks counted from the coarsest of them, coarser
        coefficients kept like samples).  With BL5/3 tiles a bordering line is
        stored by both tiles that share it (Section 3.1.1); it takes, entry by
        entry, the smaller of the two tiles' thresholds, so that both keep the
        same coefficients of it and reconstruct the same values there (the
        shared values the conservation of the totals rests on).  Corners are
        samples in both dimensions and never thresholded."""
        g = self.g
        if self.eps_patch is None and self.levels_patch is None:
            self.thr = threshold_table(g.s, g.levels, self.eps, self.rule, self.dtype)
            return
        npatch = g.npatch
        eps = [self.eps] * npatch if self.eps_patch is None else [float(e) for e in self.eps_patch]
        lev = [g.levels] * npatch if self.levels_patch is None else [int(L) for L in self.levels_patch]
        base = np.stack([threshold_table(g.s, lev[q], eps[q], self.rule, self.dtype) for q in range(npatch)])
        thr = base.copy()
        if g.wavelet == BL53:
            p = g.p
            for q in range(npatch):
                px, py = q % g.npx, q // g.npx
                left = (px - 1) % g.npx + g.npx * py
                right = (px + 1) % g.npx + g.npx * py
                down = px + g.npx * ((py - 1) % g.npx)
                up = px + g.npx * ((py + 1) % g.npx)
                thr[q, :, 0] = np.minimum(thr[q, :, 0], base[left, :, p])
                thr[q, :, p] = np.minimum(thr[q, :, p], base[right, :, 0])
                thr[q, 0, :] = np.minimum(thr[q, 0, :], base[down, p, :])
                thr[q, p, :] = np.minimum(thr[q, p, :], base[up, 0, :])
        self.thr = thr[:, None]

    def set_patch_levels(self, levels=None):
        """One threshold level count per patch (the learned control), 0 <= L_q <= L,
        or None for the single count L.  The transform keeps its L levels."""
        if self.values != "f32" and levels is not None:
            raise ValueError("per-patch level counts are for float32 records")
        if levels is not None:
            lv = np.asarray(levels, dtype=np.int64)
            if np.any(lv < 0) or np.any(lv > self.g.levels):
                raise ValueError("threshold level counts must lie in [0, L]")
        self.levels_patch = None if levels is None else np.asarray(levels, dtype=np.int64).copy()
        self._rebuild_thresholds()

    # -- compression of tiles ------------------------------------------------
    def compress_tiles(self, tiles: np.ndarray) -> np.ndarray:
        """Forward transform, hard threshold and, for a narrow value format,
        the stored (quantised) representation of the details."""
        c = forward_2d(tiles.astype(self.dtype), self.g.levels, self.g.wavelet)
        return self._store_form(hard_threshold(c, self.thr))

    def _store_form(self, c: np.ndarray) -> np.ndarray:
        self.kept = c != 0
        self.raw = c              # thresholded, before any quantisation
        if self.values == "f32":
            return c
        from .lbmz_precision import quantize_tiles
        return quantize_tiles(c, self.g.levels, self.values, self.thr)

    def decompress_tiles(self, coef: np.ndarray | None = None) -> np.ndarray:
        c = self.coef if coef is None else coef
        return inverse_2d(c, self.g.levels, self.g.wavelet)

    # -- state ---------------------------------------------------------------
    def set_grid(self, grid: np.ndarray):
        """Compress a global state ``[m, n, n]``."""
        self.coef = self.compress_tiles(extract_tiles(np.asarray(grid, dtype=self.dtype), self.g))
        self.steps = 0

    def set_patch_eps(self, eps=None):
        """One threshold constant per patch (the learned control), or None for the single eps."""
        if self.values != "f32" and eps is not None:
            raise ValueError("per-patch thresholds are for float32 records")
        self.eps_patch = None if eps is None else np.asarray(eps, dtype=np.float64).copy()
        self._rebuild_thresholds()

    def set_coefficients(self, coef: np.ndarray, threshold: bool = True):
        c = np.asarray(coef, dtype=self.dtype)
        self.coef = self._store_form(hard_threshold(c, self.thr) if threshold else c.copy())

    def grid(self) -> np.ndarray:
        """Decompressed global state ``[m, n, n]`` (owned nodes of every tile)."""
        return assemble_grid(self.decompress_tiles(), self.g)

    # -- the patch loop --------------------------------------------------------
    def step(self, n: int = 1):
        for _ in range(n):
            lossy = self.decompress_tiles()
            padded = gather_ghosts(lossy, self.g)
            new_tiles = self.scheme.update(padded).astype(self.dtype)
            self.coef = self.compress_tiles(new_tiles)
            self.steps += 1

    # -- measurements ----------------------------------------------------------
    def store(self):
        if self.values != "f32":
            from .lbmz_precision import encode_store_q
            return encode_store_q(self.raw, self.g.levels, self.values, self.thr)
        return encode_store(self.coef)

    def nnz(self) -> np.ndarray:
        """Per (patch, field): stored coefficients (float32 records) or kept
        details (narrow records, whose samples are always stored)."""
        k = self.kept.reshape(self.kept.shape[0], self.kept.shape[1], -1)
        if self.values == "f32":
            return np.count_nonzero(k, axis=-1)
        from .lbmz_precision import subband_table
        det = subband_table(self.g.s, self.g.levels).reshape(-1) != 0
        return np.count_nonzero(k & det, axis=-1)

    def store_bytes(self) -> int:
        ncoef = self.g.s * self.g.s
        if self.values != "f32":
            from .lbmz_precision import store_bytes_q
            return store_bytes_q(self.raw.astype(np.float32), self.g.levels, self.values, self.thr)
        tot = 0
        for v in self.nnz().reshape(-1):
            tot += record_layout(int(v), ncoef, self.dtype.itemsize)[3]
        return tot + self.coef.shape[0] * self.coef.shape[1] * 8

    def dense_bytes(self) -> int:
        return self.g.n * self.g.n * self.coef.shape[1] * self.dtype.itemsize

    def ratio(self) -> float:
        return self.dense_bytes() / self.store_bytes()

    def field_totals(self) -> np.ndarray:
        """Per-field trapezoid-weighted sums of the lossy state, in float64."""
        lossy = self.decompress_tiles().astype(np.float64)
        w = tile_weights(self.g)
        return (lossy * w).sum(axis=(0, 2, 3))


def whole_grid_step(run: CompressedRun):
    """The paper's protocol (Section 3.1.3): decompress everything, step, recompress.

    All patches are rebuilt into one global grid, the ghost ring comes from the
    periodic grid itself, the scheme runs on the whole grid, and the result is
    cut back into tiles and compressed.  Used to check the patch loop.
    """
    grid = run.grid()
    new_grid = dense_step(grid, run.scheme).astype(run.dtype)
    run.coef = run.compress_tiles(extract_tiles(new_grid, run.g))
    run.steps += 1


def l2_errors(sim: np.ndarray, ref: np.ndarray, cell_area: float):
    """Error measures of a state against a reference.

    Returns ``(paper_l2, rms, rel_l2, linf)``: ``paper_l2`` is equation
    "L2_error" (cell area times the sum of squared differences, no root).
    """
    d = (np.asarray(sim, dtype=np.float64) - np.asarray(ref, dtype=np.float64))
    paper = cell_area * float(np.sum(d * d))
    rms = math.sqrt(float(np.mean(d * d)))
    nref = math.sqrt(float(np.sum(np.asarray(ref, dtype=np.float64) ** 2)))
    rel = math.sqrt(float(np.sum(d * d))) / nref if nref > 0 else float("nan")
    return paper, rms, rel, float(np.max(np.abs(d)))
