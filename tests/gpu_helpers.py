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
    from paper_2302_09883_amd import decode_records
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
