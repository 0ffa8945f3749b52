"""GPU parity of the compressible-Euler Rusanov path (the precision workload's scheme).

The uncompressed reference kernel and the compressed patch loop at eps = 0
both reproduce the oracle's plain scheme; one compressed step from a common
state matches the oracle's; the four conserved totals stay constant; the
narrow value formats keep the mass exactly and shrink the store.
"""
import sys

import numpy as np
import pytest

from oracle import lbmz_oracle as O
from oracle import lbmz_precision as Q
from synth import riemann_four_quadrants

from gpu_helpers import require_gpu, torch  # noqa: F401

pytestmark = pytest.mark.gpu

G = 1.4
CFL = 0.4


def _say(*args):
    print("[case]", *args, flush=True)
    sys.stdout.flush()


@pytest.fixture(autouse=True)
def _gpu():
    require_gpu()


def _problem(n, seed=0):
    w, states = riemann_four_quadrants(n, seed=seed, gamma=G)
    smax = 2.0 * max(np.sqrt(G * p / r) for r, p in states)
    return w, smax


def _ctx(n, p, wavelet, levels, eps, smax, values="f32", reference=False):
    from paper_2302_09883_amd import Context
    return Context(n, scheme="euler_rusanov", dtype="f32", p=p, wavelet=wavelet, levels=levels, eps=eps,
                   vel=(smax, 0.0), cfl=CFL, gamma=G, values=values, reference=reference)


def _set(ctx, w):
    for f in range(4):
        ctx.set_field(f, w[f].astype(np.float32))


@pytest.mark.parametrize("p,wavelet,levels", [(64, "bl53", 5), (32, "haar", 5), (32, "bl53", 3)])
def test_eps0_equals_reference_and_oracle(p, wavelet, levels):
    n, steps = 128, 20
    _say("euler eps0", p, wavelet, levels)
    w, smax = _problem(n)
    ref = _ctx(n, p, wavelet, levels, 0.0, smax, reference=True)
    _set(ref, w)
    ref.step(steps)
    cmp = _ctx(n, p, wavelet, levels, 0.0, smax)
    _set(cmp, w)
    cmp.step(steps)
    sch = O.Scheme("euler_rusanov", vel=(smax, 0.0), cfl=CFL, gamma=G)
    plain = w.copy()
    for _ in range(steps):
        plain = O.dense_step(plain, sch)
    a, b = ref.fields().astype(np.float64), cmp.fields().astype(np.float64)
    for f in range(4):
        scale = np.max(np.abs(plain[f])) + 1e-30
        assert np.max(np.abs(a[f] - plain[f])) <= 2e-5 * max(scale, 1.0), f
        assert np.max(np.abs(b[f] - plain[f])) <= 2e-5 * max(scale, 1.0), f


@pytest.mark.parametrize("eps", [1e-4, 1e-3])
def test_one_step_from_common_state(eps):
    n, p, levels = 128, 64, 5
    _say("euler one-step", eps)
    w, smax = _problem(n, seed=1)
    sch = O.Scheme("euler_rusanov", vel=(smax, 0.0), cfl=CFL, gamma=G)
    twin = O.CompressedRun(O.Geometry(n, p, O.BL53, levels), sch, eps, O.RULE_CAPPED, np.float32)
    twin.set_grid(w)
    twin.step(3)
    table, pool = O.encode_store(twin.coef)
    ctx = _ctx(n, p, "bl53", levels, eps, smax)
    ctx.put_store(table, pool)
    ctx.step(1)
    twin.step(1)
    from gpu_helpers import decode_records
    t2, p2 = ctx.store()
    got = decode_records(t2, p2, twin.g.s, np.float32)
    want = twin.coef
    u = np.finfo(np.float32).eps
    for f in range(4):
        scale = float(np.max(np.abs(twin.grid()[f]))) + 1.0
        delta = 512 * u * scale
        d = np.abs(got[:, f].astype(np.float64) - want[:, f])
        flip = (got[:, f] != 0) != (want[:, f] != 0)
        near = np.abs(np.abs(np.where(got[:, f] != 0, got[:, f], want[:, f])) - twin.thr) <= delta
        assert np.all(near[flip]), (f, int(flip.sum()))
        assert np.max(np.where(flip, 0.0, d)) <= delta, f


def _run_totals(values, seed, rho_range=(0.1, 1.5), p_range=(0.1, 1.5), n=256, steps=50):
    p, levels, eps = 64, 5, 1e-4
    w, states = riemann_four_quadrants(n, seed=seed, gamma=G, rho_range=rho_range, p_range=p_range)
    smax = 2.0 * max(np.sqrt(G * pp / r) for r, pp in states)
    ctx = _ctx(n, p, "bl53", levels, eps, smax, values=values)
    _set(ctx, w)
    t0 = np.array(ctx.stats()["totals"])
    ctx.step(steps)
    st = ctx.stats()
    t1 = np.array(st["totals"])
    ref = np.abs(w).sum(axis=(1, 2))
    # every conserved field (mass, both momenta, energy) is kept to float32 round-off
    assert np.all(np.abs(t1 - t0) <= 2e-6 * ref + 1e-3), (t0, t1)
    fields = ctx.fields()
    assert np.all(np.isfinite(fields)) and np.all(fields[0] > 0)
    rel = None
    if values != "f32":
        base = _ctx(n, p, "bl53", levels, eps, smax)
        _set(base, w)
        base.step(steps)
        b = base.fields().astype(np.float64)
        rel = np.linalg.norm(fields - b) / np.linalg.norm(b)
        print("[case] euler", values, "rel_l2 vs float32 records", rel, "store", st["store_bytes"],
              base.stats()["store_bytes"])
    return rel


@pytest.mark.parametrize("values", ["f32", "f16"])
def test_conserved_totals_and_value_formats(values):
    _say("euler totals", values)
    rel = _run_totals(values, seed=2)
    if values == "f16":
        # binary16 keeps 11 significant bits of every detail; at the shocks the
        # details are of the order of the field itself
        assert rel <= 1e-3


def test_e4m3_on_weak_shocks():
    _say("euler e4m3 weak")
    rel = _run_totals("e4m3", seed=2, rho_range=(0.9, 1.1), p_range=(0.9, 1.1))
    assert rel <= 2e-2


def test_e4m3_on_strong_shocks_stops_cleanly_or_runs():
    # three mantissa bits on shock-sized details can undershoot the density
    # or pressure below zero; the library must then stop at the last good step
    from paper_2302_09883_amd import LbmzError
    _say("euler e4m3 strong")
    n, p, levels, eps = 256, 64, 5, 1e-4
    w, states = riemann_four_quadrants(n, seed=2, gamma=G)
    smax = 2.0 * max(np.sqrt(G * pp / r) for r, pp in states)
    ctx = _ctx(n, p, "bl53", levels, eps, smax, values="e4m3")
    _set(ctx, w)
    try:
        ctx.step(50)
    except LbmzError as e:
        assert e.code == -5                     # LBMZ_ENAN
        st = ctx.stats()
        assert 0 <= st["steps"] < 50
        f = ctx.fields()
        assert np.all(np.isfinite(f))


def test_bounded_e4m3_runs_the_strong_shocks():
    """The bounded E4M3 format keeps E4M3 codes only where their rounding
    stays within half of each subband's threshold: the shock records go to
    binary16, and the run that plain E4M3 cannot finish completes."""
    _say("euler e4m3b strong")
    rel = _run_totals("e4m3b", seed=2)
    assert rel <= 2e-3


def test_bounded_e4m3_full_precision_workload():
    """The precision workload at its size and length: 4096^2, 64^2 patches,
    BL5/3 L = 5, eps = 1e-4, four-quadrant shocks, 500 steps, bounded E4M3
    records: no non-finite stop, every conserved total kept to float32
    round-off, positive density."""
    n, p, levels, eps, steps = 4096, 64, 5, 1e-4, 500
    _say("euler e4m3b 4096^2 x 500")
    w, states = riemann_four_quadrants(n, seed=0, gamma=G)
    smax = 2.0 * max(np.sqrt(G * pp / r) for r, pp in states)
    ctx = _ctx(n, p, "bl53", levels, eps, smax, values="e4m3b")
    _set(ctx, w)
    t0 = np.array(ctx.stats()["totals"])
    ctx.step(steps)
    st = ctx.stats()
    t1 = np.array(st["totals"])
    ref = np.abs(w).sum(axis=(1, 2))
    assert st["steps"] == steps
    assert np.all(np.abs(t1 - t0) <= 2e-6 * ref + 1e-2), (t0, t1)
    rho = ctx.decompress_field(0)
    assert np.all(np.isfinite(rho)) and float(rho.min()) > 0
    print(f"[case] euler e4m3b 4096^2: ratio {st['ratio']:.1f}, mask/list records "
          f"{st['mask_records']}/{st['list_records']}", flush=True)


def test_errors_against_the_fp64_oracle():
    """Every storage format's error against the float64 oracle, on a grid the
    oracle steps in seconds: the precision workload's geometry (64^2 patches,
    BL5/3 L = 5, capped eps = 1e-4, four-quadrant shocks) on 256^2 for 100
    steps.  References: the oracle's uncompressed scheme and its compressed
    patch loop, both in float64.  The float32-record GPU run must track the
    float64 compressed run (its error against the plain scheme within 10 %);
    binary16 details add at most 10 % to that error, bounded E4M3 at most
    50 % (its codes are off by at most half a threshold)."""
    n, p, levels, eps, steps = 256, 64, 5, 1e-4, 100
    _say("euler errors vs fp64 oracle")
    w, smax = _problem(n, seed=0)
    sch = O.Scheme("euler_rusanov", vel=(smax, 0.0), cfl=CFL, gamma=G)
    plain = w.copy()
    for _ in range(steps):
        plain = O.dense_step(plain, sch)
    run64 = O.CompressedRun(O.Geometry(n, p, O.BL53, levels), sch, eps, O.RULE_CAPPED, np.float64)
    run64.set_grid(w)
    run64.step(steps)
    e64 = O.l2_errors(run64.grid(), plain, 1.0 / n ** 2)[2]
    errs = {}
    for values in ("f32", "f16", "e4m3b"):
        ctx = _ctx(n, p, "bl53", levels, eps, smax, values=values)
        _set(ctx, w)
        ctx.step(steps)
        got = ctx.fields().astype(np.float64)
        _, _, rel_plain, linf_plain = O.l2_errors(got, plain, 1.0 / n ** 2)
        rel_c64 = O.l2_errors(got, run64.grid(), 1.0 / n ** 2)[2]
        errs[values] = rel_plain
        print(f"[case] euler {values}: rel L2 vs fp64 plain {rel_plain:.3e} (Linf {linf_plain:.3e}), "
              f"vs fp64 compressed {rel_c64:.3e}; fp64 compressed vs plain {e64:.3e}; "
              f"ratio {ctx.stats()['ratio']:.1f}", flush=True)
    assert abs(errs["f32"] - e64) <= 0.1 * e64
    assert errs["f16"] <= 1.1 * errs["f32"]
    assert errs["e4m3b"] <= 1.5 * errs["f32"]
