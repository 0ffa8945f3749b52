"""Pins of the oracle's uncompressed schemes (the plain definition the method must reduce to).

Finite volumes (Section 1 and Section 3.1.2): with velocity (1, 0.5) and
CFL 0.5 the upwind update is the convex combination
0.25 W + 0.5 W_{i-1,j} + 0.25 W_{i,j-1}; a unit impulse spreads into the
trinomial distribution; the total is conserved.

D2Q9 BGK (textbook): equilibrium moments, local conservation of the collision,
the equilibrium as a fixed point, streaming as a pure shift, and the viscous
decay rate of a Taylor-Green vortex with nu = (tau - 1/2) / 3.
"""
import math

import numpy as np
import pytest

from oracle import lbmz_oracle as O
from synth import random_signal, taylor_green_macroscopic


def test_fv_upwind_is_the_convex_combination():
    w = random_signal((1, 16, 16), seed=1)
    out = O.dense_step(w, O.Scheme("fv_upwind", vel=(1.0, 0.5), cfl=0.5))
    expect = 0.25 * w + 0.5 * np.roll(w, 1, axis=2) + 0.25 * np.roll(w, 1, axis=1)
    assert np.max(np.abs(out - expect)) <= 4e-16 * np.max(np.abs(w)) * 4


def test_fv_upwind_negative_velocity_takes_the_other_side():
    w = random_signal((1, 12, 12), seed=2)
    out = O.dense_step(w, O.Scheme("fv_upwind", vel=(-1.0, 0.0), cfl=1.0))
    assert np.allclose(out, np.roll(w, -1, axis=2), rtol=0, atol=1e-15)


def test_fv_impulse_gives_trinomial_weights():
    n, steps = 32, 12
    w = np.zeros((1, n, n))
    w[0, 0, 0] = 1.0
    sch = O.Scheme("fv_upwind", vel=(1.0, 0.5), cfl=0.5)
    for _ in range(steps):
        w = O.dense_step(w, sch)
    expect = np.zeros((n, n))
    for i in range(steps + 1):
        for j in range(steps + 1 - i):
            a = steps - i - j
            expect[j, i] = (math.factorial(steps) / (math.factorial(a) * math.factorial(i) *
                            math.factorial(j))) * 0.25 ** a * 0.5 ** i * 0.25 ** j
    assert np.array_equal(w[0], expect)      # dyadic arithmetic: exact


def test_fv_conserves_total_and_max_principle():
    w = random_signal((1, 20, 20), seed=4)
    sch = O.Scheme("fv_upwind", vel=(1.0, 0.5), cfl=0.5)
    tot0, lo, hi = w.sum(), w.min(), w.max()
    for _ in range(25):
        w = O.dense_step(w, sch)
        assert lo - 1e-15 <= w.min() and w.max() <= hi + 1e-15
    assert abs(w.sum() - tot0) <= 1e-12 * np.abs(w).sum()


def test_d2q9_equilibrium_moments():
    rng = np.random.default_rng(5)
    rho = 1.0 + 0.1 * rng.standard_normal((8, 8))
    ux = 0.05 * rng.standard_normal((8, 8))
    uy = 0.05 * rng.standard_normal((8, 8))
    f = O.d2q9_equilibrium(rho, ux, uy)
    c = O.D2Q9_C
    assert np.allclose(f.sum(axis=0), rho, rtol=0, atol=1e-15)
    assert np.allclose(sum(c[i, 0] * f[i] for i in range(9)), rho * ux, rtol=0, atol=1e-15)
    assert np.allclose(sum(c[i, 1] * f[i] for i in range(9)), rho * uy, rtol=0, atol=1e-15)
    pxx = sum(c[i, 0] * c[i, 0] * f[i] for i in range(9))
    pxy = sum(c[i, 0] * c[i, 1] * f[i] for i in range(9))
    assert np.allclose(pxx, rho * (ux * ux + 1.0 / 3.0), rtol=0, atol=1e-15)
    assert np.allclose(pxy, rho * ux * uy, rtol=0, atol=1e-15)


def test_d2q9_collision_conserves_and_keeps_equilibrium():
    rng = np.random.default_rng(6)
    f = 0.1 + 0.01 * rng.uniform(size=(9, 10, 10))
    out = O.dense_step(f, O.Scheme("d2q9_bgk", tau=0.6))
    # streaming is a permutation: global moments conserved by stream + collide
    c = O.D2Q9_C
    assert abs(out.sum() - f.sum()) <= 1e-13
    for a in (0, 1):
        assert abs(sum(c[i, a] * out[i].sum() for i in range(9)) -
                   sum(c[i, a] * f[i].sum() for i in range(9))) <= 1e-13
    # a uniform equilibrium is a fixed point
    feq = O.d2q9_equilibrium(np.full((6, 6), 1.1), np.full((6, 6), 0.03), np.full((6, 6), -0.02))
    assert np.allclose(O.dense_step(feq, O.Scheme("d2q9_bgk", tau=0.7)), feq, rtol=0, atol=2e-15)


def test_d2q9_streaming_is_a_shift():
    # with an enormous relaxation time the collision does nothing, so one step
    # is pure pull streaming: population i moves by +c_i, f_i(x) <- f_i(x - c_i)
    f = 1.0 + random_signal((9, 8, 8), seed=7)
    out = O.dense_step(f, O.Scheme("d2q9_bgk", tau=1e30))
    for i in range(9):
        cx, cy = int(O.D2Q9_C[i, 0]), int(O.D2Q9_C[i, 1])
        assert np.allclose(out[i], np.roll(f[i], shift=(cy, cx), axis=(0, 1)), rtol=1e-14, atol=0)


def test_d2q9_collision_relaxes_by_one_minus_one_over_tau():
    # a spatially uniform state does not stream; its distance to equilibrium
    # shrinks by the factor (1 - 1/tau) per step
    rng = np.random.default_rng(8)
    f = np.broadcast_to((0.1 + 0.02 * rng.uniform(size=9))[:, None, None], (9, 4, 4)).copy()
    tau = 0.6
    out = O.dense_step(f, O.Scheme("d2q9_bgk", tau=tau))
    rho, ux, uy = O.d2q9_moments(f)
    feq = O.d2q9_equilibrium(rho, ux, uy)
    assert np.allclose(out - feq, (1.0 - 1.0 / tau) * (f - feq), rtol=0, atol=1e-15)


def test_d2q9_taylor_green_viscous_decay():
    n, tau, steps = 32, 0.8, 200
    rho, ux, uy = taylor_green_macroscopic(n, u0=0.01)
    f = O.d2q9_equilibrium(rho, ux, uy)
    sch = O.Scheme("d2q9_bgk", tau=tau)
    for _ in range(steps):
        f = O.dense_step(f, sch)
    _, ux2, uy2 = O.d2q9_moments(f)
    nu = (tau - 0.5) / 3.0
    k = 2.0 * math.pi / n
    decay = math.exp(-2.0 * nu * k * k * steps)
    ratio = np.sqrt((ux2 ** 2 + uy2 ** 2).sum() / (ux ** 2 + uy ** 2).sum())
    assert abs(ratio / decay - 1.0) < 0.02
