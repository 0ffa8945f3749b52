"""Pins of the oracle's compressed-Euler Rusanov scheme (the precision workload).

A hand-computed flux, the flux's consistency, exact conservation, the
symmetries of the equations (rotation by 90 degrees, mirror), a uniform state
as a fixed point and a contact discontinuity at rest keeping its pressure.
"""
import numpy as np
import pytest

from oracle import lbmz_oracle as O
from synth import riemann_four_quadrants

G = 1.4


def test_physical_flux_by_hand():
    # rho = 1, u = 2, v = 3, p = 4: E = 4 / 0.4 + 13 / 2 = 16.5
    w = O.euler_conserved(1.0, 2.0, 3.0, 4.0, G)
    assert np.allclose(w, [1.0, 2.0, 3.0, 16.5])
    f, un, c = O.euler_physical_flux(w, (1, 0), G)
    assert np.allclose(f, [2.0, 2.0 * 2.0 + 4.0, 3.0 * 2.0, (16.5 + 4.0) * 2.0])
    f, un, c = O.euler_physical_flux(w, (0, -1), G)
    assert np.allclose(f, [-3.0, -6.0, -9.0 - 4.0, -(16.5 + 4.0) * 3.0])
    assert np.isclose(c, np.sqrt(1.4 * 4.0))


def test_rusanov_consistency_and_antisymmetry():
    rng = np.random.default_rng(0)
    wl = O.euler_conserved(rng.uniform(0.5, 2, 50), rng.normal(size=50), rng.normal(size=50),
                           rng.uniform(0.5, 2, 50), G)
    wr = O.euler_conserved(rng.uniform(0.5, 2, 50), rng.normal(size=50), rng.normal(size=50),
                           rng.uniform(0.5, 2, 50), G)
    for nrm in O.NORMALS:
        f, _, _ = O.euler_physical_flux(wl, nrm, G)
        assert np.allclose(O.rusanov_flux(wl, wl, nrm, G), f)
        # the flux out of a cell through a face is the flux into its neighbour
        opp = (-nrm[0], -nrm[1])
        assert np.allclose(O.rusanov_flux(wl, wr, nrm, G), -O.rusanov_flux(wr, wl, opp, G))


def _step(w, dt_over_h=0.2):
    return O.euler_rusanov_update(O.periodic_pad(w), dt_over_h, G)


def _state(n=32, seed=1):
    w, _ = riemann_four_quadrants(n, seed=seed, gamma=G)
    rng = np.random.default_rng(seed)
    w[1] += 0.1 * rng.normal(size=(n, n)) * w[0]
    w[2] += 0.1 * rng.normal(size=(n, n)) * w[0]
    w[3] += 0.5 * (w[1] ** 2 + w[2] ** 2) / w[0]
    return w


def test_conservation_of_all_fields():
    w = _state()
    w1 = w
    for _ in range(5):
        w1 = _step(w1)
    assert np.allclose(w1.sum(axis=(1, 2)), w.sum(axis=(1, 2)), rtol=1e-13, atol=1e-12)


def test_rotation_by_90_degrees_commutes_with_the_step():
    # rotating the plane by +90 degrees maps (x, y) -> (-y, x) and (u, v) -> (-v, u)
    w = _state(seed=2)

    def rot(s):
        r = np.rot90(s, k=1, axes=(2, 1)).copy()   # array [y, x]: new[y, x] = old[x, -y]
        return np.stack([r[0], -r[2], r[1], r[3]])

    a = rot(_step(w))
    b = _step(rot(w))
    assert np.allclose(a, b, rtol=1e-13, atol=1e-13)


def test_mirror_commutes_with_the_step():
    w = _state(seed=3)

    def mir(s):
        m = s[:, :, ::-1].copy()
        m[1] = -m[1]
        return m

    assert np.allclose(mir(_step(w)), _step(mir(w)), rtol=1e-13, atol=1e-13)


def test_uniform_state_is_a_fixed_point():
    w = np.broadcast_to(O.euler_conserved(0.7, 0.3, -0.2, 1.1, G)[:, None, None], (4, 16, 16)).copy()
    assert np.allclose(_step(w), w, rtol=1e-15, atol=1e-15)


def test_contact_at_rest_keeps_uniform_pressure():
    n = 16
    rho = np.where(np.arange(n)[None, :] < n // 2, 1.0, 0.125) * np.ones((n, n))
    w = O.euler_conserved(rho, 0.0, 0.0, 1.0, G)
    w1 = _step(w)
    u = w1[1] / w1[0]
    p = (G - 1) * (w1[3] - 0.5 * (w1[1] ** 2 + w1[2] ** 2) / w1[0])
    assert np.allclose(p, 1.0, atol=1e-14) and np.allclose(u, 0.0, atol=1e-14)
    assert not np.allclose(w1[0], w[0])      # the density itself is smeared


def test_four_quadrant_generator_recipe():
    w, states = riemann_four_quadrants(8, seed=5)
    assert all(0.1 <= r <= 1.5 and 0.1 <= p <= 1.5 for r, p in states)
    assert np.allclose(w[0, 7, 7], states[0][0]) and np.allclose(w[0, 7, 0], states[1][0])
    assert np.allclose(w[0, 0, 0], states[2][0]) and np.allclose(w[0, 0, 7], states[3][0])
    assert np.all(w[1] == 0) and np.all(w[2] == 0)
    assert np.allclose(w[3, 0, 0], states[2][1] / 0.4)


@pytest.mark.parametrize("wavelet,p,levels", [("bl53", 32, 4), ("haar", 16, 3)])
def test_compressed_run_at_eps0_is_the_uncompressed_run(wavelet, p, levels):
    n = 64
    w, states = riemann_four_quadrants(n, seed=4)
    smax = 2.0 * max(np.sqrt(G * pp / r) for r, pp in states)
    sch = O.Scheme("euler_rusanov", vel=(smax, 0.0), cfl=0.4, gamma=G)
    run = O.CompressedRun(O.Geometry(n, p, wavelet, levels), sch, 0.0)
    run.set_grid(w)
    plain = w.copy()
    for _ in range(5):
        run.step(1)
        plain = O.dense_step(plain, sch)
    assert np.max(np.abs(run.grid() - plain)) <= 1e-12
    assert np.allclose(run.field_totals(), w.sum(axis=(1, 2)), rtol=1e-12)
