"""Seeded initial fields for the two hot-path workloads and for unit tests.

Workloads (cell units, periodic unit square split into ``n`` cells per side):

* transport workload: eight Gaussian bumps plus one square step, the
  scalar initial field of the first-order upwind finite-volume run;
* lattice-Boltzmann workload: a double shear layer with a small sinusoidal
  transverse perturbation, given as macroscopic density and velocity (the
  populations are built from them by each side's own equilibrium code).

Every function draws its random numbers from ``numpy.random.default_rng(seed)``
in the order its docstring states, so the recipe is reproducible from the text.
"""
from __future__ import annotations

import math

import numpy as np


def fv_gaussians_and_step(n: int = 256, seed: int = 0, n_bumps: int = 8,
                          sigma_range=(5.0, 20.0), amp_range=(0.5, 1.0),
                          step_side: int = 64) -> np.ndarray:
    """Scalar field ``[n, n]`` (float64): Gaussian bumps plus a unit square step.

    Draw order: centres ``(n_bumps, 2)`` uniform in ``[0, n)`` (x then y),
    widths ``sigma`` uniform in ``sigma_range`` cells, amplitudes uniform in
    ``amp_range``, then the step's lower-left corner as two integers in
    ``[0, n)``.  Bump ``k`` is ``A_k exp(-r^2 / (2 sigma_k^2))`` with ``r`` the
    periodic minimum-image distance between the cell index and the centre.  The
    step adds 1 on a ``step_side`` x ``step_side`` block that wraps around.
    The background is 0.
    """
    rng = np.random.default_rng(seed)
    centres = rng.uniform(0.0, n, size=(n_bumps, 2))
    sigmas = rng.uniform(sigma_range[0], sigma_range[1], size=n_bumps)
    amps = rng.uniform(amp_range[0], amp_range[1], size=n_bumps)
    corner = rng.integers(0, n, size=2)

    idx = np.arange(n, dtype=np.float64)
    field = np.zeros((n, n), dtype=np.float64)
    for (cx, cy), sg, a in zip(centres, sigmas, amps):
        dx = idx - cx
        dx = dx - n * np.round(dx / n)
        dy = idx - cy
        dy = dy - n * np.round(dy / n)
        r2 = dy[:, None] ** 2 + dx[None, :] ** 2
        field += a * np.exp(-r2 / (2.0 * sg * sg))
    side = min(step_side, n)
    xs = (corner[0] + np.arange(side)) % n
    ys = (corner[1] + np.arange(side)) % n
    field[np.ix_(ys, xs)] += 1.0
    return field


def shear_layer_macroscopic(n: int = 2048, seed: int = 0, u0: float = 0.05,
                            kappa: float = 80.0, delta: float = 0.05):
    """Double shear layer: returns ``(rho, ux, uy)``, each ``[n, n]`` float64.

    Coordinates are cell centres ``x = (i + 1/2) / n``.  ``rho = 1``;
    ``ux = u0 tanh(kappa (y - 1/4))`` for ``y <= 1/2`` and
    ``u0 tanh(kappa (3/4 - y))`` above; ``uy = delta u0 sin(2 pi (x + phi))``
    with the phase ``phi`` the single uniform ``[0, 1)`` draw of the seed.
    ``u0`` is in lattice units (0.05 keeps the Mach number near 0.09).
    """
    rng = np.random.default_rng(seed)
    phi = rng.uniform(0.0, 1.0)
    c = (np.arange(n, dtype=np.float64) + 0.5) / n
    y = c[:, None]
    x = c[None, :]
    ux_col = np.where(c <= 0.5, u0 * np.tanh(kappa * (c - 0.25)),
                      u0 * np.tanh(kappa * (0.75 - c)))
    ux = np.broadcast_to(ux_col[:, None], (n, n)).copy()
    uy = np.broadcast_to(delta * u0 * np.sin(2.0 * math.pi * (x + phi)), (n, n)).copy()
    rho = np.ones((n, n), dtype=np.float64)
    del y
    return rho, ux, uy


def taylor_green_macroscopic(n: int, u0: float = 0.02, rho0: float = 1.0):
    """Periodic 2-D Taylor-Green vortex at t = 0 (no random draw).

    ``ux = -u0 cos(kx) sin(ky)``, ``uy = u0 sin(kx) cos(ky)`` with
    ``k = 2 pi / n`` on node coordinates ``x, y = i`` (lattice units), and the
    incompressible pressure folded into the density
    ``rho = rho0 - (3 rho0 u0^2 / 4)(cos 2kx + cos 2ky)`` (``c_s^2 = 1/3``).
    """
    k = 2.0 * math.pi / n
    i = np.arange(n, dtype=np.float64)
    x = i[None, :]
    y = i[:, None]
    ux = -u0 * np.cos(k * x) * np.sin(k * y)
    uy = u0 * np.sin(k * x) * np.cos(k * y)
    rho = rho0 - 0.75 * rho0 * u0 * u0 * (np.cos(2 * k * x) + np.cos(2 * k * y))
    return rho, ux, uy


def worked_example_field(n: int = 129) -> np.ndarray:
    """The discontinuous 2-D test function of the compression section, ``[n, n]``.

    ``f(x, y) = exp(x - y) sin(2 pi (x + y)) * step(y - x^2)`` with
    ``step(s) = 1`` for ``s >= 0`` and 2 otherwise, sampled on the nodes
    ``x_i = i / n``, ``i = 0 .. n-1`` (indexed ``[y, x]``).
    """
    c = np.arange(n, dtype=np.float64) / n
    x = c[None, :]
    y = c[:, None]
    step = np.where(y - x * x >= 0.0, 1.0, 2.0)
    return np.exp(x - y) * np.sin(2.0 * math.pi * (x + y)) * step


def random_signal(shape, seed: int = 0, dtype=np.float64) -> np.ndarray:
    """Standard-normal samples of the given shape and dtype."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal(size=shape).astype(dtype)


def random_coefficient_tiles(shape, seed: int = 0, dtype=np.float32,
                             zero_frac: float = 0.3, scale_spread: float = 6.0) -> np.ndarray:
    """Random coefficient-like values with exact zeros and a wide magnitude range.

    Draw order: magnitudes ``10**U(-scale_spread, 0)``, signs from a fair coin,
    then a Bernoulli(``zero_frac``) mask of exact zeros.  About 1% of the zeros
    are made negative zero, which must behave as zero.
    """
    rng = np.random.default_rng(seed)
    mag = 10.0 ** rng.uniform(-scale_spread, 0.0, size=shape)
    sign = np.where(rng.integers(0, 2, size=shape) == 0, -1.0, 1.0)
    zero = rng.uniform(0.0, 1.0, size=shape) < zero_frac
    negz = rng.uniform(0.0, 1.0, size=shape) < 0.01
    out = (sign * mag).astype(dtype)
    out[zero] = 0.0
    out[zero & negz] = -0.0
    return out


def transport_gaussian(n: int = 128, t: float = 0.0, vel=(0.9, 0.9), lo: float = -1.0,
                       hi: float = 1.0) -> np.ndarray:
    """The paper's transport test field ``[n, n]`` (float64) at time ``t``.

    ``f(x, y, t) = 1 + exp(-30 ((x - alpha t)^2 + (y - beta t)^2))`` sampled at
    the cell centres ``lo + (i + 1/2) h``, ``h = (hi - lo) / n``, of the
    periodic square ``[lo, hi)^2``; the displaced centre is taken modulo the
    period (minimum image).  ``t = 0`` is the initial state, ``t > 0`` the exact
    solution of the transport equation with speed ``vel`` (Section 3.2,
    transport simulation).  No random numbers.
    """
    side = hi - lo
    h = side / n
    c = lo + (np.arange(n, dtype=np.float64) + 0.5) * h

    def wrapped(x):
        return (x - lo) % side + lo if side > 0 else x

    cx = wrapped(np.float64(vel[0]) * t)
    cy = wrapped(np.float64(vel[1]) * t)
    dx = c - cx
    dx = dx - side * np.round(dx / side)
    dy = c - cy
    dy = dy - side * np.round(dy / side)
    return 1.0 + np.exp(-30.0 * (dy[:, None] ** 2 + dx[None, :] ** 2))


def riemann_four_quadrants(n: int = 4096, seed: int = 0, gamma: float = 1.4,
                           rho_range=(0.1, 1.5), p_range=(0.1, 1.5)):
    """Four-quadrant Riemann problem of the compressible Euler equations.

    Returns ``(W, states)``: the conserved fields ``W[4, n, n]`` (float64;
    density, x and y momentum, total energy ``p / (gamma - 1)``, the gas at
    rest) and the quadrant states ``[(rho, p)] * 4``.  Quadrant 1 is
    ``x >= 1/2, y >= 1/2``, then counter-clockwise (2: x < 1/2, y >= 1/2;
    3: x < 1/2, y < 1/2; 4: x >= 1/2, y < 1/2) with cell centres
    ``(i + 1/2) / n`` of the periodic unit square.  Draw order: the four
    densities uniform in ``rho_range``, then the four pressures uniform in
    ``p_range``.
    """
    rng = np.random.default_rng(seed)
    rho_q = rng.uniform(rho_range[0], rho_range[1], size=4)
    p_q = rng.uniform(p_range[0], p_range[1], size=4)
    c = (np.arange(n, dtype=np.float64) + 0.5) / n
    right = c[None, :] >= 0.5
    top = c[:, None] >= 0.5
    quad = np.where(top, np.where(right, 0, 1), np.where(right, 3, 2))
    rho = rho_q[quad]
    p = p_q[quad]
    w = np.zeros((4, n, n), dtype=np.float64)
    w[0] = rho
    w[3] = p / (gamma - 1.0)
    return w, [(float(rho_q[k]), float(p_q[k])) for k in range(4)]


def shear_with_vortices(n: int = 1024, seed: int = 0, u0: float = 0.05, kappa: float = 80.0,
                        delta: float = 0.05, n_vortices: int = 12, radius_range=(0.02, 0.06),
                        strength_range=(0.5, 1.0)):
    """Double shear layer plus seeded Gaussian vortices, as ``(rho, ux, uy)``.

    The shear layer is :func:`shear_layer_macroscopic` with the same seed.
    Then, from ``default_rng(seed + 7919)``: vortex centres ``(n_vortices, 2)``
    uniform in the unit square, core radii uniform in ``radius_range``, peak
    speeds uniform in ``strength_range`` times ``u0``, signs from a fair coin.
    Vortex ``k`` adds the velocity ``s_k r_k / r * exp(1/2 - r^2 / (2 r_k^2))
    * (r / r_k)`` in the azimuthal direction (a Gaussian vortex whose speed
    peaks at ``r = r_k`` with value ``s_k``), with the periodic minimum-image
    offset ``r`` from its centre.  Density stays 1.
    """
    rho, ux, uy = shear_layer_macroscopic(n, seed=seed, u0=u0, kappa=kappa, delta=delta)
    rng = np.random.default_rng(seed + 7919)
    centres = rng.uniform(0.0, 1.0, size=(n_vortices, 2))
    radii = rng.uniform(radius_range[0], radius_range[1], size=n_vortices)
    speeds = rng.uniform(strength_range[0], strength_range[1], size=n_vortices) * u0
    signs = np.where(rng.integers(0, 2, size=n_vortices) == 0, -1.0, 1.0)
    c = (np.arange(n, dtype=np.float64) + 0.5) / n
    for (cx, cy), rk, sk, sg in zip(centres, radii, speeds, signs):
        dx = c[None, :] - cx
        dx = dx - np.round(dx)
        dy = c[:, None] - cy
        dy = dy - np.round(dy)
        r2 = dx * dx + dy * dy
        amp = sg * sk * np.exp(0.5 - r2 / (2.0 * rk * rk)) / rk
        ux = ux - amp * dy
        uy = uy + amp * dx
    return rho, ux, uy


def taylor_green_jets_3d(n: int = 768, seed: int = 0, u0: float = 0.05, n_jets: int = 4,
                         width_range=(1.0 / 32.0, 1.0 / 16.0), dtype=np.float32):
    """Macroscopic ``(rho, ux, uy, uz)``, each ``[n, n, n]`` indexed ``[z, y, x]``,
    for the 3-D lattice-Boltzmann workload: a Taylor--Green vortex plus seeded jets.

    With ``x, y, z = 2 pi (i + 1/2) / n``: ``ux = u0 sin x cos y cos z``,
    ``uy = -u0 cos x sin y cos z``, ``uz = 0``, ``rho = 1``.  Then ``n_jets``
    Gaussian jets are added; draw order: centres ``(n_jets, 3)`` uniform in
    ``[0, 1)`` (x, y, z), widths uniform in ``width_range`` (fractions of the
    box), directions ``(n_jets, 3)`` standard normal (normalised).  Jet ``k``
    adds ``u0 exp(-r^2 / (2 w_k^2)) d_k`` with ``r`` the periodic
    minimum-image distance to its centre.  The peak speed stays below
    ``(1 + n_jets) u0``; at ``u0 = 0.05`` the Mach number in lattice units is
    at most about 0.4 where jets overlap and below 0.2 elsewhere.
    """
    rng = np.random.default_rng(seed)
    centres = rng.uniform(0.0, 1.0, size=(n_jets, 3))
    widths = rng.uniform(width_range[0], width_range[1], size=n_jets)
    dirs = rng.standard_normal(size=(n_jets, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    c = (np.arange(n, dtype=np.float64) + 0.5) / n
    ph = 2.0 * math.pi * c
    sx, cx = np.sin(ph)[None, None, :], np.cos(ph)[None, None, :]
    sy, cy = np.sin(ph)[None, :, None], np.cos(ph)[None, :, None]
    cz = np.cos(ph)[:, None, None]
    ux = np.broadcast_to(u0 * sx * cy * cz, (n, n, n)).astype(np.float64)
    uy = np.broadcast_to(-u0 * cx * sy * cz, (n, n, n)).astype(np.float64)
    uz = np.zeros((n, n, n))
    for k in range(n_jets):
        d = [np.abs(c - centres[k, a]) for a in range(3)]
        d = [np.minimum(v, 1.0 - v) for v in d]
        g = [np.exp(-(v * v) / (2.0 * widths[k] ** 2)) for v in d]
        prof = u0 * g[2][:, None, None] * g[1][None, :, None] * g[0][None, None, :]
        ux += prof * dirs[k, 0]
        uy += prof * dirs[k, 1]
        uz += prof * dirs[k, 2]
    rho = np.ones((n, n, n))
    return tuple(a.astype(dtype) for a in (rho, ux, uy, uz))
