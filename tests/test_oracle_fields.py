"""The oracle's field solver and current deposition against what fixes them.

Yee advance (FP32, periodic): a standing wave of one Fourier mode follows
the closed-form solution of the discrete scheme, E(n) = E(0) cos(n theta)
with cos(theta) = 1 - (kappa dt)^2 / 2, kappa = (2/d) sin(k d / 2) (the Yee
dispersion relation), for every direction and polarisation, and differs
from the continuum solution cos(k n dt); div B is kept (div curl = 0).
Deposition (Esirkepov, TSC): the continuity equation holds node by node,
the summed current is Q v, a particle at rest or moving along one axis
deposits nothing across it, and with the solver div E - rho stays constant
(Gauss's law).
"""
import math

import numpy as np
import pytest

from oracle import oracle as O


def _mode_grid(shape, spacing, direction, pol, m):
    """Standing wave: E_pol = cos(k x_dir) on its own staggered positions, B = 0."""
    g = np.zeros((6,) + tuple(shape), np.float32)
    n = shape[direction]
    k = 2.0 * math.pi * m / (n * spacing[direction])
    # staggering of E components: E_c sits half a cell along c
    idx = np.arange(n, dtype=np.float64)
    pos = (idx + (0.5 if pol == direction else 0.0)) * spacing[direction]
    prof = np.cos(k * pos)
    sl = [None, None, None]
    sl[direction] = slice(None)
    g[pol] = np.broadcast_to(prof[tuple(sl)], shape).astype(np.float32)
    return g, k


@pytest.mark.parametrize("direction,pol", [(0, 1), (0, 2), (1, 2), (1, 0), (2, 0), (2, 1)])
def test_yee_standing_wave_follows_discrete_dispersion(direction, pol):
    shape = [4, 4, 4]
    shape[direction] = 16
    spacing = (0.4, 0.5, 0.3)
    dt = 0.2
    m = 3                                          # 16/3 cells per wavelength: strong dispersion
    g, k = _mode_grid(shape, spacing, direction, pol, m)
    e0 = g[pol].astype(np.float64).copy()
    steps = 150
    O.yee_advance(g, None, shape, spacing, dt, steps)
    d = spacing[direction]
    kappa = 2.0 / d * math.sin(k * d / 2.0)
    theta = math.acos(1.0 - (kappa * dt) ** 2 / 2.0)
    want = e0 * math.cos(steps * theta)
    assert np.max(np.abs(g[pol] - want)) < 2e-5
    # not the continuum solution
    assert np.max(np.abs(e0 * math.cos(k * steps * dt) - want)) > 0.1
    # the other E components stay zero
    for c in range(3):
        if c != pol:
            assert np.max(np.abs(g[c])) < 1e-6


def _div_b(g, spacing):
    Bx, By, Bz = (g[3 + c].astype(np.float64) for c in range(3))
    return ((np.roll(Bx, -1, 0) - Bx) / spacing[0] + (np.roll(By, -1, 1) - By) / spacing[1]
            + (np.roll(Bz, -1, 2) - Bz) / spacing[2])


def _div_e(g, spacing):
    Ex, Ey, Ez = (g[c].astype(np.float64) for c in range(3))
    return ((Ex - np.roll(Ex, 1, 0)) / spacing[0] + (Ey - np.roll(Ey, 1, 1)) / spacing[1]
            + (Ez - np.roll(Ez, 1, 2)) / spacing[2])


def test_yee_keeps_div_b():
    r = np.random.default_rng(3)
    shape, spacing = (6, 5, 7), (0.5, 0.4, 0.45)
    g = np.zeros((6,) + shape, np.float32)
    g[:3] = r.normal(size=(3,) + shape)
    O.yee_advance(g, None, shape, spacing, 0.15, 20)
    assert np.max(np.abs(g[3:])) > 0.5
    assert np.max(np.abs(_div_b(g, spacing))) < 1e-5


SHAPE, SPACING, ORIGIN = (8, 7, 6), (0.5, 0.4, 0.45), (-1.0, 0.3, 2.0)


def _moving_particles(n, seed, max_cells=0.9):
    r = np.random.default_rng(seed)
    lo = np.array(ORIGIN)
    ext = np.array(SHAPE) * np.array(SPACING)
    x0 = lo + r.uniform(0, 1, (n, 3)) * ext
    step = r.uniform(-max_cells, max_cells, (n, 3)) * np.array(SPACING)
    x1 = x0 + step
    p = {"x": x1[:, 0].copy(), "y": x1[:, 1].copy(), "z": x1[:, 2].copy(), "w": r.uniform(0.5, 2.0, n),
         "ux": r.normal(size=n), "uy": r.normal(size=n), "uz": r.normal(size=n), "tau": np.ones(n)}
    return p, x0


def _div_j(J, spacing):
    return ((J[0] - np.roll(J[0], 1, 0)) / spacing[0] + (J[1] - np.roll(J[1], 1, 1)) / spacing[1]
            + (J[2] - np.roll(J[2], 1, 2)) / spacing[2])


@pytest.mark.parametrize("q", [-1.0, 1.0])
def test_deposit_keeps_continuity(q):
    p, x0 = _moving_particles(300, 5)
    dt, js = 0.17, 0.3
    s_new = O.species_from(p)
    s_old = O.species_from(dict(p, x=x0[:, 0], y=x0[:, 1], z=x0[:, 2]))
    J, sk = O.deposit_current(s_new, (x0[:, 0], x0[:, 1], x0[:, 2]), 0, q, js, dt, SHAPE, SPACING, ORIGIN)
    assert sk == 0
    r0 = O.deposit_charge(s_old, q, js, SHAPE, SPACING, ORIGIN)
    r1 = O.deposit_charge(s_new, q, js, SHAPE, SPACING, ORIGIN)
    res = (r1 - r0) / dt + _div_j(J, SPACING)
    assert np.max(np.abs(res)) < 1e-12 * max(np.max(np.abs(r1 - r0)) / dt, 1.0)
    assert np.max(np.abs(r1 - r0)) > 0.1
    # summed current = sum Q v
    Q = q * p["w"] * js
    for c, k in enumerate("xyz"):
        want = np.sum(Q * (p[k] - x0[:, c])) / dt
        assert J[c].sum() == pytest.approx(want, rel=1e-12, abs=1e-12)


def test_deposit_rest_and_axis_motion():
    p, x0 = _moving_particles(50, 6)
    # at rest: nothing
    rest = dict(p, x=x0[:, 0], y=x0[:, 1], z=x0[:, 2])
    J, _ = O.deposit_current(O.species_from(rest), (x0[:, 0], x0[:, 1], x0[:, 2]), 0, -1.0, 1.0, 0.1, SHAPE, SPACING,
                             ORIGIN)
    assert np.max(np.abs(J)) == 0.0
    # along x only: no J_y, J_z
    along = dict(p, y=x0[:, 1], z=x0[:, 2])
    J, _ = O.deposit_current(O.species_from(along), (x0[:, 0], x0[:, 1], x0[:, 2]), 0, -1.0, 1.0, 0.1, SHAPE, SPACING,
                             ORIGIN)
    assert np.max(np.abs(J[1])) == 0.0 and np.max(np.abs(J[2])) == 0.0 and np.max(np.abs(J[0])) > 0


def test_deposit_backtracks_created_particles_and_skips_long_moves():
    dt = 0.2
    r = np.random.default_rng(2)
    n = 40
    u = r.normal(size=(n, 3)) * 3.0
    gam = np.sqrt(1 + (u * u).sum(1))
    x1 = np.array(ORIGIN) + r.uniform(0.3, 0.7, (n, 3)) * np.array(SHAPE) * np.array(SPACING)
    x0 = x1 - dt * u / gam[:, None]
    p = {"x": x1[:, 0], "y": x1[:, 1], "z": x1[:, 2], "ux": u[:, 0], "uy": u[:, 1], "uz": u[:, 2],
         "w": np.ones(n), "tau": np.ones(n)}
    s = O.species_from(p)
    Jb, _ = O.deposit_current(s, None, 0, 1.0, 1.0, dt, SHAPE, SPACING, ORIGIN)
    Jo, _ = O.deposit_current(s, (x0[:, 0], x0[:, 1], x0[:, 2]), 0, 1.0, 1.0, dt, SHAPE, SPACING, ORIGIN)
    assert np.max(np.abs(Jb - Jo)) < 1e-12 * np.max(np.abs(Jo))
    # first > 0 deposits only the tail
    Jt, _ = O.deposit_current(s, (x0[10:, 0], x0[10:, 1], x0[10:, 2]), 10, 1.0, 1.0, dt, SHAPE, SPACING, ORIGIN)
    s2 = O.species_from({k: v[10:] for k, v in p.items()})
    Jt2, _ = O.deposit_current(s2, (x0[10:, 0], x0[10:, 1], x0[10:, 2]), 0, 1.0, 1.0, dt, SHAPE, SPACING, ORIGIN)
    assert np.array_equal(Jt, Jt2)
    far = dict(p, x=x0[:, 0] + 2.6 * SPACING[0])                  # the nearest node moves by 2 or 3
    _, sk = O.deposit_current(O.species_from(far), (x0[:, 0], x0[:, 1], x0[:, 2]), 0, 1.0, 1.0, dt, SHAPE, SPACING,
                              ORIGIN)
    assert sk == n


def test_gauss_law_kept_by_solver_and_deposition():
    """Particles move for several steps; E is advanced with their currents:
    div E - rho does not change (to FP32 rounding of the grid)."""
    r = np.random.default_rng(9)
    shape, spacing, origin = (10, 9, 8), (0.5, 0.5, 0.5), (0.0, 0.0, 0.0)
    dt, js, q = 0.2, 0.05, -1.0
    n = 400
    x = np.array(origin) + r.uniform(0, 1, (n, 3)) * np.array(shape) * np.array(spacing)
    v = r.normal(size=(n, 3)) * 0.5
    v /= np.maximum(1.0, np.linalg.norm(v, axis=1) / 0.9)[:, None]        # |v| < 0.9
    g = np.zeros((6,) + shape, np.float32)
    g[:3] = 0.1 * r.normal(size=(3,) + shape)
    base = {"w": r.uniform(0.5, 1.5, n), "ux": np.zeros(n), "uy": np.zeros(n), "uz": np.zeros(n), "tau": np.ones(n)}

    def sp(pos):
        return O.species_from(dict(base, x=pos[:, 0].copy(), y=pos[:, 1].copy(), z=pos[:, 2].copy()))
    gauss0 = _div_e(g, spacing) - O.deposit_charge(sp(x), q, js, shape, spacing, origin)
    for _ in range(6):
        x1 = x + dt * v
        J, sk = O.deposit_current(sp(x1), (x[:, 0], x[:, 1], x[:, 2]), 0, q, js, dt, shape, spacing, origin)
        assert sk == 0
        O.yee_advance(g, J.astype(np.float32), shape, spacing, dt)
        x = x1
    gauss1 = _div_e(g, spacing) - O.deposit_charge(sp(x), q, js, shape, spacing, origin)
    rho_scale = np.max(np.abs(O.deposit_charge(sp(x), q, js, shape, spacing, origin)))
    assert np.max(np.abs(gauss1 - gauss0)) < 2e-5 * max(rho_scale, np.max(np.abs(_div_e(g, spacing))))
    # and without the current term it would not hold
    g2 = g.copy()
    O.yee_advance(g2, None, shape, spacing, dt)
    x2 = x + dt * v
    gauss2 = _div_e(g2, spacing) - O.deposit_charge(sp(x2), q, js, shape, spacing, origin)
    assert np.max(np.abs(gauss2 - gauss0)) > 1e-3 * rho_scale
