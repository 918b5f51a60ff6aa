"""Pins of the oracle's particle step (CPU only).

Expected values come from closed forms (Boris rotation, plane-wave invariants),
an independent ODE solve (Sokolov drag), Poisson statistics (optical-depth
Monte Carlo), exact conservation laws at events, numpy's Philox and the
numbers the paper prints for its constant-field test.
"""
import json
import math
import os

import numpy as np
import pytest
from scipy.integrate import solve_ivp

from oracle import oracle as O

HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = json.load(open(os.path.join(HERE, "golden", "paper_values.json")))
LAM = 0.8e-6
U = O.units(LAM)


# ---------------------------------------------------------------- Philox ----
def test_philox_known_answer():
    # Random123 known-answer vector for philox4x64-10, counter 0, key 0
    assert O.philox([0, 0, 0, 0], [0, 0]) == [0x16554D9ECA36314C, 0xDB20FE9D672D0FDC,
                                              0xD7E772CEE186176B, 0x7E68B68AEC7BA23B]


def test_philox_matches_numpy():
    rng = np.random.default_rng(3)
    for _ in range(200):
        ctr = [int(v) for v in rng.integers(0, 2**64, 4, dtype=np.uint64)]
        key = [int(v) for v in rng.integers(0, 2**64, 2, dtype=np.uint64)]
        # numpy's Philox increments its counter before each block
        c = sum(v << (64 * i) for i, v in enumerate(ctr))
        bg = np.random.Philox(counter=(c - 1) % 2**256, key=key[0] | (key[1] << 64))
        assert [int(v) for v in bg.random_raw(4)] == O.philox(ctr, key)


def test_uniform_open_closed():
    assert O.u01(0) == 2.0 ** -53
    assert O.u01(2**64 - 1) == 1.0


# ------------------------------------------------------------------- chi ----
def _boost(beta, E, B, u):
    """Lorentz boost of fields and of the four-velocity by velocity beta (c = 1)."""
    beta = np.asarray(beta, float)
    b2 = beta @ beta
    G = 1 / math.sqrt(1 - b2)
    k = G * G / (G + 1)
    E2 = G * (E + np.cross(beta, B)) - k * beta * (beta @ E)
    B2 = G * (B - np.cross(beta, E)) - k * beta * (beta @ B)
    g = math.sqrt(1 + u @ u)
    g2 = G * (g - beta @ u)
    u2 = u + ((G - 1) / b2) * (beta @ u) * beta - G * g * beta
    return E2, B2, u2, g2


def test_chi_lorentz_invariant():
    rng = np.random.default_rng(11)
    for _ in range(200):
        E, B = rng.normal(size=3) * 50, rng.normal(size=3) * 50
        u = rng.normal(size=3) * rng.uniform(1, 3000)
        g = math.sqrt(1 + u @ u)
        c0 = O.chi_lepton(U, u, g, E, B)
        d = rng.normal(size=3)
        beta = d / np.linalg.norm(d) * rng.uniform(0.0, 0.99)
        E2, B2, u2, g2 = _boost(beta, E, B, u)
        assert O.chi_lepton(U, u2, g2, E2, B2) == pytest.approx(c0, rel=1e-9)
        k = rng.normal(size=3) * 500
        kk = np.linalg.norm(k)
        # photon: boost the null four-vector (|k|, k)
        G = 1 / math.sqrt(1 - beta @ beta)
        kk2 = G * (kk - beta @ k)
        k2 = k + ((G - 1) / (beta @ beta)) * (beta @ k) * beta - G * kk * beta
        assert np.linalg.norm(k2) == pytest.approx(kk2, rel=1e-9)
        assert O.chi_photon(U, k2, E2, B2) == pytest.approx(O.chi_photon(U, k, E, B), rel=1e-9)


def test_chi_special_cases():
    # photon along B with no E: chi_gamma = 0; lepton with E parallel to u: chi_e = |E|/E_s
    assert O.chi_photon(U, [0, 0, 300.0], [0, 0, 0], [0, 0, 17.0]) == 0.0
    u = np.array([0.0, 0.0, 1234.5])
    assert O.chi_lepton(U, u, math.sqrt(1 + u @ u), [0, 0, 99.0], [0, 0, 0]) == pytest.approx(
        99.0 / U["Es_hat"], rel=1e-12)
    # u perpendicular to B, no E: chi_e = |u| B / E_s (the relation used in Sec. 4)
    assert O.chi_lepton(U, [1000.0, 0, 0], math.sqrt(1 + 1e6), [0, 0, 0], [0, 0, 33.0]) == pytest.approx(
        1000 * 33 / U["Es_hat"], rel=1e-14)


# --------------------------------------------------------- paper numbers ----
def test_paper_constants_and_validation_case():
    assert U["E_s"] == pytest.approx(GOLD["schwinger_field_V_per_m"]["value"], rel=0.05)
    assert 1 / U["alpha_f"] == pytest.approx(GOLD["fine_structure_inverse"]["value"], abs=0.5)
    gam = GOLD["validation_gamma"]["value"]
    Bhat = GOLD["validation_B_T"]["value"] / U["B_ref"]
    p = math.sqrt(gam * gam - 1)
    chi = O.chi_lepton(U, [p, 0, 0], gam, [0, 0, 0], [0, 0, Bhat])
    assert round(chi) == GOLD["validation_chi"]["value"]
    omega_inv_fs = gam / Bhat / U["omega_r"] * 1e15
    assert round(omega_inv_fs, 1) == GOLD["validation_inverse_gyrofrequency_fs"]["value"]
    R_um = p / Bhat * (299792458.0 / U["omega_r"]) * 1e6
    assert round(R_um, 1) == GOLD["validation_gyroradius_um"]["value"]
    # first photons: <xi> = (2/3) chi^2 g/h_rad at chi = 5.08 gives <gamma_gamma> of order 10^3
    # and <chi_gamma> close to 1
    mean_xi = (2 / 3) * chi * chi * O.g(chi) / O.h_rad(chi)
    assert 10 ** round(math.log10(mean_xi * gam)) == GOLD["first_photon_gamma_order"]["value"]
    assert round(mean_xi * chi) == GOLD["mean_photon_chi_order"]["value"]
    # pair rate at chi_gamma = 0.1 is negligible next to chi_gamma = 1
    assert O.h_pair(GOLD["pair_stall_chi"]["value"]) / O.h_pair(1.0) < 1e-11


# ----------------------------------------------------------------- field ----
def test_plane_wave_is_minus_derivative_of_potential():
    a0, N = 7.0, 10.0
    f = O.make_field(O.FIELD_PLANE_WAVE, a0=a0, n_periods=N)
    Phi = 2 * math.pi * N

    def ay(phi):
        return a0 * math.sin(math.pi * phi / Phi) ** 2 * math.sin(phi) if 0 < phi < Phi else 0.0
    for phi in (0.3, 5.0, 31.4, 50.0, 62.0):
        h = 1e-5
        d = (ay(phi + h) - ay(phi - h)) / (2 * h)
        E, B = O.field_at(f, phi + 3.0, 3.0, 0.2, -0.4)
        assert E[1] == pytest.approx(-d, rel=1e-8, abs=1e-9)
        assert B[2] == E[1] and E[0] == E[2] == B[0] == B[1] == 0.0
    assert O.field_at(f, 0.0, 5.0, 0, 0)[0][1] == 0.0          # ahead of the front


def _yee_grid(shape, fn):
    nx, ny, nz = shape
    g = np.zeros((6, nx, ny, nz), np.float32)
    st = np.array([[0.5, 0, 0], [0, 0.5, 0], [0, 0, 0.5], [0, 0.5, 0.5], [0.5, 0, 0.5], [0.5, 0.5, 0]])
    for c in range(6):
        i, j, k = np.meshgrid(np.arange(nx) + st[c, 0], np.arange(ny) + st[c, 1],
                              np.arange(nz) + st[c, 2], indexing="ij")
        g[c] = fn(c, i, j, k)
    return g


def test_yee_tsc_reproduces_linear_fields():
    shape, d, org = (12, 10, 9), (0.5, 0.25, 0.4), (-1.0, 2.0, 0.5)
    # exactly representable linear field per component, in node units
    coef = np.array([[1, 0.5, -0.25, 0.125], [2, -0.5, 0.25, 0.0], [0.5, 0.0, 0.0, 0.5],
                     [-1, 0.25, 0.5, 0.25], [0.25, 0.125, -0.5, 1], [3, 0, 0.5, -0.25]])
    g = _yee_grid(shape, lambda c, i, j, k: coef[c, 0] + coef[c, 1] * i + coef[c, 2] * j + coef[c, 3] * k)
    f = O.make_field(O.FIELD_YEE, grid=g, shape=shape, spacing=d, origin=org)
    rng = np.random.default_rng(5)
    for _ in range(50):
        gi = rng.uniform(2, np.array(shape) - 3)
        x, y, z = org[0] + gi[0] * d[0], org[1] + gi[1] * d[1], org[2] + gi[2] * d[2]
        E, B = O.field_at(f, 0.0, x, y, z)
        got = np.concatenate([E, B])
        want = coef[:, 0] + coef[:, 1] * gi[0] + coef[:, 2] * gi[1] + coef[:, 3] * gi[2]
        assert got == pytest.approx(want, rel=1e-12, abs=1e-12)
    # far outside the grid the field is zero
    E, B = O.field_at(f, 0.0, 100.0, 100.0, 100.0)
    assert not np.any(E) and not np.any(B)


def test_yee_fill_separable_is_product():
    shape = (5, 4, 3)
    rng = np.random.default_rng(1)
    tperp, tpar = rng.normal(size=(6, 12)), rng.normal(size=(6, 5))
    g = O.yee_fill_separable(shape, 3.5, tperp, tpar)
    want = ((3.5 * tperp)[:, None, :] * tpar[:, :, None]).astype(np.float32).reshape(6, 5, 4, 3)
    assert np.array_equal(g, want)


# ----------------------------------------------------------------- push -----
def _one(u, x=(0.0, 0.0, 0.0), n=1, uid0=0):
    s = O.new_species(n)
    s["x"][:], s["y"][:], s["z"][:] = x
    s["ux"][:], s["uy"][:], s["uz"][:] = u
    s["w"][:] = 1.0
    s["uid"][:] = np.arange(uid0, uid0 + n, dtype=np.uint64)
    s["n"] = n
    return s


def _run(bt, lep, field, steps, dt, q=-1.0, t0=0.0, rad=O.RAD_NONE, ph_rec=None, ph_push=None,
         seed=1, tally=None, uid_next=None, **kw):
    tally = tally or O.Tally()
    uid_next = uid_next if uid_next is not None else [10**9]
    for n in range(steps):
        st = O.make_step(t0 + n * dt, dt, seed, rad_model=rad, **kw)
        O.push_emit(bt, LAM, q, lep, field, ph_push, ph_rec, st, uid_next, tally)
    return tally


def test_boris_gyration_exact_angle(bound_tables):
    B, u0, dt, n = 40.0, 500.0, 0.05, 1000
    lep = _one((u0, 0.0, 0.0))
    f = O.make_field(O.FIELD_UNIFORM, B=(0, 0, B))
    _run(bound_tables, lep, f, n, dt)
    gam = math.sqrt(1 + u0 * u0)
    th = n * 2 * math.atan(0.5 * B * dt / gam)      # Boris rotation angle per step
    u = np.array([lep["ux"][0], lep["uy"][0], lep["uz"][0]])
    assert np.linalg.norm(u) == pytest.approx(u0, rel=1e-13)
    assert u == pytest.approx(u0 * np.array([math.cos(th), math.sin(th), 0.0]), rel=1e-9, abs=1e-9 * u0)


def _plane_wave_errors(bt, dt):
    a0, N = 5.0, 4.0
    f = O.make_field(O.FIELD_PLANE_WAVE, a0=a0, n_periods=N)
    lep = _one((-200.0, 0.0, 0.0), x=(20.0, 0.0, 0.0))
    Phi = 2 * math.pi * N
    g0 = math.sqrt(1 + 200.0 ** 2)
    h0 = None
    err_uy, err_h = 0.0, 0.0
    steps = int(round(40.0 / dt))
    for n in range(steps):
        x_old = lep["x"][0]
        _run(bt, lep, f, 1, dt, t0=n * dt)
        ux, uy = lep["ux"][0], lep["uy"][0]
        g = math.sqrt(1 + ux * ux + uy * uy)
        phi = (n + 0.5) * dt - 0.5 * (x_old + lep["x"][0])
        ay = a0 * math.sin(math.pi * phi / Phi) ** 2 * math.sin(phi) if 0 < phi < Phi else 0.0
        err_uy = max(err_uy, abs(uy - ay))                      # u_y + q a_y = 0, q = -1
        h0 = g0 + 200.0
        err_h = max(err_h, abs((g - ux) - h0) / h0)             # gamma - u_x is conserved
    return err_uy, err_h


def test_boris_plane_wave_invariants_second_order(bound_tables):
    e1 = _plane_wave_errors(bound_tables, 0.02)
    e2 = _plane_wave_errors(bound_tables, 0.01)
    assert e1[0] < 0.01 * 5.0 and e1[1] < 1e-9
    assert e1[0] / e2[0] == pytest.approx(4.0, rel=0.25)        # second order in dt


def test_sokolov_drag_matches_ode(bound_tables):
    # u perpendicular to a constant B, no E: chi = |u| B/E_s and Eqs. 4-5 give
    # d|u|/dt = -(2/3) A chi^2 g(chi) |u|/gamma (the delta_v x B term is O(1/gamma^2) smaller)
    B, u0, dt, n = 33.0, 1000.0, 0.01, 5000
    lep = _one((u0, 0.0, 0.0))
    f = O.make_field(O.FIELD_UNIFORM, B=(0, 0, B))
    tally = _run(bound_tables, lep, f, n, dt, rad=O.RAD_SOKOLOV)
    A, Es = U["A_hat"], U["Es_hat"]

    def rhs(t, y):
        p = y[0]
        chi = p * B / Es
        return [-(2 / 3) * A * chi * chi * O.g(chi) * p / math.sqrt(1 + p * p)]
    sol = solve_ivp(rhs, (0, n * dt), [u0], rtol=1e-11, atol=1e-9)
    p_end = math.sqrt(lep["ux"][0] ** 2 + lep["uy"][0] ** 2)
    assert p_end < 0.8 * u0                                     # damping is significant
    assert p_end == pytest.approx(sol.y[0, -1], rel=1e-3)
    # radiated-energy tally equals the energy lost (the Lorentz force does no work in pure B)
    assert tally.t[O.T_NAMES.index("erad")] == pytest.approx(
        math.sqrt(1 + u0 * u0) - math.sqrt(1 + p_end ** 2), rel=1e-3)


def test_hybrid_selects_by_chi(bound_tables):
    f = O.make_field(O.FIELD_UNIFORM, B=(0, 0, 1.0))
    lep = _one((1000.0, 0, 0), n=2)
    lep["ux"][1] = 10.0                      # chi = 1000/E_s ~ 3e-3 vs 10/E_s ~ 3e-5
    t = _run(bound_tables, lep, f, 1, 0.01, rad=O.RAD_HYBRID, chi_switch=1e-3)
    assert t.c[O.C_NAMES.index("mc")] == 1 and t.c[O.C_NAMES.index("sokolov")] == 1


# ------------------------------------------------------------ Monte Carlo ----
def test_optical_depth_poisson_counts(bound_tables):
    # recoil off (test switch): chi and gamma are frozen in a constant B, so the
    # number of emissions over time T is Poisson with mean W T, W = A h_rad(chi)/gamma (Eq. 6)
    n, steps, dt = 8000, 400, 0.01
    gam_target = 1000.0
    B = U["Es_hat"] / gam_target                     # chi = 1 for |u| = 1000
    lep = _one((1000.0, 0.0, 0.0), n=n)
    O.init_tau(lep, 42)
    f = O.make_field(O.FIELD_UNIFORM, B=(0, 0, B))
    _run(bound_tables, lep, f, steps, dt, rad=O.RAD_MC, seed=42, no_recoil=1, max_events=4)
    gam = math.sqrt(1 + 1000.0 ** 2)
    chi = 1000.0 * B / U["Es_hat"]
    lam = U["A_hat"] * bound_tables.h_rad(chi) / gam * steps * dt
    k = lep["n_ev"][:n].astype(float)
    assert k.mean() == pytest.approx(lam, abs=4 * math.sqrt(lam / n))
    assert k.var() / k.mean() == pytest.approx(1.0, abs=0.06)
    # chi-square against the Poisson pmf
    from scipy.stats import chisquare, poisson
    kmax = int(lam + 4 * math.sqrt(lam))
    obs = np.bincount(np.minimum(k.astype(int), kmax), minlength=kmax + 1)
    exp_ = poisson.pmf(np.arange(kmax + 1), lam) * n
    exp_[-1] += poisson.sf(kmax, lam) * n
    assert chisquare(obs, exp_).pvalue > 1e-3


def test_emission_conserves_momentum(bound_tables):
    # pure B keeps |u_L| = |u|; Eq. 8 then gives |u_after| + sum gamma_gamma = |u_before|
    n = 3000
    lep = _one((2000.0, 0.0, 300.0), n=n)
    O.init_tau(lep, 9)
    lep["tau"][:n] *= 0.01                                  # most particles emit at once
    f = O.make_field(O.FIELD_UNIFORM, B=(0, 0, 150.0))
    rec = O.new_species(4 * n)
    p0 = math.sqrt(2000.0 ** 2 + 300.0 ** 2)
    _run(bound_tables, lep, f, 1, 0.05, rad=O.RAD_MC, ph_rec=rec, seed=9, gamma_photon_min=0.0)
    k = np.sqrt(rec["ux"] ** 2 + rec["uy"] ** 2 + rec["uz"] ** 2)[:rec["n"]]
    cnt = lep["n_ev"][:n].astype(int)
    assert cnt.sum() == rec["n"] and cnt.max() >= 2
    off = np.concatenate([[0], np.cumsum(cnt)])
    for i in range(0, n, 7):
        u = np.array([lep["ux"][i], lep["uy"][i], lep["uz"][i]])
        p = np.linalg.norm(u)
        ks = k[off[i]:off[i + 1]]
        assert p + ks.sum() == pytest.approx(p0, rel=1e-12) or p == 0.0
        for j in range(off[i], off[i + 1]):
            kv = np.array([rec["ux"][j], rec["uy"][j], rec["uz"][j]])
            if p > 0:
                assert np.linalg.norm(np.cross(kv, u)) <= 1e-12 * np.linalg.norm(kv) * p
    # photons carry consecutive new ids in emission order
    assert np.array_equal(rec["uid"][:rec["n"]], 10**9 + np.arange(rec["n"], dtype=np.uint64))


def test_pair_event_conservation(bound_tables):
    n = 2000
    ph = O.new_species(n)
    ph["ux"][:n] = 4000.0
    ph["uz"][:n] = np.linspace(-100, 100, n)
    ph["w"][:n] = 0.5
    ph["tau"][:n] = 1e-12                      # every photon decays in the step
    ph["uid"][:n] = np.arange(n, dtype=np.uint64)
    ph["n"] = n
    f = O.make_field(O.FIELD_UNIFORM, B=(0, 150.0, 0))
    el, po = O.new_species(n), O.new_species(n)
    k = np.stack([ph["ux"][:n], ph["uy"][:n], ph["uz"][:n]], 1).copy()
    chig = np.array([O.chi_photon(U, kk, [0, 0, 0], [0, 150.0, 0]) for kk in k])
    tally = O.Tally()
    st = O.make_step(0.0, 0.05, 3)
    un = [5000]
    O.pair_create(bound_tables, LAM, ph, f, el, po, st, un, tally)
    assert ph["n"] == 0 and el["n"] == n and po["n"] == n
    assert tally.c[O.C_NAMES.index("pair")] == n
    kk = np.linalg.norm(k, axis=1)
    ue = np.stack([el["ux"][:n], el["uy"][:n], el["uz"][:n]], 1)
    up = np.stack([po["ux"][:n], po["uy"][:n], po["uz"][:n]], 1)
    ge, gp = np.sqrt(1 + (ue ** 2).sum(1)), np.sqrt(1 + (up ** 2).sum(1))
    assert ge + gp == pytest.approx(kk, rel=1e-13)                             # energy exact
    assert np.all(np.linalg.norm(ue + up - k, axis=1) <= 1 / (2 * ge) + 1 / (2 * gp) + 1e-9 * kk)
    assert el["chi"][:n] + po["chi"][:n] == pytest.approx(chig, rel=1e-14)    # chi_+ = chi_g - chi_-
    assert np.all(el["uid"][:n] == 5000 + 2 * np.arange(n)) and np.all(po["uid"][:n] == 5001 + 2 * np.arange(n))
    assert np.all(el["w"][:n] == 0.5)


def test_capacity_overflow_is_reported(bound_tables):
    n = 500
    lep = _one((2000.0, 0.0, 0.0), n=n)
    lep["tau"][:n] = 1e-9
    f = O.make_field(O.FIELD_UNIFORM, B=(0, 0, 150.0))
    rec = O.new_species(10)
    tally = O.Tally()
    st = O.make_step(0.0, 0.05, 1, rad_model=O.RAD_MC, gamma_photon_min=0.0)
    rc = O.push_emit(bound_tables, LAM, -1.0, lep, f, None, rec, st, [0], tally)
    assert rc == 1 and rec["n"] == 10
    assert tally.c[O.C_NAMES.index("overflow")] == tally.c[O.C_NAMES.index("rec")] - 10


def test_variant_pair_momentum_split(bound_tables):
    """Alternative reading of the pair split: the photon momentum is shared
    exactly (u_- + u_+ = k), each lepton on its mass shell, chi still adds up;
    the energy then exceeds gamma_gamma by O(1/gamma)."""
    n = 1500
    ph = O.new_species(n)
    ph["ux"][:n] = 4000.0
    ph["uz"][:n] = np.linspace(-100, 100, n)
    ph["w"][:n] = 0.5
    ph["tau"][:n] = 1e-12
    ph["uid"][:n] = np.arange(n, dtype=np.uint64)
    ph["n"] = n
    f = O.make_field(O.FIELD_UNIFORM, B=(0, 150.0, 0))
    el, po = O.new_species(n), O.new_species(n)
    k = np.stack([ph["ux"][:n], ph["uy"][:n], ph["uz"][:n]], 1).copy()
    chig = np.array([O.chi_photon(U, kk, [0, 0, 0], [0, 150.0, 0]) for kk in k])
    st = O.make_step(0.0, 0.05, 3, variants=O.VAR_PAIR_MOMENTUM)
    O.pair_create(bound_tables, LAM, ph, f, el, po, st, [5000], O.Tally())
    assert el["n"] == n and po["n"] == n
    ue = np.stack([el["ux"][:n], el["uy"][:n], el["uz"][:n]], 1)
    up = np.stack([po["ux"][:n], po["uy"][:n], po["uz"][:n]], 1)
    assert np.all(np.linalg.norm(ue + up - k, axis=1) <= 1e-13 * np.linalg.norm(k, axis=1))   # momentum exact
    ge, gp = np.sqrt(1 + (ue ** 2).sum(1)), np.sqrt(1 + (up ** 2).sum(1))
    kk = np.linalg.norm(k, axis=1)
    assert np.all(ge + gp >= kk) and np.all(ge + gp - kk <= 1 / ge + 1 / gp)
    assert el["chi"][:n] + po["chi"][:n] == pytest.approx(chig, rel=1e-14)
    # each lepton's share of k is its share of chi
    assert np.linalg.norm(ue, axis=1) / kk == pytest.approx(el["chi"][:n] / chig, rel=1e-13)


def test_variant_sokolov_g_scales_delta_v(bound_tables):
    """Alternative reading of Eq. 4 (delta_v with tau_0 g(chi)).  For E = 0 and
    u perpendicular to B, f = q v x B and v.f = 0, so delta_v = tau f and the
    q delta_v x B force is -tau B^2 v: the variant changes the new momentum
    by exactly dt tau_0 (1 - g(chi)) B^2 v, along v."""
    Bz = 300.0
    n = 8
    p = np.geomspace(50.0, 5000.0, n)
    e = {"x": np.zeros(n), "y": np.zeros(n), "z": np.zeros(n), "ux": p, "uy": np.zeros(n), "uz": np.zeros(n)}
    f = O.make_field(O.FIELD_UNIFORM, B=(0, 0, Bz))
    out = []
    for var in (0, O.VAR_SOKOLOV_G):
        s = O.species_from(e)
        st = O.make_step(0.0, 0.01, 3, rad_model=O.RAD_SOKOLOV, variants=var)
        O.push_emit(bound_tables, LAM, -1.0, s, f, None, None, st, [n], O.Tally())
        out.append(np.stack([s["ux"][:n], s["uy"][:n], s["uz"][:n]], 1))
    # the Boris rotation keeps |u|, so chi and v are those of the rotated momentum
    u_rot = out[0] / np.linalg.norm(out[0], axis=1)[:, None]            # direction, to O(tau dt)
    chi = p * Bz / U["Es_hat"]
    g = np.array([bound_tables.g(c) for c in chi])
    gam = np.sqrt(1 + p * p)
    expect = 0.01 * U["tau0_hat"] * (1 - g) * Bz ** 2 * (p / gam)       # |v| = p / gamma
    diff = out[1] - out[0]
    assert np.all(g < 1.0) and np.all(expect > 0)
    assert np.linalg.norm(diff, axis=1) == pytest.approx(expect, rel=1e-5)
    assert np.all(np.einsum("ij,ij->i", diff, u_rot) > 0)                  # less drag: along v
