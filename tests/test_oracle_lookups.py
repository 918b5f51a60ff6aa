"""Pins of the oracle's table lookups, its pair sampler and the Sokolov
correction with an electric field (CPU only).

Expected values come from outside the lookups: the direct Bessel quadrature
of the rates at the point itself (not the tables), the error law of linear
interpolation, the small-chi limits of Sec. 2, SciPy quadrature of the pair
spectrum of Eq. 3, and the closed-form Boris rotation with Eq. 4 specialised
to aligned and crossed fields.
"""
import math

import numpy as np
import pytest
import scipy.integrate as si
import scipy.special as sp

from oracle import oracle as O

LAM = 0.8e-6
U = O.units(LAM)


def _nodes(spec):
    return np.linspace(math.log(spec["chi_min"]), math.log(spec["chi_max"]), spec["n_chi"])


# ------------------------------------------------ rates between the nodes --
def _check_between_nodes(lookup, direct, lnc, segs, strip=None):
    """Lookup at fractions w of segment [lnc[i], lnc[i+1]] in ln chi against
    the direct quadrature at that chi.  Linear interpolation of a smooth
    y(ln chi) misses y by +w(1-w) D2/2 to leading order, D2 the second
    difference of y over the neighbouring nodes; the lookup's error must be
    that (to 10 % + 2e-9), which an interpolation in chi instead of ln chi, a
    shifted node or a wrong end segment all break by far more."""
    y = lambda c: math.log(direct(c)) - (strip(c) if strip else 0.0)
    for i in segs:
        d2 = 0.5 * ((y(math.exp(lnc[i - 1])) - 2 * y(math.exp(lnc[i])) + y(math.exp(lnc[i + 1]))) +
                    (y(math.exp(lnc[i])) - 2 * y(math.exp(lnc[i + 1])) + y(math.exp(lnc[i + 2]))))
        for w in (0.25, 0.5, 0.8):
            c = math.exp(lnc[i] + w * (lnc[i + 1] - lnc[i]))
            got = math.log(lookup(c)) - math.log(direct(c))
            want = 0.5 * w * (1 - w) * d2
            assert abs(got - want) <= 0.1 * abs(want) + 2e-9, (i, w, got, want)


def test_h_rad_lookup_between_nodes(bound_tables, oracle_tables):
    lnc = _nodes(oracle_tables["emit_spec"])
    _check_between_nodes(bound_tables.h_rad, O.h_rad, lnc, (1, 17, 40, 63, 90, 125))


def test_g_lookup_between_nodes(bound_tables, oracle_tables):
    lnc = _nodes(oracle_tables["emit_spec"])
    _check_between_nodes(bound_tables.g, O.g, lnc, (1, 17, 40, 63, 90, 125))


def test_h_pair_lookup_between_nodes(bound_tables, oracle_tables):
    # the table holds ln h_pair + 8/(3 chi): interpolation is linear in that
    lnc = _nodes(oracle_tables["pair_spec"])
    _check_between_nodes(bound_tables.h_pair, O.h_pair, lnc, (1, 20, 50, 80, 110, 125),
                         strip=lambda c: -8.0 / (3.0 * c))


def test_rate_lookups_at_the_table_ends(bound_tables, oracle_tables):
    es, ps = oracle_tables["emit_spec"], oracle_tables["pair_spec"]
    # the nodes themselves
    for c in (es["chi_min"], es["chi_max"]):
        assert bound_tables.h_rad(c) == pytest.approx(O.h_rad(c), rel=1e-12)
        assert bound_tables.g(c) == pytest.approx(O.g(c), rel=1e-12)
    assert bound_tables.h_pair(ps["chi_max"]) == pytest.approx(O.h_pair(ps["chi_max"]), rel=1e-12)
    # no pair rate below the pair table
    assert bound_tables.h_pair(0.999 * ps["chi_min"]) == 0.0
    # above the table the last segment is extended: at 2 chi_max its slope,
    # a little above the 2/3 of the large-chi limit, is 0.25 % high
    c = 2.0 * es["chi_max"]
    assert bound_tables.h_rad(c) == pytest.approx(O.h_rad(c), rel=5e-3)


@pytest.mark.parametrize("chi", [5e-4, 1e-4, 1e-5, 1e-6, 1e-8])
def test_g_lookup_below_table_keeps_larmor_limit(bound_tables, chi):
    """Below the first node the Sokolov step still needs g(chi) (Eq. 5): it
    must tend to 1 (classical Larmor power) with the first-order law
    g = 1 - (55 sqrt 3/16) chi, so it matches the direct quadrature."""
    g = bound_tables.g(chi)
    assert g <= 1.0
    assert g == pytest.approx(O.g(chi), rel=1e-5)
    # the slope is the node's, ln g(chi_min)/chi_min, within the O(chi_min) second-order term
    assert 1.0 - g == pytest.approx(55 * math.sqrt(3) / 16 * chi, rel=1e-2)


@pytest.mark.parametrize("chi", [5e-4, 1e-5, 1e-8])
def test_h_rad_lookup_below_table_is_classical(bound_tables, oracle_tables, chi):
    """Below the first node the photon-number rate follows the classical law,
    proportional to chi (h_rad -> 5 chi/(2 sqrt 3)), continuous at the node."""
    c0 = oracle_tables["emit_spec"]["chi_min"]
    assert bound_tables.h_rad(chi) / chi == pytest.approx(bound_tables.h_rad(c0) / c0, rel=1e-14)
    assert bound_tables.h_rad(chi) == pytest.approx(5 * chi / (2 * math.sqrt(3)), rel=1.5e-3)


# ------------------------------------------------------ pair-energy sampler --
def _pair_bracket_scipy(chi, eta):
    """Bracket of Eq. 3 (reading: y = chi_g/(3 chi_- chi_+), so 2y = delta and
    3 chi_g y = 1/(eta(1-eta))), from SciPy's Bessel routines."""
    d = 2.0 / (3.0 * chi * eta * (1.0 - eta))
    ki = si.quad(lambda u: sp.kve(1 / 3, d + u) * math.exp(-u), 0, np.inf, epsabs=0, epsrel=1e-12,
                 limit=200)[0] * math.exp(-d)
    return ki + (1.0 / (eta * (1.0 - eta)) - 2.0) * sp.kv(2 / 3, d)


def _pair_moment_scipy(chi, fn):
    """E[fn(eta)] under the pair spectrum (symmetric in eta <-> 1-eta, so
    integrate over [0, 1/2] only)."""
    pts = [1e-3, 1e-2, 0.1, 0.3]
    den = si.quad(lambda e: _pair_bracket_scipy(chi, e), 1e-12, 0.5, points=pts, epsrel=1e-10, limit=300)[0]
    num = si.quad(lambda e: fn(e) * _pair_bracket_scipy(chi, e), 1e-12, 0.5, points=pts, epsrel=1e-10,
                  limit=300)[0]
    return num / den


@pytest.mark.parametrize("chi", [0.3, 2.0, 20.0])
def test_sample_eta_moments_against_quadrature(bound_tables, chi):
    """E[(eta - 1/2)^2] and E[|eta - 1/2|] of table samples over a stratified
    grid of r, against SciPy quadrature of Eq. 3's spectrum.  The table's CDF
    error (a few 1e-4) bounds the moment error well inside 1 %."""
    r = (np.arange(20_000) + 0.5) / 20_000
    eta = np.array([bound_tables.sample_eta(chi, float(v)) for v in r])
    assert np.all((eta > 0) & (eta < 1))
    assert np.mean(eta) == pytest.approx(0.5, abs=2e-4)                 # eta <-> 1 - eta symmetry
    var = _pair_moment_scipy(chi, lambda e: (e - 0.5) ** 2)
    mad = _pair_moment_scipy(chi, lambda e: 0.5 - e)
    assert np.mean((eta - 0.5) ** 2) == pytest.approx(var, rel=1e-2)
    assert np.mean(np.abs(eta - 0.5)) == pytest.approx(mad, rel=5e-3)


def test_sample_eta_ks_against_cdf(bound_tables):
    """Table samples of eta (random r) follow the pair CDF within the table's
    interpolation error; the CDF itself is checked against SciPy here."""
    chi = 1.3
    for e in (0.05, 0.2, 0.4):
        pts = [1e-3, 1e-2, 0.1]
        den = si.quad(lambda x: _pair_bracket_scipy(chi, x), 1e-12, 0.5, points=pts, epsrel=1e-10, limit=300)[0]
        num = si.quad(lambda x: _pair_bracket_scipy(chi, x), 1e-12, e, points=[p for p in pts if p < e],
                      epsrel=1e-10, limit=300)[0]
        assert O.pair_cdf(chi, e) == pytest.approx(0.5 * num / den, rel=1e-7)
    rng = np.random.default_rng(11)
    r = rng.uniform(size=4000)
    xs = np.sort([bound_tables.sample_eta(chi, float(v)) for v in r])
    cdf = np.array([O.pair_cdf(chi, float(x)) for x in xs[::40]])
    emp = (np.arange(0, len(xs), 40) + 1) / len(xs)
    assert np.max(np.abs(cdf - emp)) < 0.03


# ------------------------------------------- Sokolov with an electric field --
def _boris_closed_form(u, E, B, q, dt):
    """u^{n+1/2} of the Boris push written as half kick, rotation of u- about
    B by 2 atan(|q B| dt/(2 gamma-)) (sense of q v x B), half kick."""
    u, E, B = (np.asarray(a, float) for a in (u, E, B))
    um = u + 0.5 * q * dt * E
    gm = math.sqrt(1 + um @ um)
    bn = np.linalg.norm(B)
    if bn == 0.0:
        return um + 0.5 * q * dt * E
    b = B / bn
    th = 2 * math.atan(abs(q) * bn * dt / (2 * gm))
    s = -math.copysign(1.0, q)                       # q v x B turns u the negative way about B for q > 0
    par = (um @ b) * b
    perp = um - par
    rot = par + perp * math.cos(th) + s * np.cross(b, perp) * math.sin(th)
    return rot + 0.5 * q * dt * E


def _sokolov_expected(u, x, E, B, q, dt, g_of):
    """One Sokolov step (Eqs. 4-5) from the closed-form Boris momentum, with
    v.f_l = q v.E (v.(v x B) = 0): delta_v = tau0 q (E + v x B - v (v.E)) /
    (1 + tau0 q v.E); chi from Eq. 1 as printed (parallel and perpendicular
    parts of E)."""
    E, B, x = (np.asarray(a, float) for a in (E, B, x))
    uL = _boris_closed_form(u, E, B, q, dt)
    gL = math.sqrt(1 + uL @ uL)
    v = uL / gL
    vn = np.linalg.norm(v)
    vh = v / vn
    Epar = (E @ vh) * vh
    Eperp = E - Epar
    w = Eperp + np.cross(v, B)
    chi = gL / U["Es_hat"] * math.sqrt(Epar @ Epar / gL ** 2 + w @ w)
    t0 = U["tau0_hat"]
    dv = t0 * q * (E + np.cross(v, B) - v * (v @ E)) / (1 + t0 * q * (v @ E))
    P = (2.0 / 3.0) * U["A_hat"] * chi * chi * g_of(chi)
    un = uL + dt * (q * np.cross(dv, B) - P * uL / gL)
    gn = math.sqrt(1 + un @ un)
    return un, x + dt * (un / gn + dv), dv, chi


def _one_step(bt, u, x, E, B, q, dt):
    s = O.new_species(1)
    s["x"][0], s["y"][0], s["z"][0] = x
    s["ux"][0], s["uy"][0], s["uz"][0] = u
    s["w"][0] = 1.0
    s["n"] = 1
    f = O.make_field(O.FIELD_UNIFORM, E=E, B=B)
    st = O.make_step(0.0, dt, 1, rad_model=O.RAD_SOKOLOV)
    O.push_emit(bt, LAM, q, s, f, None, None, st, [1], O.Tally())
    return np.array([s["ux"][0], s["uy"][0], s["uz"][0]]), np.array([s["x"][0], s["y"][0], s["z"][0]])


CASES = {
    # E along v, no B: delta_v = tau0 q E / (gamma^2 (1 + tau0 q v E)) along v,
    # so only the position sees it; chi = |E|/E_s
    "E_parallel_v": dict(u=(0.6, 0.0, 0.0), E=(1.5e5, 0.0, 0.0), B=(0.0, 0.0, 0.0)),
    # E along B, u across both: v.E != 0 after the kick, delta_v x B acts
    "E_parallel_B": dict(u=(0.0, 1.4, 0.0), E=(0.0, 0.0, 9e4), B=(0.0, 0.0, 7e4)),
    # crossed E and B, u oblique to both
    "crossed": dict(u=(0.8, -0.3, 0.5), E=(0.0, 1.2e5, 0.0), B=(0.0, 0.0, 6e4)),
}


@pytest.mark.parametrize("q", [-1.0, 1.0])
@pytest.mark.parametrize("case", sorted(CASES))
def test_sokolov_delta_v_with_electric_field(bound_tables, case, q):
    c = CASES[case]
    # strong fields over a short step (tau0 |E| ~ 2e-3, gamma ~ 2): the Sokolov
    # terms are resolved far above the 1e-12 comparison (a charge sign lost
    # from v.f, a dropped v (v.f) term or a dropped dt delta_v all show)
    dt, x0 = 1e-5, (0.0, 0.0, 0.0)
    got_u, got_x = _one_step(bound_tables, c["u"], x0, c["E"], c["B"], q, dt)
    un, xn, dv, chi = _sokolov_expected(c["u"], x0, c["E"], c["B"], q, dt, bound_tables.g)
    assert np.linalg.norm(dt * dv) > 1e-4 * np.linalg.norm(xn)
    assert 1e-2 < chi < 1.0
    assert got_u == pytest.approx(un, rel=1e-12, abs=1e-12 * np.linalg.norm(un))
    assert got_x == pytest.approx(xn, rel=1e-12, abs=1e-13 * np.linalg.norm(xn))
    if case == "E_parallel_v":
        uL = np.asarray(c["u"]) + q * dt * np.asarray(c["E"])
        gL = math.sqrt(1 + uL @ uL)
        closed = U["tau0_hat"] * q * c["E"][0] / (gL ** 2 * (1 + U["tau0_hat"] * q * c["E"][0] * uL[0] / gL))
        assert dv[0] == pytest.approx(closed, rel=1e-12) and dv[1] == dv[2] == 0.0
        assert chi == pytest.approx(c["E"][0] / U["Es_hat"], rel=1e-13)
