"""Pins of the oracle's special functions, rates and tables (CPU only).

Every expected value here comes from outside the oracle: closed forms,
textbook limits, identities, or SciPy's own Bessel routine and adaptive
quadrature evaluated on the spectrum's definition.
"""
import math

import numpy as np
import pytest
import scipy.integrate as si
import scipy.special as sp

from oracle import oracle as O

G23 = math.gamma(2.0 / 3.0)


def ki_scipy(nu, x):
    """int_x^inf K_nu with SciPy: e^{-x} int_0^inf kve(nu, x+u) e^{-u} du."""
    v = si.quad(lambda u: sp.kve(nu, x + u) * math.exp(-u), 0, np.inf, epsabs=0, epsrel=1e-13, limit=400)[0]
    return v * math.exp(-x)


# ---------------------------------------------------------------- Bessel ----
@pytest.mark.parametrize("x", [1e-8, 1e-3, 0.2, 1.0, 7.5, 40.0, 300.0])
def test_k_half_closed_form(x):
    # K_{1/2}(x) = sqrt(pi/(2x)) e^{-x}
    exact = math.sqrt(math.pi / (2 * x)) * math.exp(-x)
    assert O.bessel_k(0.5, x) == pytest.approx(exact, rel=2e-15)


@pytest.mark.parametrize("nu", [1 / 3, 2 / 3, 5 / 3])
@pytest.mark.parametrize("x", [1e-9, 1e-4, 0.05, 0.7, 3.0, 18.0, 90.0, 500.0])
def test_k_against_scipy(nu, x):
    assert O.bessel_k(nu, x) == pytest.approx(sp.kv(nu, x), rel=1e-13)


def test_integral_k13_total():
    # int_0^inf K_{1/3} = pi/sqrt(3)  (Mellin transform of K_nu at s = 1)
    assert O.bessel_ki(1 / 3, 1e-14) == pytest.approx(math.pi / math.sqrt(3), rel=1e-9)


@pytest.mark.parametrize("x", [1e-3, 0.1, 1.0, 5.0])
def test_integral_k13_against_scipy_quad(x):
    assert O.bessel_ki(1 / 3, x) == pytest.approx(ki_scipy(1 / 3, x), rel=1e-11)


@pytest.mark.parametrize("x", [1e-2, 0.3, 1.0, 4.0, 20.0])
def test_k53_identity(x):
    # K_{5/3} = -2 K_{2/3}' - K_{1/3}  =>  int_x^inf K_{5/3} = 2 K_{2/3}(x) - int_x^inf K_{1/3}
    lhs = O.bessel_ki(5 / 3, x)
    rhs = 2 * O.bessel_k(2 / 3, x) - O.bessel_ki(1 / 3, x)
    assert lhs == pytest.approx(rhs, rel=1e-13)


def test_synchrotron_function_at_one():
    # classical synchrotron function F(1) = int_1^inf K_{5/3} = 0.651422815355 (tabulated)
    assert O.bessel_ki(5 / 3, 1.0) == pytest.approx(0.651422815355, rel=1e-11)


# --------------------------------------------------------------- spectra ----
@pytest.mark.parametrize("chi", [1e-3, 0.1, 1.0, 10.0, 100.0])
def test_emit_bracket_positive_and_matches_scipy(chi):
    for xi in (1e-6, 1e-3, 0.1, 0.5, 0.9):
        b = O.emit_bracket(chi, xi)
        assert b >= 0.0
        d = 2 * xi / (3 * chi * (1 - xi))
        if d > 600:
            continue
        ki = ki_scipy(1 / 3, d)
        ref = (2 + xi * xi / (1 - xi)) * sp.kv(2 / 3, d) - ki
        assert b == pytest.approx(ref, rel=1e-9, abs=1e-300)


@pytest.mark.parametrize("chi", [0.05, 1.0, 30.0])
def test_pair_bracket_symmetric_positive(chi):
    for eta in (0.05, 0.2, 0.45):   # delta < 700 keeps the unscaled bracket representable
        a, b = O.pair_bracket(chi, eta), O.pair_bracket(chi, 1 - eta)
        assert a > 0 and a == pytest.approx(b, rel=1e-12)


# ----------------------------------------------------------------- rates ----
@pytest.mark.parametrize("chi", [1e-3, 0.1, 1.0, 10.0, 100.0])
def test_h_rad_against_scipy_quadrature(chi):
    # h_rad = (1/(pi sqrt3)) int_0^1 B_gamma dxi, with SciPy's kv and quad
    def br(xi):
        d = 2 * xi / (3 * chi * (1 - xi))
        if d > 700:
            return 0.0
        ki = ki_scipy(1 / 3, d)
        return (2 + xi * xi / (1 - xi)) * sp.kv(2 / 3, d) - ki
    pts = [min(3 * chi * k, 0.5) for k in (1e-3, 1e-2, 0.1)]
    val = si.quad(br, 0, 1, points=sorted(set(pts)), epsrel=1e-10, limit=400)[0] / (math.pi * math.sqrt(3))
    assert O.h_rad(chi) == pytest.approx(val, rel=2e-8)


def test_h_rad_classical_photon_number():
    # classical synchrotron photon rate 5 alpha_f c gamma/(2 sqrt3 R) = alpha_f/(tau_c gamma) * 5chi/(2 sqrt3)
    for chi in (1e-6, 1e-5):
        assert O.h_rad(chi) / (5 * chi / (2 * math.sqrt(3))) == pytest.approx(1.0, abs=2e-5 * chi / 1e-5 + 1e-7)


def test_g_larmor_limit_and_first_correction():
    # P_rad -> P_cl (Larmor) and g = 1 - (55 sqrt3/16) chi + O(chi^2)
    c1 = 55 * math.sqrt(3) / 16
    for chi in (1e-6, 1e-5):
        g = O.g(chi)
        assert abs(g - 1) < 7 * chi
        assert (1 - g) / chi == pytest.approx(c1, rel=1e-4)


def test_rates_large_chi_limits():
    # Small-argument K_nu(d) ~ Gamma(nu)/2 (2/d)^nu with Beta integrals give
    #   h_rad -> 14 Gamma(2/3) 3^{-7/3} chi^{2/3}
    #   g     -> 16 Gamma(2/3) 3^{2/3}/81 chi^{-4/3}
    #   h_pair-> 15 3^{2/3} Gamma(2/3)^4/(28 pi^2) chi^{2/3}
    c_h = 14 * G23 * 3 ** (-7 / 3)
    c_g = 16 * G23 * 3 ** (2 / 3) / 81
    c_p = 15 * 3 ** (2 / 3) * G23 ** 4 / (28 * math.pi ** 2)
    prev = None
    for chi in (1e4, 1e6):
        r = (O.h_rad(chi) / (c_h * chi ** (2 / 3)), O.g(chi) / (c_g * chi ** (-4 / 3)),
             O.h_pair(chi) / (c_p * chi ** (2 / 3)))
        if prev is not None:  # converging
            assert all(abs(a - 1) < abs(b - 1) for a, b in zip(r, prev))
        prev = r
    assert all(abs(v - 1) < 3e-4 for v in prev)


def test_h_pair_small_chi_limit():
    # Breit-Wheeler in a weak field: h_pair -> (3/16) sqrt(3/2) chi exp(-8/(3chi))
    prev = None
    for chi in (0.05, 0.02, 0.01):
        r = O.h_pair(chi) / (3 / 16 * math.sqrt(1.5) * chi * math.exp(-8 / (3 * chi)))
        if prev is not None:
            assert abs(r - 1) < abs(prev - 1)
        prev = r
    assert abs(prev - 1) < 2.5e-3


def test_g_baier_katkov_fit():
    # published fit g ~ [1 + 4.8(1+chi) ln(1+1.7chi) + 2.44 chi^2]^{-2/3}, a few per cent
    for chi in np.logspace(-3, 2, 11):
        fit = (1 + 4.8 * (1 + chi) * math.log(1 + 1.7 * chi) + 2.44 * chi * chi) ** (-2 / 3)
        assert O.g(chi) == pytest.approx(fit, rel=0.02)


def test_cdf_endpoints_and_monotone():
    for chi in (1e-3, 1.0, 50.0):
        xs = [1e-9, 1e-4, 0.01, 0.2, 0.6, 0.95]
        c = [O.emit_cdf(chi, x) for x in xs]
        assert all(b >= a for a, b in zip(c, c[1:]))
        assert 0 <= c[0] < 2e-2 and c[-1] <= 1
        # K_{2/3}(delta) ~ delta^{-2/3} makes B_gamma ~ xi^{-2/3}, so P ~ xi^{1/3} at small xi
        lo = 1e-9 * chi
        assert O.emit_cdf(chi, lo / 1000) / O.emit_cdf(chi, lo) == pytest.approx(0.1, rel=1e-3)
    for chi in (0.1, 3.0):
        assert O.pair_cdf(chi, 0.5) == pytest.approx(0.5, abs=1e-13)   # symmetric spectrum


def test_emit_cdf_against_scipy():
    chi, xi = 1.0, 0.3
    def br(x):
        d = 2 * x / (3 * chi * (1 - x))
        ki = ki_scipy(1 / 3, d)
        return (2 + x * x / (1 - x)) * sp.kv(2 / 3, d) - ki
    num = si.quad(br, 0, xi, points=[1e-3, 1e-2], epsrel=1e-11, limit=400)[0]
    den = si.quad(br, 0, 1, points=[1e-3, 1e-2, xi], epsrel=1e-11, limit=400)[0]
    assert O.emit_cdf(chi, xi) == pytest.approx(num / den, rel=1e-8)


# ---------------------------------------------------------------- tables ----
def test_tables_rates_match_direct(oracle_tables):
    T = oracle_tables
    ne = T["emit_spec"]["n_chi"]
    chis = np.exp(np.linspace(math.log(1e-3), math.log(1e2), ne))
    for i in (0, 37, 90, ne - 1):
        assert math.exp(T["ln_hrad"][i]) == pytest.approx(O.h_rad(chis[i]), rel=1e-13)
        assert math.exp(T["ln_g"][i]) == pytest.approx(O.g(chis[i]), rel=1e-13)
    npc = T["pair_spec"]["n_chi"]
    pch = np.exp(np.linspace(math.log(1e-2), math.log(1e2), npc))
    for i in (0, 64, npc - 1):
        v = math.exp(T["pair_lnh"][i] - 8 / (3 * pch[i]))
        assert v == pytest.approx(O.h_pair(pch[i]), rel=1e-12)


def test_tables_quantiles_invert_cdf(oracle_tables):
    T = oracle_tables
    nq = T["emit_spec"]["n_q"]
    q = T["emit_q"].reshape(-1, nq)
    chis = np.exp(np.linspace(math.log(1e-3), math.log(1e2), q.shape[0]))
    for i in (0, 50, 127):
        for k in (0, 20, 63, 64, 110, 127):
            t = -18 + 36 * k / (nq - 1)
            r = 1 / (1 + math.exp(-t))
            c = O.emit_cdf(chis[i], math.exp(q[i, k]))
            assert c == pytest.approx(r, rel=1e-10, abs=1e-14)
    pq = T["pair_q"].reshape(-1, nq)
    pch = np.exp(np.linspace(math.log(1e-2), math.log(1e2), pq.shape[0]))
    for i in (0, 100):
        for k in (0, 40, 90, 127):
            t = -18 + 36 * k / (nq - 1)
            eta = 1 / (1 + math.exp(-pq[i, k]))
            assert O.pair_cdf(pch[i], eta) == pytest.approx(1 / (1 + math.exp(-t)), rel=1e-9, abs=1e-14)
        assert pq[i] == pytest.approx(-pq[i][::-1], abs=1e-9)          # eta <-> 1-eta symmetry


def test_table_sampling_mean_fraction(bound_tables):
    # E[xi] = (2/3) chi^2 g / h_rad from the definitions of g and h_rad;
    # 2e5 table samples with a stratified uniform grid of r.
    for chi in (0.1, 1.0, 5.0):
        exact = (2 / 3) * chi * chi * O.g(chi) / O.h_rad(chi)
        r = (np.arange(200_000) + 0.5) / 200_000
        m = np.mean([bound_tables.sample_xi(chi, float(v)) for v in r[::10]])
        assert m == pytest.approx(exact, rel=3e-3)


def test_table_sampling_ks_against_cdf(bound_tables):
    # sampled xi has the CDF of Eq. 7 to within the linear-table error (~1e-3)
    chi = 0.7
    rng = np.random.default_rng(7)
    r = rng.uniform(size=4000)
    xs = np.sort([bound_tables.sample_xi(chi, float(v)) for v in r])
    cdf = np.array([O.emit_cdf(chi, float(x)) for x in xs[::40]])
    emp = (np.arange(0, len(xs), 40) + 1) / len(xs)
    assert np.max(np.abs(cdf - emp)) < 0.03
