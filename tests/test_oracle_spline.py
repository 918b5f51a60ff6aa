"""Pins of the oracle's spline option for the quantile tables (CPU only).

The paper samples the photon fraction of Eq. 7 and the pair split of Eq. 3
by inverting their CDFs but fixes no interpolation between tabulated
quantiles.  With interp = 1 the oracle reads a table through the
tensor-product natural cubic spline (zero second derivative at the table's
edges) in (ln chi, logit r).  Pinned against SciPy's natural cubic splines
applied row by row and then along ln chi, and against the CDFs themselves
computed by quadrature at the sampled point: the spline must invert them to
1e-5, where bilinear reading misses by about 1e-3.
"""
import math

import numpy as np
import pytest
from scipy.interpolate import CubicSpline

from oracle import oracle as O


def _toy(n_chi, n_q, seed, chi=(0.01, 10.0), logit_max=4.0):
    rng = np.random.default_rng(seed)
    q_e = -np.abs(rng.normal(size=(n_chi, n_q))) - 5.0     # ln xi well below 0: xi = exp(q) is not clamped
    q_p = rng.normal(size=(n_chi, n_q))
    spec = dict(chi_min=chi[0], chi_max=chi[1], n_chi=n_chi, n_q=n_q, logit_max=logit_max, interp=1)
    tabs = {"ln_hrad": np.zeros(n_chi), "ln_g": np.zeros(n_chi), "emit_q": q_e.reshape(-1),
            "pair_lnh": np.zeros(n_chi), "pair_q": q_p.reshape(-1), "emit_spec": spec, "pair_spec": dict(spec)}
    return O.BoundTables(tabs), q_e, q_p, spec


def _scipy_tensor(q, lnc, tk, c, t):
    rows = np.array([CubicSpline(tk, q[i], bc_type="natural")(t) for i in range(len(lnc))])
    return float(CubicSpline(lnc, rows, bc_type="natural")(c))


def _logit(p):
    return math.log(p) - math.log1p(-p)


@pytest.mark.parametrize("shape", [(7, 9), (5, 12), (3, 3)])
def test_spline_is_scipy_natural_tensor_product(shape):
    n_chi, n_q = shape
    bt, q_e, q_p, spec = _toy(n_chi, n_q, seed=n_chi * 100 + n_q)
    lnc = np.linspace(math.log(spec["chi_min"]), math.log(spec["chi_max"]), n_chi)
    tk = np.linspace(-spec["logit_max"], spec["logit_max"], n_q)
    rng = np.random.default_rng(5)
    for _ in range(60):
        c = rng.uniform(lnc[0], lnc[-1])
        t = rng.uniform(tk[0], tk[-1])
        r = 1.0 / (1.0 + math.exp(-t))
        got_e = math.log(bt.sample_xi(math.exp(c), r))
        got_p = _logit(bt.sample_eta(math.exp(c), r))
        assert got_e == pytest.approx(_scipy_tensor(q_e, lnc, tk, c, t), abs=1e-11)
        assert got_p == pytest.approx(_scipy_tensor(q_p, lnc, tk, c, t), abs=1e-11)


def test_curvature_tables_are_scipy_second_derivatives():
    n_chi, n_q = 6, 10
    _, q, _, spec = _toy(n_chi, n_q, seed=9)
    h_c = (math.log(spec["chi_max"]) - math.log(spec["chi_min"])) / (n_chi - 1)
    h_t = 2.0 * spec["logit_max"] / (n_q - 1)
    m = O.quantile_spline(q, n_chi, n_q, h_c, h_t)
    lnc = np.arange(n_chi) * h_c
    tk = np.arange(n_q) * h_t
    want_tt = np.array([CubicSpline(tk, q[i], bc_type="natural")(tk, 2) for i in range(n_chi)])
    want_cc = np.array([CubicSpline(lnc, q[:, j], bc_type="natural")(lnc, 2) for j in range(n_q)]).T
    want_cctt = np.array([CubicSpline(tk, want_cc[i], bc_type="natural")(tk, 2) for i in range(n_chi)])
    np.testing.assert_allclose(m[0], want_tt, atol=1e-10)
    np.testing.assert_allclose(m[1], want_cc, atol=1e-10)
    np.testing.assert_allclose(m[2], want_cctt, atol=1e-10)


def test_spline_through_nodes_and_clamped_outside():
    bt, q_e, q_p, spec = _toy(7, 9, seed=2)
    lnc = np.linspace(math.log(spec["chi_min"]), math.log(spec["chi_max"]), 7)
    tk = np.linspace(-spec["logit_max"], spec["logit_max"], 9)
    for i in (0, 3, 6):
        for j in (0, 4, 8):
            r = 1.0 / (1.0 + math.exp(-tk[j]))
            assert _logit(bt.sample_eta(math.exp(lnc[i]), r)) == pytest.approx(q_p[i, j], abs=1e-11)
    # chi below and above the table read the edge rows; r beyond the last level the edge column
    r = 0.3
    assert bt.sample_eta(spec["chi_min"] / 10, r) == bt.sample_eta(spec["chi_min"], r)
    assert bt.sample_eta(spec["chi_max"] * 10, r) == pytest.approx(bt.sample_eta(spec["chi_max"], r), rel=1e-14)
    top = 1.0 / (1.0 + math.exp(-spec["logit_max"]))
    assert bt.sample_eta(0.1, 1.0 - 1e-12) == pytest.approx(bt.sample_eta(0.1, top), rel=1e-14)


def _bound(tables, interp):
    t = dict(tables)
    t["emit_spec"] = dict(tables["emit_spec"], interp=interp)
    t["pair_spec"] = dict(tables["pair_spec"], interp=interp)
    return O.BoundTables(t)


@pytest.mark.parametrize("kind", ["emit", "pair"])
def test_spline_inverts_the_cdf_to_1e5(oracle_tables, kind):
    """Sampled xi (Eq. 7) or eta (pair spectrum) at random chi over the table
    range and levels r with logit r in [-18, 18]: the CDF at the sample,
    computed by quadrature, is r within 1e-5 with the spline; bilinear reading
    misses by more than 1e-4 somewhere on the same points."""
    spline, linear = _bound(oracle_tables, 1), _bound(oracle_tables, 0)
    spec = oracle_tables[kind + "_spec"]
    rng = np.random.default_rng(17 if kind == "emit" else 18)
    n = 90 if kind == "emit" else 200
    worst_s = worst_l = 0.0
    for k in range(n):
        chi = math.exp(rng.uniform(math.log(spec["chi_min"]), math.log(spec["chi_max"])))
        t = rng.uniform(-18.0, 18.0) if k % 3 else rng.uniform(-3.0, 3.0)
        r = 1.0 / (1.0 + math.exp(-t))
        if kind == "emit":
            cs, cl = O.emit_cdf(chi, spline.sample_xi(chi, r)), O.emit_cdf(chi, linear.sample_xi(chi, r))
        else:
            cs, cl = O.pair_cdf(chi, spline.sample_eta(chi, r)), O.pair_cdf(chi, linear.sample_eta(chi, r))
        worst_s, worst_l = max(worst_s, abs(cs - r)), max(worst_l, abs(cl - r))
    assert worst_s <= 1e-5, worst_s
    assert worst_l > 1e-4, worst_l
