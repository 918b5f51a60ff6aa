"""GPU parity of the FP32 precision form against the FP64 oracle.

One step from identical state (the FP64 oracle state rounded to FP32, fed
to both sides): the leptons' and the photons' decisions must be identical
once the particles whose decisions lie within 1e-5 of a threshold are taken
out (the optical depth against W dt, the Sokolov / Monte Carlo switch, the
photon threshold and the pushed / recorded split; for photons the pair
decision).  Those are counted and printed.  Then every count and id is
exact, and momenta and positions of the leptons, the surviving photons and
the created pairs are within 1e-5 of max(|v|, 1); chi within 1e-4 (see
CHI_TOL) and each emitted photon's momentum within 1e-5 or twice its
chi_gamma error, whichever is larger.  Whole runs: the photon and pair spectra pass a two-sample KS
test at p > 0.01 against the FP64 oracle, with the same seed and with seed +
1000, and the radiation-off momentum error over a run is reported.
"""
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import oracle as O                      # noqa: E402
from paper_1311_1107_amd import binding as B        # noqa: E402
from paper_1311_1107_amd import device as D         # noqa: E402
from paper_1311_1107_amd import sim as S            # noqa: E402
from paper_1311_1107_amd import workloads as W      # noqa: E402

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from runners import (lepton_margin_mask, oracle_lepton_step, oracle_photon_step, oracle_run,  # noqa: E402
                     photon_margin_mask, relative_vector_error)

REALS = ("x", "y", "z", "ux", "uy", "uz", "w", "chi")


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible: the gpu tests need an MI355X")


@pytest.fixture(scope="module")
def gpu_oracle_tables(oracle_tables):
    _need_gpu()
    return D.Tables(O.EMIT_SPEC, O.PAIR_SPEC, arrays=oracle_tables)


@pytest.fixture(scope="module")
def gpu_spline_tables(oracle_tables):
    _need_gpu()
    return D.Tables(dict(O.EMIT_SPEC, interp=B.QED_INTERP_SPLINE), dict(O.PAIR_SPEC, interp=B.QED_INTERP_SPLINE),
                    arrays=oracle_tables)


def _tables_for(case, request):
    """(oracle tables, device tables) of a case; '_spline' cases read the
    quantile tables through the natural bicubic spline on both sides."""
    if case.endswith("_spline"):
        return request.getfixturevalue("spline_tables"), request.getfixturevalue("gpu_spline_tables")
    return request.getfixturevalue("bound_tables"), request.getfixturevalue("gpu_oracle_tables")


def _to_f32(state: dict) -> dict:
    out = {k: np.array(v, copy=True) for k, v in state.items()}
    for k in REALS:
        if k in out:
            out[k] = out[k].astype(np.float32).astype(np.float64)
    return out


def _take(state: dict, keep: np.ndarray) -> dict:
    return {k: np.ascontiguousarray(v[keep]) for k, v in state.items()}


def _gpu_field(wl, n):
    f = wl.field
    if isinstance(f, W.PlaneWave):
        return D.plane_wave(f.a0, f.n_periods), None
    if isinstance(f, W.Uniform):
        return D.uniform(f.E, f.B), None
    nx, ny, nz = f.shape
    grid = torch.zeros(6 * nx * ny * nz, dtype=torch.float32, device="cuda")
    tperp = torch.from_numpy(np.ascontiguousarray(f.tperp)).cuda()
    tpar = torch.from_numpy(np.ascontiguousarray(f.tpar[n])).cuda()
    B.qed_yee_fill_separable(grid.data_ptr(), nx, ny, nz, f.a0, tperp.data_ptr(), tpar.data_ptr())
    torch.cuda.synchronize()
    return D.yee(grid, f.shape, f.spacing, f.origin), (grid, tperp, tpar)


def _vec_close(got, want, keys, tol, what):
    err = relative_vector_error(got, want, keys)
    assert len(err) == 0 or err.max() <= tol, f"{what} {keys}: max {err.max():.3e}"
    return float(err.max()) if len(err) else 0.0


# chi is a cancellation where E and v x B nearly cancel (leptons moving with
# the wave): there FP32 rounding of the field and of u is amplified by about
# 2 gamma^2, so chi gets a looser bound than the momenta; its error is printed
CHI_TOL = 1e-4


def _chi_close(got, want, tol, what):
    if len(want["chi"]) == 0:
        return 0.0
    err = np.abs(np.asarray(got["chi"], np.float64) - want["chi"]) / np.maximum(np.abs(want["chi"]), 1e-300)
    assert err.max() <= tol, f"{what} chi: max {err.max():.3e}"
    return float(err.max())


# ------------------------------------------------------ lepton one step ----
def _lepton_case(name, tabs):
    if name == "plane":
        wl = W.plane_wave_beam(n=3000, box_lambda=2.0, steps=700, seed=51)
        k = 399
        mid = oracle_run(wl, tabs, k, record_capacity=16 * 3000)
    else:
        wl = W.yee_beam(n=2000, steps=260, seed=13, shape=(64, 32, 32), a0=800.0, gamma_median=4000.0,
                        x_range_lambda=(3.0, 5.0), r_max_lambda=1.0, x_center0=12.0)
        k = 120
        mid = oracle_run(wl, tabs, k, photon_capacity=160 * 2000, record_capacity=8 * 2000, pair_capacity=12 * 2000)
    return wl, k, mid


@pytest.mark.parametrize("case", ["plane", "yee", "plane_spline"])
def test_fp32_lepton_one_step(request, case):
    bound_tables, gpu_oracle_tables = _tables_for(case, request)
    wl, k, mid = _lepton_case(case.replace("_spline", ""), bound_tables)
    print(f"case: FP32 lepton one step, {case}, step {k}", flush=True)
    state = _to_f32(mid["electrons"])
    m0 = len(state["x"])
    mask = lepton_margin_mask(bound_tables, wl, k, state)
    state = _take(state, ~mask)
    m = len(state["x"])
    want = oracle_lepton_step(bound_tables, wl, k, state)
    assert want["tally"]["N_emit"] > 20

    el = D.Species(m, B.QED_F32)
    el.upload(state)
    ph = D.Species(8 * m + 8, B.QED_F32) if wl.push_photons else None
    rec = D.Species(8 * m + 8, B.QED_F32) if wl.record_photons else None
    ws = D.Workspace(8 * m + 8, max_leptons=m)
    tal = D.Tally((8 * m + 8) // 64 + 2)
    uid = torch.tensor([10**9], dtype=torch.int64, device="cuda")
    field, keep_alive = _gpu_field(wl, k)
    st = D.step(k * wl.dt, wl.dt, wl.seed, chi_photon_push_min=wl.chi_photon_push_min)
    B.qed_push_emit(gpu_oracle_tables.h, ws.h, B.qed_units_init(W.LAMBDA_M), -1.0, el.struct(), field,
                    ph.struct() if ph else None, rec.struct() if rec else None, tal.s, st, uid.data_ptr(), None)
    torch.cuda.synchronize()
    ws.status()
    got = el.download()
    t = tal.reduce()
    for key, v in want["tally"].items():
        if key.startswith("N_"):
            assert t[key] == v, (key, t[key], v)
    assert np.array_equal(got["uid"], want["leptons"]["uid"])
    assert np.array_equal(got["n_ev"], want["leptons"]["n_ev"])
    eu = _vec_close(got, want["leptons"], ("ux", "uy", "uz"), 1e-5, "electrons")
    ex = _vec_close(got, want["leptons"], ("x", "y", "z"), 1e-5, "electrons")
    report = [f"excluded {int(mask.sum())} of {m0} within 1e-5 of a threshold", f"electrons u {eu:.2e} x {ex:.2e}"]
    for name, sp in (("photons", ph), ("recorded", rec)):
        if sp is None:
            continue
        g, w_ = sp.download(), want[name]
        assert len(g["x"]) == len(w_["x"]), name
        assert np.array_equal(g["uid"], w_["uid"]), name
        if len(w_["x"]):
            # the photon energy is xi gamma with xi drawn from the quantile table at the
            # FP32 chi_e: where chi_e is ill-conditioned (see CHI_TOL) the energy follows
            # it, so each photon is held to 1e-5 or twice its chi_gamma error
            ec = _chi_close(g, w_, CHI_TOL, name)
            eu = relative_vector_error(g, w_, ("ux", "uy", "uz"))
            rc = np.abs(np.asarray(g["chi"], np.float64) - w_["chi"]) / np.maximum(np.abs(w_["chi"]), 1e-300)
            assert np.all(eu <= np.maximum(1e-5, 2.0 * rc)), f"{name} momenta beyond the chi-propagated bound"
            report.append(f"{name} ({len(w_['x'])}) u {eu.max():.2e} ({int(np.sum(eu > 1e-5))} above 1e-5) "
                          f"x {_vec_close(g, w_, ('x', 'y', 'z'), 1e-5, name):.2e} chi {ec:.2e}")
    print("FP32 one step: " + "; ".join(report), flush=True)
    assert mask.mean() < 0.01


# ------------------------------------------------------ photon one step ----
def _photon_case(name, tabs):
    if name == "constant_b":
        wl = W.constant_b(n=20_000, steps=60)
        k = 60
        mid = oracle_run(wl, tabs, k, rad_model=O.RAD_MC, photon_capacity=60 * 20_000, pair_capacity=20_000)
    else:
        wl = W.yee_beam(n=2000, steps=260, seed=13, shape=(64, 32, 32), a0=800.0, gamma_median=4000.0,
                        x_range_lambda=(3.0, 5.0), r_max_lambda=1.0, x_center0=12.0)
        k = 170
        mid = oracle_run(wl, tabs, k, photon_capacity=160 * 2000, record_capacity=8 * 2000, pair_capacity=12 * 2000)
    return wl, k, mid


@pytest.mark.parametrize("case", ["constant_b", "yee", "constant_b_spline"])
def test_fp32_photon_and_pair_one_step(request, case):
    """Photon step of the FP32 form (chi_gamma, pair rate, Breit-Wheeler pair
    creation, push) from identical state against the FP64 oracle."""
    bound_tables, gpu_oracle_tables = _tables_for(case, request)
    wl, k, mid = _photon_case(case.replace("_spline", ""), bound_tables)
    print(f"case: FP32 photon one step, {case}, step {k}", flush=True)
    phs = _to_f32(mid["photons"])
    m0 = len(phs["x"])
    mask = photon_margin_mask(bound_tables, wl, k, phs)
    phs = _take(phs, ~mask)
    m = len(phs["x"])
    want = oracle_photon_step(bound_tables, wl, k, phs, m + 1)
    n_pair = want["tally"]["N_pair"]
    assert n_pair >= 20

    ph = D.Species(m + 1, B.QED_F32)
    ph.upload(phs)
    el, po = D.Species(m + 1, B.QED_F32), D.Species(m + 1, B.QED_F32)
    ws = D.Workspace(m + 1)
    tal = D.Tally(m // 64 + 2)
    uid = torch.tensor([10**9], dtype=torch.int64, device="cuda")
    field, keep_alive = _gpu_field(wl, k)
    st = D.step(k * wl.dt, wl.dt, wl.seed, chi_photon_push_min=wl.chi_photon_push_min)
    B.qed_pair_create(gpu_oracle_tables.h, ws.h, B.qed_units_init(W.LAMBDA_M), ph.struct(), field, el.struct(),
                      po.struct(), tal.s, st, uid.data_ptr(), None)
    B.qed_compact(ws.h, ph.struct(), None)
    torch.cuda.synchronize()
    ws.status()
    t = tal.reduce()
    assert t["N_pair"] == n_pair and t["N_phstep"] == want["tally"]["N_phstep"]
    report = [f"excluded {int(mask.sum())} of {m0} photons within 1e-5 of the pair decision", f"{n_pair} pairs"]
    g = ph.download()
    assert np.array_equal(g["uid"], want["photons"]["uid"])
    report.append(f"photons x {_vec_close(g, want['photons'], ('x', 'y', 'z'), 1e-5, 'photons'):.2e}")
    for name, sp in (("electrons", el), ("positrons", po)):
        g, w_ = sp.download(), want[name]
        assert len(g["x"]) == n_pair and np.array_equal(g["uid"], w_["uid"]), name
        report.append(f"{name} u {_vec_close(g, w_, ('ux', 'uy', 'uz'), 1e-5, name):.2e} "
                      f"x {_vec_close(g, w_, ('x', 'y', 'z'), 1e-5, name):.2e} chi {_chi_close(g, w_, CHI_TOL, name):.2e}")
    print("FP32 photon step: " + "; ".join(report), flush=True)
    assert mask.mean() < 0.01


# ------------------------------------------------------------ whole runs ----
def test_fp32_pair_spectrum_ks(gpu_oracle_tables, bound_tables):
    """The constant-B cascade of Sec. 4 (1e4 electrons, 120 steps, every photon
    pushed and tested for pairs) in the FP32 form against the FP64 oracle:
    the gamma spectrum of the created electrons and positrons, two-sample KS."""
    from scipy.stats import ks_2samp
    n0 = 10_000
    wl = W.constant_b(n=n0, steps=120)
    caps = dict(photon_capacity=120 * n0, pair_capacity=8 * n0)
    want = oracle_run(wl, bound_tables, wl.steps, rad_model=O.RAD_MC, **caps)

    def pair_gamma(r):
        e = r["electrons"]
        created = e["uid"] >= n0
        u = [np.concatenate([np.asarray(e[k], np.float64)[created], np.asarray(r["positrons"][k], np.float64)])
             for k in ("ux", "uy", "uz")]
        return np.sqrt(1.0 + u[0] ** 2 + u[1] ** 2 + u[2] ** 2)

    g_w = pair_gamma(want)
    assert len(g_w) > 1000
    for seed in (wl.seed, wl.seed + 1000):
        wl_s = W.constant_b(n=n0, steps=120)
        wl_s.seed = seed
        run = S.Run(wl_s, prec=B.QED_F32, tables=gpu_oracle_tables, rad_model=B.QED_RAD_MC, compact_every=5,
                    **caps)
        run.run(wl.steps)
        run.ws.status()
        g_g = pair_gamma(run.result())
        p = ks_2samp(g_g, g_w).pvalue
        print(f"FP32 pair spectrum KS seed {seed}: p = {p:.3g} ({len(g_g)} vs {len(g_w)} leptons)", flush=True)
        assert p > 0.01


def test_fp32_reduced_cascade_ks(gpu_oracle_tables, bound_tables):
    """The high-chi cascade (a0 = 1000 plane wave against gamma0 = 1e4
    electrons, 500 steps, photons with chi_gamma < 0.2 not stored) reduced to
    5000 electrons, in the FP32 form against the FP64 oracle: the gamma
    spectra of the created pairs, of the surviving photons and of all
    electrons pass a two-sample KS test, with the same seed and with seed +
    1000; pair and emission counts agree within 3 %.  The oracle creates
    about 3e4 pairs here."""
    from scipy.stats import ks_2samp
    n0 = 5000
    wl = W.cascade_beam(n=n0, steps=500)
    caps = dict(photon_capacity=200 * n0, pair_capacity=20 * n0)
    want = oracle_run(wl, bound_tables, wl.steps, compact_every=1, **caps)
    wt = want["tally"]
    assert wt["N_pair"] > 10_000 and wt["N_overflow"] == 0

    def gammas(sp, mask=None):
        u = [np.asarray(sp[k], np.float64) for k in ("ux", "uy", "uz")]
        if mask is not None:
            u = [c[mask] for c in u]
        return np.sqrt(1.0 + u[0] ** 2 + u[1] ** 2 + u[2] ** 2)

    def spectra(r):
        e, po, ph = r["electrons"], r["positrons"], r["photons"]
        created = np.asarray(e["uid"]) >= n0
        pair = np.concatenate([gammas(e, created), gammas(po)])
        k = [np.asarray(ph[c], np.float64) for c in ("ux", "uy", "uz")]
        return {"pairs": pair, "photons": np.sqrt(k[0] ** 2 + k[1] ** 2 + k[2] ** 2), "electrons": gammas(e)}

    sw = spectra(want)
    for seed in (wl.seed, wl.seed + 1000):
        wl_s = W.cascade_beam(n=n0, steps=500, seed=wl.seed)
        wl_s.seed = seed
        run = S.Run(wl_s, prec=B.QED_F32, tables=gpu_oracle_tables, compact_every=1, **caps)
        run.run(wl.steps)
        run.ws.status()
        t = run.tally.reduce()
        sg = spectra(run.result())
        dn = {k: t[k] / wt[k] - 1.0 for k in ("N_pair", "N_emit")}
        ps = {k: ks_2samp(sg[k], sw[k]).pvalue for k in sw}
        print(f"FP32 reduced cascade seed {seed}: " + ", ".join(f"{k} {v:+.2%}" for k, v in dn.items()) + "; KS "
              + ", ".join(f"{k} p = {v:.3g} ({len(sg[k])} vs {len(sw[k])})" for k, v in ps.items()), flush=True)
        assert all(abs(v) < 0.03 for v in dn.values()), dn
        assert all(v > 0.01 for v in ps.values()), ps


def test_fp32_radiation_off_momentum_error(gpu_oracle_tables, bound_tables):
    """With radiation off (Lorentz force only) the FP32 form is deterministic:
    its momentum error against the FP64 oracle over a 700-step run through the
    a0 = 100 pulse is reported (rounding of x and u to FP32 each step; the
    phase is reduced in FP64)."""
    wl = W.plane_wave_beam(n=3000, box_lambda=2.0, steps=700, seed=52)
    want = oracle_run(wl, bound_tables, wl.steps, rad_model=O.RAD_NONE, record_capacity=8)
    run = S.Run(wl, prec=B.QED_F32, tables=gpu_oracle_tables, rad_model=B.QED_RAD_NONE, record_capacity=8)
    run.run(wl.steps)
    got = run.result()["electrons"]
    eu = relative_vector_error(got, want["electrons"], ("ux", "uy", "uz"))
    ex = relative_vector_error(got, want["electrons"], ("x", "y", "z"))
    print(f"FP32 radiation-off run, 700 steps: momentum rel err max {eu.max():.2e} median {np.median(eu):.2e}; "
          f"position max {ex.max():.2e}", flush=True)
    assert eu.max() <= 1e-3 and ex.max() <= 1e-4
