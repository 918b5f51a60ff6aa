"""Oracle runs of a workload, in the same step order as the GPU driver:
electrons, positrons, then the photons that existed when the step began.
Test infrastructure: calls only oracle/ and the seeded input generators."""
from __future__ import annotations

import numpy as np

from oracle import oracle as O
from paper_1311_1107_amd.workloads import LAMBDA_M, PlaneWave, Uniform, YeePulse


def oracle_run(wl, tabs: O.BoundTables, steps: int, photon_capacity=None, record_capacity=None,
               pair_capacity=None, rad_model=O.RAD_HYBRID, chi_switch=1e-3, gamma_photon_min=2.0,
               max_events=4, start=0, lazy_grid=False, compact_every=None, sort_every=0, variants=0, threads=0):
    n0 = len(wl.electrons["x"])
    cap_pair = pair_capacity if pair_capacity is not None else (n0 if wl.push_photons else 0)
    el = O.species_from(wl.electrons, capacity=n0 + cap_pair)
    O.init_tau(el, wl.seed)
    po = O.new_species(max(cap_pair, 1))
    ph = O.new_species(photon_capacity if photon_capacity is not None else 4 * n0) if wl.push_photons else None
    rec = O.new_species(record_capacity if record_capacity is not None else 4 * n0) if wl.record_photons else None
    uid_next = [n0]
    tally = O.Tally()
    f = wl.field
    if isinstance(f, PlaneWave):
        field = O.make_field(O.FIELD_PLANE_WAVE, a0=f.a0, n_periods=f.n_periods)
    elif isinstance(f, Uniform):
        field = O.make_field(O.FIELD_UNIFORM, E=f.E, B=f.B)
    for n in range(start, start + steps):
        if isinstance(f, YeePulse) and lazy_grid:
            field = O.make_field(O.FIELD_YEE_SEPARABLE, a0=f.a0, shape=f.shape, spacing=f.spacing,
                                 origin=f.origin, tperp=f.tperp, tpar=f.tpar[n])
        elif isinstance(f, YeePulse):
            grid = O.yee_fill_separable(f.shape, f.a0, f.tperp, f.tpar[n])
            field = O.make_field(O.FIELD_YEE, grid=grid, shape=f.shape, spacing=f.spacing, origin=f.origin)
        st = O.make_step(n * wl.dt, wl.dt, wl.seed, rad_model=rad_model, chi_switch=chi_switch,
                         gamma_photon_min=gamma_photon_min, chi_photon_push_min=wl.chi_photon_push_min,
                         max_events=max_events, variants=variants)
        n_ph0 = ph["n"] if ph is not None else 0
        O.push_emit(tabs, LAMBDA_M, -1.0, el, field, ph, rec, st, uid_next, tally, threads=threads)
        O.push_emit(tabs, LAMBDA_M, +1.0, po, field, ph, rec, st, uid_next, tally, threads=threads)
        if ph is not None:
            O.pair_create(tabs, LAMBDA_M, ph, field, el, po, st, uid_next, tally, n_limit=n_ph0, threads=threads)
        if sort_every and isinstance(f, YeePulse) and (n + 1) % sort_every == 0:
            for sp in (el, po, ph):
                if sp is not None:
                    O.sort_by_cell(sp, f.shape, f.spacing, f.origin)
    return {"electrons": O.view(el), "positrons": O.view(po),
            "photons": O.view(ph) if ph is not None else None,
            "recorded": O.view(rec) if rec is not None else None,
            "tally": tally.as_dict(), "uid_next": uid_next[0]}


def assert_species_match(got: dict, want: dict, rtol=1e-12, what="", exact_keys=("uid", "n_ev")):
    """Element-wise comparison: integers bit-exact; each momentum and position
    vector within rtol of max(norm, 1); weights exact."""
    n = len(want["x"])
    assert len(got["x"]) == n, f"{what}: count {len(got['x'])} != {n}"
    for k in exact_keys:
        if k in want:
            bad = np.nonzero(got[k] != want[k])[0]
            assert bad.size == 0, f"{what}: {k} differs at {bad[:5]} ({got[k][bad[:5]]} vs {want[k][bad[:5]]})"
    # vectors (position, momentum) relative to their norm, floored at 1
    for keys in (("x", "y", "z"), ("ux", "uy", "uz")):
        g = np.stack([np.asarray(got[k], np.float64) for k in keys], 1)
        w_ = np.stack([np.asarray(want[k], np.float64) for k in keys], 1)
        err = np.linalg.norm(g - w_, axis=1) / np.maximum(np.linalg.norm(w_, axis=1), 1.0)
        i = int(np.argmax(err)) if n else 0
        assert n == 0 or err[i] <= rtol, f"{what}: {keys} rel err {err[i]:.3e} at {i}: {g[i]!r} vs {w_[i]!r}"
    g, w_ = np.asarray(got["w"], np.float64), np.asarray(want["w"], np.float64)
    assert np.array_equal(g, w_), f"{what}: weights differ"
    if "tau" in want:
        g, w_ = got["tau"], want["tau"]
        err = np.abs(g - w_) / np.maximum(np.abs(w_), 1.0)
        assert n == 0 or err.max() <= rtol * 10, f"{what}: tau rel err {err.max():.3e}"


def _field_at_step(wl, n):
    f = wl.field
    if isinstance(f, PlaneWave):
        return O.make_field(O.FIELD_PLANE_WAVE, a0=f.a0, n_periods=f.n_periods)
    if isinstance(f, Uniform):
        return O.make_field(O.FIELD_UNIFORM, E=f.E, B=f.B)
    return O.make_field(O.FIELD_YEE_SEPARABLE, a0=f.a0, shape=f.shape, spacing=f.spacing, origin=f.origin,
                        tperp=f.tperp, tpar=f.tpar[n])


def _copy_state(s: dict) -> dict:
    return {k: np.array(v, copy=True) for k, v in s.items()}


def oracle_lepton_step(tabs, wl, n, state, charge=-1.0, push=True, record=True, **step_kw):
    """One oracle step of the leptons in `state` at step n; returns the
    leptons, the pushed and recorded photons and the tally."""
    m = len(state["x"])
    s = O.species_from(_copy_state(state))
    s["tau"][:m], s["n_ev"][:m] = state["tau"], state["n_ev"]
    ph = O.new_species(8 * m + 8) if push and wl.push_photons else None
    rec = O.new_species(8 * m + 8) if record and wl.record_photons else None
    kw = dict(chi_photon_push_min=wl.chi_photon_push_min)
    kw.update(step_kw)
    st = O.make_step(n * wl.dt, wl.dt, wl.seed, **kw)
    tally = O.Tally()
    un = [10**9]
    O.push_emit(tabs, LAMBDA_M, charge, s, _field_at_step(wl, n), ph, rec, st, un, tally)
    return {"leptons": O.view(s), "photons": O.view(ph) if ph is not None else None,
            "recorded": O.view(rec) if rec is not None else None, "tally": tally.as_dict()}


def lepton_margin_mask(tabs, wl, n, state, charge=-1.0, eps=1e-5, **step_kw):
    """True for each lepton of `state` whose step-n decisions lie within a
    relative eps of a threshold: the optical depth against W dt (rates times
    1 -+ eps), the Sokolov / Monte Carlo switch at chi_switch, the photon
    threshold gamma_photon_min and the pushed / recorded split at
    chi_photon_push_min (each times 1 -+ eps).  A reduced-precision step may
    take either side of such a decision.  Each lepton is stepped on its own:
    in an external field with id-keyed draws the leptons are independent."""
    base = dict(chi_switch=1e-3, gamma_photon_min=2.0, chi_photon_push_min=wl.chi_photon_push_min)
    base.update(step_kw)
    variants = [dict(base)]
    for s in (1 - eps, 1 + eps):
        variants.append(dict(base, rate_scale=s))
        for key in ("chi_switch", "gamma_photon_min", "chi_photon_push_min"):
            variants.append(dict(base, **{key: base[key] * s}))
    m = len(state["x"])
    mask = np.zeros(m, bool)
    field = _field_at_step(wl, n)
    for i in range(m):
        sig = None
        for kw in variants:
            one = {k: v[i:i + 1] for k, v in state.items()}
            s = O.species_from(_copy_state(one))
            s["tau"][:1], s["n_ev"][:1] = one["tau"], one["n_ev"]
            ph = O.new_species(8) if wl.push_photons else None
            rec = O.new_species(8) if wl.record_photons else None
            tally = O.Tally()
            O.push_emit(tabs, LAMBDA_M, charge, s, field, ph, rec, O.make_step(n * wl.dt, wl.dt, wl.seed, **kw),
                        [10**9], tally)
            c = tally.c
            this = (int(s["n_ev"][0]), bool(s["tau"][0] == one["tau"][0]), int(c[1]), int(c[2]), int(c[4]),
                    int(c[7]))
            if sig is None:
                sig = this
            elif this != sig:
                mask[i] = True
                break
    return mask


def oracle_photon_step(tabs, wl, n, photons, n_elec_cap, **step_kw):
    """One oracle photon step (pair creation and push) of `photons` at step n."""
    m = len(photons["x"])
    ph = O.species_from(_copy_state(photons))
    ph["tau"][:m], ph["n_ev"][:m] = photons["tau"], photons["n_ev"]
    el, po = O.new_species(n_elec_cap), O.new_species(n_elec_cap)
    st = O.make_step(n * wl.dt, wl.dt, wl.seed, **step_kw)
    tally = O.Tally()
    un = [10**9]
    O.pair_create(tabs, LAMBDA_M, ph, _field_at_step(wl, n), el, po, st, un, tally, n_limit=m)
    return {"photons": O.view(ph), "electrons": O.view(el), "positrons": O.view(po), "tally": tally.as_dict()}


def photon_margin_mask(tabs, wl, n, photons, eps=1e-5):
    """True for each photon whose pair decision at step n changes when the
    pair rate is scaled by 1 -+ eps (a reduced-precision step may take either
    side)."""
    keep = []
    for s in (1.0, 1 - eps, 1 + eps):
        out = oracle_photon_step(tabs, wl, n, photons, len(photons["x"]) + 1, rate_scale=s)
        keep.append(np.isin(photons["uid"], out["photons"]["uid"]))
    return (keep[0] != keep[1]) | (keep[0] != keep[2])


def relative_vector_error(got: dict, want: dict, keys) -> np.ndarray:
    g = np.stack([np.asarray(got[k], np.float64) for k in keys], 1)
    w_ = np.stack([np.asarray(want[k], np.float64) for k in keys], 1)
    return np.linalg.norm(g - w_, axis=1) / np.maximum(np.linalg.norm(w_, axis=1), 1.0)


def compare_with_sensitivity(got: dict, want: dict, pert: dict, species, within=0.99, report=print):
    """Counts, ids and event counters exact; momenta within 1e-12 of
    max(|u|, 1) for at least `within` of each species and all within 100x
    the oracle's own sensitivity to one ulp of the initial u_x (or 1e-12).
    Returns the fraction within 1e-12 per species."""
    fractions = {}
    for sp in species:
        g, w_, p_ = got[sp], want[sp], pert[sp]
        n = len(w_["x"])
        assert len(g["x"]) == n and len(p_["x"]) == n, sp
        assert np.array_equal(g["uid"], w_["uid"]) and np.array_equal(g["n_ev"], w_["n_ev"]), sp
        if n == 0:
            fractions[sp] = 1.0
            continue
        sens = relative_vector_error(p_, w_, ("ux", "uy", "uz"))
        tol = max(1e-12, 100.0 * float(sens.max()))
        err = relative_vector_error(g, w_, ("ux", "uy", "uz"))
        fractions[sp] = float(np.mean(err <= 1e-12))
        report(f"{sp}: n={n} max err {err.max():.2e}, {int(np.sum(err > 1e-12))} above 1e-12 "
               f"(fraction within {fractions[sp]:.5f}); oracle one-ulp self-sensitivity max {sens.max():.2e}")
        assert err.max() <= tol, f"{sp}: worst {err.max():.3e} > {tol:.3e}"
        assert fractions[sp] >= within, sp
    return fractions
