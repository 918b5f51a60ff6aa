"""Oracle runs of a workload, in the same step order as the GPU driver:
electrons, positrons, then the photons that existed when the step began.
Test infrastructure: calls only oracle/ and the seeded input generators."""
from __future__ import annotations

import numpy as np

from oracle import oracle as O
from paper_1311_1107_amd.workloads import LAMBDA_M, PlaneWave, Uniform, YeePulse


def oracle_run(wl, tabs: O.BoundTables, steps: int, photon_capacity=None, record_capacity=None,
               pair_capacity=None, rad_model=O.RAD_HYBRID, chi_switch=1e-3, gamma_photon_min=2.0,
               max_events=4, start=0, lazy_grid=False, compact_every=None, sort_every=0, variants=0):
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
        O.push_emit(tabs, LAMBDA_M, -1.0, el, field, ph, rec, st, uid_next, tally)
        O.push_emit(tabs, LAMBDA_M, +1.0, po, field, ph, rec, st, uid_next, tally)
        if ph is not None:
            O.pair_create(tabs, LAMBDA_M, ph, field, el, po, st, uid_next, tally, n_limit=n_ph0)
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
