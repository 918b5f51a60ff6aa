"""The oracle's merging of super-particles (coalescence) against what fixes it.

The paper requires only that a merge keep energy and momentum.  The oracle
merges each group of (cell, energy bin, direction bin) of at least min_group
members into two particles.  Checked here:
  * the grouping against an exact brute-force partition (rational
    arithmetic, inputs away from bin edges), including which particles are
    kept unchanged and the output order;
  * per merged group: weight, momentum and energy kept, equal weights and
    equal energies of the two new particles, their momenta symmetric about
    P, the split in the plane of P and P x e_(d+1), the weighted mean
    position;
  * closed forms: identical particles merge into copies of themselves, and
    two photons (10, +-1, 0) into (10, 0, +-1);
  * leptons: the new |u| = sqrt((E/W)^2 - 1) never needs clamping (Jensen);
  * decayed photons dropped, ids and optical depths of the new particles,
    the capacity refusal.
"""
from fractions import Fraction

import numpy as np
import pytest

from oracle import oracle as O
from paper_1311_1107_amd import workloads as W

SHAPE, SPACING, ORIGIN = (4, 3, 5), (0.5, 0.5, 0.5), (-1.0, 0.0, 0.5)
OCT_MIN, N_OCT = -8, 48


def spec(massive=False, sub_bins=2, n_dir=3, min_group=3, n_oct=N_OCT):
    return O.merge_spec(ORIGIN, SPACING, SHAPE, massive, OCT_MIN, n_oct, sub_bins, n_dir, min_group)


def _exact_key(p, i, sp):
    """(cell, momentum bin, face axis) in exact arithmetic, or None if the
    particle is kept as it is; raises ValueError near a bin edge."""
    eps = Fraction(1, 10 ** 9)
    nx, ny, nz = SHAPE
    idx = []
    for c, (o, h, nn) in enumerate(zip(ORIGIN, SPACING, SHAPE)):
        g = (Fraction(float(p["xyz"[c]][i])) - Fraction(o)) / Fraction(h)
        if abs(g - round(g)) < eps:
            raise ValueError("cell edge")
        idx.append(int(np.floor(float(g))) if g >= 0 else -1)
    if not (0 <= idx[0] < nx and 0 <= idx[1] < ny and 0 <= idx[2] < nz):
        return None
    if not (p["w"][i] > 0):
        return None
    u = [Fraction(float(p[k][i])) for k in ("ux", "uy", "uz")]
    u2 = sum(v * v for v in u)
    if u2 == 0:
        return None
    # octave: 2^e <= u2 < 2^(e+1)
    e = u2.numerator.bit_length() - u2.denominator.bit_length()
    while Fraction(2) ** e > u2:
        e -= 1
    while Fraction(2) ** (e + 1) <= u2:
        e += 1
    oc = e - sp.octave_min
    if not (0 <= oc < sp.n_octaves):
        return None
    t = (u2 / Fraction(2) ** e - 1) * sp.sub_bins              # in [0, sub_bins)
    if abs(t - round(t)) < eps * sp.sub_bins or abs(u2 / Fraction(2) ** e - 1) < eps:
        raise ValueError("energy edge")
    sub = int(np.floor(float(t)))
    a = [abs(v) for v in u]
    d = 0
    if a[1] > a[d]:
        d = 1
    if a[2] > a[d]:
        d = 2
    if sorted(a)[-1] - sorted(a)[-2] < eps * a[d]:
        raise ValueError("face edge")
    face = 2 * d + (1 if u[d] < 0 else 0)
    ij = []
    for c in ((d + 1) % 3, (d + 2) % 3):
        s = (u[c] / a[d] + 1) * Fraction(sp.n_dir, 2)
        if abs(s - round(s)) < eps * sp.n_dir:
            raise ValueError("direction edge")
        ij.append(min(int(np.floor(float(s))), sp.n_dir - 1))
    cell = (idx[0] * ny + idx[1]) * nz + idx[2]
    mbin = (((oc * sp.sub_bins + sub) * 6 + face) * sp.n_dir + ij[0]) * sp.n_dir + ij[1]
    return cell, mbin, d


def _cloud(n, seed, photons=True):
    """merge_cloud (3 beams, |u| in 100 .. 150) with entries near a bin
    edge moved until none is."""
    p = W.merge_cloud(n, seed, photons=photons, shape=SHAPE, spacing=SPACING, origin=ORIGIN, n_beams=3,
                      spread=0.03, e_range=(100.0, 150.0))
    sp = spec(massive=not photons)
    r = np.random.default_rng(seed + 100)
    for i in range(n):
        for _ in range(50):
            try:
                _exact_key(p, i, sp)
                break
            except ValueError:
                for k in ("x", "y", "z"):
                    p[k][i] += r.uniform(-1e-3, 1e-3)
                for k in ("ux", "uy", "uz"):
                    p[k][i] *= 1.0 + r.uniform(-1e-3, 1e-3)
        else:
            raise AssertionError("could not move a particle off the bin edges")
    return p


def _expected(p, sp, photons):
    """Exact partition: ordered list of (kind, members, face axis) where kind
    is 'merge' or 'keep'."""
    n = len(p["x"])
    groups, kept = {}, []
    for i in range(n):
        if photons and np.isinf(p["tau"][i]) and p["tau"][i] > 0:
            continue
        k = _exact_key(p, i, sp)
        if k is None:
            kept.append(i)
        else:
            groups.setdefault((k[0], k[1]), (k[2], []))[1].append(i)
    out = []
    for key in sorted(groups):
        d, mem = groups[key]
        out.append(("merge" if len(mem) >= sp.min_group else "keep", mem, d))
    out.extend(("keep", [i], None) for i in kept)
    return out


def _energy(u, massive):
    u2 = (u * u).sum(axis=-1)
    return np.sqrt(1.0 + u2) if massive else np.sqrt(u2)


def _check_merge(p, res, sp, photons, uid0, seed):
    massive = not photons
    got = O.view(res)
    exp = _expected(p, sp, photons)
    o = 0
    fields = ("x", "y", "z", "ux", "uy", "uz", "tau", "w", "chi", "uid", "n_ev")
    n_merged = 0
    new = []
    for kind, mem, d in exp:
        if kind == "keep":
            for i in mem:
                for f in fields:
                    assert got[f][o] == p[f][i], (f, o, i)
                o += 1
            continue
        n_merged += 1
        mem = np.array(mem)
        w = p["w"][mem]
        u = np.stack([p["ux"][mem], p["uy"][mem], p["uz"][mem]], axis=1)
        Wt = w.sum()
        P = (w[:, None] * u).sum(axis=0)
        E = (w * _energy(u, massive)).sum()
        ua = np.array([got["ux"][o], got["uy"][o], got["uz"][o]])
        ub = np.array([got["ux"][o + 1], got["uy"][o + 1], got["uz"][o + 1]])
        wa, wb = got["w"][o], got["w"][o + 1]
        scale = np.abs(w[:, None] * u).sum()
        assert wa == wb and abs(wa + wb - Wt) <= 1e-13 * Wt
        assert np.allclose(wa * ua + wb * ub, P, rtol=0, atol=1e-12 * scale), "momentum"
        ea, eb = _energy(ua, massive), _energy(ub, massive)
        assert abs(wa * ea + wb * eb - E) <= 1e-12 * E, "energy"
        assert abs(ea - eb) <= 1e-12 * ea
        # symmetric about P, split along P x e_(d+1)
        diff = ua - ub
        assert abs(diff @ P) <= 1e-10 * np.linalg.norm(diff) * np.linalg.norm(P) + 1e-300
        assert abs(diff[(d + 1) % 3]) <= 1e-12 * np.linalg.norm(ua)
        for c, f in enumerate(("x", "y", "z")):
            m = (w * p[f][mem]).sum() / Wt
            assert got[f][o] == got[f][o + 1] and abs(got[f][o] - m) <= 1e-13 * (abs(m) + 1)
        assert abs(got["chi"][o] - (w * p["chi"][mem]).sum() / Wt) <= 1e-13 * 2
        for j in (o, o + 1):
            assert got["uid"][j] == uid0 + j and got["n_ev"][j] == 0
            new.append(j)
        o += 2
    assert o == res["n"]
    # fresh optical depths: the initial draw of each new id
    new = np.array(new, dtype=np.int64)
    t = O.species_from({k: got[k][new] for k in fields})
    O.init_tau(t, seed)
    assert np.array_equal(O.view(t)["tau"], got["tau"][new])
    return n_merged


@pytest.mark.parametrize("photons", [True, False])
@pytest.mark.parametrize("n,seed", [(0, 1), (1, 2), (7, 3), (400, 4), (3000, 5)])
def test_merge_matches_exact_partition(photons, n, seed):
    p = _cloud(n, seed, photons)
    sp = spec(massive=not photons)
    res, nxt = O.merge(sp, O.species_from(p), seed=11, uid_next=10 ** 6)
    assert nxt == 10 ** 6 + res["n"]
    n_merged = _check_merge(p, res, sp, photons, 10 ** 6, 11)
    if n >= 3000:
        assert n_merged > 100 and res["n"] < 0.8 * n


@pytest.mark.parametrize("sub_bins,n_dir,min_group", [(1, 1, 2), (4, 2, 3), (16, 5, 8), (64, 8, 4)])
def test_merge_bin_layouts(sub_bins, n_dir, min_group):
    p = W.merge_cloud(2000, 21, photons=True, shape=SHAPE, spacing=SPACING, origin=ORIGIN)
    sp = spec(sub_bins=sub_bins, n_dir=n_dir, min_group=min_group)
    r = np.random.default_rng(5)
    for i in range(len(p["x"])):
        for _ in range(50):
            try:
                _exact_key(p, i, sp)
                break
            except ValueError:
                for k in ("ux", "uy", "uz", "x", "y", "z"):
                    p[k][i] *= 1.0 + r.uniform(-1e-3, 1e-3)
    res, _ = O.merge(sp, O.species_from(p), seed=3, uid_next=7)
    _check_merge(p, res, sp, True, 7, 3)


@pytest.mark.parametrize("photons", [True, False])
def test_merge_conserves_totals(photons):
    p = W.merge_cloud(20000, 8, photons=photons, shape=SHAPE, spacing=SPACING, origin=ORIGIN, e_range=(10.0, 100.0))
    live = ~(np.isinf(p["tau"]) & (p["tau"] > 0)) if photons else np.ones(len(p["x"]), bool)
    res, _ = O.merge(spec(massive=not photons, sub_bins=1, n_dir=2), O.species_from(p), seed=1, uid_next=0)
    g = O.view(res)
    u0 = np.stack([p["ux"], p["uy"], p["uz"]], 1)[live]
    u1 = np.stack([g["ux"], g["uy"], g["uz"]], 1)
    w0, w1 = p["w"][live], g["w"]
    assert res["n"] < 0.5 * live.sum()
    assert abs(w1.sum() - w0.sum()) <= 1e-12 * w0.sum()
    scale = np.abs(w0[:, None] * u0).sum()
    assert np.allclose((w1[:, None] * u1).sum(0), (w0[:, None] * u0).sum(0), rtol=0, atol=1e-12 * scale)
    e0 = (w0 * _energy(u0, not photons)).sum()
    assert abs((w1 * _energy(u1, not photons)).sum() - e0) <= 1e-12 * e0


def test_merge_identical_particles_closed_form():
    n = 10
    p = {"x": np.full(n, 0.3), "y": np.full(n, 0.7), "z": np.full(n, 1.1),
         "ux": np.full(n, 3.0), "uy": np.full(n, -40.0), "uz": np.full(n, 12.0),
         "tau": np.ones(n), "w": np.full(n, 0.25), "chi": np.full(n, 0.5),
         "uid": np.arange(n, dtype=np.uint64)}
    for massive in (False, True):
        res, nxt = O.merge(spec(massive=massive), O.species_from(p), seed=2, uid_next=100)
        g = O.view(res)
        assert res["n"] == 2 and nxt == 102
        for j in range(2):
            assert np.allclose([g["ux"][j], g["uy"][j], g["uz"][j]], [3.0, -40.0, 12.0], rtol=1e-13, atol=0)
            assert g["w"][j] == 1.25
            assert np.allclose([g["x"][j], g["y"][j], g["z"][j]], [0.3, 0.7, 1.1], rtol=1e-15)


def test_merge_two_photons_closed_form():
    # (10, +-1, 0), weights 1: P = (20, 0, 0), E = 2 sqrt(101), face axis x,
    # split along P x e_y = z: the new momenta are (10, 0, +-1)
    p = {"x": np.array([0.1, 0.2]), "y": np.array([0.1, 0.1]), "z": np.array([0.6, 0.6]),
         "ux": np.array([10.0, 10.0]), "uy": np.array([1.0, -1.0]), "uz": np.zeros(2),
         "tau": np.ones(2), "w": np.ones(2), "chi": np.zeros(2), "uid": np.arange(2, dtype=np.uint64)}
    res, _ = O.merge(spec(n_dir=1, min_group=2), O.species_from(p), seed=2, uid_next=0)
    g = O.view(res)
    assert res["n"] == 2
    assert np.allclose(np.stack([g["ux"], g["uy"], g["uz"]], 1), [[10, 0, 1], [10, 0, -1]], rtol=0, atol=1e-13)
    assert g["x"][0] == pytest.approx(0.15, abs=1e-16)


def test_merge_leptons_jensen():
    # one cell, one bin: |u| spread over 4 .. 5.6 (one octave of |u|^2); |u_new| =
    # sqrt((E/W)^2 - 1) is at least the weighted mean |u|, so cos(theta) <= 1
    # without clamping, and the new gamma is E/W
    r = np.random.default_rng(4)
    n = 200
    d = np.array([1.0, 0.2, -0.1]) + 0.1 * r.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    u = d * r.uniform(4.0, 5.6, n)[:, None]
    w = r.uniform(0.1, 1.0, n)
    p = {"x": np.full(n, 0.1), "y": np.full(n, 0.1), "z": np.full(n, 0.6), "ux": u[:, 0].copy(),
         "uy": u[:, 1].copy(), "uz": u[:, 2].copy(), "tau": np.ones(n), "w": w, "chi": np.zeros(n)}
    sp = spec(massive=True, n_dir=1, sub_bins=1, n_oct=64)
    sp.octave_min = -40
    res, _ = O.merge(sp, O.species_from(p), seed=2, uid_next=0)
    g = O.view(res)
    assert res["n"] == 2
    gam = (w * np.sqrt(1 + (u * u).sum(1))).sum() / w.sum()
    un = np.sqrt(gam * gam - 1)
    assert (w * np.linalg.norm(u, axis=1)).sum() / w.sum() <= un
    P = (w[:, None] * u).sum(0)
    assert np.linalg.norm(P) < w.sum() * un
    for j in range(2):
        assert np.sqrt(1 + g["ux"][j] ** 2 + g["uy"][j] ** 2 + g["uz"][j] ** 2) == pytest.approx(gam, rel=1e-13)


def test_merge_nothing_to_merge_is_a_stable_reorder():
    p = W.merge_cloud(500, 6, photons=False, shape=SHAPE, spacing=SPACING, origin=ORIGIN)
    res, nxt = O.merge(spec(massive=True, min_group=10 ** 6), O.species_from(p), seed=1, uid_next=5)
    g = O.view(res)
    assert res["n"] == 500 and nxt == 505
    assert sorted(g["uid"].tolist()) == sorted(p["uid"].tolist())
    pos = {int(u): i for i, u in enumerate(p["uid"])}
    for j in range(500):
        i = pos[int(g["uid"][j])]
        for f in ("x", "ux", "tau", "w", "chi", "n_ev"):
            assert g[f][j] == p[f][i]


def test_merge_drops_decayed_photons_and_refuses_small_destination():
    p = W.merge_cloud(300, 7, photons=True, shape=SHAPE, spacing=SPACING, origin=ORIGIN)
    dead = np.isinf(p["tau"])
    res, _ = O.merge(spec(min_group=10 ** 6), O.species_from(p), seed=1, uid_next=0)
    assert res["n"] == 300 - dead.sum()
    assert not np.isinf(O.view(res)["tau"]).any()
    with pytest.raises(ValueError):
        O.merge(spec(min_group=10 ** 6), O.species_from(p), seed=1, uid_next=0, capacity=int(res["n"]) - 1)


def test_cascade_with_photon_merging_follows_kinetic_equations(bound_tables):
    """The Sec. 4 constant-B cascade in the oracle (3000 electrons) with the
    photons merged every 10 steps once they pass 5 % of a 160-per-electron
    buffer: the species' numbers, energies and mean chi stay on the solution
    of the kinetic equations (Eqs. 9-10) within 4 / sqrt(N_eff) + 2 %, N_eff
    the effective number of super-particles (sum w)^2 / sum w^2."""
    import math

    from oracle import kinetic as K
    from test_oracle_kinetic import B_TESLA, DT, GAMMA0, kinetic_moments
    n0, cps = 3000, (50, 100, 200, 300)
    u = O.units()
    Bh = B_TESLA / u["B_ref"]
    p0 = math.sqrt(GAMMA0 ** 2 - 1)
    el = O.species_from({"x": np.zeros(n0), "y": np.zeros(n0), "z": np.zeros(n0), "ux": np.full(n0, p0),
                         "uy": np.zeros(n0), "uz": np.zeros(n0), "w": np.ones(n0),
                         "uid": np.arange(n0, dtype=np.uint64)}, capacity=8 * n0)
    O.init_tau(el, 7)
    po, ph = O.new_species(8 * n0), O.new_species(200 * n0)
    un, tally = [n0], O.Tally()
    field = O.make_field(O.FIELD_UNIFORM, B=(0.0, 0.0, Bh))
    sp = O.merge_spec((-40, -40, -2), (4, 4, 4), (20, 20, 1), False, -8, 48, 4, 16, 4)
    mc, neff, merges = {}, {}, []
    for n in range(max(cps)):
        st = O.make_step(n * DT, DT, 7, rad_model=O.RAD_MC, chi_photon_push_min=0.0)
        n_ph0 = ph["n"]
        O.push_emit(bound_tables, 0.8e-6, -1.0, el, field, ph, None, st, un, tally)
        O.push_emit(bound_tables, 0.8e-6, +1.0, po, field, ph, None, st, un, tally)
        O.pair_create(bound_tables, 0.8e-6, ph, field, el, po, st, un, tally, n_limit=n_ph0)
        if (n + 1) % 10 == 0 and ph["n"] > 0.05 * 160 * n0:
            before = ph["n"]
            ph, un[0] = O.merge(sp, ph, 7, un[0], capacity=len(ph["x"]))
            merges.append((before, ph["n"]))
        if n + 1 in cps:
            v = {"electrons": O.view(el), "positrons": O.view(po), "photons": O.view(ph)}
            mc[n + 1] = {k: K.mc_moments(x, k == "photons", Bh, u["Es_hat"]) for k, x in v.items()}
            neff[n + 1] = {}
            for k, x in v.items():
                w = x["w"][~np.isinf(x["tau"])]
                neff[n + 1][k] = w.sum() ** 2 / max((w * w).sum(), 1e-300)
    assert len(merges) >= 10 and merges[0][1] < 0.5 * merges[0][0]
    kin = kinetic_moments(bound_tables, cps)
    for s in cps:
        for k in ("electrons", "positrons", "photons"):
            tol = 4.0 / math.sqrt(max(neff[s][k], 1.0)) + 0.02
            for q in ("n", "energy", "chi"):
                a = mc[s][k][q] / (n0 if q != "chi" else 1.0)
                assert a == pytest.approx(kin[s][k][q], rel=tol), (s, k, q)
