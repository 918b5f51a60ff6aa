"""GPU parity of the super-particle merging (qed_merge) against the oracle.

Bit-exact: the output count, the order (ids of copied and new particles),
event counters, and every field of a copied particle.  New particles:
weight, position and chi within 1e-12 relative (FP64; 1e-6 for FP32, one
rounding of an FP64 result), optical depth within 4e-16 (the log of the
same Philox draw), momentum within 1e-12 |u| plus the conditioning of the
split angle: the two implementations sum the group in different orders, so
1 - cos(theta) differs by about 1e-16 / (1 - cos(theta)) relative, which
moves u by 1e-16 |u| / sin(theta).  Conservation of weight, momentum and
energy is checked on the GPU output directly.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import oracle as O                      # noqa: E402
from paper_1311_1107_amd import binding as B        # noqa: E402
from paper_1311_1107_amd import device as D         # noqa: E402
from paper_1311_1107_amd import workloads as W      # noqa: E402

SHAPE, SPACING, ORIGIN = (4, 3, 5), (0.5, 0.5, 0.5), (-1.0, 0.0, 0.5)
FIELDS = ("x", "y", "z", "ux", "uy", "uz", "tau", "w", "chi", "uid", "n_ev")


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible: the gpu tests need an MI355X")


def _spec(massive, sub_bins=2, n_dir=3, min_group=3, octave_min=-8, n_oct=48, shape=SHAPE, spacing=SPACING,
          origin=ORIGIN):
    return (D.merge_spec(origin, spacing, shape, massive, octave_min, n_oct, sub_bins, n_dir, min_group),
            O.merge_spec(origin, spacing, shape, massive, octave_min, n_oct, sub_bins, n_dir, min_group))


def _as_prec(p, prec):
    """Inputs rounded to the species precision (the oracle sees the same values)."""
    if prec == B.QED_F64:
        return p
    q = dict(p)
    for k in ("x", "y", "z", "ux", "uy", "uz", "w", "chi"):
        q[k] = p[k].astype(np.float32).astype(np.float64)
    return q


def _gpu_merge(p, prec, spec, seed, uid0, chi=True, cap=None, calls=1):
    n = len(p["x"])
    cap = cap or max(n, 1)
    src = D.Species(cap, prec, chi=chi)
    src.upload(p)
    dst = D.Species(cap, prec, chi=chi)
    ws = D.Workspace(cap)
    mg = D.Merger(cap)
    for _ in range(calls):
        uid = torch.tensor([uid0], dtype=torch.int64, device="cuda")
        mg.merge(ws, spec, src, dst, seed, uid)
        torch.cuda.synchronize()
    ws.status()
    return dst.download(), int(uid.item())


def _check(got, want, src, prec, massive, chi=True):
    n = len(want["x"])
    assert len(got["x"]) == n, (len(got["x"]), n)
    assert np.array_equal(got["uid"], want["uid"]), "ids / order"
    assert np.array_equal(got["n_ev"], want["n_ev"])
    copied = np.isin(want["uid"], src["uid"])
    fields = [f for f in FIELDS if chi or f != "chi"]
    for f in fields:
        assert np.array_equal(got[f][copied].astype(np.float64) if f not in ("uid", "n_ev") else got[f][copied],
                              want[f][copied]), f
    new = ~copied
    if not new.any():
        return 0
    rt = 1e-12 if prec == B.QED_F64 else 1e-6
    for f in ["w", "x", "y", "z"] + (["chi"] if chi else []):
        g, w = got[f][new].astype(np.float64), want[f][new]
        assert np.all(np.abs(g - w) <= rt * np.maximum(np.abs(w), 1.0)), f
    assert np.allclose(got["tau"][new], want["tau"][new], rtol=4e-16, atol=0)
    ug = np.stack([got["ux"], got["uy"], got["uz"]], 1)[new].astype(np.float64)
    uw = np.stack([want["ux"], want["uy"], want["uz"]], 1)[new]
    m = np.linalg.norm(uw, axis=1)
    # the pair partner of each new particle is its neighbour (2k, 2k+1)
    ua, ub = uw[0::2], uw[1::2]
    s = 0.5 * np.linalg.norm(ua - ub, axis=1) / np.maximum(m[0::2], 1e-300)   # sin(theta)
    s = np.repeat(s, 2)
    tol = rt * m + 1e-15 * m / np.maximum(s, 1e-9)
    assert np.all(np.linalg.norm(ug - uw, axis=1) <= tol), "momentum"
    return int(new.sum()) // 2


def _conserved(src, got, massive):
    live = ~(np.isinf(src["tau"]) & (src["tau"] > 0))
    u0 = np.stack([src["ux"], src["uy"], src["uz"]], 1)[live].astype(np.float64)
    u1 = np.stack([got["ux"], got["uy"], got["uz"]], 1).astype(np.float64)
    w0, w1 = src["w"][live].astype(np.float64), got["w"].astype(np.float64)

    def energy(u):
        u2 = (u * u).sum(1)
        return np.sqrt(1.0 + u2) if massive else np.sqrt(u2)
    return (w0.sum(), w1.sum(), (w0[:, None] * u0).sum(0), (w1[:, None] * u1).sum(0),
            (w0 * energy(u0)).sum(), (w1 * energy(u1)).sum(), np.abs(w0[:, None] * u0).sum())


@pytest.mark.parametrize("prec", [B.QED_F64, B.QED_F32])
@pytest.mark.parametrize("massive", [False, True])
@pytest.mark.parametrize("n", [0, 1, 5, 4097, 30000])
def test_merge_matches_oracle(prec, massive, n):
    """Clustered clouds (several beams, dead, zero-weight and out-of-range
    entries); 4097 and 30000 span several 4096-key tiles with ragged tails."""
    _need_gpu()
    print(f"case: merge prec={prec} massive={massive} n={n}", flush=True)
    p = _as_prec(W.merge_cloud(n, 40 + n, photons=not massive, shape=SHAPE, spacing=SPACING, origin=ORIGIN,
                               n_beams=3, spread=0.03, e_range=(30.0, 300.0)), prec)
    gs, os_ = _spec(massive)
    got, nxt = _gpu_merge(p, prec, gs, seed=9, uid0=10 ** 9)
    want, wnxt = O.merge(os_, O.species_from(p), seed=9, uid_next=10 ** 9)
    assert nxt == wnxt
    n_merged = _check(got, O.view(want), p, prec, massive)
    if n == 30000:
        assert n_merged > 1000
    w0, w1, p0, p1, e0, e1, sc = _conserved(p, got, massive)
    rt = 1e-12 if prec == B.QED_F64 else 1e-6
    assert abs(w1 - w0) <= rt * w0 and np.all(np.abs(p1 - p0) <= rt * sc) and abs(e1 - e0) <= rt * e0


def test_merge_without_chi_and_bin_layouts():
    _need_gpu()
    p = W.merge_cloud(20000, 3, photons=False, shape=SHAPE, spacing=SPACING, origin=ORIGIN, e_range=(5.0, 50.0))
    for sub, nd, mg in ((1, 1, 2), (64, 8, 4), (4, 64, 3)):
        print(f"case: merge layout sub={sub} n_dir={nd} min_group={mg}", flush=True)
        gs, os_ = _spec(True, sub_bins=sub, n_dir=nd, min_group=mg)
        got, _ = _gpu_merge(p, B.QED_F64, gs, seed=4, uid0=10 ** 9, chi=False)
        want, _ = O.merge(os_, O.species_from(p), seed=4, uid_next=10 ** 9)
        _check(got, O.view(want), p, B.QED_F64, True, chi=False)


def test_merge_large_groups_and_reuse():
    """One cell, one bin: groups of 200000 and 3 identical particles (a wave
    walks each group many times); a second call on the same merger and
    workspace gives the same result."""
    _need_gpu()
    n = 200_000
    r = np.random.default_rng(8)
    d = np.array([0.3, -1.0, 0.2]) + 0.02 * r.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    u = d * r.uniform(46.0, 60.0, n)[:, None]                  # |u|^2 in one octave
    p = {"x": r.uniform(0.0, 0.4, n), "y": r.uniform(0.1, 0.4, n), "z": r.uniform(0.6, 0.9, n),
         "ux": u[:, 0].copy(), "uy": u[:, 1].copy(), "uz": u[:, 2].copy(), "tau": r.exponential(1.0, n),
         "w": r.uniform(0.5, 1.5, n), "chi": r.uniform(0, 1, n), "uid": np.arange(n, dtype=np.uint64)}
    for k in FIELDS[:9]:
        p[k][-3:] = p[k][0] if k != "x" else 0.7                # another cell
    gs, os_ = _spec(False, sub_bins=1, n_dir=1)
    got, nxt = _gpu_merge(p, B.QED_F64, gs, seed=1, uid0=10 ** 9, calls=2)
    want, wnxt = O.merge(os_, O.species_from(p), seed=1, uid_next=10 ** 9)
    assert nxt == wnxt and len(got["x"]) == 4
    _check(got, O.view(want), p, B.QED_F64, False)
    # the identical triple merges into two copies of its momentum
    assert np.allclose(got["ux"][2:], p["ux"][0], rtol=1e-14) and np.allclose(got["uz"][2:], p["uz"][0], rtol=1e-14)


def test_merge_nothing_merged_and_all_dead():
    _need_gpu()
    p = W.merge_cloud(9000, 5, photons=True, shape=SHAPE, spacing=SPACING, origin=ORIGIN)
    gs, os_ = _spec(False, min_group=1 << 30)
    got, _ = _gpu_merge(p, B.QED_F64, gs, seed=1, uid0=10 ** 9)
    want, _ = O.merge(os_, O.species_from(p), seed=1, uid_next=10 ** 9)
    _check(got, O.view(want), p, B.QED_F64, False)
    p["tau"][:] = np.inf
    got, nxt = _gpu_merge(p, B.QED_F64, gs, seed=1, uid0=77)
    assert len(got["x"]) == 0 and nxt == 77


def test_merge_full_size_properties():
    """1e7 FP32 photons over 64^3 cells (the cascade's scale): weight,
    momentum and energy kept, ids unique, counts consistent."""
    _need_gpu()
    n = 10_000_000
    print(f"case: merge full size n={n}", flush=True)
    p = W.merge_cloud(n, 77, photons=True, shape=(64, 64, 64), spacing=(0.25, 0.25, 0.25), origin=(0.0, 0.0, 0.0),
                      n_beams=4, spread=0.02, e_range=(10.0, 1000.0))
    gs, _ = _spec(False, sub_bins=2, n_dir=4, shape=(64, 64, 64), spacing=(0.25, 0.25, 0.25), origin=(0, 0, 0))
    got, nxt = _gpu_merge(p, B.QED_F32, gs, seed=2, uid0=1 << 40)
    m = len(got["x"])
    assert 0 < m < n and nxt == (1 << 40) + m
    assert len(np.unique(got["uid"])) == m
    w0, w1, p0, p1, e0, e1, sc = _conserved(p, got, False)
    assert abs(w1 - w0) <= 1e-6 * w0 and np.all(np.abs(p1 - p0) <= 1e-6 * sc) and abs(e1 - e0) <= 1e-6 * e0


def test_merge_rejects_bad_arguments():
    _need_gpu()
    src = D.Species(100)
    ws = D.Workspace(100)
    mg = D.Merger(100)
    uid = torch.zeros(1, dtype=torch.int64, device="cuda")
    gs, _ = _spec(False)
    with pytest.raises(B.QedError):
        mg.merge(ws, gs, src, D.Species(50), 1, uid)          # destination too small
    with pytest.raises(B.QedError):
        mg.merge(ws, gs, src, src, 1, uid)                    # aliased
    with pytest.raises(B.QedError):
        mg.merge(ws, gs, src, D.Species(100, B.QED_F32), 1, uid)
    with pytest.raises(B.QedError):
        mg.merge(ws, gs, src, D.Species(100, chi=False), 1, uid)
    with pytest.raises(B.QedError):
        D.Merger(10).merge(ws, gs, src, D.Species(100), 1, uid)
    for field, bad in (("sub_bins", 3), ("sub_bins", 128), ("n_dir", 0), ("min_group", 1), ("n_octaves", 0),
                       ("nx", 0), ("dx", 0.0), ("octave_min", 5000)):
        b, _ = _spec(False)
        setattr(b, field, bad)
        with pytest.raises(B.QedError):
            mg.merge(ws, b, src, D.Species(100), 1, uid)
    b, _ = _spec(False, shape=(2048, 2048, 1024))
    with pytest.raises(B.QedError):
        mg.merge(ws, b, src, D.Species(100), 1, uid)          # 2^32 cells


def _n_eff(v):
    w = v["w"][~np.isinf(v["tau"])].astype(np.float64)
    return float(w.sum() ** 2 / max((w * w).sum(), 1e-300))


def test_constant_b_with_photon_merging_follows_kinetic_equations(oracle_tables, bound_tables):
    """The Sec. 4 cascade (2e4 electrons, FP64) with the photons merged
    whenever they fill 5 % of their buffer: numbers, energies and mean chi of
    every species stay on the kinetic solution (Eqs. 9-10), within
    4 / sqrt(N_eff) + 2 %, N_eff = (sum w)^2 / sum w^2 the effective number of
    super-particles of unequal weights."""
    _need_gpu()
    import math
    import os
    import sys
    sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
    from test_oracle_kinetic import kinetic_moments

    from oracle import kinetic as K
    from paper_1311_1107_amd import sim as S
    n0, checkpoints = 20_000, (50, 100, 200, 300)
    wl = W.constant_b(n=n0, steps=max(checkpoints))
    print(f"case: constant B kinetic with photon merging n={n0}", flush=True)
    pol = S.MergePolicy(origin=(-40.0, -40.0, -2.0), spacing=(4.0, 4.0, 4.0), shape=(20, 20, 1), sub_bins=4,
                        n_dir=16, min_group=4, threshold=0.05, species=("ph",))
    tabs = D.Tables(O.EMIT_SPEC, O.PAIR_SPEC, arrays=oracle_tables)
    run = S.Run(wl, tables=tabs, rad_model=B.QED_RAD_MC, photon_capacity=160 * n0, pair_capacity=6 * n0,
                compact_every=8, merge=pol)
    u = O.units()
    Bh = wl.field.B[2]
    mc, parts = {}, {}
    for n in range(max(checkpoints)):
        run.step(n)
        if (n + 1) % 10 == 0:
            run.merge_if_needed()
        if n + 1 in checkpoints:
            torch.cuda.synchronize()
            sp = {"electrons": run.el.download(), "positrons": run.po.download(), "photons": run.ph.download()}
            mc[n + 1] = {k: K.mc_moments(v, k == "photons", Bh, u["Es_hat"]) for k, v in sp.items()}
            parts[n + 1] = {k: _n_eff(v) for k, v in sp.items()}
    run.ws.status()
    assert len(run.merges) >= 3 and all(m["after"] < 0.7 * m["before"] for m in run.merges), run.merges
    kin = kinetic_moments(bound_tables, checkpoints)
    for s in checkpoints:
        for sp in ("electrons", "positrons", "photons"):
            tol = 4.0 / math.sqrt(max(parts[s][sp], 1)) + 0.02
            for q in ("n", "energy", "chi"):
                a = mc[s][sp][q] / (n0 if q != "chi" else 1.0)
                b = kin[s][sp][q]
                print(f"step {s} {sp} {q}: MC {a:.5g} kinetic {b:.5g} (tol {tol:.3f}, N_eff {parts[s][sp]:.0f})")
                assert a == pytest.approx(b, rel=tol), (s, sp, q)
