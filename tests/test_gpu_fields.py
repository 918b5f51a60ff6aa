"""GPU parity of the PIC coupling (field solver and current deposition)
against the oracle.

Field solver: bit-exact (the same fmaf sequence per update, FP32 grids),
over several advances with a current, at a small grid and at the 256 x 128
x 128 grid of the Yee workload.  Deposition: the FP32 current and charge
grids within 1e-5 of the largest |value| of the oracle's FP64 sums (float
atomics in any order: each node sums a few hundred FP32-rounded terms); the
skipped count exactly; continuity on the GPU's own output.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import oracle as O                      # noqa: E402
from paper_1311_1107_amd import binding as B        # noqa: E402
from paper_1311_1107_amd import device as D         # noqa: E402


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible: the gpu tests need an MI355X")


def _geom(shape, spacing, origin=(0.0, 0.0, 0.0)):
    f = B.qed_field()
    f.kind = B.QED_FIELD_YEE
    f.grid = None
    f.nx, f.ny, f.nz = shape
    f.dx, f.dy, f.dz = spacing
    f.x0, f.y0, f.z0 = origin
    return f


@pytest.mark.parametrize("shape,steps", [((16, 12, 10), 12), ((5, 1, 7), 5), ((256, 128, 128), 2)])
def test_yee_advance_bit_exact(shape, steps):
    _need_gpu()
    print(f"case: yee advance shape={shape} steps={steps}", flush=True)
    r = np.random.default_rng(1)
    spacing, dt = (0.785, 0.6, 0.7), 0.25
    g = r.normal(size=(6,) + shape).astype(np.float32)
    J = (0.1 * r.normal(size=(3,) + shape)).astype(np.float32)
    gd = torch.from_numpy(g.copy()).cuda()
    Jd = torch.from_numpy(J).cuda()
    geo = _geom(shape, spacing)
    for s in range(steps):
        B.qed_yee_advance(gd.data_ptr(), Jd.data_ptr() if s % 2 == 0 else None, geo, dt)
        O.yee_advance(g, J if s % 2 == 0 else None, shape, spacing, dt)
    torch.cuda.synchronize()
    assert np.array_equal(gd.cpu().numpy(), g)


def test_yee_advance_rejects_courant_violation():
    _need_gpu()
    gd = torch.zeros(6 * 8, dtype=torch.float32, device="cuda")
    geo = _geom((2, 2, 2), (0.5, 0.5, 0.5))
    with pytest.raises(B.QedError):
        B.qed_yee_advance(gd.data_ptr(), None, geo, 0.3)          # limit 0.289
    bad = _geom((2, 2, 2), (0.5, 0.5, 0.5))
    bad.kind = B.QED_FIELD_UNIFORM
    with pytest.raises(B.QedError):
        B.qed_yee_advance(gd.data_ptr(), None, bad, 0.1)


SHAPE, SPACING, ORIGIN = (12, 10, 9), (0.5, 0.4, 0.45), (-1.0, 0.3, 2.0)


def _particles(n, seed, max_cells=0.95, far=0):
    r = np.random.default_rng(seed)
    lo, ext = np.array(ORIGIN), np.array(SHAPE) * np.array(SPACING)
    x0 = lo + r.uniform(-0.1, 1.1, (n, 3)) * ext                  # some start outside: periodic wrap
    x1 = x0 + r.uniform(-max_cells, max_cells, (n, 3)) * np.array(SPACING)
    if far:
        x1[:far, 0] += 2.6 * SPACING[0]
    u = r.normal(size=(n, 3)) * 2.0
    p = {"x": x1[:, 0].copy(), "y": x1[:, 1].copy(), "z": x1[:, 2].copy(), "ux": u[:, 0].copy(),
         "uy": u[:, 1].copy(), "uz": u[:, 2].copy(), "w": r.uniform(0.5, 2.0, n), "tau": np.ones(n),
         "uid": np.arange(n, dtype=np.uint64)}
    return p, x0


def _as_prec(p, x0, prec):
    if prec == B.QED_F64:
        return p, x0
    q = dict(p)
    for k in ("x", "y", "z", "ux", "uy", "uz", "w"):
        q[k] = p[k].astype(np.float32).astype(np.float64)
    return q, x0.astype(np.float32).astype(np.float64)


@pytest.mark.parametrize("prec", [B.QED_F64, B.QED_F32])
@pytest.mark.parametrize("n", [1, 777, 20000])
def test_deposit_current_matches_oracle(prec, n):
    _need_gpu()
    print(f"case: deposit prec={prec} n={n}", flush=True)
    p, x0 = _as_prec(*_particles(n, 10 + n, far=min(5, n // 100)), prec)
    dt, q, js = 0.2, -1.0, 0.7
    sp = D.Species(n, prec)
    sp.upload(p)
    dtp = torch.float64 if prec == B.QED_F64 else torch.float32
    old = [torch.from_numpy(x0[:, c].copy()).to(dtp).cuda() for c in range(3)]
    J = torch.zeros(3 * int(np.prod(SHAPE)), dtype=torch.float32, device="cuda")
    sk = torch.zeros(1, dtype=torch.int64, device="cuda")
    geo = _geom(SHAPE, SPACING, ORIGIN)
    B.qed_deposit_current(sp.struct(), [t.data_ptr() for t in old], None, q, js, dt, geo, J.data_ptr(), sk.data_ptr())
    torch.cuda.synchronize()
    want, wsk = O.deposit_current(O.species_from(p), (x0[:, 0], x0[:, 1], x0[:, 2]), 0, q, js, dt, SHAPE, SPACING,
                                  ORIGIN)
    got = J.cpu().numpy().reshape(want.shape).astype(np.float64)
    assert int(sk.item()) == wsk
    scale = np.max(np.abs(want))
    assert scale > 0
    assert np.max(np.abs(got - want)) <= 1e-5 * scale
    # continuity on the GPU's own grids
    r0 = torch.zeros(int(np.prod(SHAPE)), dtype=torch.float32, device="cuda")
    r1 = torch.zeros_like(r0)
    ok = np.ones(n, bool)
    if wsk:
        ok[:min(5, n // 100)] = False
    pk = {k: v[ok] for k, v in p.items()}
    s_new = D.Species(n, prec)
    s_new.upload(pk)
    s_old = D.Species(n, prec)
    s_old.upload(dict(pk, x=x0[ok, 0], y=x0[ok, 1], z=x0[ok, 2]))
    B.qed_deposit_charge(s_old.struct(), q, js, geo, r0.data_ptr())
    B.qed_deposit_charge(s_new.struct(), q, js, geo, r1.data_ptr())
    J2 = torch.zeros_like(J)
    old2 = [torch.from_numpy(x0[ok, c].copy()).to(dtp).cuda() for c in range(3)]
    B.qed_deposit_current(s_new.struct(), [t.data_ptr() for t in old2], None, q, js, dt, geo, J2.data_ptr())
    torch.cuda.synchronize()
    Jg = J2.cpu().numpy().reshape(want.shape).astype(np.float64)
    div = ((Jg[0] - np.roll(Jg[0], 1, 0)) / SPACING[0] + (Jg[1] - np.roll(Jg[1], 1, 1)) / SPACING[1]
           + (Jg[2] - np.roll(Jg[2], 1, 2)) / SPACING[2])
    drho = (r1.cpu().numpy().astype(np.float64) - r0.cpu().numpy().astype(np.float64)).reshape(SHAPE) / dt
    assert np.max(np.abs(drho + div)) <= 1e-5 * max(np.max(np.abs(div)), np.max(np.abs(drho)))
    # charge parity
    rw = O.deposit_charge(O.species_from(pk), q, js, SHAPE, SPACING, ORIGIN)
    assert np.max(np.abs(r1.cpu().numpy().reshape(SHAPE) - rw)) <= 1e-5 * np.max(np.abs(rw))


def test_deposit_created_particles_and_first():
    """x_old = NULL (back along u/gamma) for entries [first, n), first on the device."""
    _need_gpu()
    n, first = 3000, 1234
    p, _ = _particles(n, 3)
    dt, q, js = 0.2, 1.0, 1.0
    sp = D.Species(n)
    sp.upload(p)
    J = torch.zeros(3 * int(np.prod(SHAPE)), dtype=torch.float32, device="cuda")
    fd = torch.tensor([first], dtype=torch.int64, device="cuda")
    geo = _geom(SHAPE, SPACING, ORIGIN)
    B.qed_deposit_current(sp.struct(), None, fd.data_ptr(), q, js, dt, geo, J.data_ptr())
    torch.cuda.synchronize()
    want, _ = O.deposit_current(O.species_from(p), None, first, q, js, dt, SHAPE, SPACING, ORIGIN)
    got = J.cpu().numpy().reshape(want.shape)
    assert np.max(np.abs(got - want)) <= 1e-5 * np.max(np.abs(want))


def test_save_positions_copies_live_entries():
    _need_gpu()
    p, _ = _particles(1000, 4)
    for prec in (B.QED_F64, B.QED_F32):
        sp = D.Species(1500, prec)
        sp.upload(p)
        dtp = torch.float64 if prec == B.QED_F64 else torch.float32
        old = [torch.full((1500,), -7.0, dtype=dtp, device="cuda") for _ in range(3)]
        B.qed_save_positions(sp.struct(), [t.data_ptr() for t in old])
        torch.cuda.synchronize()
        for c, k in enumerate("xyz"):
            v = old[c].cpu().numpy()
            assert np.array_equal(v[:1000], p[k].astype(v.dtype)) and np.all(v[1000:] == -7.0)


def test_coupled_run_keeps_gauss_law():
    """A coupled run (2000 electrons against a0 = 800 on a 64 x 32 x 32 grid,
    weights of 1e9 physical electrons so that the currents matter, photons
    and pairs on): the grid is advanced by the solver with the leptons'
    currents, and div E - rho of the leptons stays what it was at step 0."""
    _need_gpu()
    from paper_1311_1107_amd import sim as S
    from paper_1311_1107_amd import workloads as W
    wl = W.yee_beam(n=2000, steps=60, seed=12, shape=(64, 32, 32), a0=800.0, gamma_median=4000.0,
                    x_range_lambda=(3.0, 5.0), r_max_lambda=1.0, x_center0=12.0)
    print("case: coupled run 2000 e- 60 steps", flush=True)
    run = S.Run(wl, photon_capacity=200 * 2000, record_capacity=200 * 2000, pair_capacity=40 * 2000, coupled=True,
                particles_per_weight=1e9, compact_every=4)
    f = wl.field
    geo = _geom(f.shape, f.spacing, f.origin)
    N = int(np.prod(f.shape))

    def gauss():
        rho = torch.zeros(N, dtype=torch.float32, device="cuda")
        B.qed_deposit_charge(run.el.struct(), -1.0, run.j_scale, geo, rho.data_ptr())
        B.qed_deposit_charge(run.po.struct(), 1.0, run.j_scale, geo, rho.data_ptr())
        torch.cuda.synchronize()
        g = run.grid.cpu().numpy().astype(np.float64).reshape((6,) + tuple(f.shape))
        dx, dy, dz = f.spacing
        div = ((g[0] - np.roll(g[0], 1, 0)) / dx + (g[1] - np.roll(g[1], 1, 1)) / dy
               + (g[2] - np.roll(g[2], 1, 2)) / dz)
        r = rho.cpu().numpy().astype(np.float64).reshape(f.shape)
        return div - r, np.max(np.abs(r)), np.max(np.abs(div))
    g0, r0, d0 = gauss()
    for n in range(wl.steps):
        run.step(n)
    g1, r1, d1 = gauss()
    run.ws.status()
    t = run.tally.reduce()
    assert t["N_emit"] > 100 and int(run.skipped.item()) == 0
    assert r1 > 1e-3 * d1                 # the charges are not negligible next to the field
    assert np.max(np.abs(g1 - g0)) <= 1e-4 * max(r1, d1)


def test_field_bound_table():
    """qed_field_bound: per 4^3-cell block, sqrt(sum over components of the
    largest |component|^2) over the block's nodes and two more each side,
    never below the exact value."""
    _need_gpu()
    r = np.random.default_rng(5)
    shape, bb = (19, 10, 13), 4
    g = r.normal(size=(6,) + shape).astype(np.float32)
    g[:, 5:9, 2:6, :] *= 50.0
    gd = torch.from_numpy(g.copy()).cuda()
    f = D.yee(gd, shape, (0.5, 0.5, 0.5), (0.0, 0.0, 0.0))
    nb = [(n + bb - 1) // bb for n in shape]
    bound = torch.zeros(2 * int(np.prod(nb)), dtype=torch.float32, device="cuda")
    B.qed_field_bound(f, bb, bound.data_ptr())
    torch.cuda.synchronize()
    got = bound.cpu().numpy().reshape(nb + [2])
    for bi in range(nb[0]):
        for bj in range(nb[1]):
            for bk in range(nb[2]):
                sl = tuple(slice(max(0, b * bb - 2), min(n, b * bb + bb + 2)) for b, n in zip((bi, bj, bk), shape))
                for fb in range(2):
                    m = [np.max(np.abs(g[3 * fb + c][sl])).astype(np.float64) for c in range(3)]
                    want = np.sqrt(sum(v * v for v in m))
                    assert want <= got[bi, bj, bk, fb] <= want * (1 + 1e-5)
    with pytest.raises(B.QedError):
        B.qed_field_bound(f, 0, bound.data_ptr())


def test_photon_step_cull_changes_nothing():
    """One photon step on the Yee grid with and without the per-block field
    bounds, from identical state: photons spread over a box whose x < L/2
    half holds no field (there every wave skips the gather) and whose other
    half holds the a0 = 800 pulse (pairs form).  Photons, pairs, ids and
    tallies are bit-identical; only the count of skipped gathers differs."""
    _need_gpu()
    from paper_1311_1107_amd import sim as S
    from paper_1311_1107_amd import workloads as W
    print("case: photon-step cull on/off, one step of 200k photons", flush=True)
    r = np.random.default_rng(17)
    n = 200_000
    res = []
    for bb in (2, 0):
        wl = W.yee_beam(n=2000, steps=260, seed=12, shape=(64, 32, 32), a0=800.0, gamma_median=4000.0,
                        x_range_lambda=(3.0, 5.0), r_max_lambda=1.0, x_center0=12.0)
        run = S.Run(wl, photon_capacity=n, record_capacity=1000, pair_capacity=4 * n, field_bound_block=bb)
        f = wl.field
        nx, ny, nz = f.shape
        run.fill_field(120)
        run.grid.view(6, nx, ny, nz)[:, : nx // 2] = 0.0
        run.field_bound()
        rr = np.random.default_rng(17)
        lo, ext = np.array(f.origin), np.array(f.shape) * np.array(f.spacing)
        pos = lo + rr.uniform(0.05, 0.95, (n, 3)) * ext
        cell = np.floor((pos - lo) / np.array(f.spacing)).astype(np.int64)
        order = np.lexsort((cell[:, 2], cell[:, 1], cell[:, 0]))
        pos = pos[order]
        kk = 10.0 ** rr.uniform(0.5, 3.5, n)
        d = np.array([-1.0, 0.0, 0.0]) + 0.05 * rr.normal(size=(n, 3))
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        k = d * kk[:, None]
        run.ph.upload({"x": pos[:, 0], "y": pos[:, 1], "z": pos[:, 2], "ux": k[:, 0], "uy": k[:, 1], "uz": k[:, 2],
                       "w": np.ones(n), "chi": np.zeros(n), "tau": rr.exponential(1.0, n) * 0.02,
                       "uid": np.arange(10 ** 6, 10 ** 6 + n, dtype=np.uint64)})
        run.uid_next.fill_(10 ** 7)
        st = D.step(120 * wl.dt, wl.dt, wl.seed, **run.step_kw)
        run.ph_snap.copy_(run.ph.count)
        B.qed_pair_create(run.tables.h, run.ws.h, run.units, run.ph_step, run.field, run.el.struct(),
                          run.po.struct(), run.tally.s, st, run.uid_next.data_ptr(), run.sched)
        torch.cuda.synchronize()
        run.ws.status()
        res.append({"ph": run.ph.download(), "el": run.el.download(), "po": run.po.download(),
                    "tally": run.tally.reduce(), "uid": int(run.uid_next.item())})
    a, b = res
    assert a["tally"].pop("N_nogather") > n // 4 and b["tally"].pop("N_nogather") == 0
    assert a["tally"] == b["tally"] and a["uid"] == b["uid"]
    assert a["tally"]["N_pair"] > 100
    for sp in ("ph", "el", "po"):
        for key in a[sp]:
            assert np.array_equal(a[sp][key], b[sp][key]), (sp, key)
