"""qed_push_emit_static, the lepton step without a workspace (its scratch in
a static device array), against qed_push_emit with a workspace on the same
inputs, through the C interface: three calls in a row on one GPU, each
smaller than the one before (6e4 electrons on a Yee grid with pushed and
recorded photons, 3000 in a plane wave, 700 in FP32), then an append past a
buffer's capacity reported through the status words.  The two entry points
run the same kernels, so particles, photons, ids, counters and tallies must
agree to the bit."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_1311_1107_amd import binding as B        # noqa: E402
from paper_1311_1107_amd import device as D         # noqa: E402
from paper_1311_1107_amd import sim as S            # noqa: E402
from paper_1311_1107_amd import workloads as W      # noqa: E402


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible: the gpu tests need an MI355X")


def _field(wl, k):
    f = wl.field
    if isinstance(f, W.PlaneWave):
        return D.plane_wave(f.a0, f.n_periods), None
    nx, ny, nz = f.shape
    grid = torch.zeros(6 * nx * ny * nz, dtype=torch.float32, device="cuda")
    tperp = torch.from_numpy(np.ascontiguousarray(f.tperp)).cuda()
    tpar = torch.from_numpy(np.ascontiguousarray(f.tpar[k])).cuda()
    B.qed_yee_fill_separable(grid.data_ptr(), nx, ny, nz, f.a0, tperp.data_ptr(), tpar.data_ptr())
    return D.yee(grid, f.shape, f.spacing, f.origin), (grid, tperp, tpar)


def _one_call(tabs, wl, k, prec, static, photon_cap, record_cap):
    n = len(wl.electrons["x"])
    units = B.qed_units_init(W.LAMBDA_M)
    el = D.Species(n, prec)
    el.upload(wl.electrons)
    B.qed_init_optical_depth(el.struct(), wl.seed)
    ph = D.Species(photon_cap, prec) if wl.push_photons else None
    rec = D.Species(record_cap, prec)
    tal = D.Tally(n // 64 + 2)
    uid = torch.tensor([n], dtype=torch.int64, device="cuda")
    field, keep = _field(wl, k)
    st = D.step(k * wl.dt, wl.dt, wl.seed, chi_photon_push_min=wl.chi_photon_push_min)
    if static:
        words = torch.zeros(6, dtype=torch.int64, device="cuda")
        B.qed_push_emit_static(tabs.h, units, -1.0, el.struct(), field, ph.struct() if ph else None, rec.struct(),
                               tal.s, st, uid.data_ptr(), words.data_ptr(), None)
        torch.cuda.synchronize()
        status = words.cpu().numpy()
    else:
        ws = D.Workspace(max(n, photon_cap, record_cap), max_leptons=n)
        B.qed_push_emit(tabs.h, ws.h, units, -1.0, el.struct(), field, ph.struct() if ph else None, rec.struct(),
                        tal.s, st, uid.data_ptr(), None)
        torch.cuda.synchronize()
        rc, rep = ws.status(raise_on_error=False)
        status = np.array([rep.flags] + list(rep.needed) + [rep.chi_above_table], dtype=np.int64)
    return {"el": el.download(), "ph": ph.download() if ph else None, "rec": rec.download(),
            "tally": tal.reduce(), "uid": int(uid.item()), "status": status,
            "energy": tal.energy.cpu().numpy(), "count": tal.count.cpu().numpy()}


def _same(a, b):
    for part in ("el", "ph", "rec"):
        if a[part] is None:
            assert b[part] is None
            continue
        assert a[part].keys() == b[part].keys()
        for k in a[part]:
            assert np.array_equal(a[part][k], b[part][k]), (part, k)
    assert a["uid"] == b["uid"]
    assert np.array_equal(a["count"], b["count"])
    assert np.array_equal(a["energy"], b["energy"])
    assert np.array_equal(a["status"], b["status"]), (a["status"], b["status"])


def test_static_entry_matches_workspace_entry():
    _need_gpu()
    tabs = D.Tables(S.EMIT_SPEC, S.PAIR_SPEC)
    calls = [
        ("Yee 6e4 e- FP64", W.yee_beam(n=60_000, steps=260, seed=12, shape=(64, 32, 32), a0=800.0,
                                         gamma_median=4000.0, x_range_lambda=(3.0, 5.0), r_max_lambda=1.0,
                                         x_center0=12.0), 150, B.QED_F64, 240_000, 30_000),
        ("plane wave 3000 e- FP64", W.plane_wave_beam(n=3000, box_lambda=2.0, steps=700, seed=11), 350,
         B.QED_F64, 8, 12_000),
        ("plane wave 700 e- FP32", W.plane_wave_beam(n=700, box_lambda=2.0, steps=700, seed=5), 350,
         B.QED_F32, 8, 3_000),
    ]
    for name, wl, k, prec, pcap, rcap in calls:
        print(f"case: static vs workspace entry, {name}, step {k}", flush=True)
        want = _one_call(tabs, wl, k, prec, False, pcap, rcap)
        got = _one_call(tabs, wl, k, prec, True, pcap, rcap)
        assert want["tally"]["N_emit"] > 0 and (len(want["rec"]["x"]) > 0)
        assert want["status"][0] == 0
        _same(got, want)
    # an append past the recorded buffer's capacity: the same sticky flag and needed count
    wl = W.plane_wave_beam(n=3000, box_lambda=2.0, steps=700, seed=11)
    print("case: static vs workspace entry, capacity overflow", flush=True)
    want = _one_call(tabs, wl, 350, B.QED_F64, False, 8, 5)
    got = _one_call(tabs, wl, 350, B.QED_F64, True, 8, 5)
    assert want["status"][0] & 1 and want["status"][2] > 5
    _same(got, want)


def test_static_entry_rejects_too_many_leptons():
    _need_gpu()
    tabs = D.Tables(S.EMIT_SPEC, S.PAIR_SPEC)
    el = D.Species(65_537)
    rec = D.Species(8)
    tal = D.Tally(4)
    uid = torch.zeros(1, dtype=torch.int64, device="cuda")
    words = torch.zeros(6, dtype=torch.int64, device="cuda")
    with pytest.raises(B.QedError) as e:
        B.qed_push_emit_static(tabs.h, B.qed_units_init(W.LAMBDA_M), -1.0, el.struct(), D.plane_wave(10.0), None,
                               rec.struct(), tal.s, D.step(0.0, W.DT, 1), uid.data_ptr(), words.data_ptr(), None)
    assert e.value.code == B.QED_ERR_ARG and "65536" in str(e.value)
    with pytest.raises(B.QedError):
        B.qed_push_emit_static(tabs.h, B.qed_units_init(W.LAMBDA_M), -1.0, D.Species(10).struct(),
                               D.plane_wave(10.0), None, rec.struct(), tal.s, D.step(0.0, W.DT, 1), uid.data_ptr(),
                               0, None)
