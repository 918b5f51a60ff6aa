"""GPU parity of the persistent loops as they run at production size.

At production size every block of a persistent kernel walks many tiles:
the lepton step's tile loop, the photon step's loop over 64-photon chunks
with the next chunk's state loaded ahead, the append passes' walks over
several tiles per wave (lepton step) and several 256-tile chunks per block
(pair append), and the scan's look-back over several 4096-tile blocks.  The
schedule's max_blocks cap makes those loops run at sizes the oracle steps
in seconds.  Same bar as the other FP64 parity tests: counts, ids and event
counters exact, momenta and positions within 1e-12.
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
from runners import assert_species_match, compare_with_sensitivity, oracle_run  # noqa: E402

CAPPED = dict(block=64, items_per_thread=1, blocks_per_cu=1, max_blocks=8)


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible: the gpu tests need an MI355X")


@pytest.fixture(scope="module")
def gpu_oracle_tables(oracle_tables):
    _need_gpu()
    return D.Tables(O.EMIT_SPEC, O.PAIR_SPEC, arrays=oracle_tables)


def _yee_small(seed=12, n=2000, steps=260):
    return W.yee_beam(n=n, steps=steps, seed=seed, shape=(64, 32, 32), a0=800.0, gamma_median=4000.0,
                      x_range_lambda=(3.0, 5.0), r_max_lambda=1.0, x_center0=12.0)


def test_yee_pairs_on_eight_blocks_fp64_parity(gpu_oracle_tables, bound_tables):
    """The Yee pair case (2000 e-, a0 = 800, 260 steps, cell order every 5
    steps, compaction every 7) with every kernel on a grid of 8 blocks of 64
    threads: each lepton block walks 4 or more tiles, each photon block
    hundreds of 64-photon chunks."""
    wl = _yee_small()
    print("case: Yee 64x32x32 n=2000 steps=260 seed=12 sort_every=5 on 8 blocks of 64", flush=True)
    caps = dict(photon_capacity=160 * 2000, record_capacity=8 * 2000, pair_capacity=12 * 2000)
    want = oracle_run(wl, bound_tables, wl.steps, sort_every=5, **caps)
    assert want["tally"]["N_pair"] > 1000 and len(want["photons"]["x"]) > 8 * 64 * 50
    wl_p = _yee_small()
    wl_p.electrons["ux"] = np.nextafter(wl_p.electrons["ux"], 0.0)
    pert = oracle_run(wl_p, bound_tables, wl.steps, sort_every=5, **caps)
    run = S.Run(wl, tables=gpu_oracle_tables, compact_every=7, sort_every=5, sched=D.schedule(**CAPPED), **caps)
    run.run(wl.steps)
    got = run.result()
    fr = compare_with_sensitivity(got, want, pert, ("electrons", "positrons", "photons", "recorded"),
                                  report=lambda s: print(s, flush=True))
    print(f"fractions within 1e-12: {fr}", flush=True)
    assert got["uid_next"] == want["uid_next"]
    for k, v in want["tally"].items():
        if k.startswith("N_"):
            assert got["tally"][k] == v, k
    run.ws.status()


@pytest.mark.parametrize("sched", [CAPPED, dict(block=256, items_per_thread=1, blocks_per_cu=8, max_blocks=0)],
                         ids=["8_blocks_of_64", "default"])
def test_large_counts_fp64_parity(gpu_oracle_tables, bound_tables, sched):
    """The constant-B cascade of Sec. 4 with 3e5 electrons for 8 steps: more
    than 4096 lepton tiles of 64 and, by the last steps, more than 2.6e5
    photons in the photon step (over 4096 tiles of 64, so two look-back
    blocks in the scan, and over 8 chunks of 256 tiles, so the pair append's
    chunk loop turns on 8 blocks).  Compaction every 3 steps."""
    n0, steps = 300_000, 8
    wl = W.constant_b(n=n0, steps=steps)
    print(f"case: constant B n={n0} steps={steps} sched={sched}", flush=True)
    caps = dict(photon_capacity=2 * n0, pair_capacity=n0 // 8)
    want = oracle_run(wl, bound_tables, steps, rad_model=O.RAD_MC, **caps)
    t = want["tally"]
    assert t["N_pair"] > 1000 and t["N_overflow"] == 0
    assert len(want["photons"]["x"]) > 4096 * 64
    run = S.Run(wl, tables=gpu_oracle_tables, rad_model=B.QED_RAD_MC, compact_every=3, sched=D.schedule(**sched),
                **caps)
    photons_stepped = []
    for n in range(steps):
        photons_stepped.append(run.ph.n())
        run.step(n)
    got = run.result()
    assert max(photons_stepped) > 4096 * 64
    for sp in ("electrons", "positrons", "photons"):
        assert_species_match(got[sp], want[sp], what=sp)
    assert got["uid_next"] == want["uid_next"]
    for k, v in t.items():
        if k.startswith("N_"):
            assert got["tally"][k] == v, k
    run.ws.status()


def test_schedule_cap_is_validated(gpu_oracle_tables):
    _need_gpu()
    wl = W.plane_wave_beam(n=100, box_lambda=2.0, steps=1, seed=3)
    run = S.Run(wl, tables=gpu_oracle_tables, record_capacity=64, sched=D.schedule(64, 1, 1, max_blocks=4))
    with pytest.raises(B.QedError) as e:
        run.step(0)
    assert e.value.code == B.QED_ERR_ARG and "max_blocks" in str(e.value)


def test_full_size_bunches_sampled_electrons(gpu_oracle_tables, bound_tables):
    """The 64-bunch workload at full size (1.376e7 electrons, 1000 steps) in
    the form bench.py times: one batched launch per step with the autotuned
    schedule, captured as a HIP graph of 10 steps and replayed.  FP64: 256
    electrons sampled by id are rerun by the oracle alone, each in its own
    bunch's plane wave (electrons in an external field with id-keyed draws
    evolve independently of one another and of where their photons go).
    Event counters exact; positions and momenta: 97 % of the sample within
    1e-12 of max(norm, 1), all within 100x the oracle's largest sensitivity to
    one ulp of the initial ux (or 1e-12).  FP32: the recorded photons' energy
    spectrum against the FP64 run's, two-sample KS at p > 0.01."""
    from scipy.stats import ks_2samp
    from paper_1311_1107_amd import batched as BT
    e, off, a0s, _ = W.bunches(n_bunches=64, seed=4)
    n = len(e["x"])
    steps = 1000
    print(f"case: full-size bunches n={n} steps={steps}", flush=True)

    def gpu_run(prec):
        bun = BT.Bunches(e, off, a0s, prec, gpu_oracle_tables, seed=4, record_capacity=20 * n)
        best, _ = bun.autotune(trial_steps=3)
        bun.capture(10)
        for _ in range(steps // 10):
            bun.replay()
        torch.cuda.synchronize()
        bun.ws.status()
        rng = np.random.default_rng(0)
        k = bun.rec.n()
        sel = torch.from_numpy(np.sort(rng.integers(0, k, size=min(200_000, k)))).cuda()
        gg = torch.sqrt(bun.rec.a["ux"][sel].double() ** 2 + bun.rec.a["uy"][sel].double() ** 2 +
                        bun.rec.a["uz"][sel].double() ** 2).cpu().numpy()
        el = bun.el.download()
        print(f"  {'FP64' if prec == B.QED_F64 else 'FP32'} batched: schedule {best.block} x {best.blocks_per_cu} "
              f"cap {best.max_blocks}, {k} photons recorded", flush=True)
        del bun
        torch.cuda.empty_cache()
        return el, gg

    el, g64 = gpu_run(B.QED_F64)
    r = np.random.default_rng(321)
    idx = np.sort(r.choice(n, 256, replace=False))
    assert np.array_equal(el["uid"][idx], e["uid"][idx])

    def oracle_sample(ux_shift):
        out = {}
        bunch_of = np.searchsorted(off, idx, side="right") - 1
        for b in np.unique(bunch_of):
            ids = idx[bunch_of == b]
            sub = {k: np.asarray(v)[ids] for k, v in e.items()}
            if ux_shift:
                sub["ux"] = np.nextafter(sub["ux"], 0.0)
            sp = O.species_from(sub)
            O.init_tau(sp, 4)
            f = O.make_field(O.FIELD_PLANE_WAVE, a0=float(a0s[b]), n_periods=10.0)
            tally, un = O.Tally(), [n]
            for k in range(steps):
                O.push_emit(bound_tables, W.LAMBDA_M, -1.0, sp, f, None, None, O.make_step(k * W.DT, W.DT, 4),
                            un, tally)
            v = O.view(sp)
            for k in v:
                out.setdefault(k, []).append(v[k])
        return {k: np.concatenate(v) for k, v in out.items()}

    print("  oracle on the sample", flush=True)
    we, pe = oracle_sample(False), oracle_sample(True)
    assert np.array_equal(we["uid"], e["uid"][idx])
    ge = {k: np.asarray(v)[idx] for k, v in el.items()}
    assert np.array_equal(ge["n_ev"], we["n_ev"])
    assert we["n_ev"].sum() > 256                          # the sample did emit
    for keys in (("x", "y", "z"), ("ux", "uy", "uz")):
        w_ = np.stack([we[k] for k in keys], 1)
        g = np.stack([ge[k].astype(np.float64) for k in keys], 1)
        p_ = np.stack([pe[k] for k in keys], 1)
        err = np.linalg.norm(g - w_, axis=1) / np.maximum(np.linalg.norm(w_, axis=1), 1.0)
        sens = np.linalg.norm(p_ - w_, axis=1) / np.maximum(np.linalg.norm(w_, axis=1), 1.0)
        tol = max(1e-12, 100.0 * float(sens.max()))
        print(f"  {keys}: max err {err.max():.2e}, {np.sum(err > 1e-12)} above 1e-12; oracle one-ulp "
              f"sensitivity max {sens.max():.2e}", flush=True)
        assert err.max() <= tol, (keys, err.max(), tol)
        assert np.mean(err <= 1e-12) >= 0.97, keys
    del el
    _, g32 = gpu_run(B.QED_F32)
    p = ks_2samp(g32, g64).pvalue
    print(f"  FP32 vs FP64 recorded-photon spectrum KS p = {p:.3g}", flush=True)
    assert p > 0.01
