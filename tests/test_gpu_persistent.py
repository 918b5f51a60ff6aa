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
