"""Determinism of the HIP path: checkpoint and restart, and split launches.

* A run saved half way and continued from the file by a freshly built run
  ends bit-identical to the run that never stopped (particles, ids, event
  counters, optical depths, id counter and FP64 tallies), with cell ordering,
  compaction, pushed photons and pairs on the Yee grid, and on a plane wave.
* Splitting the electrons of one launch into two runs (what sharding over
  GPUs does) leaves every electron bit-identical and gives the same multiset
  of recorded photons: draws are keyed by the particle's id and event counter,
  not by its place in a launch.  New particles take ids from the run's own
  counter, so only their ids differ (a shard would own a disjoint id range).

The coupled form is left out: its current deposition adds FP32 atomically,
so two runs of it agree to rounding, not to the bit.
"""
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import oracle as O                      # noqa: E402
from paper_1311_1107_amd import device as D         # noqa: E402
from paper_1311_1107_amd import sim as S            # noqa: E402
from paper_1311_1107_amd import workloads as W      # noqa: E402

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def gpu_oracle_tables(oracle_tables):
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible: the gpu tests need an MI355X")
    return D.Tables(O.EMIT_SPEC, O.PAIR_SPEC, arrays=oracle_tables)


def _yee_small():
    return W.yee_beam(n=2000, steps=200, seed=12, shape=(64, 32, 32), a0=800.0, gamma_median=4000.0,
                      x_range_lambda=(3.0, 5.0), r_max_lambda=1.0, x_center0=12.0)


def _same(a: dict, b: dict):
    for sp in ("electrons", "positrons", "photons", "recorded"):
        if a[sp] is None:
            assert b[sp] is None, sp
            continue
        assert a[sp].keys() == b[sp].keys(), sp
        for k in a[sp]:
            assert np.array_equal(a[sp][k], b[sp][k]), f"{sp}.{k}"
    assert a["uid_next"] == b["uid_next"]
    assert a["tally"] == b["tally"]


CASES = {
    "yee": (_yee_small, dict(photon_capacity=160 * 2000, record_capacity=8 * 2000, pair_capacity=12 * 2000,
                             compact_every=7, sort_every=5)),
    "plane": (lambda: W.plane_wave_beam(n=3000, box_lambda=2.0, steps=500, seed=11), dict(record_capacity=20 * 3000)),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_checkpoint_restart_is_bit_identical(gpu_oracle_tables, tmp_path, case):
    make, kw = CASES[case]
    wl = make()
    steps, half = wl.steps, wl.steps // 2 + 3          # the restart falls between two cell orderings
    print(f"case: {case} steps={steps} restart at {half}", flush=True)
    whole = S.Run(wl, tables=gpu_oracle_tables, **kw)
    whole.run(steps)
    want = whole.result()
    first = S.Run(make(), tables=gpu_oracle_tables, **kw)
    first.run(half)
    path = str(tmp_path / f"{case}.npz")
    first.save(path, half)
    del first
    second = S.Run(make(), tables=gpu_oracle_tables, **kw)
    nxt = second.load(path)
    assert nxt == half
    second.run(steps - half, start=nxt)
    got = second.result()
    if case == "yee":
        assert want["tally"]["N_pair"] > 0 and len(want["photons"]["x"]) > 0
    assert len(want["recorded"]["x"]) > 0
    _same(want, got)
    second.ws.status()


def test_checkpoint_rejects_a_mismatched_run(gpu_oracle_tables, tmp_path):
    wl = _yee_small()
    kw = CASES["yee"][1]
    run = S.Run(wl, tables=gpu_oracle_tables, **kw)
    run.run(3)
    run.ws.status()
    path = str(tmp_path / "yee.npz")
    run.save(path, 3)
    other = S.Run(W.plane_wave_beam(n=100, box_lambda=2.0, steps=10, seed=1), tables=gpu_oracle_tables)
    with pytest.raises(ValueError):
        other.load(path)


def _sorted_rows(sp: dict, keys=("x", "y", "z", "ux", "uy", "uz", "w", "chi")) -> np.ndarray:
    m = np.stack([sp[k] for k in keys], 1)
    return m[np.lexsort(m.T[::-1])]


def test_split_launches_match_one_launch(gpu_oracle_tables):
    wl = W.plane_wave_beam(n=4000, box_lambda=2.0, steps=600, seed=21)
    n = len(wl.electrons["x"])
    print(f"case: plane wave n={n} steps={wl.steps}, electrons split 1500 / 2500", flush=True)
    whole = S.Run(wl, tables=gpu_oracle_tables, record_capacity=20 * n)
    whole.run(wl.steps)
    want = whole.result()
    whole.ws.status()
    parts = []
    for idx, uid0 in ((np.arange(0, 1500), None), (np.arange(1500, n), 1 << 40)):
        run = S.Run(W.subset(wl, idx), tables=gpu_oracle_tables, record_capacity=20 * len(idx))
        run.uid_next.fill_(uid0 if uid0 is not None else n)        # disjoint id ranges for new photons
        run.run(wl.steps)
        parts.append(run.result())
        run.ws.status()
    # electrons: bit-identical, in the same order
    for k, v in want["electrons"].items():
        got = np.concatenate([p["electrons"][k] for p in parts])
        assert np.array_equal(got, v), k
    # recorded photons: the same multiset of states; ids come from each run's counter
    rec = {k: np.concatenate([p["recorded"][k] for p in parts]) for k in want["recorded"]}
    assert len(rec["x"]) == len(want["recorded"]["x"]) > 1000
    assert np.array_equal(_sorted_rows(rec), _sorted_rows(want["recorded"]))
    for k, v in want["tally"].items():
        if k.startswith("N_"):
            assert sum(p["tally"][k] for p in parts) == v, k
        else:
            assert sum(p["tally"][k] for p in parts) == pytest.approx(v, rel=1e-12, abs=1e-300), k
