"""The oracle's OpenMP drivers (used to time it on all host cores) against
its serial steps (CPU only): the same particles to the bit, in the same
order, with the same ids, event counters and counts, and energy tallies to
rounding, on a Yee grid with pushed and recorded photons, Breit-Wheeler
pairs and cell order, on thread counts that do and do not divide the
particle counts, and when appends overflow their buffers."""
import os
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_1311_1107_amd import workloads as W

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from runners import oracle_run  # noqa: E402


def _yee(n=700, steps=90):
    return W.yee_beam(n=n, steps=steps, seed=12, shape=(64, 32, 32), a0=800.0, gamma_median=4000.0,
                      x_range_lambda=(3.0, 5.0), r_max_lambda=1.0, x_center0=12.0)


def _same(a, b):
    for sp in ("electrons", "positrons", "photons", "recorded"):
        if a[sp] is None:
            assert b[sp] is None
            continue
        assert len(a[sp]["x"]) == len(b[sp]["x"]), sp
        for k in a[sp]:
            assert np.array_equal(a[sp][k], b[sp][k]), (sp, k)
    assert a["uid_next"] == b["uid_next"]
    for k, v in a["tally"].items():
        if k.startswith("N_"):
            assert b["tally"][k] == v, k
        else:
            assert b["tally"][k] == pytest.approx(v, rel=1e-12, abs=1e-300), k


@pytest.mark.parametrize("threads", [1, 3, 8])
def test_openmp_oracle_matches_serial(bound_tables, threads):
    wl = _yee()
    caps = dict(photon_capacity=160 * 700, record_capacity=8 * 700, pair_capacity=12 * 700)
    serial = oracle_run(wl, bound_tables, wl.steps, sort_every=5, lazy_grid=True, **caps)
    assert serial["tally"]["N_pair"] > 20 and serial["tally"]["N_push"] > 1000 and serial["tally"]["N_rec"] > 0
    par = oracle_run(wl, bound_tables, wl.steps, sort_every=5, lazy_grid=True, threads=threads, **caps)
    _same(serial, par)


def test_openmp_oracle_overflow_matches_serial(bound_tables):
    """Buffers too small for the appends: the same particles are kept (the
    first in serial order), the same ids consumed, the same overflow count."""
    wl = _yee(n=500, steps=70)
    caps = dict(photon_capacity=9000, record_capacity=40, pair_capacity=30)
    serial = oracle_run(wl, bound_tables, wl.steps, lazy_grid=True, **caps)
    assert serial["tally"]["N_overflow"] > 0
    par = oracle_run(wl, bound_tables, wl.steps, lazy_grid=True, threads=5, **caps)
    _same(serial, par)
