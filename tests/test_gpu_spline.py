"""GPU parity of the spline option for the quantile tables (interp = 1).

The device reads the emission and pair quantile tables through the natural
bicubic spline, from curvature tables the library derives when the tables
are loaded; the oracle derives its own and reads them through its own
spline.  Same bar as the other FP64 parity tests: counts, ids and event
counters exact, momenta and positions within 1e-12 of max(norm, 1), FP64
tallies within 1e-12.  The FP32 form with the spline is held to the FP32
bar in the one-step tests of the FP32 module.
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
from runners import assert_species_match, oracle_run  # noqa: E402


@pytest.fixture(scope="module")
def gpu_spline_tables(oracle_tables):
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible: the gpu tests need an MI355X")
    return D.Tables(dict(O.EMIT_SPEC, interp=B.QED_INTERP_SPLINE), dict(O.PAIR_SPEC, interp=B.QED_INTERP_SPLINE),
                    arrays=oracle_tables)


def _match(got, want, species, skip_energy=()):
    for sp in species:
        assert_species_match(got[sp], want[sp], what=sp)
        if sp in ("photons", "recorded") and len(want[sp]["x"]):
            c = np.abs(got[sp]["chi"] - want[sp]["chi"]) / np.maximum(np.abs(want[sp]["chi"]), 1e-300)
            assert c.max() <= 1e-11, sp
    assert got["uid_next"] == want["uid_next"]
    for k, v in want["tally"].items():
        if k.startswith("N_"):
            assert got["tally"][k] == v, k
        elif k not in skip_energy:
            assert got["tally"][k] == pytest.approx(v, rel=1e-12, abs=1e-300), k


def test_spline_tables_reject_bad_interp(oracle_tables):
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible: the gpu tests need an MI355X")
    with pytest.raises(B.QedError) as e:
        D.Tables(dict(O.EMIT_SPEC, interp=2), O.PAIR_SPEC, arrays=oracle_tables)
    assert e.value.code == B.QED_ERR_ARG


def test_spline_plane_wave_fp64_parity(gpu_spline_tables, spline_tables, bound_tables):
    """Plane-wave beam (3000 e-: 11 full tiles of 256 and a ragged tail),
    photons recorded: every emitted xi read through the spline."""
    wl = W.plane_wave_beam(n=3000, box_lambda=2.0, steps=500, seed=31)
    print("case: plane wave n=3000 steps=500 seed=31, spline quantiles", flush=True)
    want = oracle_run(wl, spline_tables, wl.steps, record_capacity=16 * 3000)
    assert want["tally"]["N_emit"] > 10000
    run = S.Run(wl, tables=gpu_spline_tables, record_capacity=16 * 3000)
    run.run(wl.steps)
    got = run.result()
    _match(got, want, ("electrons", "recorded"))
    # the spline does change the samples: the bilinear oracle run differs
    lin = oracle_run(wl, bound_tables, wl.steps, record_capacity=16 * 3000)
    n = min(len(lin["recorded"]["ux"]), len(want["recorded"]["ux"]))
    assert not np.array_equal(lin["recorded"]["ux"][:n], want["recorded"]["ux"][:n])
    run.ws.status()


def test_spline_constant_b_fp64_parity(gpu_spline_tables, spline_tables):
    """The constant-B cascade of Sec. 4 (pure Monte Carlo, every photon
    pushed and tested for pairs): emission and pair splits through the
    spline."""
    wl = W.constant_b(n=700, steps=120)
    print("case: constant B n=700 steps=120, spline quantiles", flush=True)
    caps = dict(photon_capacity=120 * 700, pair_capacity=8 * 700)
    want = oracle_run(wl, spline_tables, wl.steps, rad_model=O.RAD_MC, **caps)
    assert want["tally"]["N_pair"] > 100 and want["tally"]["N_overflow"] == 0
    run = S.Run(wl, tables=gpu_spline_tables, rad_model=B.QED_RAD_MC, compact_every=5, **caps)
    run.run(wl.steps)
    # a static magnetic field does no work: E_work holds only rounding noise (some
    # 1e-16 of the particles' energy), which no two summation orders share
    _match(run.result(), want, ("electrons", "positrons", "photons"), skip_energy=("E_work",))
    run.ws.status()
