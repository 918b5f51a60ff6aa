"""CPU checks of the HIP library: it loads, exports every entry point declared
in include/qed.h, and its host-side logic (units, FP64 table quadrature)
agrees with the oracle.  No kernel is launched here."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

from oracle import oracle as O
from paper_1311_1107_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            src = open(os.path.join(ROOT, "include", fn)).read()
            names |= set(re.findall(r"^\s*(?:qed_status|void|const char \*)\s*\*?\s*(qed_\w+)\s*\(", src, re.M))
    return names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(B.LIB_PATH):
        pytest.fail("libqed.so not built: run python -m paper_1311_1107_amd.build")
    lib = ctypes.CDLL(B.LIB_PATH)
    names = _declared()
    assert len(names) >= 19
    missing = [n for n in sorted(names) if not hasattr(lib, n)]
    assert not missing, missing
    # and the binding wraps every one of them
    assert names == set(B._SIGS), sorted(names ^ set(B._SIGS))


def test_units_match_oracle():
    u = B.qed_units_init(0.8e-6)
    o = O.units(0.8e-6)
    assert u.Es_hat == pytest.approx(o["Es_hat"], rel=1e-15)
    assert u.A_hat == pytest.approx(o["A_hat"], rel=1e-15)
    assert u.tau0_hat == pytest.approx(o["tau0_hat"], rel=1e-15)
    assert u.alpha_f == pytest.approx(o["alpha_f"], rel=1e-15)


def test_units_reject_bad_lambda():
    with pytest.raises(B.QedError):
        B.qed_units_init(-1.0)


def test_host_tables_match_oracle(oracle_tables):
    lt = B.qed_tables_compute_host(O.EMIT_SPEC, O.PAIR_SPEC)
    for k in ("ln_hrad", "ln_g", "pair_lnh"):
        assert np.max(np.abs(lt[k] - oracle_tables[k])) < 1e-13, k
    # quantiles: ln xi and logit eta to 1e-12 absolute (1e-14 relative at ln xi ~ -60)
    assert np.max(np.abs(lt["emit_q"] - oracle_tables["emit_q"])) < 1e-12
    assert np.max(np.abs(lt["pair_q"] - oracle_tables["pair_q"])) < 1e-12


def test_host_tables_reject_bad_spec():
    bad = dict(O.EMIT_SPEC, n_chi=1)
    with pytest.raises(B.QedError):
        B.qed_tables_compute_host(bad, O.PAIR_SPEC)
