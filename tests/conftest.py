import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950); calls the HIP path through the C-ABI")


@pytest.fixture(scope="session")
def oracle_tables():
    """Oracle tables at the default layout (128 chi nodes x 128 logit levels)."""
    from oracle import oracle as O
    return O.compute_tables()


@pytest.fixture(scope="session")
def bound_tables(oracle_tables):
    from oracle import oracle as O
    return O.BoundTables(oracle_tables)


@pytest.fixture(scope="session")
def spline_tables(oracle_tables):
    """The same tables read through the natural bicubic spline (interp = 1)."""
    from oracle import oracle as O
    t = dict(oracle_tables)
    t["emit_spec"] = dict(oracle_tables["emit_spec"], interp=O.INTERP_SPLINE)
    t["pair_spec"] = dict(oracle_tables["pair_spec"], interp=O.INTERP_SPLINE)
    return O.BoundTables(t)
