"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer.

A child process preloads gcc's ASan runtime and loads the oracle built with
-fsanitize=address,undefined (QED_ORACLE_SANITIZE=1).  It runs every part of
the oracle on small inputs: the tables, a plane-wave run with emission, a
Yee run with pushed photons, pairs and cell order, the banded sort, the
merge, the field solver and both depositions, and the spectrum.  Any
out-of-bounds access, use after free or undefined behaviour aborts the
child; the test requires a clean exit.
"""
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)

CHILD = r'''
import sys
import numpy as np
sys.path.insert(0, {root!r}); sys.path.insert(0, {here!r})
from oracle import oracle as O
from paper_1311_1107_amd import workloads as W
from runners import oracle_run

tabs = O.compute_tables()
bt = O.BoundTables(tabs)
wl = W.plane_wave_beam(n=64, box_lambda=2.0, steps=60, seed=3)
r = oracle_run(wl, bt, wl.steps, record_capacity=20 * 64)
assert r["tally"]["N_emit"] > 0
wl = W.yee_beam(n=60, steps=40, seed=12, shape=(16, 8, 8), a0=800.0, gamma_median=4000.0,
                x_range_lambda=(1.0, 1.5), r_max_lambda=0.4, x_center0=3.0)
r = oracle_run(wl, bt, wl.steps, photon_capacity=200 * 60, record_capacity=20 * 60, pair_capacity=20 * 60,
               sort_every=5)
p = r["photons"]
s = O.species_from(dict(p))
O.sort_by_cell(s, (16, 8, 8), wl.field.spacing, wl.field.origin, bands=4)
cloud = W.merge_cloud(400, seed=5, photons=True)
spec = O.merge_spec((-1.0, 0.0, 0.5), (0.5, 0.5, 0.5), (4, 3, 5), False, -4, 16, 2, 4, 4)
O.merge(spec, O.species_from(cloud), 7, 10**6)
shape, spacing, origin = (6, 5, 7), (0.5, 0.4, 0.45), (0.0, 0.0, 0.0)
g = np.zeros((6,) + shape, np.float32)
g[:3] = np.random.default_rng(1).normal(size=(3,) + shape)
O.yee_advance(g, None, shape, spacing, 0.15, 3)
rng = np.random.default_rng(2)
n = 50
x0 = rng.uniform(0.5, 2.0, (n, 3))
x1 = x0 + rng.uniform(-0.3, 0.3, (n, 3))
pp = dict(x=x1[:, 0], y=x1[:, 1], z=x1[:, 2], ux=rng.normal(size=n), uy=rng.normal(size=n), uz=rng.normal(size=n),
          w=np.ones(n), tau=np.ones(n))
sp = O.species_from(pp)
O.deposit_current(sp, (x0[:, 0], x0[:, 1], x0[:, 2]), 0, -1.0, 1.0, 0.2, shape, spacing, origin)
O.deposit_charge(sp, -1.0, 1.0, shape, spacing, origin)
O.spectrum(O.species_from(p), True, 1.0, 1e5, 32, 1.0)
print("sanitized oracle ok", flush=True)
'''


def test_oracle_runs_clean_under_asan_and_ubsan():
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not asan or not os.path.isabs(asan) or not os.path.exists(asan):
        pytest.skip("gcc's AddressSanitizer runtime is not installed")
    env = dict(os.environ, QED_ORACLE_SANITIZE="1", LD_PRELOAD=asan,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    code = CHILD.format(root=ROOT, here=HERE)
    res = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=600)
    tail = (res.stdout + res.stderr)[-3000:]
    assert res.returncode == 0, tail
    assert "sanitized oracle ok" in res.stdout, tail
    assert "AddressSanitizer" not in res.stderr and "runtime error" not in res.stderr, tail
