"""The oracle's log-binned spectrum against a pure-Python loop over its
definition, and its invariants (every live entry counted once)."""
import math

import numpy as np
import pytest

from oracle import oracle as O


def _brute(p, photons, e_min, e_max, n, scale):
    c = [0] * (n + 2)
    w = [0] * (n + 2)
    for i in range(len(p["ux"])):
        if photons and math.isinf(p["tau"][i]):
            continue
        u2 = p["ux"][i] ** 2 + p["uy"][i] ** 2 + p["uz"][i] ** 2
        e = math.sqrt(u2) if photons else math.sqrt(1.0 + u2)
        if e >= e_max:
            b = n + 1
        elif e >= e_min:
            b = 1 + min(n - 1, max(0, math.floor((math.log(e) - math.log(e_min)) * (n / math.log(e_max / e_min)))))
        else:
            b = 0
        c[b] += 1
        w[b] += int(round(p["w"][i] * scale))
    return np.array(c), np.array(w)


def _particles(n, seed):
    r = np.random.default_rng(seed)
    mag = 10.0 ** r.uniform(-1, 5, n)
    d = r.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    p = {"x": np.zeros(n), "y": np.zeros(n), "z": np.zeros(n),
         "ux": mag * d[:, 0], "uy": mag * d[:, 1], "uz": mag * d[:, 2],
         "w": r.choice([0.5, 1.0, 2.25], n), "tau": r.exponential(size=n)}
    p["tau"][r.random(n) < 0.1] = np.inf
    p["tau"][r.random(n) < 0.05] = -np.inf
    p["ux"][:3] = 0.0
    return p


@pytest.mark.parametrize("photons", [True, False])
def test_spectrum_matches_loop(photons):
    p = _particles(3000, 5 + photons)
    s = O.species_from(p)
    got = O.spectrum(s, photons, 2.0, 1e4, 37, 4.0)
    want = _brute(p, photons, 2.0, 1e4, 37, 4.0)
    assert np.array_equal(got[0], want[0]) and np.array_equal(got[1], want[1])
    live = np.sum(~np.isinf(p["tau"])) if photons else len(p["tau"])
    assert got[0].sum() == live
    assert got[0][0] > 0 and got[0][-1] > 0          # both open ends populated
