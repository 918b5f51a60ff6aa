"""The oracle's cell ordering against a brute-force definition.

Key of a particle: (i ny + j) nz + k of the Yee cell holding it, with
i = floor((x - x0)/dx) etc.; particles outside the grid take the key
nx ny nz.  The order is stable in the key.  Checked here against numpy's
stable argsort of keys computed independently, and by invariants (a
permutation that carries every field of a particle along)."""
import numpy as np
import pytest

from oracle import oracle as O

SHAPE = (7, 5, 6)
SPACING = (0.5, 0.25, 0.75)
ORIGIN = (-1.0, 0.5, 2.0)


def _keys(x, y, z):
    nx, ny, nz = SHAPE
    out = np.full(len(x), nx * ny * nz, dtype=np.int64)
    for t, (xx, yy, zz) in enumerate(zip(x, y, z)):
        i = np.floor((xx - ORIGIN[0]) / SPACING[0])
        j = np.floor((yy - ORIGIN[1]) / SPACING[1])
        k = np.floor((zz - ORIGIN[2]) / SPACING[2])
        if 0 <= i < nx and 0 <= j < ny and 0 <= k < nz:
            out[t] = (int(i) * ny + int(j)) * nz + int(k)
    return out


def _particles(n, seed):
    r = np.random.default_rng(seed)
    lo = np.array(ORIGIN)
    hi = lo + np.array(SHAPE) * np.array(SPACING)
    pos = r.uniform(lo - 0.3, hi + 0.3, size=(n, 3))
    # several particles per cell and exact cell faces, so that ties and edges occur
    pos[: n // 4] = lo + np.floor(r.uniform(0, 1, (n // 4, 3)) * SHAPE) * SPACING
    p = {"x": pos[:, 0], "y": pos[:, 1], "z": pos[:, 2]}
    for k in ("ux", "uy", "uz", "tau", "w", "chi"):
        p[k] = r.normal(size=n)
    p["uid"] = r.permutation(np.arange(1000, 1000 + n, dtype=np.uint64))
    p["n_ev"] = r.integers(0, 5, n).astype(np.uint32)
    return p


@pytest.mark.parametrize("n", [0, 1, 2, 517])
def test_sort_matches_stable_argsort(n):
    p = _particles(n, seed=3 + n)
    s = O.species_from(p, capacity=n + 3)
    O.sort_by_cell(s, SHAPE, SPACING, ORIGIN)
    got = O.view(s)
    order = np.argsort(_keys(p["x"], p["y"], p["z"]), kind="stable")
    for k in ("x", "y", "z", "ux", "uy", "uz", "tau", "w", "chi", "uid", "n_ev"):
        assert np.array_equal(got[k], p[k][order]), k
    assert s["n"] == n


def test_sort_keys_nondecreasing_and_stable():
    p = _particles(2000, seed=9)
    p["uid"] = np.arange(2000, dtype=np.uint64)          # uid = original index
    s = O.species_from(p)
    O.sort_by_cell(s, SHAPE, SPACING, ORIGIN)
    got = O.view(s)
    k = _keys(got["x"], got["y"], got["z"])
    assert np.all(np.diff(k) >= 0)
    same = np.diff(k) == 0
    assert np.all(np.diff(got["uid"].astype(np.int64))[same] > 0)     # ties keep their order
    assert np.sum(k == np.prod(SHAPE)) > 0 and np.sum(k < np.prod(SHAPE)) > 0


def test_sort_is_idempotent():
    p = _particles(300, seed=5)
    s = O.species_from(p)
    O.sort_by_cell(s, SHAPE, SPACING, ORIGIN)
    once = {k: v.copy() for k, v in O.view(s).items()}
    O.sort_by_cell(s, SHAPE, SPACING, ORIGIN)
    for k, v in O.view(s).items():
        assert np.array_equal(v, once[k]), k


@pytest.mark.parametrize("bands", [2, 4, 8])
def test_sort_with_energy_bands_matches_stable_argsort(bands):
    """key = cell key * bands + band, band = floor(log2 |u|^2 / 6) clamped to
    [0, bands) (edges at |u| = 8, 64, 512, ...); momenta drawn away from the
    edges so that the band is the same in any rounding."""
    n = 900
    p = _particles(n, seed=40 + bands)
    r = np.random.default_rng(bands)
    mag = 10.0 ** r.uniform(-1.0, 4.5, n)
    edges = 8.0 ** np.arange(1, 6)
    near = np.min(np.abs(mag[:, None] / edges[None, :] - 1.0), axis=1) < 1e-6
    mag[near] *= 1.01
    d = r.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    for c, k in enumerate(("ux", "uy", "uz")):
        p[k] = d[:, c] * mag
    s = O.species_from(p)
    O.sort_by_cell(s, SHAPE, SPACING, ORIGIN, bands=bands)
    got = O.view(s)
    band = np.array([min(bands - 1, max(0, int(np.floor(np.log2(m * m) / 6.0)))) for m in mag])
    keys = _keys(p["x"], p["y"], p["z"]) * bands + band
    order = np.argsort(keys, kind="stable")
    for k in ("x", "ux", "uid", "n_ev", "tau"):
        assert np.array_equal(got[k], p[k][order]), k
    assert len(set(band.tolist())) == min(bands, 5)  # every band up to |u| ~ 3e4 is used
