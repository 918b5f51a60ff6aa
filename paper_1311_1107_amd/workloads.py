"""Seeded synthetic inputs: initial particles and external laser fields.

This module holds no arithmetic of the radiation/QED step itself.  It draws
the initial super-particles (positions, momenta, weights, ids) and describes
the external field (plane-wave parameters, or the separable factors of a
focused pulse sampled on a Yee grid).  Both the HIP path and the CPU oracle
take its arrays as input; nothing here depends on either of them.

The paper's own runs (laser-electron collisions, Sec. 1, and a constant-field
test, Sec. 4) used no public dataset; these generators stand in for them.

Normalised units: time 1/omega_r, length c/omega_r (lambda = 2 pi),
momentum m c, fields m c omega_r/e.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

LAMBDA_M = 0.8e-6                   # reference wavelength [m]
TWO_PI = 2.0 * math.pi
LAM = TWO_PI                        # one wavelength in c/omega_r
DT = TWO_PI / 100.0                 # T/100
OMEGA_R = TWO_PI * 299792458.0 / LAMBDA_M


@dataclass
class PlaneWave:
    """a_y(phi) = a0 sin^2(pi phi/Phi) sin(phi), phi = t - x, Phi = 2 pi n_periods."""
    a0: float
    n_periods: float = 10.0


@dataclass
class Uniform:
    """Constant fields (normalised units)."""
    E: tuple = (0.0, 0.0, 0.0)
    B: tuple = (0.0, 0.0, 0.0)


@dataclass
class YeePulse:
    """Focused pulse on a Yee grid, value[c,i,j,k] = a0 * tperp[c,j,k] * tpar[step,c,i]."""
    shape: tuple
    spacing: tuple
    origin: tuple
    a0: float
    tperp: np.ndarray           # [6, ny*nz] float64
    tpar: np.ndarray            # [steps, 6, nx] float64


@dataclass
class Workload:
    name: str
    electrons: dict             # x y z ux uy uz w uid (float64 / uint64)
    field: object
    steps: int
    dt: float = DT
    seed: int = 1
    push_photons: bool = False
    chi_photon_push_min: float = 1e-3
    record_photons: bool = True
    extra: dict = field(default_factory=dict)


def _electrons(x, y, z, ux, uy, uz):
    n = len(x)
    return {"x": x.astype(np.float64), "y": y.astype(np.float64), "z": z.astype(np.float64),
            "ux": ux.astype(np.float64), "uy": uy.astype(np.float64), "uz": uz.astype(np.float64),
            "w": np.ones(n, np.float64), "uid": np.arange(n, dtype=np.uint64)}


def beam_in_box(n: int, gamma0: float, spread: float, rng: np.random.Generator,
                box: float = 20.0 * LAM):
    """Electrons uniform in [0, box)^3 moving along -x, |u| = gamma0 (1 + spread N(0,1))."""
    x = rng.uniform(0.0, box, n)
    y = rng.uniform(0.0, box, n)
    z = rng.uniform(0.0, box, n)
    ux = -gamma0 * (1.0 + spread * rng.standard_normal(n))
    zero = np.zeros(n)
    return _electrons(x, y, z, ux, zero, zero.copy())


def plane_wave_beam(n=100_000, a0=100.0, gamma0=2000.0, spread=0.01, steps=1000, seed=1,
                    box_lambda=20.0, push_photons=False, name="plane-wave beam") -> Workload:
    """Electrons uniform in a box of box_lambda wavelengths, gamma0 (1 % spread) along -x,
    against a 10-period plane wave.  Defaults: 1e5 electrons, gamma0 2000, a0 = 100,
    20-lambda box, 1000 steps, photons recorded."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return Workload(name, beam_in_box(n, gamma0, spread, rng, box=box_lambda * LAM), PlaneWave(a0), steps,
                    seed=seed, push_photons=push_photons)


def cascade_beam(n=50_000_000, a0=1000.0, gamma0=1.0e4, steps=500, seed=5) -> Workload:
    """5e7 electrons, gamma0 1e4 (1 % spread), a0 = 1000 plane wave, 500 steps."""
    rng = np.random.Generator(np.random.PCG64(seed))
    w = Workload("high-chi cascade", beam_in_box(n, gamma0, 0.01, rng), PlaneWave(a0), steps,
                 seed=seed, push_photons=True, chi_photon_push_min=0.2, record_photons=False)
    return w


def constant_b(n=100_000, gamma0=3000.0, b_tesla=7.48e6, steps=600, seed=7) -> Workload:
    """The validation case of Sec. 4: electrons of gamma0 = 3000 moving along x
    in a uniform B along z of 7.48 MT (chi_e ~ 5 at the start); every photon
    is pushed and may decay into a pair; 600 steps of T/100 (about 16 fs)."""
    b_ref = 9.1093837015e-31 * OMEGA_R / 1.602176634e-19      # m omega_r / e [T]
    p0 = math.sqrt(gamma0 * gamma0 - 1.0)
    e = _electrons(np.zeros(n), np.zeros(n), np.zeros(n), np.full(n, p0), np.zeros(n), np.zeros(n))
    return Workload("constant-B cascade", e, Uniform(B=(0.0, 0.0, b_tesla / b_ref)), steps, seed=seed,
                    push_photons=True, chi_photon_push_min=0.0, record_photons=False)


def bunches(n_bunches=64, seed=4, scale=1.0, lo=3.0, hi=6.0):
    """Independent bunches: sizes round(10^U(lo,hi)) (times scale), a0 ~ U(50,500),
    gamma0 ~ U(500,5000), each in the plane-wave geometry."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sizes = np.maximum(1, np.round(10.0 ** rng.uniform(lo, hi, n_bunches) * scale)).astype(np.int64)
    a0s = rng.uniform(50.0, 500.0, n_bunches)
    g0s = rng.uniform(500.0, 5000.0, n_bunches)
    parts = [beam_in_box(int(s), float(g), 0.01, rng) for s, g in zip(sizes, g0s)]
    out = {k: np.concatenate([p[k] for p in parts]) for k in parts[0]}
    out["uid"] = np.arange(len(out["x"]), dtype=np.uint64)
    offsets = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    return out, offsets, a0s, g0s


# --------------------------------------------------------------------------
# focused pulse on a Yee grid
# --------------------------------------------------------------------------
YEE_STAGGER = np.array([[0.5, 0.0, 0.0], [0.0, 0.5, 0.0], [0.0, 0.0, 0.5],
                        [0.0, 0.5, 0.5], [0.5, 0.0, 0.5], [0.5, 0.5, 0.0]])


def yee_pulse(steps: int, shape=(256, 128, 128), cells_per_lambda=8, a0=200.0, w0_lambda=3.0,
              fwhm_fs=30.0, x_center0=0.0, dt=DT) -> YeePulse:
    """Non-diffracting Gaussian pulse polarised along y, moving along +x:
    E_y = B_z = a0 exp(-(y^2+z^2)/w0^2) exp(-2 ln2 (s/tau)^2) cos(s), s = x - t - x_c0,
    tau = intensity FWHM in 1/omega_r.  Box x in [0, nx dx), y, z centred on 0."""
    nx, ny, nz = shape
    d = LAM / cells_per_lambda
    origin = (0.0, -0.5 * ny * d, -0.5 * nz * d)
    w0 = w0_lambda * LAM
    tau = fwhm_fs * 1e-15 * OMEGA_R
    tperp = np.zeros((6, ny * nz))
    tpar = np.zeros((steps, 6, nx))
    for c in (1, 5):                                   # E_y and B_z
        yy = origin[1] + (np.arange(ny) + YEE_STAGGER[c, 1]) * d
        zz = origin[2] + (np.arange(nz) + YEE_STAGGER[c, 2]) * d
        tperp[c] = np.exp(-(yy[:, None] ** 2 + zz[None, :] ** 2) / w0 ** 2).ravel()
        xx = origin[0] + (np.arange(nx) + YEE_STAGGER[c, 0]) * d
        t = np.arange(steps)[:, None] * dt
        s = xx[None, :] - t - x_center0
        tpar[:, c, :] = np.exp(-2.0 * math.log(2.0) * (s / tau) ** 2) * np.cos(s)
    return YeePulse(shape, (d, d, d), origin, a0, tperp, tpar)


def yee_beam(n=10_000_000, steps=2000, seed=2, shape=(256, 128, 128), a0=200.0, gamma_median=2000.0,
             gamma_sigma=0.3, x_range_lambda=(20.0, 28.0), r_max_lambda=2.0, x_center0=0.0,
             fwhm_fs=30.0, w0_lambda=3.0, chi_photon_push_min=1e-3) -> Workload:
    """Electrons with ln gamma0 ~ N(ln gamma_median, gamma_sigma^2), uniform in the cylinder
    r <= r_max around the axis and x in x_range (in wavelengths), moving along -x, sorted by
    grid cell (as a PIC code keeps them), against the focused pulse of yee_pulse().
    Defaults: 1e7 electrons, median 2000, sigma 0.3, a0 = 200, w0 = 3 lambda, 30 fs,
    Yee grid 256 x 128 x 128 at lambda/8, 2000 steps."""
    rng = np.random.Generator(np.random.PCG64(seed))
    pulse = yee_pulse(steps, shape=shape, a0=a0, w0_lambda=w0_lambda, fwhm_fs=fwhm_fs, x_center0=x_center0)
    d = pulse.spacing[0]
    x = rng.uniform(x_range_lambda[0] * LAM, x_range_lambda[1] * LAM, n)
    r = r_max_lambda * LAM * np.sqrt(rng.uniform(0.0, 1.0, n))
    th = rng.uniform(0.0, TWO_PI, n)
    y, z = r * np.cos(th), r * np.sin(th)
    g = np.exp(math.log(gamma_median) + gamma_sigma * rng.standard_normal(n))
    ux = -np.sqrt(g * g - 1.0)
    ci = np.floor((x - pulse.origin[0]) / d).astype(np.int64)
    cj = np.floor((y - pulse.origin[1]) / d).astype(np.int64)
    ck = np.floor((z - pulse.origin[2]) / d).astype(np.int64)
    order = np.lexsort((ck, cj, ci))
    zero = np.zeros(n)
    e = _electrons(x[order], y[order], z[order], ux[order], zero, zero.copy())
    return Workload("Yee-grid focused pulse", e, pulse, steps, seed=seed, push_photons=True,
                    chi_photon_push_min=chi_photon_push_min, record_photons=True)


def subset(wl: Workload, idx) -> Workload:
    """The same workload restricted to the electrons idx (uids kept)."""
    e = {k: v[idx].copy() for k, v in wl.electrons.items()}
    return Workload(wl.name + " (subset)", e, wl.field, wl.steps, wl.dt, wl.seed,
                    wl.push_photons, wl.chi_photon_push_min, wl.record_photons, dict(wl.extra))


# --------------------------------------------------------------------------
# particle clouds for the merging tests
# --------------------------------------------------------------------------
def merge_cloud(n: int, seed: int, photons: bool = True, shape=(4, 3, 5), spacing=(0.5, 0.5, 0.5),
                origin=(-1.0, 0.0, 0.5), n_beams: int = 5, spread: float = 0.05, e_range=(1.0, 1.0e4)):
    """Super-particles clustered in space and momentum, as after a burst of
    emission: positions uniform over a box of cells (5 % outside it),
    momenta along n_beams random directions with an angular spread and
    energies log-uniform over e_range (|k| for photons, |u| for leptons).
    A few entries are special: decayed photons (tau = +inf), zero weights
    and momenta outside a 2^-8 .. 2^40 range of |u|^2.  Returns a dict of
    numpy FP64 arrays plus uid (permuted) and n_ev."""
    r = np.random.Generator(np.random.PCG64(seed))
    lo = np.asarray(origin, float)
    hi = lo + np.asarray(shape) * np.asarray(spacing)
    pos = r.uniform(lo, hi, size=(n, 3))
    out = r.random(n) < 0.05
    pos[out] = r.uniform(lo - 1.0, hi + 1.0, size=(int(out.sum()), 3))
    dirs = r.normal(size=(n_beams, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    d = dirs[r.integers(0, n_beams, n)] + spread * r.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    mag = 10.0 ** r.uniform(math.log10(e_range[0]), math.log10(e_range[1]), n)
    u = d * mag[:, None]
    w = r.uniform(0.5, 2.0, n)
    tau = r.exponential(1.0, n)
    k = r.random(n)
    if photons:
        tau[k < 0.03] = np.inf
    w[(k >= 0.03) & (k < 0.04)] = 0.0
    u[(k >= 0.04) & (k < 0.045)] *= 2.0 ** 21          # |u|^2 above 2^40
    u[(k >= 0.045) & (k < 0.05)] *= 1e-3                # small |u|
    return {"x": pos[:, 0].copy(), "y": pos[:, 1].copy(), "z": pos[:, 2].copy(),
            "ux": u[:, 0].copy(), "uy": u[:, 1].copy(), "uz": u[:, 2].copy(),
            "tau": tau, "w": w, "chi": r.uniform(0.0, 2.0, n),
            "uid": r.permutation(np.arange(5000, 5000 + n, dtype=np.uint64)),
            "n_ev": r.integers(0, 7, n).astype(np.uint32)}
