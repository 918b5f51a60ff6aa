"""ctypes binding of the CPU oracle (``qed_oracle.c``).

TEST INFRASTRUCTURE: only the tests, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this module.  The product path
(``paper_1311_1107_amd``) never imports it.

Species are held as dicts of numpy arrays with the keys
``x y z ux uy uz tau w chi uid n_ev`` plus an integer count ``n``; the
oracle updates them in place.
"""
from __future__ import annotations

import ctypes as C
import hashlib
import math
import os
import subprocess
import tempfile

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "qed_oracle.c")
HDR = os.path.join(HERE, "qed_oracle.h")
LIB = os.path.join(HERE, "libqed_oracle.so")

RAD_NONE, RAD_SOKOLOV, RAD_MC, RAD_HYBRID = 0, 1, 2, 3
FIELD_UNIFORM, FIELD_PLANE_WAVE, FIELD_YEE, FIELD_YEE_SEPARABLE = 0, 1, 2, 3
RNG_EMIT, RNG_PAIR, RNG_INIT = 1, 2, 3

T_NAMES = ["work", "erad", "epush", "erec", "edrop", "esub", "epair", "_t7"]
C_NAMES = ["emit", "push", "rec", "drop", "sub", "cap", "range", "sokolov", "mc",
           "pair", "phstep", "nan", "overflow", "_c13", "_c14", "_c15"]


# QED_ORACLE_SANITIZE=1 selects a build with AddressSanitizer and
# UndefinedBehaviorSanitizer (the process must preload gcc's libasan).
SANITIZE = os.environ.get("QED_ORACLE_SANITIZE") == "1"
if SANITIZE:
    LIB = os.path.join(HERE, "libqed_oracle_san.so")


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain C11, FP64, no FMA contraction)."""
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= max(
            os.path.getmtime(SRC), os.path.getmtime(HDR)):
        return LIB
    tmp = LIB + ".tmp%d" % os.getpid()
    opt = (["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
            "-fno-sanitize-recover=undefined"] if SANITIZE else ["-O2"])
    cmd = ["gcc", "-std=c11"] + opt + ["-fPIC", "-shared", "-fopenmp",
                                       "-ffp-contract=off", "-fno-fast-math", "-o", tmp, SRC, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


class Units(C.Structure):
    _fields_ = [(n, C.c_double) for n in (
        "lambda_", "omega_r", "alpha_f", "E_s", "B_s", "tau_c", "tau_0",
        "Es_hat", "A_hat", "tau0_hat", "B_ref", "E_ref")]


class TableSpec(C.Structure):
    _fields_ = [("chi_min", C.c_double), ("chi_max", C.c_double),
                ("n_chi", C.c_int32), ("n_q", C.c_int32), ("logit_max", C.c_double),
                ("interp", C.c_int32), ("reserved", C.c_int32)]


_dp = C.POINTER(C.c_double)
_fp = C.POINTER(C.c_float)
_u64p = C.POINTER(C.c_uint64)
_u32p = C.POINTER(C.c_uint32)


class Tables(C.Structure):
    _fields_ = [("e_n_chi", C.c_int32), ("e_n_q", C.c_int32),
                ("e_chi_min", C.c_double), ("e_lnchi0", C.c_double), ("e_inv_dlnchi", C.c_double),
                ("e_logit_max", C.c_double), ("e_inv_dt", C.c_double),
                ("ln_hrad", _dp), ("ln_g", _dp), ("emit_q", _dp),
                ("p_n_chi", C.c_int32), ("p_n_q", C.c_int32),
                ("p_chi_min", C.c_double), ("p_lnchi0", C.c_double),
                ("p_inv_dlnchi", C.c_double), ("p_logit_max", C.c_double),
                ("p_inv_dt", C.c_double), ("pair_lnh", _dp), ("pair_q", _dp),
                ("e_interp", C.c_int32), ("p_interp", C.c_int32), ("emit_m", _dp), ("pair_m", _dp)]


class Species(C.Structure):
    _fields_ = [("n", C.c_int64), ("capacity", C.c_int64)] + [
        (n, _dp) for n in ("x", "y", "z", "ux", "uy", "uz", "tau", "w", "chi")] + [
        ("uid", _u64p), ("n_ev", _u32p)]


class MergeSpec(C.Structure):
    _fields_ = [(n, C.c_double) for n in ("x0", "y0", "z0", "dx", "dy", "dz")] + \
               [(n, C.c_int64) for n in ("nx", "ny", "nz")] + \
               [(n, C.c_int32) for n in ("massive", "octave_min", "n_octaves", "sub_bins", "n_dir", "min_group")]


class Field(C.Structure):
    _fields_ = [("kind", C.c_int32), ("E", C.c_double * 3), ("B", C.c_double * 3),
                ("a0", C.c_double), ("n_periods", C.c_double),
                ("grid", _fp * 6), ("tperp6", _dp), ("tpar6", _dp),
                ("nx", C.c_int64), ("ny", C.c_int64), ("nz", C.c_int64),
                ("dx", C.c_double), ("dy", C.c_double), ("dz", C.c_double),
                ("x0", C.c_double), ("y0", C.c_double), ("z0", C.c_double)]


class Step(C.Structure):
    _fields_ = [("t", C.c_double), ("dt", C.c_double), ("seed", C.c_uint64),
                ("rad_model", C.c_int32), ("chi_switch", C.c_double),
                ("gamma_photon_min", C.c_double), ("chi_photon_push_min", C.c_double),
                ("max_events", C.c_int32), ("no_recoil", C.c_int32), ("variants", C.c_int32),
                ("rate_scale", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = build()
        L = C.CDLL(path)
        d = C.c_double
        L.or_units_init.argtypes = [d, C.POINTER(Units)]
        for name in ("or_bessel_k", "or_bessel_ki", "or_emit_bracket", "or_pair_bracket",
                     "or_emit_cdf", "or_pair_cdf"):
            getattr(L, name).argtypes = [d, d]
            getattr(L, name).restype = d
        for name in ("or_h_rad", "or_g", "or_h_pair"):
            getattr(L, name).argtypes = [d]
            getattr(L, name).restype = d
        L.or_tables_compute.argtypes = [C.POINTER(TableSpec), C.POINTER(TableSpec)] + [_dp] * 5 + [C.c_int]
        L.or_tables_compute.restype = C.c_int
        L.or_tables_bind.argtypes = [C.POINTER(Tables), C.POINTER(TableSpec), C.POINTER(TableSpec)] + [_dp] * 5
        L.or_tables_bind_spline.argtypes = [C.POINTER(Tables), _dp, _dp]
        L.or_quantile_spline.argtypes = [_dp, C.c_int, C.c_int, C.c_double, C.c_double, _dp]
        L.or_lookup_h_rad.argtypes = [C.POINTER(Tables), d, C.POINTER(C.c_int)]
        L.or_lookup_h_rad.restype = d
        L.or_lookup_g.argtypes = [C.POINTER(Tables), d]
        L.or_lookup_g.restype = d
        L.or_lookup_h_pair.argtypes = [C.POINTER(Tables), d, C.POINTER(C.c_int)]
        L.or_lookup_h_pair.restype = d
        L.or_sample_xi.argtypes = [C.POINTER(Tables), d, d]
        L.or_sample_xi.restype = d
        L.or_sample_eta.argtypes = [C.POINTER(Tables), d, d]
        L.or_sample_eta.restype = d
        L.or_philox4x64_10.argtypes = [_u64p, _u64p, _u64p]
        L.or_u01.argtypes = [C.c_uint64]
        L.or_u01.restype = d
        L.or_field_at.argtypes = [C.POINTER(Field), d, d, d, d, _dp, _dp]
        L.or_yee_fill_separable.argtypes = [_fp, C.c_int64, C.c_int64, C.c_int64, d, _dp, _dp]
        L.or_chi_lepton.argtypes = [C.POINTER(Units), _dp, d, _dp, _dp]
        L.or_chi_lepton.restype = d
        L.or_chi_photon.argtypes = [C.POINTER(Units), _dp, _dp, _dp]
        L.or_chi_photon.restype = d
        L.or_init_tau.argtypes = [C.POINTER(Species), C.c_uint64]
        L.or_push_emit.argtypes = [C.POINTER(Tables), C.POINTER(Units), d, C.POINTER(Species),
                                   C.POINTER(Field), C.POINTER(Species), C.POINTER(Species),
                                   C.POINTER(Step), _u64p, _dp, C.POINTER(C.c_int64)]
        L.or_push_emit.restype = C.c_int
        L.or_pair_create.argtypes = [C.POINTER(Tables), C.POINTER(Units), C.POINTER(Species), C.c_int64,
                                     C.POINTER(Field), C.POINTER(Species), C.POINTER(Species),
                                     C.POINTER(Step), _u64p, _dp, C.POINTER(C.c_int64)]
        L.or_pair_create.restype = C.c_int
        L.or_push_emit_omp.argtypes = L.or_push_emit.argtypes + [C.c_int]
        L.or_push_emit_omp.restype = C.c_int
        L.or_pair_create_omp.argtypes = L.or_pair_create.argtypes + [C.c_int]
        L.or_pair_create_omp.restype = C.c_int
        L.or_sort_by_cell.argtypes = [C.POINTER(Species), C.c_int64, C.c_int64, C.c_int64, d, d, d, d, d, d]
        L.or_sort_by_cell_bands.argtypes = [C.POINTER(Species), C.c_int64, C.c_int64, C.c_int64, d, d, d, d, d, d,
                                            C.c_int32]
        L.or_yee_advance.argtypes = [_fp, _fp, C.c_int64, C.c_int64, C.c_int64, d, d, d, d]
        L.or_deposit_current.argtypes = [C.POINTER(Species), _dp, _dp, _dp, C.c_int64, d, d, d, C.c_int64, C.c_int64,
                                         C.c_int64, d, d, d, d, d, d, _dp]
        L.or_deposit_current.restype = C.c_int64
        L.or_deposit_charge.argtypes = [C.POINTER(Species), d, d, C.c_int64, C.c_int64, C.c_int64, d, d, d, d, d, d,
                                        _dp]
        L.or_merge.argtypes = [C.POINTER(MergeSpec), C.POINTER(Species), C.POINTER(Species), C.c_uint64, _u64p]
        L.or_merge.restype = C.c_int64
        _lib = L
    return _lib


# --------------------------------------------------------------------------
# scalar helpers
# --------------------------------------------------------------------------
def units(lambda_m: float = 0.8e-6) -> dict:
    u = Units()
    lib().or_units_init(lambda_m, C.byref(u))
    return {n: getattr(u, n) for n, _ in Units._fields_} | {"lambda": lambda_m}


def _units_struct(lambda_m: float) -> Units:
    u = Units()
    lib().or_units_init(lambda_m, C.byref(u))
    return u


def bessel_k(nu, x):
    return lib().or_bessel_k(nu, x)


def bessel_ki(nu, x):
    return lib().or_bessel_ki(nu, x)


def h_rad(chi):
    return lib().or_h_rad(chi)


def g(chi):
    return lib().or_g(chi)


def h_pair(chi):
    return lib().or_h_pair(chi)


def emit_bracket(chi, xi):
    return lib().or_emit_bracket(chi, xi)


def pair_bracket(chi, eta):
    return lib().or_pair_bracket(chi, eta)


def emit_cdf(chi, xi):
    return lib().or_emit_cdf(chi, xi)


def pair_cdf(chi, eta):
    return lib().or_pair_cdf(chi, eta)


def philox(ctr, key):
    c = (C.c_uint64 * 4)(*[int(v) & (2**64 - 1) for v in ctr])
    k = (C.c_uint64 * 2)(*[int(v) & (2**64 - 1) for v in key])
    o = (C.c_uint64 * 4)()
    lib().or_philox4x64_10(c, k, o)
    return [int(v) for v in o]


def u01(bits):
    return lib().or_u01(int(bits) & (2**64 - 1))


# --------------------------------------------------------------------------
# tables
# --------------------------------------------------------------------------
EMIT_SPEC = dict(chi_min=1e-3, chi_max=1e2, n_chi=128, n_q=128, logit_max=18.0)
PAIR_SPEC = dict(chi_min=1e-2, chi_max=1e2, n_chi=128, n_q=128, logit_max=18.0)


INTERP_LINEAR, INTERP_SPLINE = 0, 1


def _spec(d):
    return TableSpec(d["chi_min"], d["chi_max"], d["n_chi"], d["n_q"], d["logit_max"], d.get("interp", 0), 0)


def quantile_spline(q: np.ndarray, n_chi: int, n_q: int, h_c: float, h_t: float) -> np.ndarray:
    """Second-derivative tables of the natural bicubic spline through q
    (or_quantile_spline): shape (3, n_chi, n_q) = d2/dt2, d2/dc2, d4/dc2dt2."""
    q = np.ascontiguousarray(q, dtype=np.float64).reshape(-1)
    m = np.zeros(3 * n_chi * n_q)
    lib().or_quantile_spline(_ptr(q), n_chi, n_q, h_c, h_t, _ptr(m))
    return m.reshape(3, n_chi, n_q)


def _spacings(spec):
    h_c = (math.log(spec["chi_max"]) - math.log(spec["chi_min"])) / (spec["n_chi"] - 1)
    h_t = 2.0 * spec["logit_max"] / (spec["n_q"] - 1)
    return h_c, h_t


def compute_tables(emit=None, pair=None, threads: int | None = None, cache: bool = True) -> dict:
    """Oracle tables as numpy arrays; cached on disk per (source, spec)."""
    emit = dict(EMIT_SPEC if emit is None else emit)
    pair = dict(PAIR_SPEC if pair is None else pair)
    # the nodes do not depend on the interpolation between them
    nodes_e = {k: v for k, v in emit.items() if k != "interp"}
    nodes_p = {k: v for k, v in pair.items() if k != "interp"}
    key = hashlib.sha1((open(SRC).read() + repr(sorted(nodes_e.items())) +
                        repr(sorted(nodes_p.items()))).encode()).hexdigest()[:16]
    path = os.path.join(tempfile.gettempdir(), f"qed_oracle_tables_{key}.npz")
    if cache and os.path.exists(path):
        z = np.load(path)
        out = {k: z[k] for k in z.files}
    else:
        ne, nqe, npc, nqp = emit["n_chi"], emit["n_q"], pair["n_chi"], pair["n_q"]
        out = {"ln_hrad": np.zeros(ne), "ln_g": np.zeros(ne), "emit_q": np.zeros(ne * nqe),
               "pair_lnh": np.zeros(npc), "pair_q": np.zeros(npc * nqp)}
        se, sp = _spec(emit), _spec(pair)
        rc = lib().or_tables_compute(C.byref(se), C.byref(sp),
                                     *[_ptr(out[k]) for k in ("ln_hrad", "ln_g", "emit_q", "pair_lnh", "pair_q")],
                                     threads or os.cpu_count() or 1)
        if rc:
            raise RuntimeError("or_tables_compute failed")
        if cache:
            tmp = path + f".{os.getpid()}.npz"
            np.savez(tmp, **out)
            os.replace(tmp, path)
    out["emit_spec"] = emit
    out["pair_spec"] = pair
    return out


class BoundTables:
    """Tables bound to the oracle's lookup routines (keeps arrays alive)."""

    def __init__(self, tabs: dict):
        self.arrays = {k: np.ascontiguousarray(tabs[k], dtype=np.float64)
                       for k in ("ln_hrad", "ln_g", "emit_q", "pair_lnh", "pair_q")}
        self.se, self.sp = _spec(tabs["emit_spec"]), _spec(tabs["pair_spec"])
        self.t = Tables()
        lib().or_tables_bind(C.byref(self.t), C.byref(self.se), C.byref(self.sp),
                             *[_ptr(self.arrays[k]) for k in ("ln_hrad", "ln_g", "emit_q", "pair_lnh", "pair_q")])
        es, ps = tabs["emit_spec"], tabs["pair_spec"]
        if es.get("interp", 0) or ps.get("interp", 0):
            self.emit_m = quantile_spline(self.arrays["emit_q"], es["n_chi"], es["n_q"], *_spacings(es))
            self.pair_m = quantile_spline(self.arrays["pair_q"], ps["n_chi"], ps["n_q"], *_spacings(ps))
            lib().or_tables_bind_spline(C.byref(self.t), _ptr(self.emit_m.reshape(-1)), _ptr(self.pair_m.reshape(-1)))

    def h_rad(self, chi):
        oor = C.c_int(0)
        return lib().or_lookup_h_rad(C.byref(self.t), chi, C.byref(oor))

    def g(self, chi):
        return lib().or_lookup_g(C.byref(self.t), chi)

    def h_pair(self, chi):
        oor = C.c_int(0)
        return lib().or_lookup_h_pair(C.byref(self.t), chi, C.byref(oor))

    def sample_xi(self, chi, r):
        return lib().or_sample_xi(C.byref(self.t), chi, r)

    def sample_eta(self, chi, r):
        return lib().or_sample_eta(C.byref(self.t), chi, r)


# --------------------------------------------------------------------------
# particles, fields and the step
# --------------------------------------------------------------------------
def _ptr(a, ct=C.c_double):
    if a is None:
        return None
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(C.POINTER(ct))


FLOAT_KEYS = ("x", "y", "z", "ux", "uy", "uz", "tau", "w", "chi")


def new_species(capacity: int) -> dict:
    s = {k: np.zeros(capacity, np.float64) for k in FLOAT_KEYS}
    s["uid"] = np.zeros(capacity, np.uint64)
    s["n_ev"] = np.zeros(capacity, np.uint32)
    s["n"] = 0
    return s


def species_from(arrays: dict, capacity: int | None = None) -> dict:
    n = len(arrays["x"])
    cap = max(n, capacity or n)
    s = new_species(cap)
    for k in FLOAT_KEYS:
        if k in arrays:
            s[k][:n] = arrays[k]
    if "w" not in arrays:
        s["w"][:n] = 1.0
    s["uid"][:n] = arrays.get("uid", np.arange(n, dtype=np.uint64))
    if "n_ev" in arrays:
        s["n_ev"][:n] = arrays["n_ev"]
    s["n"] = n
    return s


def _species_struct(s: dict | None):
    if s is None:
        return None
    st = Species()
    st.n = int(s["n"])
    st.capacity = len(s["x"])
    for k in FLOAT_KEYS:
        setattr(st, k, _ptr(s[k]))
    st.uid = _ptr(s["uid"], C.c_uint64)
    st.n_ev = _ptr(s["n_ev"], C.c_uint32)
    return st


def view(s: dict) -> dict:
    """The live part of a species."""
    n = int(s["n"])
    return {k: s[k][:n] for k in FLOAT_KEYS + ("uid", "n_ev")}


def init_tau(s: dict, seed: int):
    st = _species_struct(s)
    lib().or_init_tau(C.byref(st), seed)


def make_field(kind, E=(0, 0, 0), B=(0, 0, 0), a0=0.0, n_periods=10.0, grid=None,
               shape=(0, 0, 0), spacing=(1, 1, 1), origin=(0, 0, 0), tperp=None, tpar=None):
    f = Field()
    f.kind = kind
    f.E = (C.c_double * 3)(*E)
    f.B = (C.c_double * 3)(*B)
    f.a0, f.n_periods = a0, n_periods
    keep = []
    if grid is not None:
        g6 = np.ascontiguousarray(grid, dtype=np.float32)
        keep.append(g6)
        per = g6.reshape(6, -1)
        for c in range(6):
            f.grid[c] = per[c].ctypes.data_as(_fp)
    if tperp is not None:
        tp = np.ascontiguousarray(tperp, dtype=np.float64)
        tq = np.ascontiguousarray(tpar, dtype=np.float64)
        keep += [tp, tq]
        f.tperp6, f.tpar6 = _ptr(tp), _ptr(tq)
    f.nx, f.ny, f.nz = shape
    f.dx, f.dy, f.dz = spacing
    f.x0, f.y0, f.z0 = origin
    f._keep = keep
    return f


def field_at(f: Field, t, x, y, z):
    E = (C.c_double * 3)()
    B = (C.c_double * 3)()
    lib().or_field_at(C.byref(f), t, x, y, z, E, B)
    return np.array(E[:]), np.array(B[:])


def yee_fill_separable(shape, a0, tperp6, tpar6) -> np.ndarray:
    nx, ny, nz = shape
    grid = np.zeros((6, nx, ny, nz), np.float32)
    tperp6 = np.ascontiguousarray(tperp6, dtype=np.float64)
    tpar6 = np.ascontiguousarray(tpar6, dtype=np.float64)
    lib().or_yee_fill_separable(grid.ctypes.data_as(_fp), nx, ny, nz, a0,
                                _ptr(tperp6), _ptr(tpar6))
    return grid


def chi_lepton(u_, p, gamma, E, B):
    U = _units_struct(u_["lambda"]) if isinstance(u_, dict) else u_
    arr = lambda v: (C.c_double * 3)(*[float(a) for a in v])
    return lib().or_chi_lepton(C.byref(U), arr(p), float(gamma), arr(E), arr(B))


def chi_photon(u_, k, E, B):
    U = _units_struct(u_["lambda"]) if isinstance(u_, dict) else u_
    arr = lambda v: (C.c_double * 3)(*[float(a) for a in v])
    return lib().or_chi_photon(C.byref(U), arr(k), arr(E), arr(B))


VAR_SOKOLOV_G, VAR_PAIR_MOMENTUM = 1, 2


def make_step(t, dt, seed, rad_model=RAD_HYBRID, chi_switch=1e-3, gamma_photon_min=2.0,
              chi_photon_push_min=1e-3, max_events=4, no_recoil=0, variants=0, rate_scale=1.0) -> Step:
    return Step(t, dt, seed, rad_model, chi_switch, gamma_photon_min, chi_photon_push_min,
                max_events, no_recoil, variants, rate_scale)


class Tally:
    def __init__(self):
        self.t = np.zeros(8, np.float64)
        self.c = np.zeros(16, np.int64)

    def as_dict(self):
        d = {("E_" + n): float(v) for n, v in zip(T_NAMES, self.t) if not n.startswith("_")}
        d.update({("N_" + n): int(v) for n, v in zip(C_NAMES, self.c) if not n.startswith("_")})
        return d


def push_emit(tabs: BoundTables, lambda_m, charge, lep: dict, field: Field,
              ph_push: dict | None, ph_rec: dict | None, step: Step, uid_next: list,
              tally: Tally, threads: int = 0) -> int:
    """One lepton step; threads > 0 runs it on that many OpenMP threads
    (or_push_emit_omp: the same results, energy tallies to rounding)."""
    U = _units_struct(lambda_m)
    L, P, R = _species_struct(lep), _species_struct(ph_push), _species_struct(ph_rec)
    un = (C.c_uint64 * 1)(uid_next[0])
    args = (C.byref(tabs.t), C.byref(U), float(charge), C.byref(L), C.byref(field),
            C.byref(P) if P is not None else None, C.byref(R) if R is not None else None,
            C.byref(step), un, _ptr(tally.t), tally.c.ctypes.data_as(C.POINTER(C.c_int64)))
    rc = lib().or_push_emit_omp(*args, int(threads)) if threads > 0 else lib().or_push_emit(*args)
    uid_next[0] = int(un[0])
    if P is not None:
        ph_push["n"] = P.n
    if R is not None:
        ph_rec["n"] = R.n
    return rc


def pair_create(tabs: BoundTables, lambda_m, ph: dict, field: Field, elec: dict, posi: dict,
                step: Step, uid_next: list, tally: Tally, n_limit: int | None = None, threads: int = 0) -> int:
    """One photon step; threads > 0 runs it on that many OpenMP threads."""
    U = _units_struct(lambda_m)
    P, Em, Ep = _species_struct(ph), _species_struct(elec), _species_struct(posi)
    un = (C.c_uint64 * 1)(uid_next[0])
    lim = int(ph["n"]) if n_limit is None else int(n_limit)
    args = (C.byref(tabs.t), C.byref(U), C.byref(P), lim, C.byref(field), C.byref(Em), C.byref(Ep),
            C.byref(step), un, _ptr(tally.t), tally.c.ctypes.data_as(C.POINTER(C.c_int64)))
    rc = lib().or_pair_create_omp(*args, int(threads)) if threads > 0 else lib().or_pair_create(*args)
    uid_next[0] = int(un[0])
    ph["n"], elec["n"], posi["n"] = P.n, Em.n, Ep.n
    return rc


def sort_by_cell(s: dict, shape, spacing, origin, bands: int = 1):
    st = _species_struct(s)
    lib().or_sort_by_cell_bands(C.byref(st), *[int(v) for v in shape], *[float(v) for v in spacing],
                                *[float(v) for v in origin], int(bands))


def yee_advance(grid6: np.ndarray, J3: np.ndarray | None, shape, spacing, dt: float, steps: int = 1):
    """Yee advance(s) of an FP32 grid [6][nx][ny][nz] in place (periodic), with
    the FP32 current J3 [3][nx][ny][nz] (or none)."""
    assert grid6.dtype == np.float32 and grid6.flags["C_CONTIGUOUS"]
    jp = None
    if J3 is not None:
        J3 = np.ascontiguousarray(J3, dtype=np.float32)
        jp = _ptr(J3, C.c_float)
    for _ in range(steps):
        lib().or_yee_advance(_ptr(grid6, C.c_float), jp, *[int(v) for v in shape], *[float(v) for v in spacing],
                             float(dt))


def deposit_current(s: dict, old, first: int, q: float, j_scale: float, dt: float, shape, spacing, origin,
                    J3: np.ndarray | None = None):
    """Esirkepov currents of particles [first, n) (old = (xo, yo, zo) arrays of
    their start positions, or None to go back along u/gamma); returns
    (J3 [3][nx][ny][nz] FP64, number skipped)."""
    nx, ny, nz = (int(v) for v in shape)
    if J3 is None:
        J3 = np.zeros((3, nx, ny, nz))
    ptrs = [None, None, None]
    keep = []
    if old is not None:
        for c in range(3):
            a = np.ascontiguousarray(old[c], dtype=np.float64)
            keep.append(a)
            ptrs[c] = _ptr(a)
    sk = lib().or_deposit_current(C.byref(_species_struct(s)), *ptrs, int(first), float(q), float(j_scale), float(dt),
                                  nx, ny, nz, *[float(v) for v in spacing], *[float(v) for v in origin], _ptr(J3))
    return J3, int(sk)


def deposit_charge(s: dict, q: float, j_scale: float, shape, spacing, origin, rho: np.ndarray | None = None):
    nx, ny, nz = (int(v) for v in shape)
    if rho is None:
        rho = np.zeros((nx, ny, nz))
    lib().or_deposit_charge(C.byref(_species_struct(s)), float(q), float(j_scale), nx, ny, nz,
                            *[float(v) for v in spacing], *[float(v) for v in origin], _ptr(rho))
    return rho


def merge_spec(box_origin, spacing, shape, massive: bool, octave_min: int, n_octaves: int, sub_bins: int,
               n_dir: int, min_group: int) -> MergeSpec:
    m = MergeSpec()
    m.x0, m.y0, m.z0 = (float(v) for v in box_origin)
    m.dx, m.dy, m.dz = (float(v) for v in spacing)
    m.nx, m.ny, m.nz = (int(v) for v in shape)
    m.massive = int(bool(massive))
    m.octave_min, m.n_octaves, m.sub_bins = int(octave_min), int(n_octaves), int(sub_bins)
    m.n_dir, m.min_group = int(n_dir), int(min_group)
    return m


def merge(spec: MergeSpec, s: dict, seed: int, uid_next: int, capacity: int | None = None):
    """Merging of super-particles (the oracle's or_merge).  Returns the new
    species and the advanced id counter; raises if capacity is too small."""
    dst = new_species(max(1, capacity if capacity is not None else int(s["n"])))
    u = np.array([uid_next], np.uint64)
    n = lib().or_merge(C.byref(spec), C.byref(_species_struct(s)), C.byref(_species_struct(dst)), seed,
                       _ptr(u, C.c_uint64))
    if n < 0:
        raise ValueError("or_merge: destination too small")
    dst["n"] = int(n)
    return dst, int(u[0])


def spectrum(s: dict, photons: bool, e_min: float, e_max: float, n_bins: int, weight_scale: float):
    """Log-binned energy spectrum, by its definition.  e = |u| for photons
    (|k| = gamma_gamma) or sqrt(1 + |u|^2) for leptons; bin 0 below e_min
    (and for e = 0 or non-finite e), 1 + floor(n ln(e/e_min)/ln(e_max/e_min))
    in range, n + 1 at or above e_max; decayed photons (tau = +-inf) are
    skipped.  Returns (counts, weight sums in units of 1/weight_scale)."""
    v = view(s)
    u2 = v["ux"] ** 2 + v["uy"] ** 2 + v["uz"] ** 2
    e = np.sqrt(u2) if photons else np.sqrt(1.0 + u2)
    keep = ~np.isinf(v["tau"]) if photons else np.ones(len(e), bool)
    e, w = e[keep], v["w"][keep]
    b = np.zeros(len(e), np.int64)
    with np.errstate(invalid="ignore", divide="ignore"):
        hi = e >= e_max
        mid = (e >= e_min) & ~hi
        f = np.floor((np.log(e[mid]) - np.log(e_min)) * (n_bins / np.log(e_max / e_min)))
    b[mid] = 1 + np.clip(f, 0, n_bins - 1).astype(np.int64)
    b[hi] = n_bins + 1
    counts = np.bincount(b, minlength=n_bins + 2).astype(np.int64)
    wsum = np.bincount(b, weights=None, minlength=n_bins + 2).astype(np.int64) * 0
    np.add.at(wsum, b, np.rint(w * weight_scale).astype(np.int64))
    return counts, wsum

