"""ctypes binding of libqed (include/qed.h).

The functions below carry the C names and only marshal arguments; every step
of the particle update runs in the library's HIP kernels.  PyTorch tensors
provide device memory and the current stream.  If libqed.so is missing the
first call raises: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libqed.so")

QED_OK, QED_ERR_ARG, QED_ERR_HIP, QED_ERR_CAPACITY, QED_ERR_RANGE, QED_ERR_NOMEM = 0, -1, -2, -3, -4, -5
QED_F64, QED_F32 = 0, 1
QED_FIELD_UNIFORM, QED_FIELD_PLANE_WAVE, QED_FIELD_YEE = 0, 1, 2
QED_RAD_NONE, QED_RAD_SOKOLOV, QED_RAD_MC, QED_RAD_HYBRID = 0, 1, 2, 3
QED_INTERP_LINEAR, QED_INTERP_SPLINE = 0, 1
QED_N_ENERGY, QED_N_COUNT = 8, 16

ENERGY_NAMES = ["work", "erad", "epush", "erec", "edrop", "esub", "epair", "_e7"]
COUNT_NAMES = ["emit", "push", "rec", "drop", "sub", "cap", "range", "sokolov", "mc",
               "pair", "phstep", "nan", "overflow", "nogather", "_c14", "_c15"]


class QedError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libqed error {code}: {msg}")
        self.code = code


_vp = C.c_void_p
_dp = C.POINTER(C.c_double)


class qed_units(C.Structure):
    _fields_ = [("lambda_", C.c_double), ("omega_r", C.c_double), ("alpha_f", C.c_double),
                ("Es_hat", C.c_double), ("A_hat", C.c_double), ("tau0_hat", C.c_double)]


class qed_table_spec(C.Structure):
    _fields_ = [("chi_min", C.c_double), ("chi_max", C.c_double), ("n_chi", C.c_int32),
                ("n_q", C.c_int32), ("logit_max", C.c_double), ("interp", C.c_int32), ("reserved", C.c_int32)]


class qed_species(C.Structure):
    _fields_ = [("prec", C.c_int32), ("reserved", C.c_int32),
                ("x", _vp), ("y", _vp), ("z", _vp), ("ux", _vp), ("uy", _vp), ("uz", _vp),
                ("tau", _vp), ("w", _vp), ("chi", _vp), ("uid", _vp), ("n_event", _vp),
                ("d_count", _vp), ("capacity", C.c_int64)]


class qed_field(C.Structure):
    _fields_ = [("kind", C.c_int32), ("reserved", C.c_int32), ("E", C.c_double * 3), ("B", C.c_double * 3),
                ("a0", C.c_double), ("n_periods", C.c_double), ("grid", _vp),
                ("nx", C.c_int64), ("ny", C.c_int64), ("nz", C.c_int64),
                ("dx", C.c_double), ("dy", C.c_double), ("dz", C.c_double),
                ("x0", C.c_double), ("y0", C.c_double), ("z0", C.c_double),
                ("bound", _vp), ("bound_block", C.c_int64)]


QED_VAR_SOKOLOV_G, QED_VAR_PAIR_MOMENTUM = 1, 2


class qed_merge_spec(C.Structure):
    _fields_ = [(n, C.c_double) for n in ("x0", "y0", "z0", "dx", "dy", "dz")] + \
               [(n, C.c_int64) for n in ("nx", "ny", "nz")] + \
               [(n, C.c_int32) for n in ("massive", "octave_min", "n_octaves", "sub_bins", "n_dir", "min_group")]


class qed_step(C.Structure):
    _fields_ = [("t", C.c_double), ("dt", C.c_double), ("seed", C.c_uint64),
                ("rad_model", C.c_int32), ("max_events", C.c_int32),
                ("chi_switch", C.c_double), ("gamma_photon_min", C.c_double),
                ("chi_photon_push_min", C.c_double), ("no_recoil", C.c_int32),
                ("variants", C.c_int32), ("d_step", _vp)]


class qed_tally(C.Structure):
    _fields_ = [("energy", _vp), ("count", _vp), ("n_slots", C.c_int64)]


class qed_status_report(C.Structure):
    _fields_ = [("flags", C.c_int64), ("needed", C.c_int64 * 4), ("chi_above_table", C.c_int64)]


class qed_schedule(C.Structure):
    _fields_ = [("block", C.c_int32), ("items_per_thread", C.c_int32),
                ("blocks_per_cu", C.c_int32), ("max_blocks", C.c_int32)]


class qed_bunches(C.Structure):
    _fields_ = [("n_bunches", C.c_int32), ("reserved", C.c_int32), ("offsets", _vp),
                ("a0", _vp), ("n_periods", _vp)]


_P = C.POINTER
_SIGS = {
    "qed_last_error": ([], C.c_char_p),
    "qed_units_init": ([C.c_double, _P(qed_units)], C.c_int32),
    "qed_tables_compute_host": ([_P(qed_table_spec), _P(qed_table_spec)] + [_dp] * 5, C.c_int32),
    "qed_tables_build": ([_P(qed_table_spec), _P(qed_table_spec), _P(_vp)], C.c_int32),
    "qed_tables_load": ([_P(qed_table_spec), _P(qed_table_spec)] + [_dp] * 5 + [_P(_vp)], C.c_int32),
    "qed_tables_export": ([_vp, C.c_int32, _dp, C.c_size_t], C.c_int32),
    "qed_tables_free": ([_vp], None),
    "qed_init_optical_depth": ([_P(qed_species), C.c_uint64, _vp], C.c_int32),
    "qed_yee_fill_separable": ([_vp, C.c_int64, C.c_int64, C.c_int64, C.c_double, _vp, _vp, _vp], C.c_int32),
    "qed_tally_reduce": ([_P(qed_tally), _dp, _P(C.c_int64), _vp], C.c_int32),
    "qed_workspace_create": ([C.c_int64, C.c_int64, _P(_vp)], C.c_int32),
    "qed_workspace_free": ([_vp], None),
    "qed_sync_status": ([_vp, _P(qed_status_report), C.c_int32, _vp], C.c_int32),
    "qed_push_emit": ([_vp, _vp, _P(qed_units), C.c_double, _P(qed_species), _P(qed_field),
                       _P(qed_species), _P(qed_species), _P(qed_tally), _P(qed_step), _vp,
                       _P(qed_schedule), _vp], C.c_int32),
    "qed_push_emit_static": ([_vp, _P(qed_units), C.c_double, _P(qed_species), _P(qed_field),
                              _P(qed_species), _P(qed_species), _P(qed_tally), _P(qed_step), _vp, _vp,
                              _P(qed_schedule), _vp], C.c_int32),
    "qed_pair_create": ([_vp, _vp, _P(qed_units), _P(qed_species), _P(qed_field), _P(qed_species),
                         _P(qed_species), _P(qed_tally), _P(qed_step), _vp, _P(qed_schedule), _vp], C.c_int32),
    "qed_compact": ([_vp, _P(qed_species), _P(qed_schedule), _vp], C.c_int32),
    "qed_push_emit_batched": ([_vp, _vp, _P(qed_units), C.c_double, _P(qed_species), _P(qed_bunches),
                               _P(qed_species), _P(qed_species), _P(qed_tally), _P(qed_step), _vp,
                               _P(qed_schedule), _vp], C.c_int32),
    "qed_autotune_batched": ([_vp, _vp, _P(qed_units), C.c_double, _P(qed_species), _P(qed_bunches),
                              _P(qed_species), _P(qed_step), _P(qed_schedule), C.c_int32, C.c_int32,
                              C.c_char_p, _P(qed_schedule), _dp, _vp], C.c_int32),
    "qed_step_advance": ([_vp, _vp], C.c_int32),
    "qed_spectrum": ([_P(qed_species), C.c_int32, C.c_double, C.c_double, C.c_int32, C.c_double, _vp, _vp, _vp],
                     C.c_int32),
    "qed_sorter_create": ([C.c_int64, _P(_vp)], C.c_int32),
    "qed_sorter_free": ([_vp], None),
    "qed_sort_by_cell": ([_vp, _vp, _P(qed_species), _P(qed_species), _P(qed_field), _vp], C.c_int32),
    "qed_sort_by_cell_bands": ([_vp, _vp, _P(qed_species), _P(qed_species), _P(qed_field), C.c_int32, _vp],
                               C.c_int32),
    "qed_field_bound": ([_P(qed_field), C.c_int32, _vp, _vp], C.c_int32),
    "qed_yee_advance": ([_vp, _vp, _P(qed_field), C.c_double, _vp], C.c_int32),
    "qed_deposit_current": ([_P(qed_species), _vp, _vp, _vp, _vp, C.c_double, C.c_double, C.c_double, _P(qed_field),
                             _vp, _vp, _vp], C.c_int32),
    "qed_deposit_charge": ([_P(qed_species), C.c_double, C.c_double, _P(qed_field), _vp, _vp], C.c_int32),
    "qed_save_positions": ([_P(qed_species), _vp, _vp, _vp, _vp], C.c_int32),
    "qed_merger_create": ([C.c_int64, _P(_vp)], C.c_int32),
    "qed_merger_free": ([_vp], None),
    "qed_merge": ([_vp, _vp, _P(qed_merge_spec), _P(qed_species), _P(qed_species), C.c_uint64, _vp, _vp],
                  C.c_int32),
}

_lib = None


def lib():
    """The loaded libqed.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1311_1107_amd.build`")
        L = C.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def _check(rc):
    if rc != QED_OK:
        raise QedError(rc, lib().qed_last_error().decode())
    return rc


def _ref(x):
    return C.byref(x) if x is not None else None


def _stream(stream):
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    return C.c_void_p(stream)


# ---------------------------------------------------------------- wrappers --
def qed_units_init(lambda_m: float) -> qed_units:
    u = qed_units()
    _check(lib().qed_units_init(lambda_m, C.byref(u)))
    return u


def _spec(d) -> qed_table_spec:
    if isinstance(d, qed_table_spec):
        return d
    return qed_table_spec(d["chi_min"], d["chi_max"], d["n_chi"], d["n_q"], d["logit_max"],
                          d.get("interp", QED_INTERP_LINEAR), 0)


def qed_tables_compute_host(emit: dict, pair: dict) -> dict:
    se, sp = _spec(emit), _spec(pair)
    out = {"ln_hrad": np.zeros(se.n_chi), "ln_g": np.zeros(se.n_chi), "emit_q": np.zeros(se.n_chi * se.n_q),
           "pair_lnh": np.zeros(sp.n_chi), "pair_q": np.zeros(sp.n_chi * sp.n_q)}
    _check(lib().qed_tables_compute_host(C.byref(se), C.byref(sp),
                                         *[out[k].ctypes.data_as(_dp) for k in
                                           ("ln_hrad", "ln_g", "emit_q", "pair_lnh", "pair_q")]))
    return out


def qed_tables_build(emit: dict, pair: dict) -> C.c_void_p:
    h = C.c_void_p()
    _check(lib().qed_tables_build(C.byref(_spec(emit)), C.byref(_spec(pair)), C.byref(h)))
    return h


def qed_tables_load(emit: dict, pair: dict, arrays: dict) -> C.c_void_p:
    a = {k: np.ascontiguousarray(arrays[k], dtype=np.float64) for k in
         ("ln_hrad", "ln_g", "emit_q", "pair_lnh", "pair_q")}
    h = C.c_void_p()
    _check(lib().qed_tables_load(C.byref(_spec(emit)), C.byref(_spec(pair)),
                                 *[a[k].ctypes.data_as(_dp) for k in ("ln_hrad", "ln_g", "emit_q", "pair_lnh", "pair_q")],
                                 C.byref(h)))
    return h


def qed_tables_export(handle, which: int, n: int) -> np.ndarray:
    out = np.zeros(n)
    _check(lib().qed_tables_export(handle, which, out.ctypes.data_as(_dp), n))
    return out


def qed_tables_free(handle):
    lib().qed_tables_free(handle)


def qed_workspace_create(max_particles: int, max_leptons: int) -> C.c_void_p:
    h = C.c_void_p()
    _check(lib().qed_workspace_create(int(max_particles), int(max_leptons), C.byref(h)))
    return h


def qed_workspace_free(handle):
    lib().qed_workspace_free(handle)


def qed_init_optical_depth(species: qed_species, seed: int, stream=None):
    _check(lib().qed_init_optical_depth(C.byref(species), seed, _stream(stream)))


def qed_yee_fill_separable(grid_ptr, nx, ny, nz, a0, tperp_ptr, tpar_ptr, stream=None):
    _check(lib().qed_yee_fill_separable(C.c_void_p(grid_ptr), nx, ny, nz, a0, C.c_void_p(tperp_ptr),
                                        C.c_void_p(tpar_ptr), _stream(stream)))


def qed_push_emit(tables, ws, units, charge, lep, field, ph_push, ph_rec, tally, step, uid_next_ptr,
                  sched=None, stream=None):
    _check(lib().qed_push_emit(tables, ws, C.byref(units), float(charge), C.byref(lep), C.byref(field),
                               _ref(ph_push), _ref(ph_rec), C.byref(tally), C.byref(step),
                               C.c_void_p(uid_next_ptr), _ref(sched), _stream(stream)))


def qed_push_emit_static(tables, units, charge, lep, field, ph_push, ph_rec, tally, step, uid_next_ptr,
                         status_ptr, sched=None, stream=None):
    _check(lib().qed_push_emit_static(tables, C.byref(units), float(charge), C.byref(lep), C.byref(field),
                                      _ref(ph_push), _ref(ph_rec), C.byref(tally), C.byref(step),
                                      C.c_void_p(uid_next_ptr), C.c_void_p(status_ptr), _ref(sched),
                                      _stream(stream)))


def qed_push_emit_batched(tables, ws, units, charge, lep, bunches, ph_push, ph_rec, tally, step, uid_next_ptr,
                          sched=None, stream=None):
    _check(lib().qed_push_emit_batched(tables, ws, C.byref(units), float(charge), C.byref(lep), C.byref(bunches),
                                       _ref(ph_push), _ref(ph_rec), C.byref(tally), C.byref(step),
                                       C.c_void_p(uid_next_ptr), _ref(sched), _stream(stream)))


def qed_pair_create(tables, ws, units, photons, field, elec, posi, tally, step, uid_next_ptr,
                    sched=None, stream=None):
    _check(lib().qed_pair_create(tables, ws, C.byref(units), C.byref(photons), C.byref(field), C.byref(elec),
                                 C.byref(posi), C.byref(tally), C.byref(step), C.c_void_p(uid_next_ptr),
                                 _ref(sched), _stream(stream)))


def qed_compact(ws, species, sched=None, stream=None):
    _check(lib().qed_compact(ws, C.byref(species), _ref(sched), _stream(stream)))


def qed_autotune_batched(tables, ws, units, charge, lep, bunches, ph_rec, step, candidates, trial_steps,
                         cache_path=None, stream=None):
    arr = (qed_schedule * len(candidates))(*candidates)
    best = qed_schedule()
    ms = C.c_double(0)
    _check(lib().qed_autotune_batched(tables, ws, C.byref(units), float(charge), C.byref(lep), C.byref(bunches),
                                      _ref(ph_rec), C.byref(step), arr, len(candidates), trial_steps,
                                      cache_path.encode() if cache_path else None, C.byref(best), C.byref(ms),
                                      _stream(stream)))
    return best, ms.value


def qed_sync_status(ws, clear: bool = True, stream=None, raise_on_error: bool = True):
    rep = qed_status_report()
    rc = lib().qed_sync_status(ws, C.byref(rep), 1 if clear else 0, _stream(stream))
    if raise_on_error:
        _check(rc)
    return rc, rep


def qed_tally_reduce(tally: qed_tally, stream=None):
    e = np.zeros(QED_N_ENERGY)
    c = np.zeros(QED_N_COUNT, np.int64)
    _check(lib().qed_tally_reduce(C.byref(tally), e.ctypes.data_as(_dp), c.ctypes.data_as(C.POINTER(C.c_int64)),
                                  _stream(stream)))
    return e, c


def qed_sorter_create(max_particles: int) -> C.c_void_p:
    h = C.c_void_p()
    _check(lib().qed_sorter_create(int(max_particles), C.byref(h)))
    return h


def qed_sorter_free(handle):
    lib().qed_sorter_free(handle)


def qed_sort_by_cell(sorter, ws, src, dst, grid_field, stream=None, bands=1):
    if bands == 1:
        _check(lib().qed_sort_by_cell(sorter, ws, C.byref(src), C.byref(dst), C.byref(grid_field), _stream(stream)))
    else:
        _check(lib().qed_sort_by_cell_bands(sorter, ws, C.byref(src), C.byref(dst), C.byref(grid_field), int(bands),
                                            _stream(stream)))


def qed_field_bound(field, block, bound_ptr, stream=None):
    _check(lib().qed_field_bound(C.byref(field), int(block), C.c_void_p(bound_ptr), _stream(stream)))


def qed_yee_advance(grid_ptr, J_ptr, geometry, dt, stream=None):
    _check(lib().qed_yee_advance(C.c_void_p(grid_ptr), C.c_void_p(J_ptr) if J_ptr else None, C.byref(geometry),
                                 float(dt), _stream(stream)))


def qed_deposit_current(species, old_ptrs, first_ptr, charge, j_scale, dt, geometry, J_ptr, skipped_ptr=None,
                        stream=None):
    xo, yo, zo = (C.c_void_p(p) for p in old_ptrs) if old_ptrs else (None, None, None)
    _check(lib().qed_deposit_current(C.byref(species), xo, yo, zo, C.c_void_p(first_ptr) if first_ptr else None,
                                     float(charge), float(j_scale), float(dt), C.byref(geometry), C.c_void_p(J_ptr),
                                     C.c_void_p(skipped_ptr) if skipped_ptr else None, _stream(stream)))


def qed_deposit_charge(species, charge, j_scale, geometry, rho_ptr, stream=None):
    _check(lib().qed_deposit_charge(C.byref(species), float(charge), float(j_scale), C.byref(geometry),
                                    C.c_void_p(rho_ptr), _stream(stream)))


def qed_save_positions(species, old_ptrs, stream=None):
    _check(lib().qed_save_positions(C.byref(species), *[C.c_void_p(p) for p in old_ptrs], _stream(stream)))


def qed_merger_create(max_particles: int) -> C.c_void_p:
    h = C.c_void_p()
    _check(lib().qed_merger_create(int(max_particles), C.byref(h)))
    return h


def qed_merger_free(handle):
    lib().qed_merger_free(handle)


def qed_merge(merger, ws, spec, src, dst, seed, uid_next_ptr, stream=None):
    _check(lib().qed_merge(merger, ws, C.byref(spec), C.byref(src), C.byref(dst), int(seed),
                           C.c_void_p(uid_next_ptr), _stream(stream)))


def qed_spectrum(species, photons, e_min, e_max, n_bins, weight_scale, count_ptr, wsum_ptr, stream=None):
    _check(lib().qed_spectrum(C.byref(species), 1 if photons else 0, float(e_min), float(e_max), int(n_bins),
                              float(weight_scale), C.c_void_p(count_ptr), C.c_void_p(wsum_ptr), _stream(stream)))


def qed_step_advance(d_step_ptr, stream=None):
    _check(lib().qed_step_advance(C.c_void_p(d_step_ptr), _stream(stream)))
