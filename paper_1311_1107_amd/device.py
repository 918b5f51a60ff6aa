"""Device memory for the C interface, held in torch tensors.

torch provides allocation, copies and the current stream; the particle update
itself runs only in libqed's kernels (see binding.py).
"""
from __future__ import annotations

import ctypes as C
import math

import numpy as np
import torch

from . import binding as B

FLOAT_KEYS = ("x", "y", "z", "ux", "uy", "uz", "w", "chi")


def _dtype(prec):
    return torch.float64 if prec == B.QED_F64 else torch.float32


class Species:
    """Structure-of-arrays particles in device memory with a device-side count."""

    def __init__(self, capacity: int, prec: int = B.QED_F64, chi: bool = True, device: str = "cuda"):
        self.capacity = int(capacity)
        self.prec = prec
        dt = _dtype(prec)
        n = max(self.capacity, 1)
        self.a = {k: torch.zeros(n, dtype=dt, device=device) for k in FLOAT_KEYS if (k != "chi" or chi)}
        self.a["tau"] = torch.zeros(n, dtype=torch.float64, device=device)
        self.a["uid"] = torch.zeros(n, dtype=torch.int64, device=device)      # uint64 bit patterns
        self.a["n_ev"] = torch.zeros(n, dtype=torch.int32, device=device)     # uint32 bit patterns
        self.count = torch.zeros(1, dtype=torch.int64, device=device)
        self._struct = None

    def struct(self) -> B.qed_species:
        if self._struct is None:
            s = B.qed_species()
            s.prec = self.prec
            for k in ("x", "y", "z", "ux", "uy", "uz", "tau", "w"):
                setattr(s, k, self.a[k].data_ptr())
            s.chi = self.a["chi"].data_ptr() if "chi" in self.a else None
            s.uid = self.a["uid"].data_ptr()
            s.n_event = self.a["n_ev"].data_ptr()
            s.d_count = self.count.data_ptr()
            s.capacity = self.capacity
            self._struct = s
        return self._struct

    def view(self, start: int, count_ptr: int, capacity: int) -> B.qed_species:
        """A qed_species over entries [start, start+capacity) whose count lives at count_ptr."""
        s = B.qed_species()
        s.prec = self.prec
        for k in ("x", "y", "z", "ux", "uy", "uz", "tau", "w"):
            t = self.a[k]
            setattr(s, k, t.data_ptr() + start * t.element_size())
        s.chi = self.a["chi"].data_ptr() + start * self.a["chi"].element_size() if "chi" in self.a else None
        s.uid = self.a["uid"].data_ptr() + start * 8
        s.n_event = self.a["n_ev"].data_ptr() + start * 4
        s.d_count = count_ptr
        s.capacity = capacity
        return s

    def upload(self, arrays: dict, n: int | None = None):
        n = len(arrays["x"]) if n is None else n
        if n > self.capacity:
            raise ValueError("more particles than capacity")
        for k, v in arrays.items():
            if k not in self.a or v is None:
                continue
            if k == "uid":
                t = torch.from_numpy(np.ascontiguousarray(v, dtype=np.uint64).view(np.int64))
            elif k == "n_ev":
                t = torch.from_numpy(np.ascontiguousarray(v, dtype=np.uint32).view(np.int32))
            else:
                t = torch.from_numpy(np.ascontiguousarray(v)).to(self.a[k].dtype)
            self.a[k][:n].copy_(t[:n])
        if "w" not in arrays:
            self.a["w"][:n] = 1.0
        self.count.fill_(n)

    def n(self) -> int:
        return int(self.count.item())

    def download(self, n: int | None = None) -> dict:
        n = self.n() if n is None else n
        out = {}
        for k, t in self.a.items():
            v = t[:n].cpu().numpy()
            if k == "uid":
                v = v.view(np.uint64)
            elif k == "n_ev":
                v = v.view(np.uint32)
            out[k] = v
        return out


class Tally:
    def __init__(self, n_slots: int, device: str = "cuda"):
        self.energy = torch.zeros(max(1, n_slots) * B.QED_N_ENERGY, dtype=torch.float64, device=device)
        self.count = torch.zeros(B.QED_N_COUNT, dtype=torch.int64, device=device)
        self.s = B.qed_tally(self.energy.data_ptr(), self.count.data_ptr(), max(1, n_slots))

    def zero(self):
        self.energy.zero_()
        self.count.zero_()

    def reduce(self) -> dict:
        e, c = B.qed_tally_reduce(self.s)
        d = {"E_" + k: float(v) for k, v in zip(B.ENERGY_NAMES, e) if not k.startswith("_")}
        d.update({"N_" + k: int(v) for k, v in zip(B.COUNT_NAMES, c) if not k.startswith("_")})
        return d


class Tables:
    """Rate and quantile tables on the device (built here, or loaded from arrays)."""

    def __init__(self, emit: dict, pair: dict, arrays: dict | None = None):
        self.emit, self.pair = dict(emit), dict(pair)
        self.h = B.qed_tables_load(emit, pair, arrays) if arrays is not None else B.qed_tables_build(emit, pair)

    def export(self) -> dict:
        ne, nq = self.emit["n_chi"], self.emit["n_q"]
        npc, npq = self.pair["n_chi"], self.pair["n_q"]
        sizes = [ne, ne, ne * nq, npc, npc * npq]
        names = ["ln_hrad", "ln_g", "emit_q", "pair_lnh", "pair_q"]
        return {k: B.qed_tables_export(self.h, i, n) for i, (k, n) in enumerate(zip(names, sizes))}

    def __del__(self):
        try:
            if self.h:
                B.qed_tables_free(self.h)
        except Exception:
            pass


class Workspace:
    def __init__(self, max_particles: int, max_leptons: int | None = None):
        self.h = B.qed_workspace_create(max_particles, max_particles if max_leptons is None else max_leptons)

    def status(self, clear=True, raise_on_error=True):
        return B.qed_sync_status(self.h, clear=clear, raise_on_error=raise_on_error)

    def __del__(self):
        try:
            if self.h:
                B.qed_workspace_free(self.h)
        except Exception:
            pass


class Sorter:
    """Scratch of the cell ordering (qed_sort_by_cell) for up to max_particles."""

    def __init__(self, max_particles: int):
        self.max_particles = int(max_particles)
        self.h = B.qed_sorter_create(self.max_particles)

    def sort(self, ws: "Workspace", src: Species, dst: Species, grid_field: B.qed_field, bands: int = 1):
        B.qed_sort_by_cell(self.h, ws.h, src.struct(), dst.struct(), grid_field, bands=bands)

    def __del__(self):
        h, self.h = getattr(self, "h", None), None
        if h:
            B.qed_sorter_free(h)


class Merger:
    """Scratch of the super-particle merging (qed_merge) for up to max_particles."""

    def __init__(self, max_particles: int):
        self.max_particles = int(max_particles)
        self.h = B.qed_merger_create(self.max_particles)

    def merge(self, ws: "Workspace", spec: B.qed_merge_spec, src: Species, dst: Species, seed: int,
              uid_next: torch.Tensor):
        B.qed_merge(self.h, ws.h, spec, src.struct(), dst.struct(), seed, uid_next.data_ptr())

    def __del__(self):
        h, self.h = getattr(self, "h", None), None
        if h:
            B.qed_merger_free(h)


def merge_spec(origin, spacing, shape, massive: bool, octave_min: int, n_octaves: int, sub_bins: int, n_dir: int,
               min_group: int) -> B.qed_merge_spec:
    m = B.qed_merge_spec()
    m.x0, m.y0, m.z0 = (float(v) for v in origin)
    m.dx, m.dy, m.dz = (float(v) for v in spacing)
    m.nx, m.ny, m.nz = (int(v) for v in shape)
    m.massive = int(bool(massive))
    m.octave_min, m.n_octaves, m.sub_bins = int(octave_min), int(n_octaves), int(sub_bins)
    m.n_dir, m.min_group = int(n_dir), int(min_group)
    return m


def plane_wave(a0: float, n_periods: float = 10.0) -> B.qed_field:
    f = B.qed_field()
    f.kind = B.QED_FIELD_PLANE_WAVE
    f.a0, f.n_periods = a0, n_periods
    return f


def uniform(E=(0, 0, 0), Bf=(0, 0, 0)) -> B.qed_field:
    f = B.qed_field()
    f.kind = B.QED_FIELD_UNIFORM
    f.E = (C.c_double * 3)(*E)
    f.B = (C.c_double * 3)(*Bf)
    return f


def yee(grid: torch.Tensor, shape, spacing, origin) -> B.qed_field:
    f = B.qed_field()
    f.kind = B.QED_FIELD_YEE
    f.grid = grid.data_ptr()
    f.nx, f.ny, f.nz = shape
    f.dx, f.dy, f.dz = spacing
    f.x0, f.y0, f.z0 = origin
    return f


def step(t, dt, seed, rad_model=B.QED_RAD_HYBRID, chi_switch=1e-3, gamma_photon_min=2.0,
         chi_photon_push_min=1e-3, max_events=4, no_recoil=0, d_step=None, variants=0) -> B.qed_step:
    s = B.qed_step()
    s.t, s.dt, s.seed = t, dt, seed
    s.rad_model, s.max_events = rad_model, max_events
    s.chi_switch, s.gamma_photon_min, s.chi_photon_push_min = chi_switch, gamma_photon_min, chi_photon_push_min
    s.no_recoil = no_recoil
    s.variants = variants
    s.d_step = d_step
    return s


def schedule(block=256, items_per_thread=1, blocks_per_cu=8, max_blocks=0) -> B.qed_schedule:
    return B.qed_schedule(block, items_per_thread, blocks_per_cu, max_blocks)
