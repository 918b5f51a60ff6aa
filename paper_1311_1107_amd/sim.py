"""A run of the QED step on one GPU: electrons, positrons and photons in a
laser field, advanced step by step through libqed.

Order within step n (time t = n dt):
  1. (Yee field) sample the pulse onto the grid for step n
  2. electrons: push + emission            (qed_push_emit, charge -1)
  3. positrons: push + emission            (qed_push_emit, charge +1)
  4. photons alive at the start of the step: pair creation and push
     (qed_pair_create); photons emitted in 2-3 are stored at level n+1 and
     are first advanced at step n+1, as are the pairs created in 4
  5. every `compact_every` steps, decayed photons are removed (qed_compact)
  6. (Yee field) every `sort_every` steps the leptons, and every
     `photon_sort_every` steps the photons, are put in stable cell order
     (qed_sort_by_cell), which also drops decayed photons
Between steps, merge_if_needed() merges the super-particles of a species
that fills more than a set fraction of its buffer (qed_merge, keeping weight,
momentum and energy).

Coupled form (coupled=True, Yee field): the pulse is sampled onto the grid
once, at step 0, and from then on the grid is advanced by the field solver
with the leptons' currents:
  1. the leptons' positions are saved (qed_save_positions)
  2-3. electrons and positrons are pushed with the field at step n
  then their charge-conserving currents over the step are deposited
  4. photons are stepped; the pairs they create deposit the current of
     their motion from the photon's position (qed_deposit_current, x_old
     NULL, from the lepton counts before the photon step)
  5. qed_yee_advance takes E and B from step n to n+1 with that current
Weights are numbers of physical particles times particles_per_weight.
"""
from __future__ import annotations

import ctypes as C
import math
from dataclasses import dataclass

import numpy as np
import torch

from . import binding as B
from . import device as D
from .workloads import LAMBDA_M, PlaneWave, Uniform, Workload, YeePulse

EMIT_SPEC = dict(chi_min=1e-3, chi_max=1e2, n_chi=128, n_q=128, logit_max=18.0)
PAIR_SPEC = dict(chi_min=1e-2, chi_max=1e2, n_chi=128, n_q=128, logit_max=18.0)


@dataclass
class MergePolicy:
    """When and how to merge super-particles: a species holding more than
    `threshold` of its capacity is merged over the cells of the box
    (origin, spacing, shape) and the momentum bins given (see qed_merge)."""
    origin: tuple
    spacing: tuple
    shape: tuple
    octave_min: int = -8
    n_octaves: int = 48
    sub_bins: int = 2
    n_dir: int = 8
    min_group: int = 4
    threshold: float = 0.5
    species: tuple = ("ph", "el", "po")


class Run:
    def __init__(self, wl: Workload, prec: int = B.QED_F64, tables: D.Tables | None = None,
                 photon_capacity: int | None = None, record_capacity: int | None = None,
                 pair_capacity: int | None = None, rad_model: int = B.QED_RAD_HYBRID,
                 chi_switch: float = 1e-3, gamma_photon_min: float = 2.0, max_events: int = 4,
                 sched: B.qed_schedule | None = None, compact_every: int = 16, sort_every: int = 0,
                 photon_sort_every: int | None = None,
                 deterministic_tally: bool = True, variants: int = 0, merge: MergePolicy | None = None,
                 coupled: bool = False, particles_per_weight: float = 1.0, field_bound_block: int = 0,
                 device: str = "cuda"):
        self.wl = wl
        self.prec = prec
        self.units = B.qed_units_init(LAMBDA_M)
        self.tables = tables or D.Tables(EMIT_SPEC, PAIR_SPEC)
        n0 = len(wl.electrons["x"])
        self.n0 = n0
        push = wl.push_photons
        self.push = push
        cap_ph = photon_capacity if photon_capacity is not None else (4 * n0 if push else 0)
        cap_rec = record_capacity if record_capacity is not None else (4 * n0 if wl.record_photons else 0)
        cap_pair = pair_capacity if pair_capacity is not None else (n0 if push else 0)
        self.el = D.Species(n0 + cap_pair, prec, chi=True, device=device)
        self.po = D.Species(cap_pair, prec, chi=True, device=device)
        self.ph = D.Species(cap_ph, prec, chi=True, device=device) if push else None
        self.rec = D.Species(cap_rec, prec, chi=True, device=device) if wl.record_photons else None
        caps = [n0 + cap_pair, cap_pair, cap_ph, cap_rec, 1]
        self.ws = D.Workspace(max(caps), max_leptons=n0 + cap_pair)
        # one energy slot per tile (64 photons in the photon step) keeps the sums reproducible
        slots = (max(caps) + 63) // 64 + 1 if deterministic_tally else 4096
        self.tally = D.Tally(slots, device=device)
        self.uid_next = torch.tensor([n0], dtype=torch.int64, device=device)
        self.ph_snap = torch.zeros(1, dtype=torch.int64, device=device)
        self.sched = sched
        self.compact_every = compact_every
        self.step_kw = dict(rad_model=rad_model, chi_switch=chi_switch, gamma_photon_min=gamma_photon_min,
                            chi_photon_push_min=wl.chi_photon_push_min, max_events=max_events,
                            variants=variants)
        self.el.upload(wl.electrons)
        B.qed_init_optical_depth(self.el.struct(), wl.seed)
        # field
        f = wl.field
        if isinstance(f, PlaneWave):
            self.field = D.plane_wave(f.a0, f.n_periods)
            self.grid = None
        elif isinstance(f, Uniform):
            self.field = D.uniform(f.E, f.B)
            self.grid = None
        elif isinstance(f, YeePulse):
            nx, ny, nz = f.shape
            self.grid = torch.zeros(6 * nx * ny * nz, dtype=torch.float32, device=device)
            self.tperp = torch.from_numpy(np.ascontiguousarray(f.tperp)).to(device)
            self.tpar = torch.from_numpy(np.ascontiguousarray(f.tpar)).to(device)
            self.field = D.yee(self.grid, f.shape, f.spacing, f.origin)
            # per-block field bounds let the photon step skip the gather of waves in which no
            # pair can form (opt-in: on the Yee workload too few waves qualify to pay for it)
            self.bound_block = int(field_bound_block)
            if self.bound_block:
                nb = [(n + self.bound_block - 1) // self.bound_block for n in f.shape]
                self.bound = torch.zeros(2 * nb[0] * nb[1] * nb[2], dtype=torch.float32, device=device)
                self.field.bound = self.bound.data_ptr()
                self.field.bound_block = self.bound_block
        else:
            raise TypeError("unknown field description")
        # cell ordering (Yee field only): a second buffer per species, swapped after each sort
        self.sort_every = sort_every if self.grid is not None else 0
        # photons move together at c, and those emitted in one step are appended in the
        # cell order of their parents, so their order decays more slowly than the leptons'
        pse = sort_every if photon_sort_every is None else photon_sort_every
        self.photon_sort_every = pse if (self.grid is not None and self.ph is not None) else 0
        if self.sort_every or self.photon_sort_every:
            self.sorter = D.Sorter(max(caps))
            self.alt = {"el": D.Species(self.el.capacity, prec, chi=True, device=device),
                        "po": D.Species(self.po.capacity, prec, chi=True, device=device)}
            if self.ph is not None:
                self.alt["ph"] = D.Species(self.ph.capacity, prec, chi=True, device=device)
        # coupling to the field solver
        self.coupled = bool(coupled)
        if self.coupled:
            if self.grid is None:
                raise ValueError("the coupled form needs a Yee grid")
            nx, ny, nz = f.shape
            self.J = torch.zeros(3 * nx * ny * nz, dtype=torch.float32, device=device)
            dt_ = D._dtype(prec)
            self.x_old = {k: [torch.zeros(max(1, sp.capacity), dtype=dt_, device=device) for _ in range(3)]
                          for k, sp in (("el", self.el), ("po", self.po))}
            self.lep_snap = {k: torch.zeros(1, dtype=torch.int64, device=device) for k in ("el", "po")}
            self.skipped = torch.zeros(1, dtype=torch.int64, device=device)
            # one physical particle per unit weight: charge density unit n_c over a cell of dx dy dz (c/omega_r)^3
            eps0, me, c, e = 8.8541878128e-12, 9.1093837015e-31, 299792458.0, 1.602176634e-19
            omega = 2.0 * math.pi * c / LAMBDA_M
            nc_cube = eps0 * me * c ** 3 / (e * e * omega)
            self.j_scale = particles_per_weight / (nc_cube * f.spacing[0] * f.spacing[1] * f.spacing[2])
            self.fill_field(0)
        # merging: second buffers (shared with the cell ordering) made on first use
        self.merge_policy = merge
        self.merger = D.Merger(max(caps)) if merge is not None else None
        self.merges = []
        if not (self.sort_every or self.photon_sort_every):
            self.alt = {}
        self._photon_view()

    def _photon_view(self):
        # photon view whose count is the snapshot taken at the start of a step
        if self.ph is not None:
            s = self.ph.struct()
            self.ph_step = B.qed_species()
            C.memmove(C.addressof(self.ph_step), C.addressof(s), C.sizeof(s))
            self.ph_step.d_count = self.ph_snap.data_ptr()

    def sort(self, leptons: bool = True, photons: bool = True):
        """Stable cell order of the leptons and/or the photons (drops decayed photons);
        photons by (cell, energy band) when the field bounds are on."""
        for name in ("el", "po", "ph"):
            src = getattr(self, name)
            if src is None or not (photons if name == "ph" else leptons):
                continue
            dst = self.alt[name]
            # with field bounds, photons of one cell are grouped by energy band so that whole
            # waves can skip the gather
            bands = 4 if (name == "ph" and self.bound_block) else 1
            self.sorter.sort(self.ws, src, dst, self.field, bands=bands)
            setattr(self, name, dst)
            self.alt[name] = src
        self._photon_view()

    # ------------------------------------------------------------------
    def fill_field(self, n: int):
        if self.grid is not None:
            f = self.wl.field
            nx, ny, nz = f.shape
            tp = self.tpar[n].reshape(-1)
            B.qed_yee_fill_separable(self.grid.data_ptr(), nx, ny, nz, f.a0, self.tperp.data_ptr(), tp.data_ptr())
            self.field_bound()

    def field_bound(self):
        """Recompute the per-block field bounds (after every change of the grid)."""
        if self.grid is not None and self.bound_block:
            B.qed_field_bound(self.field, self.bound_block, self.bound.data_ptr())

    def step(self, n: int, timed=None):
        """Step n.  `timed(kind, fn)`, if given, wraps every launch (for timing)."""
        run = timed or (lambda kind, fn: fn())
        st = D.step(n * self.wl.dt, self.wl.dt, self.wl.seed, **self.step_kw)
        if self.coupled:
            run("save", self._save_positions)
        elif self.grid is not None:
            run("fill", lambda: self.fill_field(n))
        if self.ph is not None:
            self.ph_snap.copy_(self.ph.count)
        pp = self.ph.struct() if self.ph is not None else None
        pr = self.rec.struct() if self.rec is not None else None
        uid = self.uid_next.data_ptr()
        run("push_e", lambda: B.qed_push_emit(self.tables.h, self.ws.h, self.units, -1.0, self.el.struct(),
                                              self.field, pp, pr, self.tally.s, st, uid, self.sched))
        run("push_p", lambda: B.qed_push_emit(self.tables.h, self.ws.h, self.units, +1.0, self.po.struct(),
                                              self.field, pp, pr, self.tally.s, st, uid, self.sched))
        sort_lep = bool(self.sort_every) and (n + 1) % self.sort_every == 0
        sort_ph = bool(self.photon_sort_every) and (n + 1) % self.photon_sort_every == 0
        if self.coupled:
            run("deposit", self._deposit_pushed)
        if self.ph is not None:
            run("pair", lambda: B.qed_pair_create(self.tables.h, self.ws.h, self.units, self.ph_step, self.field,
                                                  self.el.struct(), self.po.struct(), self.tally.s, st, uid,
                                                  self.sched))
            if self.coupled:
                run("deposit", self._deposit_created)
            # the cell sort drops decayed photons itself
            if self.compact_every and (n + 1) % self.compact_every == 0 and not sort_ph:
                run("compact", self.compact)
        if self.coupled:
            run("field", lambda: (B.qed_yee_advance(self.grid.data_ptr(), self.J.data_ptr(), self.field, self.wl.dt),
                                  self.field_bound()))
        if sort_lep or sort_ph:
            run("sort", lambda: self.sort(leptons=sort_lep, photons=sort_ph))

    # ------------------------------------------------------------------
    def _save_positions(self):
        for k in ("el", "po"):
            sp = getattr(self, k)
            B.qed_save_positions(sp.struct(), [t.data_ptr() for t in self.x_old[k]])
            self.lep_snap[k].copy_(sp.count)

    def _deposit_pushed(self):
        self.J.zero_()
        for k, q in (("el", -1.0), ("po", 1.0)):
            B.qed_deposit_current(getattr(self, k).struct(), [t.data_ptr() for t in self.x_old[k]], None, q,
                                  self.j_scale, self.wl.dt, self.field, self.J.data_ptr(), self.skipped.data_ptr())

    def _deposit_created(self):
        for k, q in (("el", -1.0), ("po", 1.0)):
            B.qed_deposit_current(getattr(self, k).struct(), None, self.lep_snap[k].data_ptr(), q, self.j_scale,
                                  self.wl.dt, self.field, self.J.data_ptr(), self.skipped.data_ptr())

    def merge_if_needed(self) -> list:
        """Merge every species of the policy that holds more than its threshold
        (reads the counts: one host synchronisation).  Returns what was done."""
        pol = self.merge_policy
        if pol is None:
            return []
        done = []
        for name in pol.species:
            src = getattr(self, name)
            if src is None or src.capacity == 0:
                continue
            n = src.n()
            if n <= pol.threshold * src.capacity:
                continue
            dst = self.alt.get(name)
            if dst is None:
                dst = self.alt[name] = D.Species(src.capacity, self.prec, chi=True, device=src.count.device)
            spec = D.merge_spec(pol.origin, pol.spacing, pol.shape, name != "ph", pol.octave_min, pol.n_octaves,
                                pol.sub_bins, pol.n_dir, pol.min_group)
            self.merger.merge(self.ws, spec, src, dst, self.wl.seed, self.uid_next)
            setattr(self, name, dst)
            self.alt[name] = src
            rec = {"species": name, "before": n, "after": dst.n()}
            done.append(rec)
            self.merges.append(rec)
        if done:
            self._photon_view()
        return done

    # ------------------------------------------------------------------
    # Checkpoint and restart.  What carries over from one step to the next is
    # saved: the live particles of every species with their ids, event counters
    # and optical depths, the id counter, the tallies and, in the coupled form,
    # the grid.  A run built again from the same workload and options and
    # loaded from the file continues bit-identically: draws are keyed by id and
    # event counter, and the step schedule (compaction, cell order) by step.
    _SPECIES = ("el", "po", "ph", "rec")

    def save(self, path: str, next_step: int):
        """Write a checkpoint (numpy .npz) to continue from step `next_step`."""
        torch.cuda.synchronize()
        out = {"next_step": np.array(next_step, dtype=np.int64),
               "uid_next": self.uid_next.cpu().numpy(),
               "tally_energy": self.tally.energy.cpu().numpy(),
               "tally_count": self.tally.count.cpu().numpy()}
        for name in self._SPECIES:
            sp = getattr(self, name)
            if sp is None:
                continue
            for k, v in sp.download().items():
                out[f"{name}.{k}"] = v
        if self.coupled:
            out["grid"] = self.grid.cpu().numpy()
            out["skipped"] = self.skipped.cpu().numpy()
        np.savez(path, **out)

    def load(self, path: str) -> int:
        """Restore a checkpoint written by save() into this run (built with the
        same workload and options); returns the step to continue from."""
        with np.load(path, allow_pickle=False) as z:
            for name in self._SPECIES:
                sp = getattr(self, name)
                keys = [k for k in z.files if k.startswith(name + ".")]
                if sp is None:
                    if keys:
                        raise ValueError(f"checkpoint holds species {name!r}, which this run does not")
                    continue
                arrays = {k.split(".", 1)[1]: z[k] for k in keys}
                sp.upload(arrays, len(arrays["x"]))
            if self.tally.energy.numel() != z["tally_energy"].size:
                raise ValueError("checkpoint tally has a different number of slots")
            self.uid_next.copy_(torch.from_numpy(z["uid_next"]))
            self.tally.energy.copy_(torch.from_numpy(z["tally_energy"]))
            self.tally.count.copy_(torch.from_numpy(z["tally_count"]))
            if self.coupled:
                self.grid.copy_(torch.from_numpy(z["grid"]))
                self.skipped.copy_(torch.from_numpy(z["skipped"]))
                self.field_bound()
            nxt = int(z["next_step"])
        torch.cuda.synchronize()
        return nxt

    def compact(self):
        if self.ph is not None:
            B.qed_compact(self.ws.h, self.ph.struct(), self.sched)

    def run(self, steps: int, start: int = 0):
        for n in range(start, start + steps):
            self.step(n)

    def counts(self) -> dict:
        return {"electrons": self.el.n(), "positrons": self.po.n(),
                "photons": self.ph.n() if self.ph is not None else 0,
                "recorded": self.rec.n() if self.rec is not None else 0}

    def result(self) -> dict:
        self.compact()
        torch.cuda.synchronize()
        out = {"electrons": self.el.download(), "positrons": self.po.download(),
               "photons": self.ph.download() if self.ph is not None else None,
               "recorded": self.rec.download() if self.rec is not None else None,
               "tally": self.tally.reduce(), "uid_next": int(self.uid_next.item())}
        return out
