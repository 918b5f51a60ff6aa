"""The batched form on one GPU: many independent electron bunches, each in its
own plane wave, advanced together.

Two ways to step the same bunches:
  * plain:   one qed_push_emit per bunch per step (a view of the bunch and its
             own field), launched eagerly;
  * batched: one qed_push_emit_batched per step over all bunches, with the
             schedule picked by qed_autotune_batched and the step sequence
             captured once in a HIP graph and replayed.  The step time comes
             from a device counter (qed_step.d_step) that qed_step_advance
             increments inside the graph.
Both append the emitted photons to one recorded-photon buffer in bunch order,
then particle order, and hand out ids from one device counter, so they give
the same events.
"""
from __future__ import annotations

import numpy as np
import torch

from . import binding as B
from . import device as D
from .workloads import DT, LAMBDA_M

# schedules the autotuner chooses from: block size, workgroups per CU and a cap
# on the persistent grid (0 = none; a cap makes each block walk more tiles)
CANDIDATES = [(64, 8, 0), (128, 8, 0), (256, 8, 0), (256, 4, 0), (256, 2, 0), (128, 16, 0), (64, 16, 0),
              (256, 16, 0), (256, 8, 1024), (256, 8, 512), (128, 8, 1024)]


class Bunches:
    def __init__(self, electrons: dict, offsets: np.ndarray, a0s: np.ndarray, prec: int, tables: D.Tables,
                 seed: int = 4, n_periods: float = 10.0, record_capacity: int | None = None,
                 rad_model: int = B.QED_RAD_HYBRID, device: str = "cuda"):
        n = len(electrons["x"])
        self.n, self.prec, self.seed, self.tables = n, prec, seed, tables
        self.offsets = np.asarray(offsets, dtype=np.int64)
        self.a0s = np.asarray(a0s, dtype=np.float64)
        self.nb = len(self.a0s)
        self.units = B.qed_units_init(LAMBDA_M)
        self.rad_model = rad_model
        self.el = D.Species(n, prec, chi=False, device=device)
        self.el.upload(electrons)
        B.qed_init_optical_depth(self.el.struct(), seed)
        cap = record_capacity if record_capacity is not None else 16 * n
        self.rec = D.Species(cap, prec, device=device)
        self.ws = D.Workspace(max(n, cap), max_leptons=n)
        self.tally = D.Tally((n + 63) // 64 + 2, device=device)
        self.uid = torch.tensor([n], dtype=torch.int64, device=device)
        self.d_step = torch.zeros(1, dtype=torch.int64, device=device)
        self.d_off = torch.from_numpy(self.offsets).to(device)
        self.d_a0 = torch.from_numpy(np.ascontiguousarray(self.a0s)).to(device)
        self.d_np = torch.full((self.nb,), float(n_periods), dtype=torch.float64, device=device)
        self.counts = torch.from_numpy(np.diff(self.offsets)).to(device)
        self.bun = B.qed_bunches(self.nb, 0, self.d_off.data_ptr(), self.d_a0.data_ptr(), self.d_np.data_ptr())
        self.views = [self.el.view(int(self.offsets[b]), self.counts[b:b + 1].data_ptr(),
                                   int(self.offsets[b + 1] - self.offsets[b])) for b in range(self.nb)]
        self.fields = [D.plane_wave(float(a), n_periods) for a in self.a0s]
        self.n_periods = float(n_periods)
        self.sched = None
        self.graph = None
        self.graph_steps = 0

    # -------------------------------------------------------------- plain --
    def step_plain(self, n: int, sched=None):
        st = D.step(n * DT, DT, self.seed, rad_model=self.rad_model)
        for v, f in zip(self.views, self.fields):
            B.qed_push_emit(self.tables.h, self.ws.h, self.units, -1.0, v, f, None, self.rec.struct(),
                            self.tally.s, st, self.uid.data_ptr(), sched)

    # ------------------------------------------------------------ batched --
    def _batched_step_struct(self):
        return D.step(0.0, DT, self.seed, rad_model=self.rad_model, d_step=self.d_step.data_ptr())

    def step_batched(self):
        """One eager batched step at the time held by the device step counter."""
        B.qed_push_emit_batched(self.tables.h, self.ws.h, self.units, -1.0, self.el.struct(), self.bun, None,
                                self.rec.struct(), self.tally.s, self._batched_step_struct(), self.uid.data_ptr(),
                                self.sched)
        B.qed_step_advance(self.d_step.data_ptr())

    def autotune(self, trial_steps: int = 3, cache_path: str | None = None, trial_time: float | None = None):
        """Pick the schedule of the batched step.  The candidates are timed on a
        scratch copy of the state at trial_time, by default one pulse length
        (2 pi n_periods): the pulse then covers about half of each bunch's
        box, so the trial steps emit as the run does in the pulse."""
        cands = [D.schedule(b, 1, bpc, cap) for b, bpc, cap in CANDIDATES]
        t = trial_time if trial_time is not None else 2.0 * np.pi * self.n_periods
        st = D.step(t, DT, self.seed, rad_model=self.rad_model)
        best, ms = B.qed_autotune_batched(self.tables.h, self.ws.h, self.units, -1.0, self.el.struct(), self.bun,
                                          self.rec.struct(), st, cands, trial_steps, cache_path)
        self.sched = best
        return best, ms

    def capture(self, steps: int):
        """Capture `steps` batched steps (and their step-counter advances) in a graph."""
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        s = torch.cuda.Stream()
        with torch.cuda.graph(g, stream=s):
            for _ in range(steps):
                self.step_batched()
        torch.cuda.synchronize()
        self.graph, self.graph_steps = g, steps
        return g

    def replay(self):
        self.graph.replay()

    # ------------------------------------------------------------ results --
    def result(self) -> dict:
        torch.cuda.synchronize()
        return {"electrons": self.el.download(), "recorded": self.rec.download(), "tally": self.tally.reduce(),
                "uid_next": int(self.uid.item())}
