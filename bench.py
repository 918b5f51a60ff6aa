"""Throughput of the QED particle step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--start S] [--workload yee|coupled|plane|batched|cascade]

Default workload: 1e7 electrons (ln gamma0 ~ N(ln 2000, 0.3^2)) colliding with
a focused a0 = 200 pulse (w0 = 3 lambda, 30 fs) sampled on a 256 x 128 x 128
FP32 Yee grid, FP64 step, photon emission, photons with chi_gamma > 1e-3 pushed
and tested for Breit-Wheeler pairs; the collision lasts 2000 steps.

The run is advanced, untimed, to step S - W (default S = 1000, mid-collision,
where the beam is inside the pulse and the photon population is building
up); W warm-up steps follow, then the K timed steps [S, S + K) (default
K = 1000, the rest of the collision), every input resident in HBM: field
sampling onto the grid, electron and positron push/emission, photon
push/pair creation, periodic compaction and cell order.  The metric counts
particles advanced per second (leptons plus pushed photons) in the timed
steps.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=None)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--start", type=int, default=1000,
                   help="first timed step (Yee workloads): the run is advanced untimed to start - warmup")
    p.add_argument("--workload", default="yee", choices=["yee", "coupled", "plane", "batched", "batched-fp32",
                                                          "cascade"])
    p.add_argument("--electrons", type=int, default=None, help="override the electron count")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-sample", type=int, default=1500, help="electrons in the oracle sample")
    p.add_argument("--cpu-min-seconds", type=float, default=1.0,
                   help="the oracle repeats the timed window from its start state until this much time has passed")
    p.add_argument("--copy-calibration", action="store_true",
                   help="run a 1 GiB device copy first (reference for the traffic counters)")
    p.add_argument("--compact-every", type=int, default=16)
    p.add_argument("--no-merge", action="store_true",
                   help="cascade: stop at the first full buffer instead of merging super-particles")
    p.add_argument("--sort-every", type=int, default=16, help="cell-order the leptons every k steps (Yee)")
    p.add_argument("--photon-sort-every", type=int, default=None,
                   help="cell-order the photons every k steps (Yee; default: as the leptons)")
    p.add_argument("--bound-block", type=int, default=0,
                   help="Yee: per-block field bounds (block edge in cells) so that photon waves with no possible "
                        "pair skip the gather; 0 = off")
    p.add_argument("--batched-steps", type=int, default=1000,
                   help="steps of the FP32-batched vs FP64-plain comparison (0 skips it)")
    p.add_argument("--no-graph", action="store_true",
                   help="batched forms: eager launches instead of HIP-graph replays (for counter collection)")
    return p.parse_args()


TRAFFIC_SUMMARIES = {
    "pair": os.path.join(ROOT, "profiles", "qed_pair_create_yee1e7_f64_window_traffic.md"),
    "push": os.path.join(ROOT, "profiles", "qed_push_emit_yee1e7_f64_window_traffic.md"),
}
KERNEL_SOURCES = ["paper_1311_1107_amd/csrc/qed_kernels.hip", "paper_1311_1107_amd/csrc/qed_kernels.h",
                  "paper_1311_1107_amd/csrc/qed_device.h"]


def kernel_source_sha256() -> str:
    import hashlib
    h = hashlib.sha256()
    for src in KERNEL_SOURCES:
        with open(os.path.join(ROOT, src), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(call: str):
    """Copy-calibrated HBM bytes per call of the timed window from the
    committed counter summary of the driver's command, or None if there is
    none or the kernel sources have changed since the counters were taken."""
    try:
        lines = open(TRAFFIC_SUMMARIES[call]).read().splitlines()
    except (OSError, KeyError):
        return None
    vals = dict(l.split(": ", 1) for l in lines if l.startswith(("traffic_bytes_per_call: ", "kernel_source_sha256: ")))
    if vals.get("kernel_source_sha256") != kernel_source_sha256() or "traffic_bytes_per_call" not in vals:
        return None
    return float(vals["traffic_bytes_per_call"])


def device_copy_gbs(reps: int = 10) -> float:
    """Bandwidth of a plain 1 GiB device-to-device copy (read + write bytes / time)."""
    import torch
    a = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    return 2.0 * (1 << 30) / (ms * 1e-3) / 1e9


def host_cpu() -> dict:
    """The host's CPU model and core counts."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"model": model, "nproc": os.cpu_count(), "affinity": len(os.sched_getaffinity(0))}


def oracle_threads() -> int:
    """Threads for the all-core oracle leg: OMP_NUM_THREADS if set, else the CPUs this process may use."""
    v = os.environ.get("OMP_NUM_THREADS", "")
    return int(v) if v.isdigit() and int(v) > 0 else len(os.sched_getaffinity(0))


def cpu_baseline(wl, n_sample: int, start: int, steps: int, min_seconds: float, caps=(2, 1, 80, 20)):
    """The oracle on a fixed uid subset of the same workload.  The subset is
    advanced (untimed, on all host cores) to the first timed step; the timed
    window [start, start + steps) then runs single-threaded (the oracle as
    written) and on all host cores (its OpenMP driver: the same particles),
    each repeated from a copy of the start state until min_seconds have
    passed.  Leptons are independent in an external field with id-keyed
    draws, so the subset evolves as it does inside the full run.  caps: the
    electron, positron, pushed- and recorded-photon buffers in units of the
    subset's size."""
    import numpy as np

    from oracle import oracle as O
    from paper_1311_1107_amd import workloads as W

    n = len(wl.electrons["x"])
    idx = np.linspace(0, n - 1, min(n_sample, n)).astype(np.int64)
    sub = W.subset(wl, idx)
    bt = O.BoundTables(O.compute_tables())
    m = len(idx)
    el = O.species_from(sub.electrons, capacity=m * caps[0])
    O.init_tau(el, wl.seed)
    po = O.new_species(m * caps[1])
    ph = O.new_species(caps[2] * m) if wl.push_photons else None
    rec = O.new_species(caps[3] * m) if wl.record_photons else None
    un = [n]
    f = wl.field
    threads = oracle_threads()

    def field_at(k):
        if isinstance(f, W.YeePulse):
            return O.make_field(O.FIELD_YEE_SEPARABLE, a0=f.a0, shape=f.shape, spacing=f.spacing,
                                origin=f.origin, tperp=f.tperp, tpar=f.tpar[k])
        return O.make_field(O.FIELD_PLANE_WAVE, a0=f.a0, n_periods=f.n_periods)

    def run(species, k0, k1, th, tally):
        e, p, g, r = species
        for k in range(k0, k1):
            field = field_at(k)
            st = O.make_step(k * wl.dt, wl.dt, wl.seed, chi_photon_push_min=wl.chi_photon_push_min)
            n_ph0 = g["n"] if g is not None else 0
            O.push_emit(bt, W.LAMBDA_M, -1.0, e, field, g, r, st, un, tally, threads=th)
            O.push_emit(bt, W.LAMBDA_M, +1.0, p, field, g, r, st, un, tally, threads=th)
            if g is not None:
                O.pair_create(bt, W.LAMBDA_M, g, field, e, p, st, un, tally, n_limit=n_ph0, threads=th)

    t0 = time.perf_counter()
    run((el, po, ph, rec), 0, start, threads, O.Tally())
    advance_s = time.perf_counter() - t0
    state = (el, po, ph, rec)
    uid0 = un[0]
    live0 = {name: (sp["n"] if sp is not None else 0) for name, sp in zip(("electrons", "positrons", "photons"), state)}

    def window(th):
        total_s, total_ps, reps = 0.0, 0, 0
        while reps == 0 or total_s < min_seconds:
            copy = tuple({k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in sp.items()}
                         if sp is not None else None for sp in state)
            un[0] = uid0
            tally = O.Tally()
            t1 = time.perf_counter()
            run(copy, start, start + steps, th, tally)
            total_s += time.perf_counter() - t1
            c = tally.as_dict()
            total_ps += c["N_mc"] + c["N_sokolov"] + c["N_nan"] + c["N_phstep"]
            reps += 1
        return total_ps / total_s, total_ps // reps, reps, total_s

    v1, ps1, r1, s1 = window(0)
    va, psa, ra, sa = window(threads)
    cpu = host_cpu()
    return {"value": v1, "unit": "particle-steps/s", "cores": 1, "kind": "oracle",
            "sample": (f"all {m} electrons of the workload" if m == n else
                       f"{m} electrons (uid subset) of the same workload") + f", advanced to step {start} "
                      f"({live0['electrons']} e-, {live0['positrons']} e+, {live0['photons']} pushed photons there, "
                      f"{advance_s:.1f} s on {threads} threads, untimed), then steps [{start}, {start + steps}): "
                      f"{ps1} particle-steps per pass, {r1} passes in {s1:.2f} s, single thread",
            "cpu": cpu["model"], "nproc": cpu["nproc"], "cpus_allowed": cpu["affinity"],
            "all_cores": {"value": va, "unit": "particle-steps/s", "cores": threads, "kind": "oracle (OpenMP driver)",
                          "sample": f"the same window, {psa} particle-steps per pass, {ra} passes in {sa:.2f} s",
                          "speedup_over_one_core": va / v1}}


def cpu_bunch_baseline(steps: int, seed: int = 4, every: int = 8, per_bunch: int = 2000, min_seconds: float = 1.0):
    """The oracle on a fixed subset of the bunch workload: every `every`-th of
    the 64 bunches, up to per_bunch electrons of each (evenly spaced ids), each
    bunch in its own plane wave, steps [0, steps), photons recorded; one oracle
    call per bunch per step (about 75 us of call overhead each, included);
    single-threaded and on all host cores, repeated from the initial state
    until min_seconds have passed."""
    import numpy as np

    from oracle import oracle as O
    from paper_1311_1107_amd import workloads as W

    e, off, a0s, _ = W.bunches(n_bunches=64, seed=seed)
    n = len(e["x"])
    bt = O.BoundTables(O.compute_tables())
    threads = oracle_threads()
    parts = []
    for b in range(0, len(a0s), every):
        idx = np.linspace(off[b], off[b + 1] - 1, min(per_bunch, int(off[b + 1] - off[b]))).astype(np.int64)
        parts.append(({k: v[idx] for k, v in e.items()}, O.make_field(O.FIELD_PLANE_WAVE, a0=float(a0s[b]),
                                                                       n_periods=10.0)))
    m = sum(len(p[0]["x"]) for p in parts)

    def window(th):
        total_s, total_ps, reps = 0.0, 0, 0
        while reps == 0 or total_s < min_seconds:
            tally = O.Tally()
            states = []
            for el_d, _ in parts:
                el = O.species_from(el_d, capacity=len(el_d["x"]))
                O.init_tau(el, seed)
                states.append((el, O.new_species(40 * len(el_d["x"]))))
            un = [n]
            t1 = time.perf_counter()
            for k in range(steps):
                st = O.make_step(k * W.DT, W.DT, seed)
                for (el, rec), (_, field) in zip(states, parts):
                    O.push_emit(bt, W.LAMBDA_M, -1.0, el, field, None, rec, st, un, tally, threads=th)
            total_s += time.perf_counter() - t1
            c = tally.as_dict()
            total_ps += c["N_mc"] + c["N_sokolov"] + c["N_nan"]
            reps += 1
        return total_ps / total_s, total_ps // reps, reps, total_s

    v1, ps1, r1, s1 = window(0)
    va, psa, ra, sa = window(threads)
    return {"value": v1, "unit": "particle-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"{m} electrons (up to {per_bunch} evenly spaced ids of each of {len(parts)} of the "
                      f"{len(a0s)} bunches, every {every}th, each in its own plane wave), steps [0, {steps}): "
                      f"{ps1} particle-steps per pass, {r1} passes in {s1:.2f} s, single thread",
            "all_cores": {"value": va, "unit": "particle-steps/s", "cores": threads, "kind": "oracle (OpenMP driver)",
                          "sample": f"the same subset, {psa} particle-steps per pass, {ra} passes in {sa:.2f} s"}}


def batched_comparison(steps: int, seed: int = 4, cpu: bool = True, graph: bool = True, only_fp32: bool = False):
    """The batched-form bunches (64 bunches, sizes log-uniform 1e3..1e6,
    a0 ~ U(50, 500), gamma0 ~ U(500, 5000), plane waves): FP64 plain (one
    launch per bunch per step, eager) against FP32 batched (one persistent
    launch per step, autotuned schedule, HIP-graph replays), and the KS test
    of their photon spectra (same seed, and seed + 1000 for the FP32 run)."""
    import numpy as np
    import torch
    from scipy import stats

    from paper_1311_1107_amd import batched as BT
    from paper_1311_1107_amd import binding as B
    from paper_1311_1107_amd import device as D
    from paper_1311_1107_amd import sim as S
    from paper_1311_1107_amd import workloads as W

    e, off, a0s, _ = W.bunches(n_bunches=64, seed=seed)
    n = len(e["x"])
    tabs = D.Tables(S.EMIT_SPEC, S.PAIR_SPEC)
    cap = 40 * n
    stream = torch.cuda.current_stream()

    def timed(fn):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a.record(stream)
        fn()
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b)

    def photon_gamma(bun, m=400_000):
        k = bun.rec.n()
        rng = np.random.default_rng(0)
        idx = torch.from_numpy(np.sort(rng.integers(0, k, size=min(m, k)))).cuda()
        g = torch.sqrt(bun.rec.a["ux"][idx].double() ** 2 + bun.rec.a["uy"][idx].double() ** 2 +
                       bun.rec.a["uz"][idx].double() ** 2)
        return g.cpu().numpy()

    def finish(bun, ms, prec):
        rc, _ = bun.ws.status(raise_on_error=False)
        tal = bun.tally.reduce()
        ps = tal["N_mc"] + tal["N_sokolov"] + tal["N_nan"]
        # algorithmic bytes, as for the lepton call of the Yee line: x, u read and written and w
        # read per lepton-step; tau read and written per Monte Carlo step; id and event counter
        # per emission; x, k, w, chi, tau, id, event counter per recorded photon
        es = 4 if prec == B.QED_F32 else 8
        byts = ps * 13 * es + tal["N_mc"] * 16 + tal["N_emit"] * 16 + tal["N_rec"] * (8 * es + 20)
        gbs = byts / (ms * 1e-3) / 1e9
        return {"ms_per_step": ms / steps, "particle_steps_per_s": ps / (ms * 1e-3), "photons": bun.rec.n(),
                "emissions": tal["N_emit"], "status": int(rc),
                "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                             "frac": gbs / HBM_PEAK_GBS, "bytes_per_step": byts / steps}}

    def batched(sd, prec=B.QED_F32):
        bun = BT.Bunches(e, off, a0s, prec, tabs, seed=sd, record_capacity=cap)
        best, _ = bun.autotune(trial_steps=3)
        chunk = 10
        if graph:
            bun.capture(chunk)
            ms = timed(lambda: [bun.replay() for _ in range(steps // chunk)])
        else:
            ms = timed(lambda: [bun.step_batched() for _ in range(steps // chunk * chunk)])
        out = finish(bun, ms, prec)
        out["schedule"] = {"block": best.block, "blocks_per_cu": best.blocks_per_cu, "max_blocks": best.max_blocks}
        out["graph_steps"] = chunk if graph else 0
        return bun, out

    if only_fp32:
        # the FP32 batched form alone (counter collection on its kernels)
        bun, r_b = batched(seed)
        return {"workload": f"{len(a0s)} bunches, {n} e-, {steps} steps, FP32 batched form only",
                "fp32_batched_graph" if graph else "fp32_batched_eager": r_b}
    # FP64 plain
    plain = BT.Bunches(e, off, a0s, B.QED_F64, tabs, seed=seed, record_capacity=cap)
    ms = timed(lambda: [plain.step_plain(k) for k in range(steps)])
    r_plain = finish(plain, ms, B.QED_F64)
    g_plain = photon_gamma(plain)
    del plain
    torch.cuda.empty_cache()
    print("bench: FP64 plain bunches done", file=sys.stderr, flush=True)

    bun, r_b = batched(seed)
    g_b = photon_gamma(bun)
    del bun
    torch.cuda.empty_cache()
    bun, r_c = batched(seed + 1000)
    g_c = photon_gamma(bun)
    del bun
    torch.cuda.empty_cache()
    print("bench: FP32 batched bunches done", file=sys.stderr, flush=True)
    # the FP64 form in the batched launch too: separates the gain of batching from that of FP32
    bun, r_d = batched(seed, B.QED_F64)
    del bun
    torch.cuda.empty_cache()
    print("bench: FP64 batched bunches done", file=sys.stderr, flush=True)
    return {
        "workload": f"{len(a0s)} bunches, {n} e- (sizes 10^U(3,6)), a0 ~ U(50,500), gamma0 ~ U(500,5000), "
                    f"plane waves, {steps} steps, photons recorded",
        "fp64_plain": r_plain, "fp32_batched_graph": r_b, "fp64_batched_graph": r_d,
        "speedup": r_plain["ms_per_step"] / r_b["ms_per_step"],
        "speedup_of_batching_fp64": r_plain["ms_per_step"] / r_d["ms_per_step"],
        "speedup_of_fp32_batched": r_d["ms_per_step"] / r_b["ms_per_step"],
        "ks_photon_gamma_same_seed_p": float(stats.ks_2samp(g_plain, g_b).pvalue),
        "ks_photon_gamma_seed_plus_1000_p": float(stats.ks_2samp(g_plain, g_c).pvalue),
        "ks_sample": len(g_plain),
        "cpu_baseline": cpu_bunch_baseline(steps, seed) if cpu else None,
    }


def _timed_steps(run, K, stream):
    """K steps of a sim.Run with HIP events around every library call."""
    import torch

    evs = {}

    def timed(kind, fn):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        fn()
        b.record(stream)
        evs.setdefault(kind, []).append((a, b))

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for n in range(K):
        run.step(n, timed=timed)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kernel_ms = {k: sum(a.elapsed_time(b) for a, b in v) for k, v in evs.items() if v}
    return wall, kernel_ms, {k: len(v) for k, v in evs.items() if v}


def _energy_balance(run, res, init_el):
    """|dK - W_field + E_rad + E_gamma + E_sub - E_pair| / (E_rad + E_gamma + E_sub) over a run."""
    import numpy as np

    def kin(sp):
        u2 = sp["ux"].astype(np.float64) ** 2 + sp["uy"].astype(np.float64) ** 2 + sp["uz"].astype(np.float64) ** 2
        return float(np.sum(sp["w"].astype(np.float64) * (np.sqrt(1.0 + u2) - 1.0)))

    t = res["tally"]
    k0 = kin(init_el)
    k1 = kin(res["electrons"]) + kin(res["positrons"])
    e_gamma = t["E_epush"] + t["E_erec"] + t["E_edrop"]
    # pairs: the created leptons carry E_pair - 2 (rest mass) per pair weight; E_pair is the photons' energy
    denom = t["E_erad"] + e_gamma + t["E_esub"]
    return abs((k1 - k0) - t["E_work"] + t["E_erad"] + e_gamma + t["E_esub"] - t["E_epair"]) / max(denom, 1e-300)


def bench_plane(args):
    """Plane-wave beam (1e5 e-, gamma0 2000, a0 = 100, 1000 steps, photons
    recorded): the FP64 plain form and the FP32 form on the same electrons."""
    import numpy as np
    import torch
    from scipy import stats

    from paper_1311_1107_amd import binding as B
    from paper_1311_1107_amd import sim as S
    from paper_1311_1107_amd import workloads as W

    stream = torch.cuda.current_stream()
    res = {}
    for name, prec, seed in (("f64", B.QED_F64, 1), ("f32", B.QED_F32, 1), ("f32_seed1001", B.QED_F32, 1001)):
        wl = W.plane_wave_beam(n=args.electrons or 100_000)
        wl.seed = seed
        n0 = len(wl.electrons["x"])
        K = min(args.steps or wl.steps, wl.steps)
        run = S.Run(wl, prec=prec, record_capacity=40 * n0)
        init_el = run.el.download()
        wall, kms, nl = _timed_steps(run, K, stream)
        rc, _ = run.ws.status(raise_on_error=False)
        r = run.result()
        t = r["tally"]
        ps = t["N_mc"] + t["N_sokolov"] + t["N_nan"]
        rec = r["recorded"]
        gam = np.sqrt(rec["ux"].astype(np.float64) ** 2 + rec["uy"].astype(np.float64) ** 2 + rec["uz"].astype(np.float64) ** 2)
        res[name] = {"pss": ps / wall, "ms_per_step": wall * 1e3 / K, "kernel_ms": kms, "launches": nl,
                     "photons": len(gam), "emissions": t["N_emit"], "status": int(rc),
                     "energy_balance": _energy_balance(run, r, init_el), "gamma": gam, "K": K, "n0": n0,
                     "lep_steps": ps, "N_mc": t["N_mc"], "N_push": t["N_push"], "N_rec": t["N_rec"],
                     "N_emit": t["N_emit"]}
        del run
        torch.cuda.empty_cache()
    f64, f32 = res["f64"], res["f32"]
    es = 8
    # tau is read and written by Monte Carlo steps only (the Sokolov branch leaves it alone)
    lep_bytes = (f64["lep_steps"] * 13 * es + f64["N_mc"] * 16 + f64["N_emit"] * 16
                 + (f64["N_push"] + f64["N_rec"]) * (8 * es + 20))
    push_ms = f64["kernel_ms"].get("push_e", 0.0)
    achieved = lep_bytes / (push_ms * 1e-3) / 1e9 if push_ms > 0 else 0.0
    n_l = f64["launches"].get("push_e", 1)
    out = {
        "metric": "QED particle-steps/s", "value": f64["pss"], "unit": "particle-steps/s", "n_gpus": 1,
        "steps": f64["K"], "warmup": 0, "ms_per_step": f64["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{f64['n0']} e- gamma0 2000 (1% spread) vs a0=100 10-period plane wave, "
                               f"{f64['K']} steps, photons recorded (FP64 plain)"},
        "roofline": {"bound": "hbm", "kernel": "qed_push_emit (lepton step)", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "bytes_per_launch": lep_bytes / n_l, "avg_launch_ms": push_ms / n_l,
                     "note": "working set ~11 MB per step: cache-resident and launch-bound"},
        "fp32_form": {"value": f32["pss"], "ms_per_step": f32["ms_per_step"], "speedup": f32["pss"] / f64["pss"],
                      "ks_photon_gamma_same_seed_p": float(stats.ks_2samp(f64["gamma"], f32["gamma"]).pvalue),
                      "ks_photon_gamma_seed_plus_1000_p": float(stats.ks_2samp(f64["gamma"], res["f32_seed1001"]["gamma"]).pvalue),
                      "photons_f64": f64["photons"], "photons_f32": f32["photons"],
                      "energy_balance_f64": f64["energy_balance"], "energy_balance_f32": f32["energy_balance"]},
        "detail": {k: {kk: vv for kk, vv in v.items() if kk != "gamma"} for k, v in res.items()},
        # the oracle on the whole workload (every electron, every step), one thread and all cores
        "cpu_baseline": None if args.no_cpu_baseline else cpu_baseline(
            W.plane_wave_beam(n=args.electrons or 100_000), args.electrons or 100_000, 0,
            min(args.steps or 1000, 1000), 1.0, caps=(1, 1, 0, 40)),
    }
    return out


def bench_cascade(args):
    """High-chi cascade: 5e7 e-, gamma0 1e4, a0 = 1000 plane wave, 500 steps,
    FP32 form; photons with chi_gamma > 0.2 at creation are pushed and tested
    for pairs, the rest tallied; decayed photons compacted every step.  Every
    10 steps a species past half of its buffer is merged (qed_merge over
    lambda/2 cells), unless --no-merge: then the run stops at the first step
    whose appends did not fit."""
    import torch

    from paper_1311_1107_amd import binding as B
    from paper_1311_1107_amd import sim as S
    from paper_1311_1107_amd import workloads as W

    wl = W.cascade_beam(n=args.electrons or 50_000_000)
    n0 = len(wl.electrons["x"])
    K = min(args.steps or wl.steps, wl.steps)
    lam = W.LAM
    pol = None if args.no_merge else S.MergePolicy(
        origin=(-10.0 * lam, -2.0 * lam, -2.0 * lam), spacing=(0.5 * lam,) * 3, shape=(60, 48, 48), sub_bins=4,
        n_dir=16, min_group=4, threshold=0.5)
    run = S.Run(wl, prec=B.QED_F32, photon_capacity=4 * n0, pair_capacity=4 * n0, compact_every=1, merge=pol)
    stream = torch.cuda.current_stream()
    growth = []
    chunk = 10
    wall = 0.0
    kms, nl = {}, {}
    done = 0
    stopped = None
    merge_ms = 0.0
    while done < K:
        k = min(chunk, K - done)
        # the chunk's steps continue the run's step numbering
        w, km, n_ = _timed_steps(_Offset(run, done), k, stream)
        wall += w
        for key, v in km.items():
            kms[key] = kms.get(key, 0.0) + v
        for key, v in n_.items():
            nl[key] = nl.get(key, 0) + v
        done += k
        rc, rep = run.ws.status(clear=False, raise_on_error=False)
        if rc != 0:
            # a buffer is full: stop and report the growth up to this step
            growth.append({"step": done, **run.counts()})
            stopped = {"step": done, "status": int(rc)}
            break
        if pol is not None:
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            a.record(stream)
            m = run.merge_if_needed()
            b.record(stream)
            torch.cuda.synchronize()
            wall += time.perf_counter() - t0
            if m:
                merge_ms += a.elapsed_time(b)
                nl["merge"] = nl.get("merge", 0) + len(m)
        if done % 50 == 0:
            growth.append({"step": done, **run.counts()})
            print(f"bench: cascade step {done}/{K}", file=sys.stderr, flush=True)
    if merge_ms:
        kms["merge"] = merge_ms
    rc, _ = run.ws.status(raise_on_error=False)
    t = run.tally.reduce()
    lep = t["N_mc"] + t["N_sokolov"] + t["N_nan"]
    ph = t["N_phstep"]
    es = 4
    rec_bytes = 8 * es + 20
    lep_bytes = lep * 13 * es + t["N_mc"] * 16 + t["N_emit"] * 16 + (t["N_push"] + t["N_rec"]) * rec_bytes
    ph_bytes = ph * (9 * es + 16) + t["N_pair"] * (7 * es + 8 + 2 * rec_bytes)
    push_ms = kms.get("push_e", 0.0) + kms.get("push_p", 0.0)
    pair_ms = kms.get("pair", 0.0)
    total_bytes = lep_bytes + ph_bytes
    kern_ms = push_ms + pair_ms
    achieved = total_bytes / (kern_ms * 1e-3) / 1e9 if kern_ms > 0 else 0.0
    merging = "merging every 10 steps past half a buffer" if pol is not None else "no merging"
    return {
        "metric": "QED particle-steps/s", "value": (lep + ph) / wall, "unit": "particle-steps/s", "n_gpus": 1,
        "steps": done, "warmup": 0, "ms_per_step": wall * 1e3 / done, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": f"{n0} e- gamma0 1e4 (1% spread) vs a0=1000 10-period plane wave, {K} steps, "
                               "FP32 form, photons with chi_gamma>0.2 pushed + pairs, compaction every step, "
                               + merging},
        "roofline": {"bound": "hbm", "kernel": "qed_push_emit + qed_pair_create", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None},
        "detail": {"growth": growth, "stopped_at_capacity": stopped, "kernel_ms": kms, "launches": nl,
                   "merges": run.merges, "status": int(rc), "tally": t},
        # the oracle on 1000 of the electrons over the same steps (the subset's cascade grows
        # about tenfold in leptons and photons; its buffers hold that without merging)
        "cpu_baseline": None if args.no_cpu_baseline else cpu_baseline(wl, 1000, 0, K, 1.0, caps=(12, 12, 40, 0)),
    }


class _Offset:
    """A sim.Run whose step numbers start at `start` (for a run timed in chunks)."""

    def __init__(self, run, start):
        self.run, self.start = run, start

    def step(self, n, timed=None):
        self.run.step(self.start + n, timed=timed)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: the library has no multi-GPU path (asked for --gpus {args.gpus}).",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_1311_1107_amd import binding as B
    from paper_1311_1107_amd import device as D
    from paper_1311_1107_amd import sim as S
    from paper_1311_1107_amd import workloads as W

    assert torch.cuda.is_available(), "bench.py needs the GPU"
    torch.cuda.set_device(0)

    if args.copy_calibration:
        a = torch.empty(1 << 27, dtype=torch.float64, device="cuda")     # 1 GiB
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    if args.workload in ("plane", "cascade", "batched", "batched-fp32"):
        if args.workload == "plane":
            out = bench_plane(args)
        elif args.workload == "cascade":
            out = bench_cascade(args)
        else:
            out = batched_comparison(args.steps or 1000, cpu=not args.no_cpu_baseline, graph=not args.no_graph,
                                     only_fp32=args.workload == "batched-fp32")
        print(json.dumps(out), flush=True)
        return
    coupled = args.workload == "coupled"
    wl = W.yee_beam(n=args.electrons or 10_000_000)
    n0 = len(wl.electrons["x"])
    caps = dict(photon_capacity=42 * n0, record_capacity=6 * n0, pair_capacity=n0 // 4)
    prec = B.QED_F64
    desc = ("1e7 e- (ln gamma0 ~ N(ln 2000, 0.3^2), r <= 2 lambda, x in [20,28) lambda) vs focused pulse "
            "a0=200 w0=3 lambda 30 fs on a 256x128x128 FP32 Yee grid, TSC gather, FP64, photons with "
            "chi_gamma>1e-3 pushed + Breit-Wheeler pairs, 2000-step collision")
    if coupled:
        desc += ("; coupled: the pulse sampled once, then advanced by the Yee solver with the leptons' "
                 "Esirkepov currents (1000 physical electrons per unit weight)")
    W_ = max(0, args.warmup)
    start = max(W_, min(args.start, wl.steps - 1))
    K = args.steps if args.steps is not None else 1000
    K = max(1, min(K, wl.steps - start))

    run = S.Run(wl, prec=prec, compact_every=args.compact_every, sort_every=args.sort_every,
                photon_sort_every=args.photon_sort_every, coupled=coupled,
                particles_per_weight=1000.0, field_bound_block=args.bound_block, **caps)
    # untimed advance into the collision, then the warm-up steps
    for k in range(start):
        run.step(k)
        if (k + 1) % 250 == 0:
            torch.cuda.synchronize()
            print(f"bench: advanced to step {k + 1}/{start}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    tal0 = run.tally.reduce()
    counts0 = run.counts()

    # per-call event timing on the stream the kernels run on
    stream = torch.cuda.current_stream()
    evs = {}

    def timed(kind, fn):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        fn()
        b.record(stream)
        evs.setdefault(kind, []).append((a, b))

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for n in range(start, start + K):
        run.step(n, timed=timed)
        if (n + 1 - start) % 250 == 0:                 # the host runs at most a queue's depth ahead
            print(f"bench: step {n + 1}/{start + K} enqueued", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    rc, rep = run.ws.status(raise_on_error=False)
    tal1 = run.tally.reduce()
    tal = {k: tal1[k] - tal0[k] for k in tal1}           # the timed steps only
    counts = run.counts()
    kernel_ms = {k: sum(a.elapsed_time(b) for a, b in v) for k, v in evs.items() if v}
    n_launch = {k: len(v) for k, v in evs.items() if v}

    lepton_steps = tal["N_mc"] + tal["N_sokolov"] + tal["N_nan"]
    photon_steps = tal["N_phstep"]
    psteps = lepton_steps + photon_steps
    # algorithmic bytes per unit (es = 8 for FP64 reals; tau is always FP64):
    #   lepton-step: x, u read and written 12 es, weight read es (energy tally)
    #   Monte Carlo step: tau read and written 16 B (the Sokolov branch leaves tau alone)
    #   emission event: uid read 8 B, n_event read and written 8 B
    #   stored photon: x, k, w, chi 8 es, tau 8 B, uid 8 B, n_event 4 B written
    #   photon-step: x, k, tau read 6 es + 8 B; x, tau written 3 es + 8 B
    #   pair event: photon x, k, w read 7 es, tau written 8 B, two leptons written 2 (8 es + 20 B)
    # (the grid nodes the gathers read are not counted: the counters measure them)
    es = 8
    rec_bytes = 8 * es + 20
    lep_bytes = (lepton_steps * 13 * es + tal["N_mc"] * 16 + tal["N_emit"] * 16
                 + (tal["N_push"] + tal["N_rec"]) * rec_bytes)
    ph_bytes = photon_steps * (9 * es + 16) + tal["N_pair"] * (7 * es + 8 + 2 * rec_bytes)
    calls = {
        "qed_push_emit (lepton step: k_lepton_stream, k_scan_tiles, k_lepton_events, k_scan_tiles, k_push_append; electrons and positrons)":
            (lep_bytes, kernel_ms.get("push_e", 0.0) + kernel_ms.get("push_p", 0.0),
             n_launch.get("push_e", 0) + n_launch.get("push_p", 0), "push"),
        "qed_pair_create (photon step: k_pair_create, k_scan_tiles, k_pair_append)":
            (ph_bytes, kernel_ms.get("pair", 0.0), n_launch.get("pair", 0), "pair"),
    }
    per_call = {}
    for name, (byts, ms, nl, key) in calls.items():
        ach = byts / (ms * 1e-3) / 1e9 if ms > 0 else 0.0
        per_call[key] = {"call": name, "bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": ach / HBM_PEAK_GBS, "bytes_per_launch": byts / max(nl, 1),
                         "avg_launch_ms": ms / max(nl, 1), "launches": nl}
    dom = max(per_call, key=lambda k: per_call[k]["avg_launch_ms"] * per_call[k]["launches"])
    roof = dict(per_call[dom])
    roof["kernel"] = roof.pop("call")
    # counters are taken on the driver's command (1e7 electrons, steps [1000, 1020), 5 warm-up steps)
    default_cfg = (n0 == 10_000_000 and start == 1000 and K == 20 and W_ == 5 and args.sort_every == 16
                   and run.photon_sort_every == 16 and args.compact_every == 16 and not coupled
                   and args.bound_block == 0)
    for key, pc in per_call.items():
        t_ = measured_traffic(key) if default_cfg else None
        pc["traffic"] = t_
        if t_:
            pc["traffic_ratio"] = t_ / pc["bytes_per_launch"]
    tr = per_call[dom]["traffic"]
    roof["traffic"] = tr
    if tr:
        roof["traffic_ratio"] = tr / roof["bytes_per_launch"]

    out = {
        "metric": "QED particle-steps/s",
        "value": psteps / wall,
        "unit": "particle-steps/s",
        "n_gpus": 1, "steps": K, "warmup": W_,
        "ms_per_step": wall * 1e3 / K,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": desc, "electrons": n0, "grid": list(wl.field.shape),
                   "steps_timed": [start, start + K], "advanced_untimed_to": start - W_, "dt": wl.dt,
                   "compact_every": args.compact_every, "sort_every": args.sort_every,
                   "photon_sort_every": run.photon_sort_every, "bound_block": args.bound_block},
        "roofline": roof,
        "roofline_calls": per_call,
        "detail": {"lepton_steps": lepton_steps, "photon_steps": photon_steps, "kernel_ms": kernel_ms,
                   "launches": n_launch, "counts_at_start": counts0, "counts_at_end": counts,
                   "emissions": tal["N_emit"], "pairs": tal["N_pair"], "status": int(rc),
                   "lepton_bytes": lep_bytes, "photon_bytes": ph_bytes,
                   "photon_steps_without_gather": tal.get("N_nogather", 0)},
    }
    if coupled:
        out["detail"]["deposit_skipped"] = int(run.skipped.item())
    del run
    torch.cuda.empty_cache()
    if args.batched_steps > 0 and not coupled:
        out["batched_vs_plain"] = batched_comparison(args.batched_steps, cpu=not args.no_cpu_baseline,
                                                     graph=not args.no_graph)
    # measured copy bandwidth on this GPU (after the timed region), for the ratio to it
    copy_gbs = device_copy_gbs()
    out["roofline"]["copy_GBs"] = copy_gbs
    out["roofline"]["frac_of_copy"] = out["roofline"]["achieved"] / copy_gbs if copy_gbs > 0 else None
    if not args.no_cpu_baseline and not coupled:
        print("bench: oracle CPU baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(wl, args.cpu_sample, start, K, args.cpu_min_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
