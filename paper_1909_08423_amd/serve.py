"""Continuous-batching VMC serving loop.

Many independent VMC jobs (different molecules, electron counts, walker
counts) arrive over time.  Each admitted job keeps its walkers, parameters
and AdamW moments resident in device memory and advances one VMC step at a
time (Metropolis move, local energy, clipping, Hermitian gradient, AdamW;
Methods, "Ansatz optimization").  Jobs are admitted in arrival order while
their device bytes (pn_job_bytes) fit the memory budget and a slot is free;
a finished job frees its memory and slot for the next arrival.

Two ways to advance the active jobs, behind one scheduler:
  grouped   every step is one pn_serve_step launch sequence over all active
            jobs on the server's stream (the grouped proposal, acceptance,
            clipping and AdamW launches cover every slot); jobs join and
            leave at step boundaries, and up to two grouped steps are in
            flight so the host prepares the next while the device runs;
  per job   every active job has one pn_vmc_step in flight on a stream of
            its own, so steps of different jobs overlap on the device.
Either way a job's results do not depend on what else runs: every step is
deterministic and draws from a counter-based RNG keyed by the job's seed.

Contexts are created once per job (at its arrival) and destroyed when the
server closes, so no device-wide synchronisation of a free happens while
steps are in flight.  The scheduler is backend-agnostic: `GpuBackend` drives
the HIP library; tests drive the same scheduler with CPU backends.
"""

from __future__ import annotations

import dataclasses
import time
from typing import Dict, List, Optional

import numpy as np


@dataclasses.dataclass
class JobSpec:
    job_id: int
    arrival_s: float
    n_steps: int
    system: object
    net: object
    params: np.ndarray
    walkers: np.ndarray
    seed: int


@dataclasses.dataclass
class JobRecord:
    job_id: int
    n_walkers: int
    n_elec: int
    admitted_s: float = float("nan")
    finished_s: float = float("nan")
    step_ms: List[float] = dataclasses.field(default_factory=list)
    step_after_admission: List[bool] = dataclasses.field(default_factory=list)
    stats: Optional[np.ndarray] = None    # [n_steps, 8]
    params: Optional[np.ndarray] = None   # final parameters
    eloc: Optional[np.ndarray] = None     # final local energies
    rejected: bool = False


class GpuBackend:
    """Runs jobs through the HIP library: grouped steps (pn_serve_step on one
    stream) or one pn_vmc_step per job on per-slot streams."""

    def __init__(self, prec: int = 1, grouped: bool = True, n_streams: int = 16, hparams: Optional[dict] = None,
                 device="cuda"):
        import torch

        from . import _lib
        self.torch = torch
        self.lib = _lib
        self.prec = prec
        self.hp = hparams
        self.device = device
        self.grouped = grouped
        self.stream = torch.cuda.Stream(device=device)
        self.free_streams = [torch.cuda.Stream(device=device) for _ in range(n_streams)]
        self.ctxs = {}

    def _ctx(self, spec: JobSpec):
        ctx = self.ctxs.get(spec.job_id)
        if ctx is None:
            ctx = self.lib.PauliNetContext(spec.system, spec.net)
            self.ctxs[spec.job_id] = ctx
        return ctx

    def bytes(self, spec: JobSpec) -> int:
        res, scr = self.lib.job_bytes(self._ctx(spec), spec.walkers.shape[0], self.prec)
        return res + scr + 8 * 8 * spec.n_steps  # + the per-step statistics history

    def start(self, spec: JobSpec):
        t = self.torch
        ctx = self._ctx(spec)
        dev = self.device
        st = {
            "ctx": ctx,
            "r": t.tensor(spec.walkers, dtype=t.float64, device=dev),
            "params": t.tensor(spec.params, dtype=t.float64, device=dev),
            "adam_m": t.zeros(spec.params.shape[0], dtype=t.float64, device=dev),
            "adam_v": t.zeros(spec.params.shape[0], dtype=t.float64, device=dev),
            "eloc": t.empty(spec.walkers.shape[0], dtype=t.float64, device=dev),
            "hist": t.full((spec.n_steps, 8), float("nan"), dtype=t.float64, device=dev),
            "ws": t.empty(self.lib.vmc_workspace_bytes(ctx, spec.walkers.shape[0], self.prec), dtype=t.uint8,
                          device=dev),
            "seed": spec.seed,
            "step": 0,
        }
        st["stream"] = self.stream if self.grouped else self.free_streams.pop()
        # make the uploads visible to the job's stream
        st["stream"].wait_stream(t.cuda.current_stream())
        return st

    # -- grouped steps --
    def step_group(self, states):
        t = self.torch
        ev0 = t.cuda.Event(enable_timing=True)
        ev1 = t.cuda.Event(enable_timing=True)
        ev0.record(self.stream)
        for st in states:
            st["stats"] = st["hist"][st["step"]]
        self.lib.serve_step(states, self.prec, self.hp, stream=self.stream)
        ev1.record(self.stream)
        for st in states:
            st["step"] += 1
        return (ev0, ev1, time.perf_counter())

    # -- one step of one job --
    def step(self, st):
        t = self.torch
        s = st["stream"]
        ev0 = t.cuda.Event(enable_timing=True)
        ev1 = t.cuda.Event(enable_timing=True)
        ev0.record(s)
        st["stats"] = st["hist"][st["step"]]
        self.lib.vmc_step(st["ctx"], st, self.prec, self.hp, stream=s)
        ev1.record(s)
        st["step"] += 1
        return (ev0, ev1, time.perf_counter())

    def ready(self, token) -> bool:
        return token[1].query()

    def latency_ms(self, token) -> float:
        """Device time of the step (from its first to its last launch)."""
        return token[0].elapsed_time(token[1])

    def finish_async(self, st):
        """Copy the job's results to pinned host memory behind its last step;
        returns a token for `collect`."""
        t = self.torch
        s = st["stream"]
        out = {}
        with t.cuda.stream(s):
            for k, src in (("stats", st["hist"]), ("params", st["params"]), ("eloc", st["eloc"])):
                h = t.empty(src.shape, dtype=src.dtype, pin_memory=True)
                h.copy_(src, non_blocking=True)
                out[k] = h
        ev = t.cuda.Event()
        ev.record(s)
        if not self.grouped:
            self.free_streams.append(s)
        return {"event": ev, "out": out, "state": st}

    def collected(self, tok) -> bool:
        return tok["event"].query()

    def collect(self, tok) -> Dict[str, np.ndarray]:
        tok["event"].synchronize()
        return {k: v.numpy().copy() for k, v in tok["out"].items()}

    def finish(self, st) -> Dict[str, np.ndarray]:
        return self.collect(self.finish_async(st))

    def close(self):
        self.torch.cuda.synchronize()
        for ctx in self.ctxs.values():
            ctx.close()
        self.ctxs = {}


class Server:
    """Admission by memory budget and slot count, in arrival order; either
    grouped steps over all active jobs (backends with `step_group`) or one
    step in flight per active job."""

    def __init__(self, backend, mem_budget_bytes: int, max_active: int = 16, clock=time.monotonic,
                 sleep=time.sleep, max_inflight: int = 2):
        self.backend = backend
        self.budget = int(mem_budget_bytes)
        self.max_active = max_active
        self.max_inflight = max_inflight
        self.clock = clock
        self.sleep = sleep
        self.log: List[tuple] = []
        self.max_concurrency = 0
        self.max_bytes_in_use = 0

    def _admit(self, pending, active, records, sizes, used, now):
        """Admit arrived jobs in order while they fit; returns (used, admitted
        any).  A job that can never fit is rejected."""
        admitted = False
        while pending and pending[0].arrival_s <= now:
            s = pending[0]
            if s.job_id not in sizes:
                sizes[s.job_id] = self.backend.bytes(s)
            need = sizes[s.job_id]
            if need > self.budget:
                records[s.job_id].rejected = True
                self.log.append(("reject", s.job_id, now))
                pending.pop(0)
                continue
            if len(active) >= self.max_active or used + need > self.budget:
                break
            pending.pop(0)
            st = self.backend.start(s)
            st["completed"] = 0
            used += need
            self.max_bytes_in_use = max(self.max_bytes_in_use, used)
            active[s.job_id] = [s, st, None]
            records[s.job_id].admitted_s = now
            self.log.append(("admit", s.job_id, now))
            admitted = True
        return used, admitted

    def run(self, specs: List[JobSpec], time_scale: float = 1.0) -> Dict[int, JobRecord]:
        if getattr(self.backend, "grouped", False) and hasattr(self.backend, "step_group"):
            return self._run_grouped(specs, time_scale)
        pending = sorted(specs, key=lambda s: (s.arrival_s, s.job_id))
        records = {s.job_id: JobRecord(s.job_id, s.walkers.shape[0], s.walkers.shape[1]) for s in specs}
        sizes = {}
        active = {}  # job_id -> [spec, state, token or None]
        used = 0
        t0 = self.clock()
        while pending or active:
            now = (self.clock() - t0) / time_scale
            used, adm = self._admit(pending, active, records, sizes, used, now)
            self.max_concurrency = max(self.max_concurrency, len(active))
            # launch a step for every active job that has none in flight
            for jid, ent in active.items():
                s, st, tok = ent
                if tok is None and st["step"] < s.n_steps:
                    ent[2] = self.backend.step(st)
                    records[jid].step_after_admission.append(adm)
            # retire finished steps
            progressed = False
            for jid in list(active):
                s, st, tok = active[jid]
                if tok is not None and self.backend.ready(tok):
                    records[jid].step_ms.append(self.backend.latency_ms(tok))
                    active[jid][2] = None
                    progressed = True
                    if st["step"] >= s.n_steps:
                        out = self.backend.finish(st)
                        rec = records[jid]
                        rec.stats, rec.params, rec.eloc = out["stats"], out["params"], out["eloc"]
                        rec.finished_s = (self.clock() - t0) / time_scale
                        used -= sizes[jid]
                        del active[jid]
                        self.log.append(("finish", jid, rec.finished_s))
            if not progressed:
                if not active and pending:
                    wait = pending[0].arrival_s - (self.clock() - t0) / time_scale
                    if wait > 0:
                        self.sleep(min(wait * time_scale, 0.05))
                else:
                    self.sleep(0.0002)
        return records

    def _run_grouped(self, specs: List[JobSpec], time_scale: float) -> Dict[int, JobRecord]:
        """Every step of the active jobs is one grouped launch sequence; up to
        max_inflight grouped steps are queued on the device.  A job's results
        are copied out behind its last step without stopping the queue."""
        be = self.backend
        pending = sorted(specs, key=lambda s: (s.arrival_s, s.job_id))
        records = {s.job_id: JobRecord(s.job_id, s.walkers.shape[0], s.walkers.shape[1]) for s in specs}
        sizes = {}
        active = {}      # job_id -> [spec, state, None]
        inflight = []    # (token, member job ids, admitted since the previous launch)
        finishing = []   # (job id, copy token)
        used = 0
        admitted_since = False
        t0 = self.clock()
        while pending or active or inflight or finishing:
            now = (self.clock() - t0) / time_scale
            used, adm = self._admit(pending, active, records, sizes, used, now)
            admitted_since = admitted_since or adm
            self.max_concurrency = max(self.max_concurrency, len(active))
            progressed = False
            if len(inflight) < self.max_inflight:
                members = [jid for jid, (s, st, _) in active.items() if st["step"] < s.n_steps]
                if members:
                    tok = be.step_group([active[j][1] for j in members])
                    inflight.append((tok, members, admitted_since))
                    admitted_since = False
                    progressed = True
            if inflight and be.ready(inflight[0][0]):
                tok, members, adm_flag = inflight.pop(0)
                lat = be.latency_ms(tok)
                for jid in members:
                    rec = records[jid]
                    rec.step_ms.append(lat)
                    rec.step_after_admission.append(adm_flag)
                    s, st, _ = active[jid]
                    st["completed"] += 1
                    if st["completed"] >= s.n_steps:
                        finishing.append((jid, be.finish_async(st)))
                        del active[jid]
                progressed = True
            for item in list(finishing):
                jid, ctok = item
                if be.collected(ctok):
                    out = be.collect(ctok)
                    rec = records[jid]
                    rec.stats, rec.params, rec.eloc = out["stats"], out["params"], out["eloc"]
                    rec.finished_s = (self.clock() - t0) / time_scale
                    used -= sizes[jid]
                    finishing.remove(item)
                    self.log.append(("finish", jid, rec.finished_s))
                    progressed = True
            if not progressed:
                if not active and not inflight and not finishing and pending:
                    wait = pending[0].arrival_s - (self.clock() - t0) / time_scale
                    if wait > 0:
                        self.sleep(min(wait * time_scale, 0.05))
                else:
                    self.sleep(0.0002)
        return records


def summarize(records: Dict[int, JobRecord], wall_s: float) -> dict:
    lat = np.concatenate([np.asarray(r.step_ms) for r in records.values() if r.step_ms] or [np.zeros(0)])
    adm = np.concatenate([np.asarray(r.step_after_admission[:len(r.step_ms)], bool)
                          for r in records.values() if r.step_ms] or [np.zeros(0, bool)])
    walker_steps = sum(r.n_walkers * len(r.step_ms) for r in records.values())

    def pct(x, q):
        return float(np.percentile(x, q)) if x.size else None

    return {
        "jobs_done": sum(1 for r in records.values() if r.stats is not None),
        "jobs_rejected": sum(1 for r in records.values() if r.rejected),
        "steps": int(lat.size),
        "p50_step_ms": pct(lat, 50),
        "p99_step_ms": pct(lat, 99),
        "p50_step_ms_after_admission": pct(lat[adm], 50) if adm.size == lat.size else None,
        "p99_step_ms_after_admission": pct(lat[adm], 99) if adm.size == lat.size else None,
        "p99_step_ms_no_admission": pct(lat[~adm], 99) if adm.size == lat.size else None,
        "walker_steps_per_s": walker_steps / wall_s if wall_s > 0 else None,
        "wall_s": wall_s,
    }
