"""Continuous-batching VMC serving loop.

Many independent VMC jobs (different molecules, electron counts, walker
counts) arrive over time.  Each admitted job keeps its walkers, parameters
and AdamW moments resident in device memory and advances one VMC step at a
time (Metropolis move, local energy, clipping, Hermitian gradient, AdamW;
Methods, "Ansatz optimization").  Jobs are admitted while their device bytes
fit the memory budget and a slot is free; every active job has one step in
flight on its own stream, so steps of different jobs overlap on the device;
a finished job frees its memory and slot for the next arrival.

The scheduler is backend-agnostic: `GpuBackend` drives the HIP library;
tests drive the same scheduler with a CPU backend.  Results of a job do not
depend on what else runs (each step is deterministic and uses a
counter-based RNG keyed by the job's seed).
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
    stats: Optional[np.ndarray] = None    # [n_steps, 8]
    params: Optional[np.ndarray] = None   # final parameters
    eloc: Optional[np.ndarray] = None     # final local energies
    rejected: bool = False


class GpuBackend:
    """Runs jobs through pn_vmc_step on a pool of HIP streams."""

    def __init__(self, prec: int = 1, n_streams: int = 8, hparams: Optional[dict] = None, device="cuda"):
        import torch

        from . import _lib
        self.torch = torch
        self.lib = _lib
        self.prec = prec
        self.hp = hparams
        self.device = device
        self.streams = [torch.cuda.Stream(device=device) for _ in range(n_streams)]
        self._next = 0

    def bytes(self, spec: JobSpec) -> int:
        B, N = spec.walkers.shape[0], spec.walkers.shape[1]
        n_par = spec.params.shape[0]
        ctx = self.lib.PauliNetContext(spec.system, spec.net)
        ws = self.lib.vmc_workspace_bytes(ctx, B, self.prec)
        ctx.close()
        resident = 8 * (B * N * 3 + 3 * n_par + B + spec.n_steps * 8)
        return ws + resident

    def start(self, spec: JobSpec):
        t = self.torch
        ctx = self.lib.PauliNetContext(spec.system, spec.net)
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
            "stream": self.streams[self._next % len(self.streams)],
        }
        self._next += 1
        # make the uploads visible to the job's stream
        st["stream"].wait_stream(t.cuda.current_stream())
        return st

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
        return (ev0, ev1)

    def ready(self, token) -> bool:
        return token[1].query()

    def latency_ms(self, token) -> float:
        return token[0].elapsed_time(token[1])

    def finish(self, st) -> Dict[str, np.ndarray]:
        st["stream"].synchronize()
        out = {"stats": st["hist"].cpu().numpy(), "params": st["params"].cpu().numpy(),
               "eloc": st["eloc"].cpu().numpy()}
        st["ctx"].close()
        return out


class Server:
    """Admission by memory budget and slot count; one step in flight per
    active job; steps of all active jobs overlap on the device."""

    def __init__(self, backend, mem_budget_bytes: int, max_active: int = 16, clock=time.monotonic,
                 sleep=time.sleep):
        self.backend = backend
        self.budget = int(mem_budget_bytes)
        self.max_active = max_active
        self.clock = clock
        self.sleep = sleep
        self.log: List[tuple] = []
        self.max_concurrency = 0
        self.max_bytes_in_use = 0

    def run(self, specs: List[JobSpec], time_scale: float = 1.0) -> Dict[int, JobRecord]:
        pending = sorted(specs, key=lambda s: (s.arrival_s, s.job_id))
        records = {s.job_id: JobRecord(s.job_id, s.walkers.shape[0], s.walkers.shape[1]) for s in specs}
        sizes = {s.job_id: self.backend.bytes(s) for s in specs}
        active = {}  # job_id -> (spec, state, token or None)
        used = 0
        t0 = self.clock()
        while pending or active:
            now = (self.clock() - t0) / time_scale
            # admission, in arrival order (no overtaking)
            while pending and pending[0].arrival_s <= now:
                s = pending[0]
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
                used += need
                self.max_bytes_in_use = max(self.max_bytes_in_use, used)
                active[s.job_id] = [s, st, None]
                records[s.job_id].admitted_s = now
                self.log.append(("admit", s.job_id, now))
            self.max_concurrency = max(self.max_concurrency, len(active))
            # launch a step for every active job that has none in flight
            for jid, ent in active.items():
                s, st, tok = ent
                if tok is None and st["step"] < s.n_steps:
                    ent[2] = self.backend.step(st)
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


def summarize(records: Dict[int, JobRecord], wall_s: float) -> dict:
    lat = np.concatenate([np.asarray(r.step_ms) for r in records.values() if r.step_ms] or [np.zeros(0)])
    walker_steps = sum(r.n_walkers * len(r.step_ms) for r in records.values())
    return {
        "jobs_done": sum(1 for r in records.values() if r.stats is not None),
        "jobs_rejected": sum(1 for r in records.values() if r.rejected),
        "steps": int(lat.size),
        "p50_step_ms": float(np.percentile(lat, 50)) if lat.size else None,
        "p99_step_ms": float(np.percentile(lat, 99)) if lat.size else None,
        "walker_steps_per_s": walker_steps / wall_s if wall_s > 0 else None,
        "wall_s": wall_s,
    }
