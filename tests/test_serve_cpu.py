"""Serving scheduler logic on the CPU, with fake backends: admission by
memory budget and slot count, rejection of jobs that can never fit,
arrival order, completion of every admitted job, and results of a job that
do not depend on the other jobs in the mix (CPU oracle backend)."""

import numpy as np
import pytest
import torch

from paper_1909_08423_amd.serve import JobSpec, Server, summarize
from synth import make_config


class VirtualClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 1e-4)


class TimedFakeBackend:
    """Each step takes `step_s` of virtual time; bytes = walkers * 1 KiB."""

    def __init__(self, clock, step_s=0.01):
        self.clock = clock
        self.step_s = step_s
        self.in_use = 0
        self.peak = 0
        self.started = []

    def bytes(self, spec):
        return spec.walkers.shape[0] * 1024

    def start(self, spec):
        self.in_use += self.bytes(spec)
        self.peak = max(self.peak, self.in_use)
        self.started.append(spec.job_id)
        return {"step": 0, "spec": spec}

    def step(self, st):
        st["step"] += 1
        return self.clock.t + self.step_s

    def ready(self, tok):
        return self.clock.t >= tok

    def latency_ms(self, tok):
        return self.step_s * 1e3

    def finish(self, st):
        self.in_use -= self.bytes(st["spec"])
        return {"stats": np.zeros((st["spec"].n_steps, 8)), "params": np.zeros(1), "eloc": np.zeros(1)}


def _specs(n, walkers, gaps, steps=3):
    w = make_config(1, n_walkers=2)
    out, t = [], 0.0
    for j in range(n):
        t += gaps[j % len(gaps)]
        out.append(JobSpec(j, t, steps, w.system, w.net, w.params, np.zeros((walkers[j % len(walkers)], 2, 3)),
                           seed=j))
    return out


def test_admission_respects_budget_and_slots():
    clk = VirtualClock()
    be = TimedFakeBackend(clk)
    specs = _specs(12, [256, 512, 1024], [0.001, 0.0, 0.002])
    srv = Server(be, mem_budget_bytes=1024 * 1500, max_active=3, clock=clk, sleep=clk.sleep)
    recs = srv.run(specs)
    assert all(r.stats is not None for r in recs.values())
    assert be.peak <= 1024 * 1500
    assert srv.max_concurrency <= 3
    # admitted in arrival order (no overtaking)
    assert be.started == sorted(be.started)
    s = summarize(recs, clk.t)
    assert s["jobs_done"] == 12 and s["steps"] == 36


def test_oversized_job_is_rejected_others_run():
    clk = VirtualClock()
    be = TimedFakeBackend(clk)
    specs = _specs(4, [256, 4096, 256, 256], [0.0])
    srv = Server(be, mem_budget_bytes=1024 * 1024, max_active=4, clock=clk, sleep=clk.sleep)
    recs = srv.run(specs)
    assert recs[1].rejected and recs[1].stats is None
    assert all(recs[j].stats is not None for j in (0, 2, 3))


def test_jobs_arriving_later_join_while_others_run():
    clk = VirtualClock()
    be = TimedFakeBackend(clk, step_s=0.01)
    specs = _specs(3, [256], [0.0, 0.015, 0.015], steps=5)
    srv = Server(be, mem_budget_bytes=1 << 30, max_active=8, clock=clk, sleep=clk.sleep)
    recs = srv.run(specs)
    # job 1 is admitted before job 0 has finished: the two run concurrently
    assert recs[1].admitted_s < recs[0].finished_s
    assert srv.max_concurrency >= 2


class OracleBackend:
    """CPU backend built from the oracle's VMC pieces (tiny jobs only)."""

    def __init__(self):
        from oracle import Oracle  # noqa: F401

    def bytes(self, spec):
        return 1

    def start(self, spec):
        from oracle import Oracle
        o = Oracle(spec.system, spec.net, spec.params)
        return {"o": o, "r": torch.tensor(spec.walkers), "th": torch.tensor(spec.params), "step": 0,
                "m": torch.zeros(spec.params.shape[0], dtype=torch.float64),
                "v": torch.zeros(spec.params.shape[0], dtype=torch.float64), "seed": spec.seed,
                "stats": [], "spec": spec}

    def step(self, st):
        from oracle.vmc import adamw_step, energy_gradient, metropolis_randoms, metropolis_step
        o, r = st["o"], st["r"]
        B, N = r.shape[0], r.shape[1]
        with torch.no_grad():
            la = o.log_psi(r)[0]
        xi, u = metropolis_randoms(st["seed"], st["step"], B, 3 * N)
        r, _, acc = metropolis_step(o, r, la, xi, u, 0.3)
        el = o.evaluate(r)["eloc"]
        g, L, _ = energy_gradient(o, r, el)
        th, st["m"], st["v"] = adamw_step(st["th"], g, st["m"], st["v"], st["step"])
        st["th"], st["r"] = th, r
        o.set_params(th)
        st["eloc"] = el
        st["stats"].append([float(el.mean()), float(L), float(acc.double().mean())])
        st["step"] += 1
        return True

    def ready(self, tok):
        return True

    def latency_ms(self, tok):
        return 0.0

    def finish(self, st):
        return {"stats": np.asarray(st["stats"]), "params": st["th"].numpy(), "eloc": st["eloc"].numpy()}


@pytest.mark.slow
def test_result_same_alone_and_in_the_mix_cpu_oracle():
    w1 = make_config(1, n_walkers=6)
    w2 = make_config(2, n_walkers=3)
    a = JobSpec(0, 0.0, 2, w1.system, w1.net, w1.params, w1.walkers, seed=11)
    b = JobSpec(1, 0.0, 2, w2.system, w2.net, w2.params, w2.walkers, seed=12)
    alone = Server(OracleBackend(), 1 << 30).run([a])[0]
    mix = Server(OracleBackend(), 1 << 30).run([b, a])[0]
    np.testing.assert_array_equal(alone.params, mix.params)
    np.testing.assert_array_equal(alone.eloc, mix.eloc)


class GroupedFakeBackend(TimedFakeBackend):
    """Grouped steps: one step of every member takes `step_s` of virtual
    time; results are collected after a copy that completes at once."""

    grouped = True

    def __init__(self, clock, step_s=0.01):
        super().__init__(clock, step_s)
        self.groups = []

    def step_group(self, states):
        self.groups.append(sorted(st["spec"].job_id for st in states))
        for st in states:
            st["step"] += 1
        return self.clock.t + self.step_s

    def finish_async(self, st):
        return st

    def collected(self, tok):
        return True

    def collect(self, st):
        return self.finish(st)


def test_grouped_steps_admit_at_step_boundaries():
    """Grouped stepping: every admitted job finishes its steps, later
    arrivals join the running group at a step boundary, the budget and the
    slot limit hold, and steps that follow an admission are flagged."""
    clk = VirtualClock()
    be = GroupedFakeBackend(clk, step_s=0.01)
    specs = _specs(6, [256, 512, 1024], [0.0, 0.012, 0.03], steps=8)
    srv = Server(be, mem_budget_bytes=1024 * 1800, max_active=3, clock=clk, sleep=clk.sleep)
    recs = srv.run(specs)
    assert all(r.stats is not None and len(r.step_ms) == 8 for r in recs.values())
    assert be.peak <= 1024 * 1800 and srv.max_concurrency <= 3
    assert be.started == sorted(be.started)
    # a group holds several jobs, and some job joins a group already running
    assert max(len(g) for g in be.groups) >= 2
    assert any(set(a) < set(b) for a, b in zip(be.groups, be.groups[1:]))
    s = summarize(recs, clk.t)
    assert s["steps"] == 48 and s["p99_step_ms_after_admission"] is not None
    assert sum(sum(r.step_after_admission) for r in recs.values()) >= 1
