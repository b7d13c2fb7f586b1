"""GPU tests of the serving VMC step (pn_vmc_step) and of continuous
batching: one step against the CPU oracle's Metropolis / E_loc / clipping /
Hermitian gradient / AdamW, and a job's results identical alone and in a mix
of concurrently running jobs."""

import numpy as np
import pytest
import torch

from gpu_util import announce
from synth import make_config

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pn():
    import paper_1909_08423_amd as pn
    assert torch.cuda.is_available(), "no ROCm device"
    pn.load_library()
    return pn


def _state(pn, ctx, w, prec, seed, n_hist=1):
    dev = "cuda"
    return {
        "r": torch.tensor(w.walkers, dtype=torch.float64, device=dev),
        "params": torch.tensor(w.params, dtype=torch.float64, device=dev),
        "adam_m": torch.zeros(w.params.shape[0], dtype=torch.float64, device=dev),
        "adam_v": torch.zeros(w.params.shape[0], dtype=torch.float64, device=dev),
        "eloc": torch.empty(w.walkers.shape[0], dtype=torch.float64, device=dev),
        "stats": torch.zeros(8, dtype=torch.float64, device=dev),
        "ws": torch.empty(pn.vmc_workspace_bytes(ctx, w.walkers.shape[0], prec), dtype=torch.uint8, device=dev),
        "seed": seed, "step": 0,
    }


@pytest.mark.parametrize("idx", [1, 2, 6, 7])
def test_vmc_step_matches_oracle(pn, idx):
    from oracle import Oracle
    from oracle.vmc import adamw_step, energy_gradient, metropolis_randoms, metropolis_step
    w = make_config(idx, n_walkers=48)
    seed = 987654321987 + idx
    announce(f"vmc step vs oracle, workload {idx}")
    ctx = pn.PauliNetContext(w.system, w.net)
    st = _state(pn, ctx, w, pn.PN_PREC_FP64, seed)
    pn.vmc_step(ctx, st, pn.PN_PREC_FP64)
    torch.cuda.synchronize()
    # oracle
    o = Oracle(w.system, w.net, w.params)
    r0 = torch.tensor(w.walkers)
    B, N = r0.shape[0], r0.shape[1]
    with torch.no_grad():
        la0 = o.log_psi(r0)[0]
    xi, u = metropolis_randoms(seed, 0, B, 3 * N)
    r1, _, acc = metropolis_step(o, r0, la0, xi, u, 0.3)
    out = o.evaluate(r1)
    g, L, ec = energy_gradient(o, r1, out["eloc"])
    th1, _, _ = adamw_step(torch.tensor(w.params), g, torch.zeros_like(g), torch.zeros_like(g), 0)
    np.testing.assert_allclose(st["r"].cpu().numpy(), r1.numpy(), rtol=0, atol=1e-12)
    stats = st["stats"].cpu().numpy()
    assert abs(stats[2] - float(acc.double().mean())) < 1e-15
    e_gpu = st["eloc"].cpu().numpy()
    e_ref = out["eloc"].numpy()
    scale = np.maximum(1.0, np.abs(out["lap"].numpy()) + (out["grad"].numpy() ** 2).sum((1, 2)))
    assert np.max(np.abs(e_gpu - e_ref) / scale) < 1e-6
    assert abs(stats[3] - float(L)) < 1e-6 * max(1.0, abs(float(L)))
    assert stats[5] == 1.0
    th_gpu = st["params"].cpu().numpy()
    big = np.abs(g.numpy()) > 1e-5 * np.abs(g.numpy()).max()
    np.testing.assert_allclose(th_gpu[big], th1.numpy()[big], rtol=0, atol=1e-9)
    assert np.max(np.abs(th_gpu - th1.numpy())) <= 2.1 * 0.01  # the rest differ at most by the sign of a ~0 step


@pytest.mark.parametrize("grouped", [True, False])
def test_job_same_alone_and_in_the_mix(pn, grouped):
    """Continuous batching: job A's walkers, parameters and E_loc after 4
    steps are bit-identical whether it runs alone or together with three
    other jobs (one admitted mid-run), in grouped steps or per-job steps."""
    from paper_1909_08423_amd.serve import GpuBackend, JobSpec, Server
    specs = []
    wa = make_config(2, n_walkers=512)
    specs.append(JobSpec(0, 0.0, 4, wa.system, wa.net, wa.params, wa.walkers, seed=5))
    for j, (idx, B) in enumerate([(3, 768), (7, 256), (6, 1024)], start=1):
        wj = make_config(idx, n_walkers=B)
        specs.append(JobSpec(j, 0.0 if j < 3 else 0.02, 3, wj.system, wj.net, wj.params, wj.walkers, seed=100 + j))
    announce(f"alone vs mix, grouped={grouped}")
    be = GpuBackend(prec=1, grouped=grouped)
    alone = Server(be, 1 << 36).run([specs[0]])[0]
    be.close()
    be2 = GpuBackend(prec=1, grouped=grouped)
    srv = Server(be2, 1 << 36)
    mix = srv.run(specs)
    be2.close()
    assert srv.max_concurrency >= 2
    np.testing.assert_array_equal(alone.params, mix[0].params)
    np.testing.assert_array_equal(alone.eloc, mix[0].eloc)
    np.testing.assert_array_equal(alone.stats, mix[0].stats)
    assert all(mix[j].stats is not None and np.all(mix[j].stats[:, 5] == 1.0) for j in range(4))


def test_grouped_step_equals_per_job_steps(pn):
    """pn_serve_step over three jobs of different systems (a 10-electron atom,
    the odd H7 chain, H2) gives, for every job and two steps in a row, the
    bits pn_vmc_step gives on the same state."""
    jobs = [(2, 384, 11), (7, 256, 12), (1, 512, 13)]
    states_g, states_1 = [], []
    for idx, B, seed in jobs:
        w = make_config(idx, n_walkers=B)
        ctx = pn.PauliNetContext(w.system, w.net)
        for lst in (states_g, states_1):
            st = _state(pn, ctx, w, pn.PN_PREC_NET_FP32, seed)
            st["ctx"] = ctx
            lst.append(st)
    announce("grouped step vs per-job steps")
    for step in range(2):
        pn.serve_step(states_g, pn.PN_PREC_NET_FP32)
        for st in states_1:
            pn.vmc_step(st["ctx"], st, pn.PN_PREC_NET_FP32)
        torch.cuda.synchronize()
        for a, b in zip(states_g, states_1):
            for k in ("r", "params", "adam_m", "adam_v", "eloc", "stats"):
                assert torch.equal(a[k], b[k]), (step, k)
            a["step"] += 1
            b["step"] += 1


def test_job_bytes_cover_the_job(pn):
    """pn_job_bytes: the resident bytes are the job's state and the scratch
    is the step workspace."""
    w = make_config(2, n_walkers=300)
    ctx = pn.PauliNetContext(w.system, w.net)
    res, scr = pn.job_bytes(ctx, 300, pn.PN_PREC_NET_FP32)
    assert scr == pn.vmc_workspace_bytes(ctx, 300, pn.PN_PREC_NET_FP32)
    assert res == 8 * (300 * w.system.n_elec * 3 + 3 * ctx.param_count + 300 + 8)


def test_serving_admission_by_memory(pn):
    """With a budget that fits two jobs at a time, every job still completes,
    in arrival order, and the bytes in use never exceed the budget."""
    from paper_1909_08423_amd.serve import GpuBackend, JobSpec, Server
    specs = []
    for j in range(5):
        wj = make_config(1 + (j % 2), n_walkers=256)
        specs.append(JobSpec(j, 0.0, 2, wj.system, wj.net, wj.params, wj.walkers, seed=j))
    be = GpuBackend(prec=1)
    sizes = sorted(be.bytes(s) for s in specs)
    budget = sizes[-1] + sizes[-2]
    announce("admission by memory")
    srv = Server(be, budget)
    recs = srv.run(specs)
    assert all(r.stats is not None for r in recs.values())
    assert srv.max_bytes_in_use <= budget
    order = [e[1] for e in srv.log if e[0] == "admit"]
    assert order == sorted(order)
    be.close()
