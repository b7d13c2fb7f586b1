"""Benchmark of the PauliNet walker-evaluation hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload 5] [--prec fp32]

One step = one pn_eval over the whole batch with every output: ln|psi|,
sign, gradient, Laplacian and E_loc per walker, inputs resident in HBM.  The
headline is walker E_loc evaluations per second of the mixed-precision form
(network in FP32, determinants, their derivatives and E_loc in FP64) on the
largest single-GPU workload, the 30-electron diatomic (16384 walkers); the
plain FP64 GPU path is timed on the same batch and the E_loc difference
between the two is reported in hartree beside the batch standard error.

Also reported, each outside the timed region of the headline:
  - per-stage HIP-event times (recorded by the library on the call's stream
    over a separate timed pass), the roofline of the dominant kernel (the
    network tangent pass) and the whole-pass roofline fraction
    t_roof / t_measured with t_roof summed over the pass's units;
  - the other workloads (H2, Ne-like, H10 in BF16 / FP32 / FP64);
  - the VMC step, Langevin sampling, the full adjoint;
  - the serving stream with p50 / p99 step latency;
  - the FP64 CPU oracle on a bounded sample (all host threads and one).
"""

import argparse
import json
import math
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "walker E_loc evals/s (logψ,∇,∇²) vs FP64 path at stated Ha error; p50/p99 step"
PEAKS = {  # MI355X published dense peaks (TFLOP/s) and HBM (GB/s)
    "fp64": 78.6, "fp32": 157.3, "bf16": 2500.0, "hbm": 8000.0,
}


# ------------------------------------------------------------ work counts --
def tangent_flops_per_walker(s, net):
    """Algorithmic flops of the network tangent pass for one walker: the 3N
    first-derivative columns and one Laplacian column (3N + 1 jet columns;
    the value column belongs to the value pass) through the h and g products,
    the pair sums of the messages, and the backflow and Jastrow heads."""
    N, NN, M = s.n_elec, s.n_nuc, s.n_mo
    DX, DZ, L = net.dim_x, net.dim_z, net.n_layers
    C = 3 * N + 1
    R = N * C
    f = (L - 1) * 2 * R * DX * DZ           # h on layers 1..L-1 (layer 0 has no tangents)
    f += L * 3 * 2 * R * DZ * DX            # g, three channels
    f += L * R * DZ * 2 * (N - 1 + NN)      # pair sums of the messages
    f += 2 * R * (2 * DX * DX + DX * M)     # kappa head
    f += 2 * C * (2 * DX * DX + DX)         # eta head
    return f


def network_flops_per_walker(s, net):
    """All network work of one walker on J = 3N + 2 jet columns (value,
    3N tangents, Laplacian): h, g, filters, messages, kappa and eta."""
    N, NN, M = s.n_elec, s.n_nuc, s.n_mo
    DX, DZ, L, K = net.dim_x, net.dim_z, net.n_layers, net.n_feat
    J = 3 * N + 2
    n_pairs = N * (N - 1) // 2 + N * NN
    f = sum(2 * N * (1 if n == 0 else J) * DX * DZ for n in range(L))
    f += 6 * L * N * J * DZ * DX
    f += 6 * L * n_pairs * (K * DZ + DZ * DZ)
    f += L * 2 * N * (N - 1 + NN) * DZ * J
    f += 2 * N * J * (2 * DX * DX + DX * M)
    f += 2 * J * (2 * DX * DX + DX)
    return f


def det_flops_per_walker(s, lowrank):
    """FP64 determinant work of one walker.  Member by member: per
    (determinant, spin) the LU, G T_a for the 3N coordinates and the traces.
    Low-rank: the first determinant's LU, T_a G_0 on its rows and the virtual
    rows, Xi_a = B_a - Theta N_a, S, the traces, and Lambda."""
    N, P = s.n_elec, s.n_det
    ncoord = 3 * N
    tot = 0
    for n, dets in ((s.n_up, s.det_up), (s.n_down, s.det_down)):
        if n == 0:
            continue
        if not lowrank:
            tot += P * (2 * n ** 3 * (ncoord + 1) + 6 * N * n ** 2 + 2 * n ** 3)
        else:
            ref = set(int(x) for x in dets[0])
            nv = len({int(o) for d in dets for o in d if int(o) not in ref})
            per_a = 2 * (n + nv) * n * n + 2 * nv * n * n + 2 * nv * n * n + 2 * n * n
            tot += 2 * n ** 3 + ncoord * per_a + 2 * (n + nv) * n * n
    return tot


# ------------------------------------------------------------- counters ----
TANGENT_SOURCES = ["k_tangent_impl.h", "k_tangent_f32.hip", "k_tangent_f64.hip", "mfma_gemm.h", "gemm_lds.h"]
COUNTERS_FILE = os.path.join(ROOT, "profiles", "k_net_tangent_cfg5_counters.md")


def tangent_source_digest():
    """sha256 over the sources of the tangent kernel (counters taken on
    another build of it do not describe this one)."""
    import hashlib
    h = hashlib.sha256()
    for f in TANGENT_SOURCES:
        with open(os.path.join(ROOT, "paper_1909_08423_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def stored_traffic(prec, T, tile, walkers):
    """HBM bytes per launch of the tangent kernel from the committed counter
    summary, or None when that summary was taken on other kernel sources or
    another launch configuration."""
    try:
        with open(COUNTERS_FILE) as fh:
            text = fh.read()
    except OSError:
        return None
    for line in text.splitlines():
        if line.startswith("traffic-record: "):
            rec = json.loads(line[len("traffic-record: "):])
            if (rec.get("sha256") == tangent_source_digest() and rec.get("prec") == prec
                    and rec.get("chunk_coords") == T and rec.get("tile_walkers") == tile
                    and rec.get("walkers") == walkers):
                return rec["hbm_bytes_per_launch"]
    return None


def copy_probe(mib, torch):
    """A plain device-to-device copy of known size, run so that a counter
    pass over this program also reads the counters for it (the scale factor
    of FETCH_SIZE / WRITE_SIZE against bytes actually moved)."""
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    return {"bytes_read": 4 * n, "bytes_written": 4 * n, "reps": 3}


# --------------------------------------------------------------- timing ----
def time_path(ctx, r, th, prec, steps, warmup, torch):
    """K timed pn_eval calls over the batch (all outputs), bracketed by
    device synchronisation; per-call HIP events on the call's stream give the
    median.  Returns (elapsed s, per-call ms list, outputs)."""
    out = ctx.eval(r, th, prec)
    ws = ctx.workspace(r.shape[0], prec, r.device)
    for _ in range(warmup):
        ctx.eval(r, th, prec, out=out, ws=ws)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for a, b in ev:
        a.record()
        ctx.eval(r, th, prec, out=out, ws=ws)
        b.record()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return dt, [a.elapsed_time(b) for a, b in ev], out


def stage_pass(ctx, r, th, prec, steps, torch):
    """Per-stage kernel times from the library's HIP events on the call's
    stream, over `steps` further calls (outside the headline's timed region)."""
    out = ctx.eval(r, th, prec)
    ws = ctx.workspace(r.shape[0], prec, r.device)
    torch.cuda.synchronize()
    ctx.stage_timing(True)
    for _ in range(steps):
        ctx.eval(r, th, prec, out=out, ws=ws)
    torch.cuda.synchronize()
    st = ctx.stage_times()
    ctx.stage_timing(False)
    return st


def clipped_mean(e, q=5.0):
    """Batch mean of E_loc clipped as the VMC update clips it (Methods,
    "Ansatz optimization"): logarithmic growth outside q mean absolute
    deviations from the median."""
    e = np.asarray(e, dtype=np.float64)
    m = np.median(e)
    w = q * np.mean(np.abs(e - m))
    dev = np.abs(e - m)
    if w == 0:
        return float(e.mean())
    ec = np.where(dev <= w, e, m + np.sign(e - m) * w * (1.0 + np.log(np.maximum(dev, w) / w)))
    return float(ec.mean())


def error_stats(e_mix, e_64):
    de = np.abs(e_mix - e_64)
    B = e_64.shape[0]
    return {
        "mean_eloc_fp64": float(e_64.mean()),
        "abs_dmean_eloc_Ha": float(abs(e_mix.mean() - e_64.mean())),
        "abs_dclipped_mean_Ha": float(abs(clipped_mean(e_mix) - clipped_mean(e_64))),
        "stderr_eloc_Ha": float(e_64.std() / math.sqrt(B)),
        "p50_abs_deloc_Ha": float(np.percentile(de, 50)),
        "p99_abs_deloc_Ha": float(np.percentile(de, 99)),
        "max_abs_deloc_Ha": float(de.max()),
    }


def output_error_stats(o_mix, o_64):
    """Per output p50 / p99 / max of the parity ratios of the mixed form
    against the FP64 GPU path (the ratios of the FP64 parity criterion)."""
    la, rla = o_mix["logabs"], o_64["logabs"]
    g, rg = o_mix["grad"].reshape(la.shape[0], -1), o_64["grad"].reshape(la.shape[0], -1)
    gn = np.linalg.norm(rg, axis=1)
    kin = np.abs(o_64["lap"]) + gn ** 2
    rat = {
        "logabs": np.abs(la - rla) / np.maximum(1, np.abs(rla)),
        "grad": np.linalg.norm(g - rg, axis=1) / np.maximum(1, gn),
        "lap": np.abs(o_mix["lap"] - o_64["lap"]) / np.maximum(1, kin),
        "eloc": np.abs(o_mix["eloc"] - o_64["eloc"]) / np.maximum(1, kin + np.abs(o_64["eloc"])),
    }
    return {k: [float(np.percentile(v, 50)), float(np.percentile(v, 99)), float(v.max())] for k, v in rat.items()}


def other_workloads(pn, torch, steps=3, warmup=1):
    """The other synthetic systems at their full batch sizes: H2 (launch
    bound: microseconds per batch), the Ne-like atom in FP32 / FP64 and H10
    in BF16 / FP32 / FP64; walker E_loc evaluations per second and the E_loc
    difference to the FP64 path."""
    from synth import make_config
    P = pn._lib.PRECISIONS
    plan = {1: ["fp64"], 2: ["fp32", "fp64"], 3: ["bf16", "fp32", "fp64"]}
    out = {}
    for idx, precs in plan.items():
        w = make_config(idx)
        ctx = pn.PauliNetContext(w.system, w.net)
        r = torch.tensor(w.walkers, dtype=torch.float64, device="cuda")
        th = torch.tensor(w.params, dtype=torch.float64, device="cuda")
        B = w.walkers.shape[0]
        rec = {"walkers": B}
        o64 = None
        for prec in reversed(precs):  # FP64 first, as the reference of the others
            dt, ms, o = time_path(ctx, r, th, P[prec], steps, warmup, torch)
            o = {k: v.double().cpu().numpy().copy() for k, v in o.items()}
            if prec == "fp64":
                o64 = o
            ent = {"walker_evals_per_s": B * steps / dt, "us_per_batch": float(np.median(ms)) * 1e3}
            if prec != "fp64" and o64 is not None:
                ent["eloc_error_vs_fp64"] = error_stats(o["eloc"], o64["eloc"])
                ent["output_ratios_p50_p99_max"] = output_error_stats(o, o64)
            rec[prec] = ent
        if "bf16" in rec and "fp32" in rec:
            rec["bf16"]["speedup_over_fp32"] = rec["bf16"]["walker_evals_per_s"] / rec["fp32"]["walker_evals_per_s"]
        ctx.close()
        out[w.name] = rec
    return out


def cpu_info():
    model = platform.processor() or "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, os.cpu_count()


def cpu_baseline(workload_idx, budget_s=15.0, chunk=2, single_s=8.0):
    """The FP64 CPU oracle (PyTorch CPU autograd, as written for checking, not
    tuned) on the first walkers of the same workload: chunks of `chunk`
    walkers until `budget_s` elapse with all host threads, then a shorter run
    on one thread."""
    import torch
    from oracle import Oracle
    from synth import make_config
    w = make_config(workload_idx)
    o = Oracle(w.system, w.net, w.params)
    threads = torch.get_num_threads()

    def run(budget):
        n, t0 = 0, time.perf_counter()
        while True:
            o.evaluate(w.walkers[n:n + chunk])
            n += chunk
            if time.perf_counter() - t0 > budget or n >= w.walkers.shape[0]:
                break
        return n, time.perf_counter() - t0

    n, dt = run(budget_s)
    torch.set_num_threads(1)
    try:
        n1, dt1 = run(single_s)
    finally:
        torch.set_num_threads(threads)
    model, ncpu = cpu_info()
    return {"value": n / dt, "unit": "walker-evals/s", "cores": threads, "kind": "oracle",
            "sample": f"first {n} walkers of the same workload, {chunk} per call, {dt:.1f} s",
            "cpu_model": model, "host_cpus": ncpu,
            "single_core": {"value": n1 / dt1, "sample": f"first {n1} walkers, one thread, {dt1:.1f} s"}}


def time_vmc_step(pn, ctx, w, prec, steps, warmup, torch):
    """Full VMC step of one job (Metropolis + E_loc + clipping + gradient +
    AdamW) on the benchmark batch."""
    st = {
        "r": torch.tensor(w.walkers, dtype=torch.float64, device="cuda"),
        "params": torch.tensor(w.params, dtype=torch.float64, device="cuda"),
        "adam_m": torch.zeros(w.params.shape[0], dtype=torch.float64, device="cuda"),
        "adam_v": torch.zeros(w.params.shape[0], dtype=torch.float64, device="cuda"),
        "eloc": torch.empty(w.walkers.shape[0], dtype=torch.float64, device="cuda"),
        "stats": torch.zeros(8, dtype=torch.float64, device="cuda"),
        "ws": torch.empty(pn.vmc_workspace_bytes(ctx, w.walkers.shape[0], prec), dtype=torch.uint8, device="cuda"),
        "seed": 1234, "step": 0,
    }
    for _ in range(warmup):
        pn.vmc_step(ctx, st, prec)
        st["step"] += 1
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        pn.vmc_step(ctx, st, prec)
        st["step"] += 1
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return {"walker_steps_per_s": w.walkers.shape[0] * steps / dt, "ms_per_step": dt / steps * 1e3,
            "steps": steps, "last_stats": st["stats"].cpu().numpy().tolist()}


def time_backward(ctx, r, th, prec, steps, warmup, torch, full):
    """Parameter adjoint over the benchmark batch: the value-path adjoint
    (cotangent on ln|psi|, what the Hermitian estimator needs) or the full
    adjoint (cotangent on E_loc: determinant and tangent-pass adjoints too).
    Each call recomputes the forward pass."""
    B = r.shape[0]
    ct = torch.ones(B, dtype=torch.float64, device="cuda") / B
    ws = ctx.workspace(B, prec, r.device, full=full)
    g = torch.zeros(ctx.param_count, dtype=torch.float64, device="cuda")
    kw = {"ct_eloc": ct} if full else {}
    first = None if full else ct
    for _ in range(warmup):
        ctx.eval_backward(r, th, first, prec, grad_params=g, ws=ws, **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.eval_backward(r, th, first, prec, grad_params=g, ws=ws, **kw)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return {"walkers_per_s": B * steps / dt, "ms_per_call": dt / steps * 1e3, "steps": steps,
            "workspace_GiB": ws.numel() / 2**30}


def time_langevin(pn, ctx, w, prec, steps, torch):
    """Langevin sampling (drift-diffusion + Metropolis-Hastings, adaptive
    step) on the benchmark batch: walker-steps per second."""
    r = torch.tensor(w.walkers, dtype=torch.float64, device="cuda")
    th = torch.tensor(w.params, dtype=torch.float64, device="cuda")
    tau = torch.tensor([0.05], dtype=torch.float64, device="cuda")
    pn.langevin_run(ctx, r, th, prec, tau, 2, seed=11, step0=0)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = pn.langevin_run(ctx, r, th, prec, tau, steps, seed=11, step0=2)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    st = st.cpu().numpy()
    return {"walker_steps_per_s": r.shape[0] * steps / dt, "ms_per_step": dt / steps * 1e3, "steps": steps,
            "last_acceptance": float(st[-1, 0]), "last_tau": float(st[-1, 1])}


def time_line_scan(pn, torch, idx=3, n_points=1001, reps=20):
    """Latency of a one-dimensional scan (electron 0 moved along the
    molecular axis with the other electrons fixed, every output at every
    point, FP64): median over `reps` scans, walker batch built on the device."""
    from paper_1909_08423_amd.scan import line_scan
    from synth import make_config
    w = make_config(idx, n_walkers=4)
    ctx = pn.PauliNetContext(w.system, w.net)
    th = torch.tensor(w.params, dtype=torch.float64, device="cuda")
    z = w.system.nuc_xyz[:, 2]
    a, b = [0.013, -0.011, float(z.min()) - 2.0], [0.013, -0.011, float(z.max()) + 2.0]
    ws = ctx.workspace(n_points, pn.PN_PREC_FP64, torch.device("cuda"))
    line_scan(ctx, th, w.walkers[0], 0, a, b, n_points, ws=ws)
    ms = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        line_scan(ctx, th, w.walkers[0], 0, a, b, n_points, ws=ws)
        e1.record()
        torch.cuda.synchronize()
        ms.append(e0.elapsed_time(e1))
    ctx.close()
    return {"workload": w.name, "points": n_points, "median_ms_per_scan": float(np.median(ms)),
            "p99_ms_per_scan": float(np.percentile(ms, 99)), "reps": reps}


def run_serving(pn, prec, n_jobs, n_steps, torch, mean_gap_s=0.25, budget_gib=64):
    """The serving stream (H-chains and atoms, 2-18 electrons, 1-32
    determinants, 1024-8192 walkers, Poisson arrivals): n_jobs jobs of
    n_steps steps, mean inter-arrival mean_gap_s, device-memory budget
    budget_gib for admission."""
    from paper_1909_08423_amd.serve import GpuBackend, JobSpec, Server, summarize
    from synth import make_serving_jobs
    jobs = make_serving_jobs(n_jobs=n_jobs, n_steps=n_steps, mean_gap_s=mean_gap_s)
    specs = [JobSpec(j.job_id, j.arrival_s, j.n_steps, j.workload.system, j.workload.net, j.workload.params,
                     j.workload.walkers, seed=1000 + j.job_id) for j in jobs]
    be = GpuBackend(prec=prec)
    srv = Server(be, mem_budget_bytes=int(budget_gib * 2**30), max_active=16)
    t0 = time.perf_counter()
    recs = srv.run(specs)
    torch.cuda.synchronize()
    out = summarize(recs, time.perf_counter() - t0)
    out.update({"jobs": n_jobs, "steps_per_job": n_steps, "max_concurrency": srv.max_concurrency,
                "mean_gap_s": mean_gap_s, "mem_budget_GiB": budget_gib,
                "max_bytes_in_use_GiB": srv.max_bytes_in_use / 2**30})
    be.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--fp64-steps", type=int, default=5, help="timed calls of the FP64 comparison path")
    ap.add_argument("--bf16-steps", type=int, default=5, help="timed calls of the BF16 form (0: skip)")
    ap.add_argument("--stage-steps", type=int, default=3, help="calls of the per-stage timing pass")
    ap.add_argument("--workload", type=int, default=5)
    ap.add_argument("--prec", default="fp32", choices=["fp32", "bf16", "fp64"])
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--serve-jobs", type=int, default=64)
    ap.add_argument("--serve-steps", type=int, default=100)
    ap.add_argument("--serve-gap", type=float, default=0.25, help="mean inter-arrival time (s)")
    ap.add_argument("--serve-budget-gib", type=float, default=64.0)
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-backward", action="store_true")
    ap.add_argument("--no-other", action="store_true", help="skip the other workloads")
    ap.add_argument("--only-headline", action="store_true",
                    help="the headline, the FP64 path and the stage pass only (profiling runs)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="first run a plain device copy of MIB MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU (asked for {args.gpus}): the walker batch shards "
              "trivially across GPUs, but this build measures the single-GPU path only.", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1909_08423_amd as pn
    from synth import make_config

    if not torch.cuda.is_available():
        print("no ROCm device", file=sys.stderr)
        sys.exit(1)
    pn.load_library()
    probe = copy_probe(args.copy_probe, torch) if args.copy_probe > 0 else None
    w = make_config(args.workload)
    s, net = w.system, w.net
    B = w.walkers.shape[0]
    ctx = pn.PauliNetContext(s, net)
    r = torch.tensor(w.walkers, dtype=torch.float64, device="cuda")
    th = torch.tensor(w.params, dtype=torch.float64, device="cuda")
    P = pn._lib.PRECISIONS
    pmix, p64 = P[args.prec], P["fp64"]

    # ---- headline: K timed calls of the mixed form, then the FP64 path ----
    dt_mix, ms_mix, out_mix = time_path(ctx, r, th, pmix, args.steps, args.warmup, torch)
    o_mix = {k: v.double().cpu().numpy().copy() for k, v in out_mix.items()}
    dt_64, ms_64, out_64 = time_path(ctx, r, th, p64, args.fp64_steps, 1, torch)
    o_64 = {k: v.double().cpu().numpy().copy() for k, v in out_64.items()}
    value = B * args.steps / dt_mix
    plan_mix, plan_64 = ctx.plan(B, pmix), ctx.plan(B, p64)
    # the BF16 form (BF16 operands in the tangent products) on the same batch
    alt = None
    if args.prec == "fp32" and args.bf16_steps > 0:
        dt_b, ms_b, out_b = time_path(ctx, r, th, P["bf16"], args.bf16_steps, 1, torch)
        o_b = {k: v.double().cpu().numpy().copy() for k, v in out_b.items()}
        alt = {"value": B * args.bf16_steps / dt_b, "median_ms_per_step": float(np.median(ms_b)),
               "speedup_over_fp32": (B * args.bf16_steps / dt_b) / value,
               "eloc_error_vs_fp64": error_stats(o_b["eloc"], o_64["eloc"]),
               "output_ratios_vs_fp64_p50_p99_max": output_error_stats(o_b, o_64)}
        del out_b

    # ---- per-stage times (separate pass) and rooflines ----
    st_mix = stage_pass(ctx, r, th, pmix, args.stage_steps, torch)
    st_64 = stage_pass(ctx, r, th, p64, max(1, args.stage_steps - 1), torch)
    per_step = lambda st, n: {k: v[0] / n for k, v in st.items() if v[1] > 0}  # noqa: E731
    stages_mix = per_step(st_mix, args.stage_steps)
    stages_64 = per_step(st_64, max(1, args.stage_steps - 1))
    tan_ms_launch = st_mix["net_tangent"][0] / st_mix["net_tangent"][1]
    tan_launches = st_mix["net_tangent"][1] // args.stage_steps
    tan_fl = tangent_flops_per_walker(s, net)
    peak_net = PEAKS["fp64" if args.prec == "fp64" else ("bf16" if args.prec == "bf16" else "fp32")]
    walkers_per_launch = B / tan_launches
    ach = tan_fl * walkers_per_launch / (tan_ms_launch * 1e-3) / 1e12
    roof = {"kernel": "k_net_tangent", "bound": "mfma", "achieved": ach, "peak": peak_net, "unit": "TFLOP/s",
            "frac": ach / peak_net,
            "traffic": stored_traffic(args.prec, plan_mix["chunk_coords"], plan_mix["tile_walkers"], B),
            "flops_per_walker": tan_fl, "jet_columns": 3 * s.n_elec + 1, "walkers_per_launch": walkers_per_launch,
            "avg_launch_ms": tan_ms_launch, "launches_per_step": tan_launches,
            "chunk_coords": plan_mix["chunk_coords"]}
    net_fl = network_flops_per_walker(s, net)
    det_fl = det_flops_per_walker(s, plan_mix["lowrank"])
    t_roof_ms = B * (net_fl / (peak_net * 1e12) + det_fl / (PEAKS["fp64"] * 1e12)) * 1e3
    t_meas_ms = float(np.median(ms_mix))
    pass_roof = {"t_roof_ms": t_roof_ms, "t_measured_ms": t_meas_ms, "frac": t_roof_ms / t_meas_ms,
                 "network_flops_per_walker": net_fl, "network_peak_TFLOPs": peak_net,
                 "det_flops_per_walker_fp64": det_fl, "det_path": "low-rank" if plan_mix["lowrank"] else "direct",
                 "det_flops_per_walker_direct": det_flops_per_walker(s, False)}

    model, ncpu = cpu_info()
    res = {
        "metric": METRIC,
        "value": value,
        "unit": "walker-evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt_mix / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32": "f32 net + f64 det", "bf16": "bf16 net + f64 det", "fp64": "f64"}[args.prec],
        "data": "synthetic",
        "config": {"workload": f"{w.name}: two Z={int(s.charge[0])} nuclei at (0,0,+-2.0) bohr, "
                               f"{s.n_up}+{s.n_down} electrons, {s.n_det} determinants, 10 s + 8 p GTOs per atom, "
                               f"width {net.dim_x}, {net.n_layers} layers, {net.n_feat} features"
                   if args.workload == 5 else f"{w.name} (N={s.n_elec}, {s.n_det} determinants)",
                   "walkers": B, "precision": args.prec},
        "median_ms_per_step": t_meas_ms,
        "walker_evals_per_s_median": B / (t_meas_ms * 1e-3),
        "plan": plan_mix,
        "fp64_path": {"value": B * args.fp64_steps / dt_64, "ms_per_step": dt_64 / args.fp64_steps * 1e3,
                      "median_ms_per_step": float(np.median(ms_64)), "steps": args.fp64_steps, "plan": plan_64},
        "speedup_vs_fp64": (B * args.steps / dt_mix) / (B * args.fp64_steps / dt_64),
        "eloc_error_vs_fp64": error_stats(o_mix["eloc"], o_64["eloc"]),
        "output_ratios_vs_fp64_p50_p99_max": output_error_stats(o_mix, o_64),
        "bf16_form": alt,
        "stages_ms_per_step": stages_mix,
        "stages_ms_per_step_fp64": stages_64,
        "roofline": roof,
        "pass_roofline": pass_roof,
        "host": {"cpu_model": model, "cpus": ncpu},
    }
    if probe is not None:
        res["copy_probe"] = probe
    print(json.dumps({"progress": "headline done", "value": value}), file=sys.stderr, flush=True)
    if args.only_headline:
        print(json.dumps(res), flush=True)
        return
    res["vmc_step"] = time_vmc_step(pn, ctx, w, pmix, 3, 1, torch)
    if not args.no_backward:
        res["value_adjoint"] = {args.prec: time_backward(ctx, r, th, pmix, 3, 1, torch, False)}
        res["full_adjoint_eloc"] = {args.prec: time_backward(ctx, r, th, pmix, 2, 1, torch, True)}
    res["langevin"] = time_langevin(pn, ctx, w, pmix, 5, torch)
    ctx.close()
    del r, th, out_mix, out_64
    torch.cuda.empty_cache()
    if not args.no_other:
        res["other_workloads"] = other_workloads(pn, torch)
        res["line_scan"] = time_line_scan(pn, torch)
    print(json.dumps({"progress": "side measurements done"}), file=sys.stderr, flush=True)
    if not args.no_serve:
        res["serving"] = run_serving(pn, pmix, args.serve_jobs, args.serve_steps, torch, args.serve_gap,
                                     args.serve_budget_gib)
    if not args.no_cpu:
        res["cpu_baseline"] = cpu_baseline(args.workload, args.cpu_seconds)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
