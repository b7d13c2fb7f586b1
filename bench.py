"""Benchmark of the PauliNet walker-evaluation hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload 2] [--prec fp32]

One step = one pn_eval over the whole batch: ln|psi|, sign, gradient,
Laplacian and E_loc for every walker (inputs resident in HBM).  The headline
value is walker E_loc evaluations per second of the mixed-precision form
(network in FP32, determinants and E_loc in FP64) on the Ne-like workload
(B = 4096); the plain FP64 GPU path is timed beside it on the same batch and
the E_loc difference between the two is reported in hartree.

Also reported: the roofline of the dominant kernel (per-stage HIP events
recorded by the library on the call's stream during the timed region), and
the FP64 CPU oracle timed on a bounded sample of the same workload.
"""

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAKS = {  # MI355X published dense peaks (TFLOP/s) and HBM (GB/s)
    "fp64": 78.6, "fp32": 157.3, "bf16": 2500.0, "hbm": 8000.0,
}


def tangent_flops_per_walker(s, net, T):
    """Algorithmic flops of the network tangent pass for one walker with
    coordinate chunks of T (each chunk carries T first-derivative columns
    and one partial-Laplacian column)."""
    N, NN, M = s.n_elec, s.n_nuc, s.n_mo
    DX, DZ, L = net.dim_x, net.dim_z, net.n_layers
    total = 0
    for a0 in range(0, 3 * N, T):
        C = min(T, 3 * N - a0) + 1
        R = N * C
        f = (L - 1) * 2 * R * DX * DZ           # h on layers 1..L-1 (layer 0 has no tangents)
        f += L * 3 * 2 * R * DZ * DX            # g, three channels
        f += L * R * DZ * 2 * (N - 1 + NN)      # pair sums of the messages
        f += 2 * R * (2 * DX * DX + DX * M)     # kappa head
        f += 2 * C * (2 * DX * DX + DX)         # eta head
        total += f
    return total


def chunk_T(s, net, prec):
    """Same chunk choice as the library's planner (LDS budget per block)."""
    N, DX, DZ, NN = s.n_elec, net.dim_x, net.dim_z, s.n_nuc
    n_ee = N * (N - 1) // 2
    tn = 8 if prec == "fp64" else 4
    pad = 16 // tn
    LDX, LDZ = DX + pad, DZ + pad
    LDHZ = max(2 * LDZ, LDX)

    def lds(T, stage):
        C = T + 1
        R = N * C
        NCE = min(N, T // 3 + 2)
        e = N * DZ + R * (LDX + LDHZ) + max(2 * C * LDX, NCE * C * LDZ) + NCE * (N + NN) * 4
        if stage:
            e += n_ee * DZ + 2 * NCE * (N + NN) * DZ
        return 3 * 64 * 8 + ((N * N + 3) & ~3) * 4 + e * tn

    def pick(budget):
        for nc in range(1, 3 * N + 1):
            T = -(-3 * N // nc)
            if T not in (1, 2, 3, 4, 5, 6, 8, 9, 10, 12, 15):
                continue
            for stage in (True, False):
                if lds(T, stage) <= budget or (not stage and T == 1):
                    return T
        return 1

    T = pick(80 * 1024)
    if T < 3:
        T2 = pick(160 * 1024)
        if T2 >= 2 * T:
            T = T2
    return T


TANGENT_SOURCES = ["k_tangent_impl.h", "k_tangent_f32.hip", "k_tangent_f64.hip", "mfma_gemm.h", "gemm_lds.h"]
COUNTERS_FILE = os.path.join(ROOT, "profiles", "k_net_tangent_ne4096_counters.md")


def tangent_source_digest():
    """sha256 over the sources of the tangent kernel (counters taken on
    another build of it do not describe this one)."""
    import hashlib
    h = hashlib.sha256()
    for f in TANGENT_SOURCES:
        with open(os.path.join(ROOT, "paper_1909_08423_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def stored_traffic(prec, T, B):
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
                    and rec.get("chunk_coords") == T and rec.get("walkers") == B):
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


def time_path(ctx, r, th, prec, steps, warmup, torch):
    out = ctx.eval(r, th, prec)
    ws = ctx.workspace(r.shape[0], prec, r.device)
    for _ in range(warmup):
        ctx.eval(r, th, prec, out=out, ws=ws)
    torch.cuda.synchronize()
    ctx.stage_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.eval(r, th, prec, out=out, ws=ws)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    stages = ctx.stage_times()
    ctx.stage_timing(False)
    return dt, out, stages


def other_workloads(pn, torch, steps=3, warmup=1):
    """The other synthetic systems at their full batch sizes: H2 (launch
    bound: microseconds per batch), H10 in BF16 / FP32 / FP64 and the
    30-electron diatomic in FP32 / FP64; walker E_loc evaluations per
    second and the mean E_loc difference to the FP64 path."""
    from synth import make_config
    P = pn._lib.PRECISIONS
    plan = {1: ["fp64"], 3: ["bf16", "fp32", "fp64"], 5: ["fp32", "fp64"]}
    out = {}
    for idx, precs in plan.items():
        w = make_config(idx)
        ctx = pn.PauliNetContext(w.system, w.net)
        r = torch.tensor(w.walkers, dtype=torch.float64, device="cuda")
        th = torch.tensor(w.params, dtype=torch.float64, device="cuda")
        B = w.walkers.shape[0]
        rec = {"walkers": B}
        e64 = None
        for prec in reversed(precs):  # FP64 first, as the reference of the others
            dt, o, _ = time_path(ctx, r, th, P[prec], steps, warmup, torch)
            e = o["eloc"].double().cpu().numpy().copy()
            if prec == "fp64":
                e64 = e
            ent = {"walker_evals_per_s": B * steps / dt, "us_per_batch": dt / steps * 1e6}
            if prec != "fp64" and e64 is not None:
                de = np.abs(e - e64)
                ent["abs_dmean_eloc_Ha"] = float(abs(e.mean() - e64.mean()))
                ent["p99_abs_deloc_Ha"] = float(np.percentile(de, 99))
            rec[prec] = ent
        ctx.close()
        out[w.name] = rec
    return out


def cpu_baseline(workload_idx, budget_s=15.0, chunk=8):
    import torch
    from oracle import Oracle
    from synth import make_config
    w = make_config(workload_idx)
    o = Oracle(w.system, w.net, w.params)
    n, t0 = 0, time.perf_counter()
    while True:
        o.evaluate(w.walkers[n:n + chunk])
        n += chunk
        if time.perf_counter() - t0 > budget_s or n >= w.walkers.shape[0]:
            break
    dt = time.perf_counter() - t0
    return {"value": n / dt, "unit": "walker-evals/s", "cores": torch.get_num_threads(), "kind": "oracle",
            "sample": f"first {n} walkers of the same workload, {chunk} per call, {dt:.1f} s"}


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


def time_full_adjoint(ctx, r, th, prec, steps, warmup, torch):
    """Full parameter adjoint (cotangent on E_loc: the forward recomputation,
    the determinant and tangent-pass adjoints and the value-path adjoint)
    over the benchmark batch."""
    B = r.shape[0]
    ce = torch.ones(B, dtype=torch.float64, device="cuda") / B
    ws = ctx.workspace(B, prec, r.device, full=True)
    g = torch.zeros(ctx.param_count, dtype=torch.float64, device="cuda")
    for _ in range(warmup):
        ctx.eval_backward(r, th, None, prec, grad_params=g, ws=ws, ct_eloc=ce)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.eval_backward(r, th, None, prec, grad_params=g, ws=ws, ct_eloc=ce)
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


def run_serving(pn, prec, n_jobs, n_steps, torch, mean_gap_s=0.05, budget_gib=64):
    """The serving stream (H-chains and atoms, 2-18 electrons, 1-32
    determinants, 1024-8192 walkers, Poisson arrivals): n_jobs jobs of
    n_steps steps, mean inter-arrival mean_gap_s, device-memory budget
    budget_gib for admission."""
    from paper_1909_08423_amd.serve import GpuBackend, JobSpec, Server, summarize
    from synth import make_serving_jobs
    jobs = make_serving_jobs(n_jobs=n_jobs, n_steps=n_steps, mean_gap_s=mean_gap_s)
    specs = [JobSpec(j.job_id, j.arrival_s, j.n_steps, j.workload.system, j.workload.net, j.workload.params,
                     j.workload.walkers, seed=1000 + j.job_id) for j in jobs]
    be = GpuBackend(prec=prec, n_streams=8)
    srv = Server(be, mem_budget_bytes=int(budget_gib * 2**30), max_active=16)
    t0 = time.perf_counter()
    recs = srv.run(specs)
    torch.cuda.synchronize()
    out = summarize(recs, time.perf_counter() - t0)
    out.update({"jobs": n_jobs, "steps_per_job": n_steps, "max_concurrency": srv.max_concurrency,
                "mean_gap_s": mean_gap_s, "mem_budget_GiB": budget_gib,
                "max_bytes_in_use_GiB": srv.max_bytes_in_use / 2**30, "electrons": [int(s.walkers.shape[1]) for s in specs],
                "walkers": [int(s.walkers.shape[0]) for s in specs]})
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", type=int, default=2)
    ap.add_argument("--prec", default="fp32", choices=["fp32", "bf16", "fp64"])
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--serve-jobs", type=int, default=12)
    ap.add_argument("--serve-steps", type=int, default=10)
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--serve-gap", type=float, default=0.05, help="mean inter-arrival time (s)")
    ap.add_argument("--serve-budget-gib", type=float, default=64.0)
    ap.add_argument("--no-full-adjoint", action="store_true")
    ap.add_argument("--no-other", action="store_true", help="skip the other workloads")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="first run a plain device copy of MIB MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU (asked for {args.gpus}): the walker batch shards "
              "trivially across GPUs but this build measures the single-GPU path only.", file=sys.stderr)
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

    dt_mix, out_mix, st_mix = time_path(ctx, r, th, P[args.prec], args.steps, args.warmup, torch)
    e_mix = out_mix["eloc"].double().cpu().numpy().copy()
    dt_64, out_64, st_64 = time_path(ctx, r, th, P["fp64"], args.steps, args.warmup, torch)
    e_64 = out_64["eloc"].double().cpu().numpy().copy()

    ms_step = dt_mix / args.steps * 1e3
    value = B * args.steps / dt_mix
    de = np.abs(e_mix - e_64)
    err = {
        "mean_eloc_fp64": float(e_64.mean()),
        "abs_dmean_eloc_Ha": float(abs(e_mix.mean() - e_64.mean())),
        "stderr_eloc_Ha": float(e_64.std() / math.sqrt(B)),
        "p50_abs_deloc_Ha": float(np.percentile(de, 50)),
        "p99_abs_deloc_Ha": float(np.percentile(de, 99)),
        "max_abs_deloc_Ha": float(de.max()),
    }

    # roofline of the dominant kernel of the headline path
    stages = {k: v for k, v in st_mix.items() if v[1] > 0}
    dom = max(stages, key=lambda k: stages[k][0])
    avg_ms = stages[dom][0] / stages[dom][1]
    roof = None
    if dom == "net_tangent":
        T = chunk_T(s, net, args.prec)
        fl = tangent_flops_per_walker(s, net, T) * B
        peak = PEAKS["fp64" if args.prec == "fp64" else ("bf16" if args.prec == "bf16" else "fp32")]
        ach = fl / (avg_ms * 1e-3) / 1e12
        roof = {"kernel": "k_net_tangent", "bound": "alu" if args.prec != "bf16" else "mfma",
                "achieved": ach, "peak": peak, "unit": "TFLOP/s", "frac": ach / peak,
                "traffic": stored_traffic(args.prec, T, B),
                "flops_per_walker": fl / B, "avg_launch_ms": avg_ms, "chunk_coords": T}
    else:
        roof = {"kernel": dom, "bound": "unknown", "achieved": None, "peak": None, "unit": None, "frac": None,
                "traffic": None, "avg_launch_ms": avg_ms}

    res = {
        "metric": "walker E_loc evals/s (ln psi, grad, lap, E_loc)",
        "value": value,
        "unit": "walker-evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32": "f32 net + f64 det", "bf16": "bf16 net + f64 det", "fp64": "f64"}[args.prec],
        "data": "synthetic",
        "config": {"workload": f"{w.name} (N={s.n_elec}, {s.n_det} determinants, width {net.dim_x}, "
                               f"{net.n_layers} layers, {net.n_feat} features)", "walkers": B,
                   "precision": args.prec},
        "fp64_path": {"value": B * args.steps / dt_64, "ms_per_step": dt_64 / args.steps * 1e3},
        "speedup_vs_fp64": (B * args.steps / dt_mix) / (B * args.steps / dt_64),
        "eloc_error_vs_fp64": err,
        "stages_ms_per_step": {k: v[0] / max(v[1], 1) for k, v in st_mix.items() if v[1] > 0},
        "stages_ms_per_step_fp64": {k: v[0] / max(v[1], 1) for k, v in st_64.items() if v[1] > 0},
        "roofline": roof,
    }
    if probe is not None:
        res["copy_probe"] = probe
    res["vmc_step"] = time_vmc_step(pn, ctx, w, P[args.prec], max(3, args.steps // 4), 1, torch)
    if not args.no_other:
        res["other_workloads"] = other_workloads(pn, torch)
    res["langevin"] = time_langevin(pn, ctx, w, P[args.prec], max(5, args.steps // 2), torch)
    if not args.no_full_adjoint:
        res["full_adjoint_eloc"] = {
            args.prec: time_full_adjoint(ctx, r, th, P[args.prec], max(3, args.steps // 4), 1, torch),
            "fp64": time_full_adjoint(ctx, r, th, P["fp64"], max(3, args.steps // 4), 1, torch)}
    if not args.no_serve:
        res["serving"] = run_serving(pn, P[args.prec], args.serve_jobs, args.serve_steps, torch, args.serve_gap,
                                     args.serve_budget_gib)
    if not args.no_cpu:
        res["cpu_baseline"] = cpu_baseline(args.workload, args.cpu_seconds)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
