"""Write the oracle reference values used by the GPU parity tests.

    python tests/golden/make_oracle_fixtures.py            (forward, value adjoint)
    python tests/golden/make_oracle_fixtures.py --full     (full adjoint)

Inputs come from the seeded generators in `synth`; expected values come only
from the CPU oracle in `oracle/`.  Nothing here touches the HIP library.
Each fixture holds, per workload, a ragged batch of walkers (the first
walkers of the workload plus copies moved close to a nucleus, inside the
cusp-correction radius, and close to another electron) and the oracle's
ln|psi|, sign, gradient, Laplacian and local energy for them, plus oracle
values for a sample of walkers of the full-size batch.
"""

import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import Oracle  # noqa: E402
from synth import make_config  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))

# (workload, ragged batch size, number of sampled walkers from the full batch)
PLAN = {1: (67, 16), 2: (67, 16), 3: (37, 8), 5: (5, 3), 6: (37, 8), 7: (37, 8)}


def special_walkers(w, base):
    """Copies of walker 0 with an electron inside the cusp radius of a
    nucleus, and with two electrons close together."""
    s = w.system
    out = []
    u = np.array([0.6, -0.48, 0.64])
    for I, t in ((0, 0.05), (s.n_nuc - 1, 0.013)):
        r = base.copy()
        r[0] = s.nuc_xyz[I] + t * u
        out.append(r)
    r = base.copy()
    r[s.n_elec - 1] = s.nuc_xyz[0] + 0.07 * u[::-1]
    out.append(r)
    if s.n_elec > 1:
        r = base.copy()
        r[s.n_elec - 1] = r[0] + 0.01 * u  # opposite spins (0 is up, last is down)
        out.append(r)
    return np.stack(out)


def run(idx):
    B, n_sample = PLAN[idx]
    full = make_config(idx)
    w = make_config(idx, n_walkers=B)
    o = Oracle(w.system, w.net, w.params)
    walkers = np.concatenate([w.walkers, special_walkers(w, w.walkers[0])])
    t0 = time.time()
    out = o.evaluate(walkers)
    rng = np.random.default_rng(77 + idx)
    sample = np.sort(rng.choice(full.walkers.shape[0], n_sample, replace=False))
    out_s = o.evaluate(full.walkers[sample])
    # parameter gradient of sum_w ct_w ln|psi_w| on a few walkers (value-path adjoint)
    nb = min(6, walkers.shape[0])
    ct = np.random.default_rng(500 + idx).standard_normal(nb)
    bwd = o.param_grad_logabs(walkers[:nb], ct).numpy()
    path = os.path.join(HERE, f"oracle_cfg{idx}.npz")
    np.savez_compressed(
        path, walkers=walkers, bwd_ct=ct, bwd_grad=bwd,
        logabs=out["logabs"].numpy(), sign=out["sign"].numpy(), grad=out["grad"].numpy(),
        lap=out["lap"].numpy(), eloc=out["eloc"].numpy(),
        full_sample=sample, full_logabs=out_s["logabs"].numpy(), full_sign=out_s["sign"].numpy(),
        full_grad=out_s["grad"].numpy(), full_lap=out_s["lap"].numpy(), full_eloc=out_s["eloc"].numpy())
    print(f"cfg {idx}: {walkers.shape[0]} + {n_sample} walkers in {time.time() - t0:.1f}s -> {path}")


# full adjoint (cotangents on ln|psi|, grad, lap and E_loc): workload -> walkers
FULL_PLAN = {1: 6, 2: 5, 3: 4, 5: 2}


def run_full(idx):
    """Parameter gradients of sum_w ct . (ln|psi|, grad, lap, E_loc) for four
    cotangent sets: gradient only, Laplacian only, E_loc only, all four."""
    nb = FULL_PLAN[idx]
    w = make_config(idx, n_walkers=67)
    o = Oracle(w.system, w.net, w.params)
    walkers = np.concatenate([w.walkers[:nb - 1], special_walkers(w, w.walkers[0])[:1]])
    B, N = walkers.shape[0], walkers.shape[1]
    rng = np.random.default_rng(900 + idx)
    ca, cg, cl, ce = rng.standard_normal(B), rng.standard_normal((B, N, 3)), rng.standard_normal(B), \
        rng.standard_normal(B)
    t0 = time.time()
    sets = {"grad": (None, cg, None, None), "lap": (None, None, cl, None), "eloc": (None, None, None, ce),
            "all": (ca, cg, cl, ce)}
    res = {k: o.param_grad_full(walkers, *v).numpy() for k, v in sets.items()}
    path = os.path.join(HERE, f"oracle_full_adjoint_cfg{idx}.npz")
    np.savez_compressed(path, walkers=walkers, ct_logabs=ca, ct_grad=cg, ct_lap=cl, ct_eloc=ce,
                        **{"g_" + k: v for k, v in res.items()})
    print(f"cfg {idx} full adjoint: {B} walkers in {time.time() - t0:.1f}s -> {path}")


if __name__ == "__main__":
    args = sys.argv[1:]
    if args and args[0] == "--full":
        for idx in (int(a) for a in args[1:]) if len(args) > 1 else FULL_PLAN:
            run_full(idx)
    else:
        for idx in (int(a) for a in args) if args else PLAN:
            run(idx)
