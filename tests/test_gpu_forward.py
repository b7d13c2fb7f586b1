"""GPU parity of the forward path (ln|psi|, sign, grad, Laplacian, E_loc)
against the FP64 oracle, through the C ABI.

Oracle values are stored fixtures written by tests/golden/make_oracle_fixtures.py
(which calls only oracle/).  FP64 bar: per walker
  |d ln|psi|| <= 1e-6 max(1, |ln|psi||),  ||d grad|| <= 1e-6 max(1, ||grad||),
  |d lap| and |d E_loc| <= 1e-6 x the scale of the cancelling kinetic terms,
  signs equal.
"""

import numpy as np
import pytest
import torch

from gpu_util import announce, load_fixture, parity_ratios, summarize
from synth import make_config

pytestmark = pytest.mark.gpu

TOL64 = 1e-6


@pytest.fixture(scope="module")
def pn():
    import paper_1909_08423_amd as pn
    assert torch.cuda.is_available(), "no ROCm device"
    pn.load_library()
    return pn


def _run(pn, w, walkers, prec, derivs=True):
    ctx = pn.PauliNetContext(w.system, w.net)
    r = torch.tensor(walkers, dtype=torch.float64, device="cuda")
    th = torch.tensor(w.params, dtype=torch.float64, device="cuda")
    out = ctx.eval(r, th, prec, want_derivs=derivs)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}, ctx


@pytest.mark.parametrize("idx", [1, 2, 3, 5, 6, 7])
def test_fp64_parity_ragged_batch(pn, idx):
    try:
        fx = load_fixture(idx)
    except FileNotFoundError:
        pytest.skip(f"no oracle fixture for workload {idx}")
    w = make_config(idx, n_walkers=4)
    announce(f"fp64 parity workload {idx} B={fx['walkers'].shape[0]}")
    out, _ = _run(pn, w, fx["walkers"], pn.PN_PREC_FP64)
    np.testing.assert_array_equal(out["sign"], fx["sign"])
    rat = parity_ratios(out, fx)
    for k, v in rat.items():
        assert v.max() <= TOL64, f"{k}: worst {v.max():.3e} at walker {int(v.argmax())}; {summarize(rat)}"


@pytest.mark.parametrize("idx", [1, 2, 3, 5, 6, 7])
def test_fp64_parity_full_batch_sample(pn, idx):
    """Full-size batch in the benchmark's launch configuration; the oracle
    values of a sample of walkers are compared one by one.  The 30-electron
    batch (16384 walkers) is processed in several walker tiles, the sample
    reaching into the last one."""
    fx = load_fixture(idx)
    w = make_config(idx)
    announce(f"fp64 full batch workload {idx} B={w.walkers.shape[0]}")
    out, _ = _run(pn, w, w.walkers, pn.PN_PREC_FP64)
    s = fx["full_sample"]
    sub = {k: out[k][s] for k in out}
    ref = {k: fx["full_" + k] for k in ("logabs", "sign", "grad", "lap", "eloc")}
    np.testing.assert_array_equal(sub["sign"], ref["sign"])
    rat = parity_ratios(sub, ref)
    for k, v in rat.items():
        assert v.max() <= TOL64, f"{k}: worst {v.max():.3e}; {summarize(rat)}"
    assert np.all(np.isfinite(out["eloc"]))


def test_value_only_matches_full(pn):
    w = make_config(2, n_walkers=100)
    announce("value-only vs full, workload 2")
    a, _ = _run(pn, w, w.walkers, pn.PN_PREC_FP64, derivs=False)
    b, _ = _run(pn, w, w.walkers, pn.PN_PREC_FP64, derivs=True)
    np.testing.assert_array_equal(a["logabs"], b["logabs"])
    np.testing.assert_array_equal(a["sign"], b["sign"])


@pytest.mark.parametrize("idx", [2, 5])
def test_value_only_workspace(pn, idx):
    """pn_workspace_bytes with out_mask PN_OUT_LOGABS sizes a workspace for
    value-only calls (no tangent buffers): smaller than the one for calls
    with derivatives and the value-path adjoint, enough for a value-only pn_eval (ln|psi| and sign bit
    for bit those of the full call, the low-rank determinant path included),
    and refused for a call with derivatives; bits outside PN_OUT_ALL are
    invalid arguments."""
    w = make_config(idx, n_walkers=37)
    announce(f"value-only workspace, workload {idx}")
    ctx = pn.PauliNetContext(w.system, w.net)
    prec = pn.PN_PREC_NET_FP32 if idx == 5 else pn.PN_PREC_FP64
    B = len(w.walkers)
    small = ctx.workspace_bytes(B, prec, out_mask=pn.PN_OUT_LOGABS)
    big = ctx.workspace_bytes(B, prec, out_mask=pn.PN_OUT_ALL)
    fwd = ctx.workspace_bytes(B, prec, out_mask=pn.PN_OUT_LOGABS | pn.PN_OUT_ELOC)
    assert small < fwd <= big
    assert ctx.plan(B, prec, pn.PLAN_VALUE_ONLY)["workspace_bytes"] <= small
    r = torch.tensor(w.walkers, dtype=torch.float64, device="cuda")
    th = torch.tensor(w.params, dtype=torch.float64, device="cuda")
    ws = torch.empty(small, dtype=torch.uint8, device="cuda")
    a = ctx.eval(r, th, prec, want_derivs=False, ws=ws)
    b = ctx.eval(r, th, prec)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(a["logabs"].cpu().numpy(), b["logabs"].cpu().numpy())
    np.testing.assert_array_equal(a["sign"].cpu().numpy(), b["sign"].cpu().numpy())
    with pytest.raises(pn.PauliNetError, match="(?i)workspace"):
        ctx.eval(r, th, prec, ws=ws)
    with pytest.raises(pn.PauliNetError):
        ctx.workspace_bytes(B, prec, out_mask=32)
    ctx.close()


def test_deterministic_bits(pn):
    w = make_config(3, n_walkers=300)
    announce("determinism, workload 3")
    a, _ = _run(pn, w, w.walkers, pn.PN_PREC_FP64)
    b, _ = _run(pn, w, w.walkers, pn.PN_PREC_FP64)
    for k in a:
        np.testing.assert_array_equal(a[k], b[k])


def test_antisymmetry_on_gpu(pn):
    """Same-spin exchange: sign flips, ln|psi|, lap and E_loc unchanged,
    gradient permuted (Results, eq. "antisymmetry")."""
    w = make_config(2, n_walkers=64)
    announce("antisymmetry, workload 2")
    a, _ = _run(pn, w, w.walkers, pn.PN_PREC_FP64)
    rs = w.walkers.copy()
    rs[:, [1, 4]] = rs[:, [4, 1]]
    b, _ = _run(pn, w, rs, pn.PN_PREC_FP64)
    np.testing.assert_array_equal(b["sign"], -a["sign"])
    np.testing.assert_allclose(b["logabs"], a["logabs"], rtol=1e-12, atol=1e-12)
    gp = a["grad"].copy()
    gp[:, [1, 4]] = gp[:, [4, 1]]
    np.testing.assert_allclose(b["grad"], gp, rtol=1e-9, atol=1e-9)
    np.testing.assert_allclose(b["eloc"], a["eloc"], rtol=1e-9, atol=1e-9)


# p99 ratios measured on the fixture batches (ln|psi|, E_loc; gradient,
# Laplacian), about 3x as the gate: FP32 cfg2 1.4e-6 / 2.1e-7; 3.6e-5 /
# 3.6e-5, cfg3 1.0e-7 / 6.3e-8; 1.4e-6 / 1.4e-6, cfg5 4.3e-6 / 2.9e-6;
# 2.9e-4 / 2.1e-4; BF16 tangent products cfg2 1.4e-6 / 6.6e-6; 1.0e-4 /
# 5.2e-5, cfg3 1.0e-7 / 4.2e-6; 2.2e-5 / 1.0e-5, cfg5 4.3e-6 / 3.5e-4;
# 3.6e-3 / 1.9e-3.
@pytest.mark.parametrize("idx,prec,bound,gbound,lbound", [
    (2, "fp32", 5e-6, 1.1e-4, 1.1e-4), (3, "fp32", 3e-7, 4.5e-6, 4.5e-6), (5, "fp32", 1.5e-5, 9e-4, 6.5e-4),
    (2, "bf16", 2e-5, 3e-4, 1.6e-4), (3, "bf16", 1.5e-5, 6.5e-5, 3.2e-5), (5, "bf16", 1.1e-3, 1.1e-2, 5.7e-3)])
def test_mixed_precision_error_statement(pn, idx, prec, bound, gbound, lbound):
    """Mixed modes: the network in FP32 (or, in the tangent products, BF16
    operands with FP32 accumulation), determinants and E_loc in FP64.  The
    per-output error against the FP64 oracle is printed; the p99 of each
    output's ratio (ln|psi|, E_loc, gradient, Laplacian) must stay within
    about three times what was measured."""
    fx = load_fixture(idx)
    w = make_config(idx, n_walkers=4)
    announce(f"{prec} error statement workload {idx}")
    out, _ = _run(pn, w, fx["walkers"], pn._lib.PRECISIONS[prec])
    rat = parity_ratios(out, fx)
    summ = summarize(rat)
    print(f"[{prec} cfg{idx}] p50/p99/max: {summ}")
    np.testing.assert_array_equal(out["sign"], fx["sign"])
    assert summ["eloc"][1] < bound and summ["logabs"][1] < bound
    assert summ["grad"][1] < gbound and summ["lap"][1] < lbound


def test_fp32_deterministic_bits(pn):
    """The FP32 tangent pass at the 30-electron system (row blocks of the
    pair sums, the chunk electron's own-row terms split over the waves and
    added in a fixed order) gives the same bits on every run."""
    w = make_config(5, n_walkers=64)
    announce("fp32 determinism, workload 5")
    a, _ = _run(pn, w, w.walkers, pn.PN_PREC_NET_FP32)
    b, _ = _run(pn, w, w.walkers, pn.PN_PREC_NET_FP32)
    for k in a:
        np.testing.assert_array_equal(a[k], b[k])


# ------------------------------------------------------------- backward ----
@pytest.mark.parametrize("idx", [1, 2, 3, 5, 6, 7])
def test_backward_fp64_matches_oracle(pn, idx):
    """Value-path adjoint grad += sum_w ct_w d ln|psi_w| / d theta (the
    gradient the Hermitian estimator of Methods eq. "trainig" needs) against
    the oracle's autograd gradient.  FP64 bar: ||d g|| <= 1e-8 ||g|| and
    every component within 1e-7 max|g|."""
    fx = load_fixture(idx)
    w = make_config(idx, n_walkers=4)
    ct = fx["bwd_ct"]
    nb = ct.shape[0]
    announce(f"fp64 backward workload {idx} B={nb}")
    ctx = pn.PauliNetContext(w.system, w.net)
    r = torch.tensor(fx["walkers"][:nb], dtype=torch.float64, device="cuda")
    th = torch.tensor(w.params, dtype=torch.float64, device="cuda")
    g0 = torch.full((ctx.param_count,), 0.5, dtype=torch.float64, device="cuda")
    g = ctx.eval_backward(r, th, torch.tensor(ct, device="cuda"), pn.PN_PREC_FP64, grad_params=g0.clone())
    torch.cuda.synchronize()
    got = g.cpu().numpy() - 0.5  # the call accumulates
    ref = fx["bwd_grad"]
    assert np.linalg.norm(got - ref) <= 1e-8 * np.linalg.norm(ref)
    assert np.max(np.abs(got - ref)) <= 1e-7 * np.max(np.abs(ref))


@pytest.mark.parametrize("idx,prec", [(2, "fp32"), (3, "fp32"), (3, "bf16")])
def test_backward_mixed_error_statement(pn, idx, prec):
    fx = load_fixture(idx)
    w = make_config(idx, n_walkers=4)
    ct = fx["bwd_ct"]
    nb = ct.shape[0]
    announce(f"{prec} backward workload {idx}")
    ctx = pn.PauliNetContext(w.system, w.net)
    r = torch.tensor(fx["walkers"][:nb], dtype=torch.float64, device="cuda")
    th = torch.tensor(w.params, dtype=torch.float64, device="cuda")
    g = ctx.eval_backward(r, th, torch.tensor(ct, device="cuda"), pn._lib.PRECISIONS[prec])
    torch.cuda.synchronize()
    got, ref = g.cpu().numpy(), fx["bwd_grad"]
    rel = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    print(f"[{prec} backward cfg{idx}] relative L2 error {rel:.3e}")
    assert rel < (3e-4 if idx == 2 else 1e-6)  # measured 8.5e-5 (cfg2), 2.9e-7 (cfg3, FP32 and BF16)


def test_backward_deterministic_and_batch_split(pn):
    """Two identical calls give identical bits; two half batches accumulated
    into one buffer equal the full batch to rounding."""
    w = make_config(2, n_walkers=600)
    announce("backward determinism, workload 2, B=600")
    ctx = pn.PauliNetContext(w.system, w.net)
    r = torch.tensor(w.walkers, dtype=torch.float64, device="cuda")
    th = torch.tensor(w.params, dtype=torch.float64, device="cuda")
    ct = torch.tensor(np.random.default_rng(3).standard_normal(600), device="cuda")
    a = ctx.eval_backward(r, th, ct, pn.PN_PREC_FP64)
    b = ctx.eval_backward(r, th, ct, pn.PN_PREC_FP64)
    c = torch.zeros_like(a)
    ctx.eval_backward(r[:300].contiguous(), th, ct[:300].contiguous(), pn.PN_PREC_FP64, grad_params=c)
    ctx.eval_backward(r[300:].contiguous(), th, ct[300:].contiguous(), pn.PN_PREC_FP64, grad_params=c)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    assert float(torch.linalg.norm(a - c)) <= 1e-12 * float(torch.linalg.norm(a))


def test_backward_against_finite_differences(pn):
    """Central differences of sum_w ct_w ln|psi_w| computed by the GPU value
    path, for 24 random parameters of the H10 workload (FP64)."""
    w = make_config(3, n_walkers=32)
    announce("backward vs finite differences, workload 3")
    ctx = pn.PauliNetContext(w.system, w.net)
    r = torch.tensor(w.walkers, dtype=torch.float64, device="cuda")
    th = torch.tensor(w.params, dtype=torch.float64, device="cuda")
    ct = torch.tensor(np.random.default_rng(9).standard_normal(32), device="cuda")
    g = ctx.eval_backward(r, th, ct, pn.PN_PREC_FP64).cpu().numpy()
    idx = np.random.default_rng(10).choice(th.numel(), 24, replace=False)
    h = 1e-6
    for k in idx:
        e = torch.zeros_like(th)
        e[int(k)] = h
        fp = float((ct * ctx.eval(r, th + e, pn.PN_PREC_FP64, want_derivs=False)["logabs"]).sum())
        fm = float((ct * ctx.eval(r, th - e, pn.PN_PREC_FP64, want_derivs=False)["logabs"]).sum())
        fd = (fp - fm) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(fd)), (int(k), fd, g[k])


def test_param_layout_matches_blob_order(pn):
    """pn_param_layout names every tensor of the blob at the offsets and
    shapes the oracle's unpacking of the same blob uses."""
    from oracle.network import Params
    w = make_config(2, n_walkers=4)
    ctx = pn.PauliNetContext(w.system, w.net)
    lay = ctx.param_layout()
    n = ctx.param_count
    p = Params(torch.arange(n, dtype=torch.float64), w.system.nuc_xyz.shape[0], w.system.n_mo, w.net)
    ref = [("x0", p.x0), ("Y", p.Y)]
    for l, L in enumerate(p.layers):
        for c, cn in zip("+-n", ("same", "opp", "nuc")):
            ref += [(f"l{l}.w_{cn}.{k}", t) for k, t in zip(("W1", "b1", "W2", "b2"), L["w"][c])]
        ref += [(f"l{l}.h.W", L["h"][0]), (f"l{l}.h.b", L["h"][1])]
        for c, cn in zip("+-n", ("same", "opp", "nuc")):
            ref += [(f"l{l}.g_{cn}.W", L["g"][c][0]), (f"l{l}.g_{cn}.b", L["g"][c][1])]
    ref += [(f"eta.{k}", t) for k, t in zip(("W1", "b1", "W2", "b2", "W3", "b3"), p.eta)]
    ref += [(f"kappa.{k}", t) for k, t in zip(("W1", "b1", "W2", "b2", "W3", "b3"), p.kappa)]
    assert [e[0] for e in lay] == [r[0] for r in ref]
    for (name, off, shape), (_, t) in zip(lay, ref):
        assert off == int(t.reshape(-1)[0]), name
        assert shape == tuple(t.shape), name


def test_edge_batches(pn):
    """An empty batch is a no-op; a single walker gives bit for bit what it
    gets inside a ragged batch (walkers are independent all the way)."""
    w = make_config(2, n_walkers=67)
    announce("edge batches, workload 2")
    ctx = pn.PauliNetContext(w.system, w.net)
    th = torch.tensor(w.params, dtype=torch.float64, device="cuda")
    r0 = torch.zeros(0, w.system.n_elec, 3, dtype=torch.float64, device="cuda")
    out0 = ctx.eval(r0, th, pn.PN_PREC_FP64)
    assert out0["eloc"].numel() == 0
    g = torch.zeros(ctx.param_count, dtype=torch.float64, device="cuda")
    ctx.eval_backward(r0, th, torch.zeros(0, dtype=torch.float64, device="cuda"), pn.PN_PREC_FP64, grad_params=g)
    torch.cuda.synchronize()
    assert float(g.abs().max()) == 0.0
    full, _ = _run(pn, w, w.walkers, pn.PN_PREC_FP64)
    for k in (0, 66):
        one, _ = _run(pn, w, w.walkers[k:k + 1], pn.PN_PREC_FP64)
        for key in one:
            np.testing.assert_array_equal(one[key][0], full[key][k])


@pytest.mark.parametrize("idx", [2, 5])
def test_autograd_logabs_only_takes_value_adjoint(pn, idx):
    """A loss on ln|psi| alone (the Hermitian estimator's surrogate, Methods
    eq. "trainig") through the autograd Function equals the oracle's
    value-path gradient, and the call sizes its workspace for the value-path
    adjoint, not for the full adjoint through the coordinate derivatives."""
    fx = load_fixture(idx)
    w = make_config(idx, n_walkers=4)
    ct = fx["bwd_ct"]
    nb = ct.shape[0]
    announce(f"autograd ln|psi|-only loss, workload {idx} B={nb}")
    ctx = pn.PauliNetContext(w.system, w.net)
    r = torch.tensor(fx["walkers"][:nb], dtype=torch.float64, device="cuda")
    th = torch.tensor(w.params, dtype=torch.float64, device="cuda", requires_grad=True)
    la, _, _, _, _ = pn.paulinet_eval(ctx, r, th, pn.PN_PREC_FP64)
    (torch.tensor(ct, device="cuda") * la).sum().backward()
    torch.cuda.synchronize()
    got, ref = th.grad.cpu().numpy(), fx["bwd_grad"]
    assert np.linalg.norm(got - ref) <= 1e-8 * np.linalg.norm(ref)
    used = max(t.numel() for t in ctx._ws.values())
    assert used == ctx.workspace_bytes(nb, pn.PN_PREC_FP64, full=False)
    assert used < ctx.workspace_bytes(nb, pn.PN_PREC_FP64, full=True)
