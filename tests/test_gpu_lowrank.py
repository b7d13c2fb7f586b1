"""GPU parity of the low-rank determinant path (one LU of the first
determinant per spin, the other members as excitations of it) and of the
member-by-member path it replaces, both against the FP64 oracle, which
evaluates every determinant of the expansion on its own (Results, eq.
"ansatz": the multideterminant sum).

FP64 bar as in the forward tests: per walker ratios <= 1e-6, signs equal.
"""

import dataclasses

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


def _ctx(pn, w, direct=False):
    net = dataclasses.replace(w.net, flags=w.net.flags | (pn._lib.PN_DET_DIRECT if direct else 0))
    return pn.PauliNetContext(w.system, net)


def _eval(ctx, w, walkers, prec):
    r = torch.tensor(walkers, dtype=torch.float64, device="cuda")
    th = torch.tensor(w.params, dtype=torch.float64, device="cuda")
    out = ctx.eval(r, th, prec)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


@pytest.mark.parametrize("idx", [2, 3, 5, 6, 7])
def test_plan_takes_lowrank_path(pn, idx):
    w = make_config(idx, n_walkers=4)
    B = make_config(idx).walkers.shape[0]
    assert _ctx(pn, w).plan(B, pn.PN_PREC_FP64)["lowrank"]
    assert not _ctx(pn, w, direct=True).plan(B, pn.PN_PREC_FP64)["lowrank"]
    ctx = _ctx(pn, w)
    assert not ctx.plan(B, pn.PN_PREC_FP64, pn._lib.PLAN_VALUE_ADJOINT)["lowrank"]


def test_single_determinant_takes_direct_path(pn):
    w = make_config(1, n_walkers=4)
    assert not _ctx(pn, w).plan(512, pn.PN_PREC_FP64)["lowrank"]


@pytest.mark.parametrize("idx", [2, 3, 5, 6, 7])
@pytest.mark.parametrize("direct", [False, True])
def test_both_determinant_paths_match_oracle(pn, idx, direct):
    fx = load_fixture(idx)
    w = make_config(idx, n_walkers=4)
    announce(f"fp64 {'direct' if direct else 'low-rank'} determinants, workload {idx} B={fx['walkers'].shape[0]}")
    out = _eval(_ctx(pn, w, direct), w, fx["walkers"], pn.PN_PREC_FP64)
    np.testing.assert_array_equal(out["sign"], fx["sign"])
    rat = parity_ratios(out, fx)
    for k, v in rat.items():
        assert v.max() <= TOL64, f"{k}: worst {v.max():.3e} at walker {int(v.argmax())}; {summarize(rat)}"


@pytest.mark.parametrize("idx", [2, 5])
def test_lowrank_full_batch_against_direct(pn, idx):
    """The whole benchmark batch through both paths: the two agree within the
    parity bar on every walker (the low-rank path hands walkers with an
    ill-conditioned first determinant to the direct kernels)."""
    w = make_config(idx)
    announce(f"fp64 low-rank vs direct, full batch of workload {idx}")
    a = _eval(_ctx(pn, w), w, w.walkers, pn.PN_PREC_FP64)
    b = _eval(_ctx(pn, w, direct=True), w, w.walkers, pn.PN_PREC_FP64)
    np.testing.assert_array_equal(a["sign"], b["sign"])
    rat = parity_ratios(a, b)
    print(f"[low-rank vs direct cfg{idx}] p50/p99/max: {summarize(rat)}")
    for k, v in rat.items():
        assert v.max() <= TOL64, f"{k}: worst {v.max():.3e}"


def _near_reference_node(w, o, e=0, rho_min=1.2e4, psi_min=0.2):
    """A walker of workload w moved so that the first determinant of electron
    e's spin block is small against another member (ratio above rho_min, just
    past the hand-back threshold of 1e4) while the determinant sum is not
    (|sum_p c_p D_p| above psi_min max_p |c_p D_p|, so the walker is away from
    a node of psi), by bisecting on the sign of that determinant between two
    positions of the electron.  Uses the oracle's Slater matrices only."""
    from oracle.network import jastrow_backflow
    spin = 0 if e < w.system.n_up else 1
    ci = np.asarray(w.system.ci)

    def dets(r):
        rt = torch.tensor(r[None])
        with torch.no_grad():
            _, f = jastrow_backflow(rt, o.R, o.n_up, o.p, o.net)
            (su, lu), (sd, ld) = o.slater_logdets(rt, f)
        s, l = (su, lu) if spin == 0 else (sd, ld)
        lt = np.log(np.abs(ci)) + lu[0].numpy() + ld[0].numpy()
        st = np.sign(ci) * su[0].numpy() * sd[0].numpy()
        rel = abs(np.sum(st * np.exp(lt - lt.max())))
        return float(s[0, 0]), l[0].numpy(), rel

    base = w.walkers[0].copy()
    rng = np.random.default_rng(3)
    for _ in range(400):
        a, b = base.copy(), base.copy()
        b[e] = base[e] + rng.normal(0.0, 1.0, 3)
        sa, _, _ = dets(a)
        sb, _, _ = dets(b)
        if sa * sb > 0:
            continue
        for _ in range(80):
            m = 0.5 * (a + b)
            sm, lm, rel = dets(m)
            if np.max(lm[1:] - lm[0]) > np.log(rho_min):
                break
            if sm * sa > 0:
                a = m
            else:
                b = m
        if np.max(lm[1:] - lm[0]) > np.log(rho_min) and rel > psi_min:
            return m
    raise AssertionError("no point on the first determinant's node away from a node of psi")


def test_walker_at_first_determinant_node_is_handed_back(pn):
    """Walkers whose first determinant nearly vanishes: the low-rank path
    hands them to the direct kernels, so their outputs equal the direct
    path's bit for bit, and they match the oracle.  Near that node every
    member-by-member FP64 evaluation loses digits (det 0's gradient squared
    and Laplacian terms cancel), so for those two walkers the bar is the
    larger of 1e-6 and 20 times the oracle's own scatter under 1e-12 bohr
    jitter of the positions; the other walkers keep the 1e-6 bar."""
    from oracle import Oracle
    w = make_config(2, n_walkers=8)
    o = Oracle(w.system, w.net, w.params)
    near = [_near_reference_node(w, o, 0), _near_reference_node(w, o, w.system.n_up)]
    rs = np.stack(near + list(w.walkers[1:4]))
    announce("low-rank hand-back near the first determinant's node, workload 2")
    ref = {k: v.numpy() for k, v in o.evaluate(rs).items()}
    jit = np.concatenate([np.stack(near) + 1e-12 * np.random.default_rng(k).standard_normal((2,) + rs.shape[1:])
                          for k in range(3)])
    oj = {k: v.numpy() for k, v in o.evaluate(jit).items()}
    scatter = {k: np.zeros(2) for k in ("logabs", "grad", "lap", "eloc")}
    for j in range(3):
        rj = parity_ratios({k: oj[k][2 * j:2 * j + 2] for k in oj}, {k: ref[k][:2] for k in ref})
        for k in scatter:
            scatter[k] = np.maximum(scatter[k], rj[k])
    a = _eval(_ctx(pn, w), w, rs, pn.PN_PREC_FP64)
    b = _eval(_ctx(pn, w, direct=True), w, rs, pn.PN_PREC_FP64)
    for k in ("logabs", "sign", "grad", "lap", "eloc"):
        np.testing.assert_array_equal(a[k][:2], b[k][:2])
    np.testing.assert_array_equal(a["sign"], ref["sign"])
    rat = parity_ratios(a, ref)
    print(f"[hand-back] oracle jitter scatter {scatter}; ratios {summarize(rat)}")
    for k, v in rat.items():
        bar = np.concatenate([np.maximum(TOL64, 20 * scatter[k]), np.full(3, TOL64)])
        assert np.all(v <= bar), f"{k}: {v} over {bar}"
