"""GPU parity of the ansatz variants (Results: single- vs multi-determinant,
Jastrow factor only, Jastrow and backflow) against the FP64 oracle evaluated
live on the same walkers, through the C ABI.  FP64 bar as for the full
ansatz: per walker ratios <= 1e-6; gradients <= 1e-8 relative L2."""

import copy
import dataclasses

import numpy as np
import pytest
import torch

from gpu_util import announce, parity_ratios
from oracle import Oracle
from synth import make_config

pytestmark = pytest.mark.gpu

TOL64 = 1e-6


@pytest.fixture(scope="module")
def pn():
    import paper_1909_08423_amd as pn
    assert torch.cuda.is_available(), "no ROCm device"
    pn.load_library()
    return pn


def _walkers(w, B):
    r = w.walkers[:B].copy()
    r[-1, 0] = w.system.nuc_xyz[0] + 0.03 * np.array([0.6, -0.48, 0.64])  # inside the cusp radius
    return r


def _single_det(system):
    s = copy.deepcopy(system)
    s.det_up, s.det_down, s.ci = s.det_up[:1].copy(), s.det_down[:1].copy(), s.ci[:1].copy()
    return s


def _gpu_eval(pn, system, net, params, r, prec):
    ctx = pn.PauliNetContext(system, net)
    out = ctx.eval(torch.tensor(r, dtype=torch.float64, device="cuda"),
                   torch.tensor(params, dtype=torch.float64, device="cuda"), prec)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}, ctx


@pytest.mark.parametrize("flags,single", [(1, False), (2, False), (3, False), (0, True), (2, True)])
def test_variant_forward_fp64_matches_oracle(pn, flags, single):
    w = make_config(2, n_walkers=12)
    system = _single_det(w.system) if single else w.system
    net = dataclasses.replace(w.net, flags=flags)
    r = _walkers(w, 12)
    announce(f"variant flags={flags} single_det={single} workload 2 B=12")
    ref = {k: v.numpy() for k, v in Oracle(system, net, w.params).evaluate(r).items()}
    out, _ = _gpu_eval(pn, system, net, w.params, r, pn.PN_PREC_FP64)
    rat = parity_ratios(out, ref)
    for k, v in rat.items():
        assert v.max() <= TOL64, (k, float(v.max()))
    assert np.array_equal(out["sign"], ref["sign"])


@pytest.mark.parametrize("flags", [1, 2])
def test_variant_value_adjoint_matches_oracle(pn, flags):
    w = make_config(2, n_walkers=4)
    net = dataclasses.replace(w.net, flags=flags)
    r = _walkers(w, 4)
    ct = np.array([0.7, -1.1, 0.4, 0.9])
    announce(f"variant flags={flags} value adjoint")
    ref = Oracle(w.system, net, w.params).param_grad_logabs(r, ct).numpy()
    ctx = pn.PauliNetContext(w.system, net)
    g = ctx.eval_backward(torch.tensor(r, device="cuda"), torch.tensor(w.params, device="cuda"),
                          torch.tensor(ct, device="cuda"), pn.PN_PREC_FP64).cpu().numpy()
    assert np.linalg.norm(g - ref) <= 1e-8 * np.linalg.norm(ref)


def test_variant_full_adjoint_matches_oracle(pn):
    w = make_config(2, n_walkers=3)
    net = dataclasses.replace(w.net, flags=2)
    r = _walkers(w, 3)
    ce = np.array([0.5, -0.8, 1.3])
    announce("variant flags=2 full adjoint (E_loc cotangent)")
    ref = Oracle(w.system, net, w.params).param_grad_full(r, ct_eloc=ce).numpy()
    ctx = pn.PauliNetContext(w.system, net)
    g = ctx.eval_backward(torch.tensor(r, device="cuda"), torch.tensor(w.params, device="cuda"), None,
                          pn.PN_PREC_FP64, ct_eloc=torch.tensor(ce, device="cuda")).cpu().numpy()
    assert np.linalg.norm(g - ref) <= 1e-8 * np.linalg.norm(ref)


def test_variant_without_network_has_no_parameter_gradient(pn):
    w = make_config(2, n_walkers=4)
    net = dataclasses.replace(w.net, flags=3)
    ctx = pn.PauliNetContext(w.system, net)
    g = ctx.eval_backward(torch.tensor(w.walkers, device="cuda"), torch.tensor(w.params, device="cuda"),
                          torch.ones(4, dtype=torch.float64, device="cuda"), pn.PN_PREC_FP64,
                          ct_eloc=torch.ones(4, dtype=torch.float64, device="cuda"))
    torch.cuda.synchronize()
    assert float(g.abs().max()) == 0.0


@pytest.mark.parametrize("idx", [2, 3])
def test_cusp_value_gradient_matches_oracle(pn, idx):
    """d ln|psi| / d s0 (orbital values at the nuclei) for walkers with
    electrons inside the cusp radius, FP64, against the oracle's autograd
    gradient (itself pinned by finite differences)."""
    w = make_config(idx, n_walkers=5)
    r = w.walkers.copy()
    u = np.array([0.6, -0.48, 0.64])
    nuc = w.system.nuc_xyz
    r[0, 0] = nuc[0] + 0.05 * u
    r[1, 3] = nuc[-1] + 0.02 * u[::-1]
    r[2, 1] = nuc[0] + 0.08 * u
    r[3, 4] = nuc[len(nuc) // 2] + 0.03 * u
    ct = np.array([1.0, -0.6, 0.8, 0.3, 1.2])
    announce(f"cusp value gradient workload {idx}")
    ref = Oracle(w.system, w.net, w.params).cusp_value_grad(r, ct).numpy()
    ctx = pn.PauliNetContext(w.system, w.net)
    g = ctx.eval_backward_cusp(torch.tensor(r, device="cuda"), torch.tensor(w.params, device="cuda"),
                               torch.tensor(ct, device="cuda"), pn.PN_PREC_FP64).cpu().numpy()
    assert np.abs(ref).max() > 0
    assert np.linalg.norm(g - ref) <= 1e-8 * np.linalg.norm(ref), (np.abs(g - ref).max(), np.abs(ref).max())
