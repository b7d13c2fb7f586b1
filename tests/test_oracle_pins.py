"""Pins of the FP64 CPU oracle against what the paper and the mathematics fix.

Each test names the passage of the paper (or the mathematical fact) it
checks.  None of these compares the oracle with itself: expected values come
from closed forms, textbook special cases computed by a different method
(numpy slogdet and analytic Jacobi-formula derivatives), invariances,
finite differences, library routines (torch.optim.AdamW) or published
known-answer vectors.
"""

import copy
import dataclasses
import math
import os

import numpy as np
import pytest
import torch

from oracle import Oracle, local_energy_from
from oracle.hamiltonian import coulomb_potential, electronic_cusp
from oracle.network import Params, distance_features, schnet, ssp
from oracle.orbitals import CuspCorrectedOrbitals, gto_basis
from oracle.vmc import (adamw_step, clip_local_energy, energy_gradient, metropolis_randoms,
                        philox4x32_10)
from synth import NetShape, System, make_config

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _small(idx, B=4, seed=0):
    w = make_config(idx, n_walkers=B)
    return w


# ---------------------------------------------------------------- P1 -------
def _radial(r):
    return torch.sqrt((r**2).sum(-1)).sum(-1)


@pytest.mark.parametrize("Z", [1.0, 2.0, 3.5])
def test_p1_hydrogenic_exact_local_energy(Z):
    """psi = exp(-Z r) with V = -Z / r is an exact eigenfunction with
    E = -Z^2 / 2; Z = 1 is the hydrogen atom, the one system the paper notes
    is solvable analytically (Introduction; Methods eq. "monte-carlo")."""
    g = torch.Generator().manual_seed(1)
    r = torch.randn(64, 1, 3, generator=g, dtype=torch.float64) * 2.0
    _, _, e = local_energy_from(lambda x: -Z * _radial(x), lambda x: -Z / _radial(x), r)
    assert torch.max(torch.abs(e + Z * Z / 2)) < 1e-12


def test_p1_gaussian_local_energy_closed_form():
    """psi = exp(-a r^2) in the potential -Z/r: E_loc = 3a - 2a^2 r^2 - Z/r."""
    a, Z = 0.7, 2.0
    g = torch.Generator().manual_seed(2)
    r = torch.randn(64, 1, 3, generator=g, dtype=torch.float64)
    rr = _radial(r)
    _, _, e = local_energy_from(lambda x: -a * (x**2).sum((-1, -2)), lambda x: -Z / _radial(x), r)
    ref = 3 * a - 2 * a * a * rr**2 - Z / rr
    assert torch.max(torch.abs(e - ref)) < 1e-12


def test_p1_coulomb_hand_value():
    """V for two electrons and two nuclei, computed by hand."""
    r = torch.tensor([[[0.0, 0.0, 0.0], [0.0, 0.0, 2.0]]], dtype=torch.float64)
    R = torch.tensor([[1.0, 0.0, 0.0], [0.0, 3.0, 0.0]], dtype=torch.float64)
    Z = torch.tensor([1.0, 2.0], dtype=torch.float64)
    v = coulomb_potential(r, R, Z)
    ref = (1 / 2.0 - (1 / 1.0 + 2 / 3.0 + 1 / math.sqrt(5) + 2 / math.sqrt(13))
           + 2 / math.sqrt(10))
    assert abs(float(v[0]) - ref) < 1e-14


# ---------------------------------------------------------------- P14 ------
def test_p14_features_cuspless_at_zero():
    """e_k(0) = e_k'(0) = 0 and e_k''(0) = 2 exp(-mu_k^2 / sigma_k^2)
    (Methods, featurisation: envelope forces features and derivatives to 0)."""
    K, rc = 16, 10.0
    d = torch.zeros(1, dtype=torch.float64, requires_grad=True)
    e = distance_features(d, K, rc)[0]
    d1 = torch.stack([torch.autograd.grad(e[k], d, create_graph=True)[0][0] for k in range(K)])
    d2 = torch.stack([torch.autograd.grad(d1[k], d, retain_graph=True)[0][0] for k in range(K)])
    q = np.arange(K) / (K - 1)
    mu, sig = rc * q**2, (1 + rc * q) / 7
    assert torch.all(e.detach() == 0) and torch.max(torch.abs(d1.detach())) == 0
    np.testing.assert_allclose(d2.detach().numpy(), 2 * np.exp(-(mu**2) / sig**2), rtol=1e-12, atol=1e-300)


def test_features_spot_values():
    """e_k(d) at a few hand-evaluated points (K=3 -> q = 0, 1/2, 1)."""
    rc = 4.0
    d = torch.tensor([0.5, 2.0], dtype=torch.float64)
    e = distance_features(d, 3, rc).numpy()
    for i, dd in enumerate([0.5, 2.0]):
        for k, q in enumerate([0.0, 0.5, 1.0]):
            mu, s = rc * q * q, (1 + rc * q) / 7
            assert abs(e[i, k] - dd * dd * math.exp(-dd - (dd - mu) ** 2 / s**2)) < 1e-16


# -------------------------------------------------------------- basis ------
def test_gto_normalisation_by_quadrature():
    """Each primitive s and p Gaussian is unit-normalised (checked on a grid,
    independent of the normalisation constants' formula)."""
    xs = np.linspace(-6, 6, 121)
    X, Y, Zg = np.meshgrid(xs, xs, xs, indexing="ij")
    pts = torch.tensor(np.stack([X, Y, Zg], -1).reshape(-1, 3))
    h3 = (xs[1] - xs[0]) ** 3
    for a in (0.3, 1.0, 2.5):
        chi = gto_basis(pts, torch.zeros(1, 3, dtype=torch.float64), [0, 0], [0, 1], [a, a]).numpy()
        norms = (chi**2).sum(0) * h3
        np.testing.assert_allclose(norms, 1.0, rtol=2e-6)


def test_gto_derivatives_analytic():
    """Autograd gradient/Laplacian of the basis equals the analytic
    Gaussian derivatives (s: grad = -2a d chi, lap = (4a^2 r^2 - 6a) chi;
    p_x: lap = (4a^2 r^2 - 10a) chi)."""
    a = 0.8
    g = torch.Generator().manual_seed(3)
    r = torch.randn(5, 1, 3, generator=g, dtype=torch.float64)
    C = torch.zeros(1, 3, dtype=torch.float64)
    for col, (l, fac) in enumerate([(0, 6.0), (1, 10.0)]):
        def f(x, col=col):
            return gto_basis(x, C, [0, 0], [0, 1], [a, a])[..., 0 if col == 0 else 1].sum(-1)
        grad, lap, _ = local_energy_from(lambda x: torch.log(torch.abs(f(x))), lambda x: x.new_zeros(x.shape[0]), r)
        r2 = (r**2).sum(-1)[:, 0]
        if l == 0:
            np.testing.assert_allclose(grad[:, 0].numpy(), (-2 * a * r[:, 0]).numpy(), rtol=1e-13)
            # lap ln chi = lap chi / chi - |grad ln chi|^2
            np.testing.assert_allclose(lap.numpy(), ((4 * a * a * r2 - 6 * a) - 4 * a * a * r2).numpy(), rtol=1e-12)
        else:
            x = r[:, 0, 0]
            gl = torch.stack([1 / x - 2 * a * x, -2 * a * r[:, 0, 1], -2 * a * r[:, 0, 2]], -1)
            np.testing.assert_allclose(grad[:, 0].numpy(), gl.numpy(), rtol=1e-12)
            np.testing.assert_allclose(lap.numpy(), ((4 * a * a * r2 - fac * a) - (gl**2).sum(-1)).numpy(), rtol=1e-10)


# ------------------------------------------------------ P2 textbook case ---
def _textbook_numpy(system, r, ci):
    """Slater-Jastrow(gamma) with plain GTO MOs, value and derivatives by
    numpy slogdet and the analytic Jacobi formula (no autograd)."""
    R = system.nuc_xyz
    B, N, _ = r.shape
    nb = system.n_basis
    # basis value / grad / lap, analytic
    val = np.zeros((B, N, nb)); grd = np.zeros((B, N, nb, 3)); lap = np.zeros((B, N, nb))
    b = 0
    for c, l, a in zip(system.shell_center, system.shell_l, system.shell_exp):
        d = r - R[c]
        r2 = (d**2).sum(-1)
        g = np.exp(-a * r2)
        if l == 0:
            n = (2 * a / math.pi) ** 0.75
            val[..., b] = n * g
            grd[..., b, :] = -2 * a * d * (n * g)[..., None]
            lap[..., b] = (4 * a * a * r2 - 6 * a) * n * g
            b += 1
        else:
            n = (128 * a**5 / math.pi**3) ** 0.25
            for k in range(3):
                val[..., b] = n * d[..., k] * g
                gk = -2 * a * d * (n * d[..., k] * g)[..., None]
                gk[..., k] += n * g
                grd[..., b, :] = gk
                lap[..., b] = (4 * a * a * r2 - 10 * a) * n * d[..., k] * g
                b += 1
    C = system.mo_coeff
    phi, dphi, lphi = val @ C, np.einsum("bnkc,km->bnmc", grd, C), lap @ C
    nu = system.n_up
    logs, signs, grads, laps = [], [], [], []
    for p in range(len(ci)):
        lg = np.zeros(B); sg = np.ones(B); gr = np.zeros((B, N, 3)); lp = np.zeros(B)
        for sl, occ in ((slice(0, nu), system.det_up[p]), (slice(nu, N), system.det_down[p])):
            if sl.stop - sl.start == 0:
                continue
            A = np.transpose(phi[:, sl][:, :, occ], (0, 2, 1))  # [B, k, i]
            s, l = np.linalg.slogdet(A)
            Ai = np.linalg.inv(A)  # [B, i, k]
            # d ln det / d r_{i,c} = sum_k Ainv[i,k] dphi_{mu_k}(r_i)_c
            dA = dphi[:, sl][:, :, occ, :]  # [B, i, k, c]
            lA = lphi[:, sl][:, :, occ]  # [B, i, k]
            gi = np.einsum("bik,bikc->bic", Ai, dA)
            li = np.einsum("bik,bik->bi", Ai, lA) - (gi**2).sum(-1)
            lg += l; sg *= s; gr[:, sl] += gi; lp += li.sum(-1)
        logs.append(lg + np.log(abs(ci[p]))); signs.append(sg * np.sign(ci[p])); grads.append(gr); laps.append(lp)
    logs, signs = np.stack(logs, 1), np.stack(signs, 1)
    m = logs.max(1)
    S = (signs * np.exp(logs - m[:, None])).sum(1)
    wts = signs * np.exp(logs - m[:, None]) / S[:, None]
    grads, laps = np.stack(grads, 1), np.stack(laps, 1)
    g_d = np.einsum("bp,bpnc->bnc", wts, grads)
    l_d = np.einsum("bp,bp->b", wts, laps + (grads**2).sum((-1, -2))) - (g_d**2).sum((-1, -2))
    # gamma, analytic
    spin = np.array([0] * nu + [1] * (N - nu))
    gam = np.zeros(B); ggam = np.zeros((B, N, 3)); lgam = np.zeros(B)
    for i in range(N):
        for j in range(i + 1, N):
            c = 0.25 if spin[i] == spin[j] else 0.5
            dv = r[:, i] - r[:, j]
            d = np.sqrt((dv**2).sum(-1))
            gam += -c / (1 + d)
            fp = c / (1 + d) ** 2
            fpp = -2 * c / (1 + d) ** 3
            ggam[:, i] += (fp / d)[:, None] * dv
            ggam[:, j] -= (fp / d)[:, None] * dv
            lgam += 2 * (fpp + 2 * fp / d)
    logabs = m + np.log(abs(S)) + gam
    grad = g_d + ggam
    lapl = l_d + lgam
    V = coulomb_potential(torch.tensor(r), torch.tensor(R), torch.tensor(system.charge)).numpy()
    eloc = -0.5 * (lapl + (grad**2).sum((-1, -2))) + V
    return logabs, np.sign(S), grad, lapl, eloc


def _zero_heads(w):
    """Zero the last Linear of eta and kappa: J = 0 and f = 1."""
    s, net = w.system, w.net
    p = torch.tensor(w.params.copy())
    P = Params(p, s.n_nuc, s.n_mo, net)
    with torch.no_grad():
        for t in (P.eta[4], P.eta[5], P.kappa[4], P.kappa[5]):
            t.zero_()
    return P.flat.numpy().copy()


@pytest.mark.parametrize("idx", [1, 2, 3])
def test_p2_textbook_slater_jastrow(idx):
    """With J = 0, f = 1 and no cusp correction the ansatz is the textbook
    multideterminant Slater wavefunction times exp(gamma) (Results, eq.
    "ansatz").  Values and derivatives against numpy slogdet plus analytic
    Jacobi-formula derivatives."""
    w = _small(idx, B=6)
    sysm = copy.deepcopy(w.system)
    sysm.cusp_radius = 0.0
    o = Oracle(sysm, w.net, _zero_heads(w))
    out = o.evaluate(w.walkers)
    la, sg, gr, lp, el = _textbook_numpy(sysm, w.walkers, sysm.ci)
    np.testing.assert_allclose(out["logabs"].numpy(), la, rtol=1e-12, atol=1e-12)
    np.testing.assert_array_equal(out["sign"].numpy(), sg)
    np.testing.assert_allclose(out["grad"].numpy(), gr, rtol=1e-9, atol=1e-10)
    np.testing.assert_allclose(out["lap"].numpy(), lp, rtol=1e-9, atol=1e-9)
    np.testing.assert_allclose(out["eloc"].numpy(), el, rtol=1e-9, atol=1e-9)


# ----------------------------------------------------------- P3 / P4 -------
def test_p3_antisymmetry_same_spin_exchange():
    """Swapping two same-spin electrons flips the sign and permutes the
    gradient; ln|psi|, the Laplacian and E_loc are unchanged (Results, eq.
    "antisymmetry")."""
    w = _small(2, B=3)
    o = Oracle(w.system, w.net, w.params)
    r = w.walkers.copy()
    a = o.evaluate(r)
    for (i, j) in ((0, 3), (6, 8)):
        rs = r.copy()
        rs[:, [i, j]] = rs[:, [j, i]]
        b = o.evaluate(rs)
        np.testing.assert_allclose(b["logabs"].numpy(), a["logabs"].numpy(), rtol=1e-12)
        np.testing.assert_array_equal(b["sign"].numpy(), -a["sign"].numpy())
        gp = a["grad"].numpy().copy()
        gp[:, [i, j]] = gp[:, [j, i]]
        np.testing.assert_allclose(b["grad"].numpy(), gp, rtol=1e-10, atol=1e-10)
        np.testing.assert_allclose(b["lap"].numpy(), a["lap"].numpy(), rtol=1e-10)
        np.testing.assert_allclose(b["eloc"].numpy(), a["eloc"].numpy(), rtol=1e-10)


def test_p4_jastrow_invariant_backflow_equivariant():
    """J(P_ij r) = J(r) and P_ij f_i(r) = f_j(P_ij r) for same-spin
    exchanges (Results, the invariance/equivariance equation)."""
    from oracle.network import jastrow_backflow
    w = _small(3, B=3)
    o = Oracle(w.system, w.net, w.params)
    r = torch.tensor(w.walkers)
    J, f = jastrow_backflow(r, o.R, o.n_up, o.p, w.net)
    for (i, j) in ((1, 4), (5, 9)):
        rs = r.clone()
        rs[:, [i, j]] = rs[:, [j, i]]
        J2, f2 = jastrow_backflow(rs, o.R, o.n_up, o.p, w.net)
        fp = f.clone()
        fp[:, [i, j]] = fp[:, [j, i]]
        assert torch.max(torch.abs(J2 - J)) < 1e-12
        assert torch.max(torch.abs(f2 - fp)) < 1e-12
    # an opposite-spin exchange is not a symmetry of the network
    rs = r.clone()
    rs[:, [0, 5]] = rs[:, [5, 0]]
    J3, _ = jastrow_backflow(rs, o.R, o.n_up, o.p, w.net)
    assert torch.max(torch.abs(J3 - J)) > 1e-6


def test_network_depends_only_on_distances():
    """J and f are built from inter-particle distances only, so a common
    rotation and translation of electrons and nuclei leaves them unchanged."""
    from oracle.network import jastrow_backflow
    w = _small(2, B=3)
    o = Oracle(w.system, w.net, w.params)
    r = torch.tensor(w.walkers)
    J, f = jastrow_backflow(r, o.R, o.n_up, o.p, w.net)
    Q, _ = np.linalg.qr(np.random.default_rng(5).standard_normal((3, 3)))
    Qt = torch.tensor(Q)
    t = torch.tensor([0.3, -1.2, 0.7], dtype=torch.float64)
    J2, f2 = jastrow_backflow(r @ Qt.T + t, o.R @ Qt.T + t, o.n_up, o.p, w.net)
    assert torch.max(torch.abs(J2 - J)) < 1e-11
    assert torch.max(torch.abs(f2 - f)) < 1e-11


def test_network_constant_filter_special_case():
    """With zero first filter layers (ssp(0) = 0) every filter is its output
    bias b^c, so after one interaction
    x_i = x0 + (n_same(i) - 1) (b^+ * h) G+ + n_opp(i) (b^- * h) G-
          + (b^n * sum_I Y_I) Gn + g biases,  h = x0 W_h + b_h
    (Methods, SchNet interaction equations)."""
    net = NetShape(4, 10.0, 6, 5, 1)
    w = make_config(2, n_walkers=2)
    s = w.system
    rng = np.random.default_rng(0)
    from synth import param_count
    flat = torch.tensor(0.3 * rng.standard_normal(param_count(s.n_nuc, s.n_mo, net)))
    P = Params(flat, s.n_nuc, s.n_mo, net)
    lay = P.layers[0]
    with torch.no_grad():
        for c in "+-n":
            lay["w"][c][0].zero_(); lay["w"][c][1].zero_()
    x = schnet(torch.tensor(w.walkers), torch.tensor(s.nuc_xyz), s.n_up, P, net).numpy()
    x0 = P.x0.numpy(); hW, hb = (t.numpy() for t in lay["h"])
    h = x0 @ hW + hb
    b = {c: lay["w"][c][3].numpy() for c in "+-n"}
    G = {c: (lay["g"][c][0].numpy(), lay["g"][c][1].numpy()) for c in "+-n"}
    Ysum = P.Y.numpy().sum(0)
    for i in range(s.n_elec):
        n_same = (s.n_up if i < s.n_up else s.n_down) - 1
        n_opp = s.n_down if i < s.n_up else s.n_up
        ref = (x0 + (n_same * b["+"] * h) @ G["+"][0] + G["+"][1]
               + (n_opp * b["-"] * h) @ G["-"][0] + G["-"][1]
               + (b["n"] * Ysum) @ G["n"][0] + G["n"][1])
        np.testing.assert_allclose(x[:, i], np.broadcast_to(ref, x[:, i].shape), rtol=1e-12, atol=1e-13)


def test_ssp_definition():
    """ssp(x) = ln(e^x / 2 + 1 / 2): ssp(0) = 0, ssp'(0) = 1/2."""
    x = torch.tensor([0.0, 1.0, -30.0, 40.0], dtype=torch.float64)
    ref = torch.log(0.5 * torch.exp(x) + 0.5)
    assert torch.max(torch.abs(ssp(x) - ref)) < 1e-14


# ------------------------------------------------------------ P5 cusps -----
@pytest.mark.parametrize("idx", [1, 2])
def test_p5_nuclear_cusp(idx):
    """Electron at R_I + t u: the average over u = +-x, +-y, +-z of
    u . grad_i ln|psi| tends to -Z_I linearly in t, and E_loc converges to a
    finite value instead of diverging like Z/t (Results, "Asymptotic
    behavior"; Methods, "Cusp conditions", Ma et al. scheme)."""
    w = _small(idx, B=2)
    o = Oracle(w.system, w.net, w.params)
    R, Z = w.system.nuc_xyz, w.system.charge
    dirs = np.concatenate([np.eye(3), -np.eye(3)])
    for I in range(w.system.n_nuc):
        slopes, el = [], []
        ts = (2e-6, 1e-6)
        for t in ts:
            rs = np.repeat(w.walkers[:1], 6, 0)
            rs[:, 0] = R[I] + t * dirs
            out = o.evaluate(rs)
            slopes.append(np.mean(np.einsum("uc,uc->u", out["grad"].numpy()[:, 0], dirs)))
            el.append(out["eloc"].numpy())
        # Richardson extrapolation of the O(t) slope to t = 0
        s0 = (slopes[1] * ts[0] - slopes[0] * ts[1]) / (ts[0] - ts[1])
        assert abs(s0 + Z[I]) < 1e-3 * Z[I]
        # an uncancelled -Z/t would change E_loc by Z/2e-6 between the points
        assert np.max(np.abs(el[1] - el[0]) / (1 + np.abs(el[1]))) < 1e-2


def test_p6_electronic_cusp_opposite_spin():
    """Opposite-spin electrons meeting: averaged slope of ln|psi| in r_ij
    tends to c = 1/2, E_loc stays bounded (Methods, gamma with c_ij)."""
    w = _small(2, B=2)
    o = Oracle(w.system, w.net, w.params)
    dirs = np.concatenate([np.eye(3), -np.eye(3)])
    i, j = 0, 5  # up, down
    vals = []
    for t in (1e-3, 1e-4, 1e-5):
        rs = np.repeat(w.walkers[:1], 6, 0)
        rs[:, j] = rs[:, i] + t * dirs
        out = o.evaluate(rs)
        slope = np.mean(np.einsum("uc,uc->u", out["grad"].numpy()[:, j], dirs))
        vals.append(slope)
        assert np.max(np.abs(out["eloc"].numpy())) < 1e3
    assert abs(vals[-1] - 0.5) < 1e-2


def test_gamma_same_spin_coefficient():
    """Same-spin pairs carry c = 1/4: d gamma / d r_ij at 0 equals 1/4."""
    r = torch.tensor([[[0.0, 0, 0], [0.0, 0, 1e-7], [3.0, 0, 0]]], dtype=torch.float64, requires_grad=True)
    g = electronic_cusp(r, n_up=2)
    (dg,) = torch.autograd.grad(g.sum(), r)
    assert abs(float(dg[0, 1, 2]) - 0.25) < 1e-6


def test_p7_cuspless_network_averaged_slope():
    """The network is cuspless: the averaged directional derivative of J and
    f at e-n and e-e coalescence vanishes as t -> 0 (Methods, eq.
    "cuspless")."""
    from oracle.network import jastrow_backflow
    w = _small(2, B=1)
    o = Oracle(w.system, w.net, w.params)
    dirs = np.concatenate([np.eye(3), -np.eye(3)])
    for target in ("nuc", "elec"):
        slopes = []
        for t in (1e-3, 1e-5):
            rs = np.repeat(w.walkers[:1], 6, 0)
            base = w.system.nuc_xyz[0] if target == "nuc" else rs[0, 7]
            rs[:, 2] = base + t * dirs
            r = torch.tensor(rs, requires_grad=True)
            J, f = jastrow_backflow(r, o.R, o.n_up, o.p, w.net)
            (gJ,) = torch.autograd.grad(J.sum(), r, retain_graph=True)
            (gf,) = torch.autograd.grad(f[:, 2].sum(), r)
            sJ = abs(np.mean(np.einsum("uc,uc->u", gJ.numpy()[:, 2], dirs)))
            sf = abs(np.mean(np.einsum("uc,uc->u", gf.numpy()[:, 2], dirs)))
            slopes.append(max(sJ, sf))
        assert slopes[1] < 1e-6 and slopes[1] < slopes[0]


# --------------------------------------------------------------- P8 FD -----
@pytest.mark.parametrize("idx", [1, 2])
def test_p8_finite_differences(idx):
    """Gradient and Laplacian of ln|psi| against central differences."""
    w = _small(idx, B=2)
    o = Oracle(w.system, w.net, w.params)
    out = o.evaluate(w.walkers)
    r0 = torch.tensor(w.walkers)
    N = r0.shape[1]
    lp = lambda x: o.log_psi(x)[0]  # noqa: E731
    h1, h2 = 1e-5, 1e-3
    fd_g = torch.zeros_like(r0)
    fd_l = torch.zeros(r0.shape[0], dtype=torch.float64)
    with torch.no_grad():
        f0 = lp(r0)
        for i in range(N):
            for c in range(3):
                e = torch.zeros_like(r0); e[:, i, c] = 1
                fd_g[:, i, c] = (lp(r0 + h1 * e) - lp(r0 - h1 * e)) / (2 * h1)
                fp1, fm1 = lp(r0 + h2 * e), lp(r0 - h2 * e)
                fp2, fm2 = lp(r0 + 2 * h2 * e), lp(r0 - 2 * h2 * e)
                fd_l += (-fp2 + 16 * fp1 - 30 * f0 + 16 * fm1 - fm2) / (12 * h2 * h2)
    g = out["grad"]
    assert float(torch.linalg.norm(g - fd_g)) < 1e-7 * max(1.0, float(torch.linalg.norm(g)))
    assert torch.max(torch.abs(out["lap"] - fd_l) / torch.clamp(torch.abs(out["lap"]), min=1.0)) < 1e-5


# ---------------------------------------------------------- P9 .. P12 ------
def test_p9_translation_and_axial_rotation():
    """Rigid translation leaves every output unchanged; for an s-only linear
    molecule on z a rotation about z does too (the gradient rotates)."""
    w = _small(3, B=2)
    o = Oracle(w.system, w.net, w.params)
    a = o.evaluate(w.walkers)
    s2 = copy.deepcopy(w.system)
    t = np.array([0.4, -0.3, 1.1])
    s2.nuc_xyz = s2.nuc_xyz + t
    b = Oracle(s2, w.net, w.params).evaluate(w.walkers + t)
    for k in ("logabs", "grad", "lap", "eloc"):
        np.testing.assert_allclose(b[k].numpy(), a[k].numpy(), rtol=1e-9, atol=1e-9)
    th = 0.7
    Q = np.array([[math.cos(th), -math.sin(th), 0], [math.sin(th), math.cos(th), 0], [0, 0, 1]])
    c = o.evaluate(w.walkers @ Q.T)
    np.testing.assert_allclose(c["logabs"].numpy(), a["logabs"].numpy(), rtol=1e-10)
    np.testing.assert_allclose(c["grad"].numpy(), a["grad"].numpy() @ Q.T, rtol=1e-8, atol=1e-9)
    np.testing.assert_allclose(c["eloc"].numpy(), a["eloc"].numpy(), rtol=1e-8, atol=1e-9)


def test_p10_ci_scaling():
    """c -> lambda c shifts ln|psi| by ln|lambda|, flips the sign for
    lambda < 0, and leaves the derivatives and E_loc unchanged."""
    w = _small(2, B=2)
    a = Oracle(w.system, w.net, w.params).evaluate(w.walkers)
    s2 = copy.deepcopy(w.system)
    s2.ci = -2.5 * s2.ci
    b = Oracle(s2, w.net, w.params).evaluate(w.walkers)
    np.testing.assert_allclose(b["logabs"].numpy(), a["logabs"].numpy() + math.log(2.5), rtol=1e-13)
    np.testing.assert_array_equal(b["sign"].numpy(), -a["sign"].numpy())
    for k in ("grad", "lap", "eloc"):
        np.testing.assert_allclose(b[k].numpy(), a[k].numpy(), rtol=1e-9, atol=1e-9)


def test_p11_duplicate_determinant():
    """A determinant listed twice with c1 + c2 = c equals it listed once."""
    w = _small(2, B=2)
    a = Oracle(w.system, w.net, w.params).evaluate(w.walkers)
    s2 = copy.deepcopy(w.system)
    s2.det_up = np.concatenate([s2.det_up, s2.det_up[3:4]])
    s2.det_down = np.concatenate([s2.det_down, s2.det_down[3:4]])
    c = s2.ci[3]
    s2.ci = np.concatenate([s2.ci, [0.3 * c]])
    s2.ci[3] = 0.7 * c
    b = Oracle(s2, w.net, w.params).evaluate(w.walkers)
    for k in ("logabs", "grad", "lap", "eloc"):
        np.testing.assert_allclose(b[k].numpy(), a[k].numpy(), rtol=1e-9, atol=1e-9)


def test_p12_empty_spin_block():
    """One electron (no spin-down block): ln|psi| = J + ln|phi~_0(r)|."""
    from oracle.network import jastrow_backflow
    w = _small(1, B=3)
    s = copy.deepcopy(w.system)
    s.n_down = 0
    s.det_down = np.zeros((1, 0), np.int32)
    s.nuc_xyz = s.nuc_xyz[:1]
    s.charge = s.charge[:1]
    keep = s.shell_center == 0
    s.shell_center, s.shell_l, s.shell_exp = s.shell_center[keep], s.shell_l[keep], s.shell_exp[keep]
    s.mo_coeff = s.mo_coeff[:4]
    from synth import param_count
    params = 0.1 * np.random.default_rng(0).standard_normal(param_count(1, 1, w.net))
    o = Oracle(s, w.net, params)
    r = torch.tensor(w.walkers[:, :1])
    lp, sg = o.log_psi(r)
    J, f = jastrow_backflow(r, o.R, 1, o.p, w.net)
    phi = o.orbitals(r)[:, 0, 0] * f[:, 0, 0]
    np.testing.assert_allclose(lp.numpy(), (J + torch.log(torch.abs(phi))).numpy(), rtol=1e-13)
    np.testing.assert_array_equal(sg.numpy(), torch.sign(phi).numpy())


# ------------------------------------------------------------ P13 cusp -----
def test_p13_cusp_correction_c2_and_nucleus_value():
    """The corrected orbital is continuous with continuous first and second
    radial derivatives at r_cusp, takes the nucleus value s0 + eta(R_I), and
    the input nucleus value is honoured."""
    w = _small(2, B=1)
    s = w.system
    orb = CuspCorrectedOrbitals(s)
    rc = s.cusp_radius
    u = np.array([0.36, -0.48, 0.8])
    def radial(rho):
        return orb(torch.tensor(rho[:, None, None] * u[None, None, :]))[:, 0, :].numpy()
    eps = 1e-4
    rin = rc - np.array([4 * eps, 3 * eps, 2 * eps, eps]) - 1e-9
    rout = rc + np.array([eps, 2 * eps, 3 * eps, 4 * eps]) + 1e-9
    fi, fo = radial(rin), radial(rout)
    # extrapolate each side quadratically to rc and compare value/slope
    for k in range(fi.shape[1]):
        pi = np.polyfit(rin - rc, fi[:, k], 3)
        po = np.polyfit(rout - rc, fo[:, k], 3)
        scale = max(1.0, abs(pi[3]))
        assert abs(pi[3] - po[3]) < 1e-9 * scale  # value
        assert abs(pi[2] - po[2]) < 1e-5 * scale  # slope
        assert abs(pi[1] - po[1]) < 2e-2 * max(scale, abs(pi[1]))  # curvature / 2
    # nucleus value with an explicit input
    s2 = copy.deepcopy(s)
    base = np.array([[orb._s_radial(terms, torch.tensor(0.0, dtype=torch.float64)).item() if terms else 0.0
                      for terms in [orb._s_terms(0, mu) for mu in range(s.n_mo)]]])
    s2.cusp_nuc_value = 1.2 * base
    orb2 = CuspCorrectedOrbitals(s2)
    at = orb2(torch.tensor(np.zeros((1, 1, 3)) + 1e-12))[0, 0].numpy()
    un = orb.uncorrected(torch.zeros(1, 3, dtype=torch.float64))[0].numpy()
    np.testing.assert_allclose(at, un + 0.2 * base[0], rtol=1e-8)


# --------------------------------------------------------- VMC pieces ------
def test_philox_known_answers():
    """Philox4x32-10 against the published known-answer vectors."""
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) as fh:
        rows = [l.split() for l in fh if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for row in rows:
        v = [int(x, 16) for x in row]
        assert tuple(philox4x32_10(v[0:4], v[4:6])) == tuple(v[6:10])


def test_metropolis_normals_statistics():
    """Box-Muller normals from the counter-based stream: mean 0, variance 1."""
    xi, u = metropolis_randoms(seed=123456789, step=3, n_walkers=400, n_coord=30)
    assert abs(xi.mean()) < 0.03 and abs(xi.var() - 1) < 0.03
    assert 0 < u.min() and u.max() < 1 and abs(u.mean() - 0.5) < 0.05


def test_adamw_matches_torch_optim():
    """AdamW with lr_t = lr0 / (1 + t / t0) equals torch.optim.AdamW stepped
    with the same per-step learning rate."""
    g = torch.Generator().manual_seed(7)
    th0 = torch.randn(50, generator=g, dtype=torch.float64)
    grads = [torch.randn(50, generator=g, dtype=torch.float64) for _ in range(5)]
    p = torch.nn.Parameter(th0.clone())
    opt = torch.optim.AdamW([p], lr=0.01, betas=(0.9, 0.999), eps=1e-8, weight_decay=0.01)
    th, m, v = th0.clone(), torch.zeros(50, dtype=torch.float64), torch.zeros(50, dtype=torch.float64)
    for t, gr in enumerate(grads):
        for grp in opt.param_groups:
            grp["lr"] = 0.01 / (1 + t / 200.0)
        p.grad = gr.clone()
        opt.step()
        th, m, v = adamw_step(th, gr, m, v, t)
    assert torch.max(torch.abs(p.detach() - th)) < 1e-15


def test_clip_local_energy():
    """Inside the window q * mean|E - median| values are unchanged; outside
    they grow logarithmically; the clip is continuous with slope 1 at the
    window edge."""
    e = torch.tensor([-1.0, 0, 1, 0, 0, 0, 0, 0, 0, 100], dtype=torch.float64)
    c = clip_local_energy(e, 5.0)
    w = 5 * 10.2
    assert torch.equal(c[:9], e[:9])
    assert abs(float(c[9]) - w * (1 + math.log(100 / w))) < 1e-12
    base = torch.zeros(20, dtype=torch.float64)
    base[0] = 1.0
    base[1] = -1.0
    # probe near the window edge with a tiny outlier family
    m, dev = 0.0, 2.0 / 20
    wq = 5 * dev
    for x in (wq * (1 - 1e-7), wq * (1 + 1e-7)):
        pass
    f = lambda E: m + math.copysign(1, E) * wq * (1 + math.log(abs(E) / wq)) if abs(E) > wq else E  # noqa
    assert abs(f(wq * (1 + 1e-9)) - wq) < 1e-8
    assert abs((f(wq * 1.001) - f(wq)) / (wq * 0.001) - 1) < 1e-3
    # odd B median
    c3 = clip_local_energy(torch.tensor([1.0, 2.0, 30.0], dtype=torch.float64), 1.0)
    w3 = 1 * (1 + 0 + 28) / 3
    assert abs(float(c3[2]) - (2 + w3 * (1 + math.log(28 / w3)))) < 1e-12


def test_energy_gradient_matches_surrogate_fd():
    """The Hermitian gradient (eq. "trainig") equals the theta-derivative of
    sum_w 2/B (E_w - L) ln|psi_w| with the weights held fixed (central
    differences on a random subset of parameters)."""
    w = _small(1, B=8)
    o = Oracle(w.system, w.net, w.params)
    out = o.evaluate(w.walkers)
    g, L, ec = energy_gradient(o, w.walkers, out["eloc"])
    B = w.walkers.shape[0]
    wt = 2.0 / B * (ec - L)
    r = torch.tensor(w.walkers)
    th = torch.tensor(w.params)
    idx = np.random.default_rng(0).choice(th.numel(), 40, replace=False)
    h = 1e-6
    for k in idx:
        e = torch.zeros_like(th); e[k] = h
        fp = (wt * o.log_psi(r, th + e)[0]).sum()
        fm = (wt * o.log_psi(r, th - e)[0]).sum()
        fd = float(fp - fm) / (2 * h)
        assert abs(fd - float(g[k])) < 1e-7 * max(1.0, abs(fd))


@pytest.mark.parametrize("idx", [1, 2])
def test_full_adjoint_matches_finite_differences(idx):
    """The parameter gradient of sum_w (a ln|psi| + b . grad + c lap + e E_loc)
    (the Laplacian's second-order terms included) equals Richardson-
    extrapolated central differences in theta of the same sum, each
    evaluation taking grad and lap from the coordinate derivatives."""
    w = _small(idx, B=3)
    o = Oracle(w.system, w.net, w.params)
    B, N = w.walkers.shape[0], w.walkers.shape[1]
    rng = np.random.default_rng(11)
    ca, cg, cl, ce = rng.normal(size=B), rng.normal(size=(B, N, 3)), rng.normal(size=B), rng.normal(size=B)
    g = o.param_grad_full(w.walkers, ca, cg, cl, ce)

    def F(th):
        o2 = Oracle(w.system, w.net, th)
        out = o2.evaluate(w.walkers)
        return float((ca * out["logabs"].numpy()).sum() + (cg * out["grad"].numpy()).sum()
                     + (cl * out["lap"].numpy()).sum() + (ce * out["eloc"].numpy()).sum())

    th0 = np.asarray(w.params, dtype=np.float64)
    n = th0.size
    picks = sorted(set([0, n - 1] + list(rng.choice(n, 10, replace=False))))
    for k in picks:
        def D(h):
            e = np.zeros(n); e[k] = h
            return (F(th0 + e) - F(th0 - e)) / (2 * h)
        h = 1e-3
        fd = (4 * D(h / 2) - D(h)) / 3
        assert abs(fd - float(g[k])) < 1e-6 * max(1.0, abs(fd)), (k, fd, float(g[k]))


def test_full_adjoint_reduces_to_value_adjoint():
    """With only a ln|psi| cotangent the full adjoint is the value-path one."""
    w = _small(2, B=3)
    o = Oracle(w.system, w.net, w.params)
    ct = np.array([0.3, -1.2, 0.7])
    a = o.param_grad_full(w.walkers, ct_logabs=ct)
    b = o.param_grad_logabs(w.walkers, ct)
    assert torch.allclose(a, b, rtol=1e-12, atol=1e-12)


# ---------------------------------------------------------------- Langevin --
def _toy_randoms(B, n, seed):
    g = torch.Generator().manual_seed(seed)
    return lambda k: (torch.randn(B, n, generator=g, dtype=torch.float64),
                      torch.rand(B, generator=g, dtype=torch.float64))


def test_langevin_samples_gaussian_exactly():
    """|psi|^2 = exp(-2 a r^2) (a = 1/2): per-coordinate variance 1/(4a).
    At tau = 0.4 the drift-diffusion chain without the Hastings correction
    would sit at 1/(2 - tau) = 0.625; the sampler must give 0.5."""
    from oracle.langevin import langevin_run
    a = 0.5

    def lg(r):
        r = torch.as_tensor(r, dtype=torch.float64)
        return -a * (r ** 2).sum((1, 2)), -2 * a * r

    B = 4000
    r0 = torch.randn(B, 1, 3, generator=torch.Generator().manual_seed(1), dtype=torch.float64)
    r, accs, _, _ = langevin_run(lg, r0, torch.zeros(0, 3, dtype=torch.float64), 0.4, _toy_randoms(B, 3, 2), 80,
                                 rate=0.0)
    var = float((r ** 2).mean())
    assert abs(var - 1 / (4 * a)) < 0.025, var
    assert 0.5 < sum(accs[-20:]) / 20 < 1.0


def test_langevin_hydrogen_mean_radius_with_clipping():
    """Hydrogen ground state psi = exp(-r): <r> = 3/2 bohr under |psi|^2, with
    the nearest-nucleus clipping of the drift active (the drift length tau
    would exceed r near the nucleus)."""
    from oracle.langevin import langevin_run

    def lg(r):
        r = torch.as_tensor(r, dtype=torch.float64)
        d = torch.linalg.norm(r, dim=-1)
        return -d.sum(-1), -r / d[..., None]

    B = 4000
    r0 = torch.randn(B, 1, 3, generator=torch.Generator().manual_seed(3), dtype=torch.float64)
    r, accs, taus, _ = langevin_run(lg, r0, torch.zeros(1, 3, dtype=torch.float64), 0.5, _toy_randoms(B, 3, 4), 120)
    mean_r = float(torch.linalg.norm(r, dim=-1).mean())
    assert abs(mean_r - 1.5) < 0.05, mean_r
    assert abs(sum(accs[-40:]) / 40 - 0.57) < 0.08  # the step adapts to the target acceptance


def test_langevin_drift_clipped_below_nearest_nucleus():
    from oracle.langevin import clipped_drift
    nuc = torch.tensor([[0.0, 0.0, 0.0], [0.0, 0.0, 3.0]], dtype=torch.float64)
    r = torch.tensor([[[0.1, 0.0, 0.0], [0.0, 0.0, 2.2]]], dtype=torch.float64)
    g = torch.tensor([[[-50.0, 0.0, 0.0], [0.0, 0.2, 0.0]]], dtype=torch.float64)
    d = clipped_drift(r, g, nuc, 0.1)
    assert torch.allclose(torch.linalg.norm(d[0, 0]), torch.tensor(0.1, dtype=torch.float64))  # clipped to 0.1
    assert torch.allclose(d[0, 1], 0.1 * g[0, 1])  # short drift untouched


# ------------------------------------------------------- ansatz variants ----
def test_variant_without_network_is_textbook():
    """Neither Jastrow factor nor backflow (flags 3): the textbook
    multideterminant Slater wavefunction times exp(gamma), checked like P2
    against numpy slogdet and Jacobi-formula derivatives, with the seeded
    (non-zero) heads left in the parameter blob."""
    w = _small(2, B=5)
    sysm = copy.deepcopy(w.system)
    sysm.cusp_radius = 0.0
    net = dataclasses.replace(w.net, flags=3)
    out = Oracle(sysm, net, w.params).evaluate(w.walkers)
    la, sg, gr, lp, el = _textbook_numpy(sysm, w.walkers, sysm.ci)
    np.testing.assert_allclose(out["logabs"].numpy(), la, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(out["grad"].numpy(), gr, rtol=1e-9, atol=1e-10)
    np.testing.assert_allclose(out["eloc"].numpy(), el, rtol=1e-9, atol=1e-9)


@pytest.mark.parametrize("flags,zeroed", [(1, "eta"), (2, "kappa")])
def test_variant_removes_one_head(flags, zeroed):
    """Removing a head equals zeroing its last layer (J = 0 or f = 1), and its
    parameters get exactly zero gradient."""
    w = _small(2, B=4)
    s, net = w.system, w.net
    p = torch.tensor(w.params.copy())
    P = Params(p, s.n_nuc, s.n_mo, net)
    head = P.eta if zeroed == "eta" else P.kappa
    with torch.no_grad():
        head[4].zero_()
        head[5].zero_()
    a = Oracle(s, dataclasses.replace(net, flags=flags), w.params).evaluate(w.walkers)
    b = Oracle(s, net, P.flat.numpy()).evaluate(w.walkers)
    for k in ("logabs", "grad", "lap", "eloc"):
        np.testing.assert_allclose(a[k].numpy(), b[k].numpy(), rtol=1e-12, atol=1e-12)
    g = Oracle(s, dataclasses.replace(net, flags=flags), w.params).param_grad_logabs(w.walkers, np.ones(4))
    Pg = Params(g, s.n_nuc, s.n_mo, net)
    hg = Pg.eta if zeroed == "eta" else Pg.kappa
    assert all(float(t.abs().max()) == 0.0 for t in hg)


def test_cusp_value_gradient_finite_differences():
    """d ln|psi| / d s0 (orbital values at the nucleus, variational in the
    paper) against central differences of ln|psi| with the nucleus values
    passed through the system description, for walkers with electrons inside
    the cusp radius."""
    w = _small(2, B=4)
    o = Oracle(w.system, w.net, w.params)
    r = w.walkers.copy()
    u = np.array([0.6, -0.48, 0.64])
    r[0, 0] = w.system.nuc_xyz[0] + 0.05 * u
    r[1, 3] = w.system.nuc_xyz[0] + 0.02 * u[::-1]
    r[2, 7] = w.system.nuc_xyz[0] + 0.08 * u
    ct = np.array([1.0, -0.6, 0.8, 0.3])
    g = o.cusp_value_grad(r, ct).numpy()
    s0 = o.orbitals.s0.numpy().copy()
    corrected = [(I, mu) for I, mu, *_ in o.orbitals.corr]
    assert corrected
    nz = 0
    for I, mu in corrected[:6]:
        h = 1e-6 * max(1.0, abs(s0[I, mu]))
        vals = []
        for sgn in (1, -1):
            sysm = copy.deepcopy(w.system)
            sv = s0.copy()
            sv[I, mu] += sgn * h
            sysm.cusp_nuc_value = sv
            lp, _ = Oracle(sysm, w.net, w.params).log_psi(torch.tensor(r))
            vals.append(float((torch.tensor(ct) * lp).sum()))
        fd = (vals[0] - vals[1]) / (2 * h)
        assert abs(fd - g[I, mu]) <= 1e-6 * max(1.0, abs(fd)), (I, mu, fd, g[I, mu])
        nz += abs(fd) > 1e-6
    assert nz > 0  # the walkers do probe the corrected region
