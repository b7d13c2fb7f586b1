"""PauliNet wavefunction, its coordinate derivatives and the local energy
(oracle; test infrastructure).

psi(r) = exp(gamma(r) + J(r)) sum_p c_p det[phi~_up] det[phi~_down],
phi~_{mu i} = phi_mu(r_i) f_{mu i}(r)                (Results, eq. "ansatz")

E_loc = H psi / psi = -1/2 (lap ln|psi| + |grad ln|psi||^2) + V
                                        (Methods, eq. "monte-carlo"; H is
                                         the electronic Hamiltonian)

Derivatives: autograd.  grad = d ln|psi| / d r; the Laplacian is the sum over
the 3N coordinates of the diagonal second derivatives, each taken by a second
autograd pass.

Readings (listed in the design notes): electrons 0..n_up-1 are spin up;
A_p^sigma[k, i] = phi~_{mu_p^sigma(k)}(r_i) over the electrons of spin sigma in
ascending index; an empty spin block has determinant 1; the determinant sum
is taken in signed log-sum-exp form (ln|psi_d| = -inf, sign 0 on exact
cancellation).

Parity pins: exact E_loc for hydrogen-like and Gaussian test functions
through `local_energy_from`; the textbook Slater-Jastrow special case against
numpy slogdet and analytic Jacobi-formula derivatives; antisymmetry; CI
scaling; duplicate determinants; empty spin block; nuclear and electronic
cusps; finite differences of ln|psi| (tests).
"""

import torch

from .hamiltonian import coulomb_potential, electronic_cusp
from .network import Params, jastrow_backflow
from .orbitals import CuspCorrectedOrbitals


def local_energy_from(logpsi_fn, potential_fn, r: torch.Tensor):
    """E_loc for any log|psi| provider: returns (grad [B,N,3], lap [B],
    E_loc [B]).  logpsi_fn maps r [B,N,3] -> [B] with walkers independent."""
    r = r.detach().clone().requires_grad_(True)
    B = r.shape[0]
    lp = logpsi_fn(r)
    (g,) = torch.autograd.grad(lp.sum(), r, create_graph=True)
    gf = g.reshape(B, -1)
    lap = torch.zeros(B, dtype=r.dtype)
    for a in range(gf.shape[1]):
        (h,) = torch.autograd.grad(gf[:, a].sum(), r, retain_graph=True)
        lap = lap + h.reshape(B, -1)[:, a]
    V = potential_fn(r.detach())
    eloc = -0.5 * (lap + (gf.detach() ** 2).sum(-1)) + V
    return g.detach(), lap.detach(), eloc.detach()


class Oracle:
    """Evaluates the ansatz for one system, network shape and parameter blob."""

    def __init__(self, system, net, params):
        self.system = system
        self.net = net
        self.R = torch.as_tensor(system.nuc_xyz, dtype=torch.float64)
        self.Z = torch.as_tensor(system.charge, dtype=torch.float64)
        self.n_up, self.n_down = int(system.n_up), int(system.n_down)
        self.orbitals = CuspCorrectedOrbitals(system)
        self.det_up = torch.as_tensor(system.det_up, dtype=torch.long)
        self.det_down = torch.as_tensor(system.det_down, dtype=torch.long)
        self.ci = torch.as_tensor(system.ci, dtype=torch.float64)
        self.set_params(params)

    def set_params(self, params):
        flat = torch.as_tensor(params, dtype=torch.float64)
        self.flat = flat
        self.p = Params(flat, self.R.shape[0], self.system.n_mo, self.net)

    # -- pieces --------------------------------------------------------------
    def slater_logdets(self, r, f, cusp_s0=None):
        """Per determinant and spin: (sign, ln|det|) of A_p^sigma."""
        phi = self.orbitals(r, cusp_s0)  # [B, N, M]
        phit = phi * f
        out = []
        for sl, dets in ((slice(0, self.n_up), self.det_up),
                         (slice(self.n_up, self.n_up + self.n_down), self.det_down)):
            n = sl.stop - sl.start
            if n == 0:
                B, P = r.shape[0], dets.shape[0]
                out.append((torch.ones(B, P, dtype=r.dtype), torch.zeros(B, P, dtype=r.dtype)))
                continue
            blk = phit[:, sl, :]  # [B, n, M]  (electron i, orbital mu)
            A = blk[:, :, dets].permute(0, 2, 3, 1)  # [B, P, k, i]
            s, l = torch.linalg.slogdet(A)
            out.append((s, l))
        return out

    def log_psi(self, r, params=None, cusp_s0=None):
        """(ln|psi| [B], sign [B]) for r [B, N, 3]; cusp_s0 optionally
        replaces the orbital values at the nuclei of the cusp correction."""
        if params is not None:
            p = Params(params, self.R.shape[0], self.system.n_mo, self.net)
        else:
            p = self.p
        gamma = electronic_cusp(r, self.n_up)
        flags = int(getattr(self.net, "flags", 0))
        if flags & 3 == 3:  # neither head: the network does not enter
            J, f = torch.zeros(r.shape[0], dtype=r.dtype), torch.ones(r.shape[0], r.shape[1], self.system.n_mo,
                                                                        dtype=r.dtype)
            J = J + 0.0 * p.flat.sum()  # keep the parameters in the graph (zero gradient)
        else:
            J, f = jastrow_backflow(r, self.R, self.n_up, p, self.net)
            if flags & 1:  # variant without Jastrow factor: J = 0
                J = 0.0 * J
            if flags & 2:  # variant without backflow: f = 1
                f = 1.0 + 0.0 * f
        (su, lu), (sd, ld) = self.slater_logdets(r, f, cusp_s0)
        lc = torch.log(torch.abs(self.ci))
        l_p = lc + lu + ld
        s_p = torch.sign(self.ci) * su * sd
        m = torch.max(l_p, dim=-1).values
        m = torch.where(torch.isfinite(m), m, torch.zeros_like(m))
        S = (s_p * torch.exp(l_p - m[:, None])).sum(-1)
        log_d = m + torch.log(torch.abs(S))
        return gamma + J + log_d, torch.sign(S)

    def potential(self, r):
        return coulomb_potential(r, self.R, self.Z)

    def evaluate(self, r):
        """Full hot-path outputs: ln|psi|, sign, grad [B,N,3], lap, E_loc."""
        r = torch.as_tensor(r, dtype=torch.float64)
        with torch.no_grad():
            lp, sg = self.log_psi(r)
        g, lap, el = local_energy_from(lambda x: self.log_psi(x)[0], self.potential, r)
        return {"logabs": lp, "sign": sg, "grad": g, "lap": lap, "eloc": el}

    def param_grad_full(self, r, ct_logabs=None, ct_grad=None, ct_lap=None, ct_eloc=None):
        """sum_w of the cotangents times the parameter derivatives of the
        outputs: ln|psi_w|, its coordinate gradient [N,3], its Laplacian and
        E_loc (each cotangent may be None = zero).  V does not depend on the
        parameters, so d E_loc / d theta = -1/2 d(lap + |grad|^2) / d theta:
        the Laplacian's second-order terms enter through a third autograd
        level (the Laplacian graph is kept with create_graph)."""
        r = torch.as_tensor(r, dtype=torch.float64)
        B = r.shape[0]
        th = self.flat.detach().clone().requires_grad_(True)
        rr = r.detach().clone().requires_grad_(True)
        lp, _ = self.log_psi(rr, th)
        (g,) = torch.autograd.grad(lp.sum(), rr, create_graph=True)
        gf = g.reshape(B, -1)
        lap = torch.zeros(B, dtype=torch.float64)
        for a in range(gf.shape[1]):
            (h,) = torch.autograd.grad(gf[:, a].sum(), rr, create_graph=True)
            lap = lap + h.reshape(B, -1)[:, a]
        loss = torch.zeros((), dtype=torch.float64)
        t = lambda x: torch.as_tensor(x, dtype=torch.float64)
        if ct_logabs is not None:
            loss = loss + (t(ct_logabs) * lp).sum()
        if ct_grad is not None:
            loss = loss + (t(ct_grad).reshape(B, -1) * gf).sum()
        if ct_lap is not None:
            loss = loss + (t(ct_lap) * lap).sum()
        if ct_eloc is not None:
            loss = loss + (t(ct_eloc) * (-0.5) * (lap + (gf ** 2).sum(-1))).sum()
        if not loss.requires_grad:
            return torch.zeros_like(th)
        (gth,) = torch.autograd.grad(loss, th)
        return gth

    def cusp_value_grad(self, r, cotangent):
        """sum_w cotangent_w d ln|psi_w| / d s0[I, mu] for the orbital values
        at the nuclei of the cusp correction (Methods, "Cusp conditions": the
        paper optimizes them); zero for pairs that are not corrected."""
        r = torch.as_tensor(r, dtype=torch.float64)
        s0 = self.orbitals.s0.detach().clone().requires_grad_(True)
        lp, _ = self.log_psi(r, cusp_s0=s0)
        (g,) = torch.autograd.grad((lp * torch.as_tensor(cotangent, dtype=torch.float64)).sum(), s0,
                                   allow_unused=True)
        return torch.zeros_like(s0) if g is None else g

    def param_grad_logabs(self, r, cotangent):
        """sum_w cotangent_w * d ln|psi_w| / d theta (value-path adjoint)."""
        r = torch.as_tensor(r, dtype=torch.float64)
        th = self.flat.detach().clone().requires_grad_(True)
        lp, _ = self.log_psi(r, th)
        (gth,) = torch.autograd.grad((lp * torch.as_tensor(cotangent, dtype=torch.float64)).sum(), th)
        return gth
