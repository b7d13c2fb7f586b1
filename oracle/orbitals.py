"""Gaussian-orbital baseline with nuclear cusp correction (oracle; test
infrastructure).

The molecular orbitals phi_mu come from a (multireference) Hartree-Fock
calculation in a Gaussian basis (Results, "Hartree-Fock baseline"; Methods,
"Computational details") and are corrected at the nuclei with the scheme of
Ma et al. (J. Chem. Phys. 122, 224322, 2005), with the orbital value at each
nucleus as a variational input (Methods, "Cusp conditions").

Readings taken where the paper is silent (each listed in the design notes):
  * primitive (uncontracted) normalised s and p Gaussians, basis order =
    shell order then (x, y, z);
  * per nucleus I and MO mu, the on-centre s part s(rho) (s shells on I) is
    replaced for rho = |r - R_I| < r_cusp by sign(s0) exp(p(rho)),
    p = a0 + a1 rho + ... + a4 rho^4, with a0 = ln|s0|,
    a1 = -Z_I (eta(R_I) + s0) / s0 (cusp of the full orbital; eta is the rest
    of the orbital), and a2..a4 matching value, slope and curvature of ln|s|
    at r_cusp; no shift constant;
  * a (nucleus, MO) pair is corrected only if the nucleus carries s shells,
    s0 != 0 and s(r_cusp) has the sign of s0; otherwise it is left as is.

Parity pins:
  gto_basis          pinned: normalisation integrals by quadrature, analytic
                     gradient/Laplacian of a Gaussian (tests).
  cusp coefficients  pinned: C^2 continuity at r_cusp, and the spherically
                     averaged slope -Z at the nucleus (tests).
"""

import math

import torch


def gto_basis(r: torch.Tensor, centers: torch.Tensor, shell_center, shell_l, shell_exp):
    """chi_b(r_i) for every electron and basis function.  r: [..., 3];
    returns [..., n_basis]."""
    out = []
    for c, l, a in zip(shell_center, shell_l, shell_exp):
        d = r - centers[int(c)]
        r2 = (d**2).sum(-1)
        g = torch.exp(-a * r2)
        if int(l) == 0:
            out.append((2 * a / math.pi) ** 0.75 * g)
        elif int(l) == 1:
            norm = (128 * a**5 / math.pi**3) ** 0.25
            for k in range(3):
                out.append(norm * d[..., k] * g)
        else:
            raise ValueError("only s and p shells")
    return torch.stack(out, -1)


class CuspCorrectedOrbitals:
    """phi_mu(r_i) with the nuclear cusp correction applied."""

    def __init__(self, system):
        self.R = torch.as_tensor(system.nuc_xyz, dtype=torch.float64)
        self.Z = torch.as_tensor(system.charge, dtype=torch.float64)
        self.sc = [int(x) for x in system.shell_center]
        self.sl = [int(x) for x in system.shell_l]
        self.se = [float(x) for x in system.shell_exp]
        self.C = torch.as_tensor(system.mo_coeff, dtype=torch.float64)
        self.rc = float(system.cusp_radius)
        self.n_mo = self.C.shape[1]
        # basis index of each s shell
        idx, self.s_index = 0, []
        for c, l in zip(self.sc, self.sl):
            if l == 0:
                self.s_index.append((c, idx))
            idx += 2 * l + 1
        nuc_val = None if system.cusp_nuc_value is None else torch.as_tensor(
            system.cusp_nuc_value, dtype=torch.float64)
        self.corr = []  # (I, mu, sign, alpha[5], [(exp, coef*norm)])
        if self.rc > 0:
            self._setup(nuc_val)

    def _s_terms(self, I, mu):
        terms = []
        for (c, b) in self.s_index:
            if c == I:
                a = self.se[self._shell_of_basis(b)]
                terms.append((a, float(self.C[b, mu]) * (2 * a / math.pi) ** 0.75))
        return terms

    def _shell_of_basis(self, b):
        idx = 0
        for s, l in enumerate(self.sl):
            if idx == b:
                return s
            idx += 2 * l + 1
        raise KeyError(b)

    @staticmethod
    def _s_radial(terms, rho):
        return sum(cn * torch.exp(-a * rho**2) for a, cn in terms)

    def _setup(self, nuc_val):
        self.s0 = torch.zeros(self.R.shape[0], self.n_mo, dtype=torch.float64)
        for I in range(self.R.shape[0]):
            phi_at_nuc = self.uncorrected(self.R[I][None])[0]  # [n_mo]
            for mu in range(self.n_mo):
                terms = self._s_terms(I, mu)
                if not terms:
                    continue
                s_at0 = float(self._s_radial(terms, torch.zeros((), dtype=torch.float64)))
                s0 = s_at0 if nuc_val is None else float(nuc_val[I, mu])
                self.s0[I, mu] = s0
                eta0 = float(phi_at_nuc[mu]) - s_at0
                # value, slope and curvature of s at r_cusp by autograd
                rho = torch.tensor(self.rc, dtype=torch.float64, requires_grad=True)
                s = self._s_radial(terms, rho)
                (ds,) = torch.autograd.grad(s, rho, create_graph=True)
                (d2s,) = torch.autograd.grad(ds, rho)
                s, ds, d2s = float(s.detach()), float(ds.detach()), float(d2s)
                if s0 == 0.0 or s * s0 <= 0.0:
                    continue
                X1, X2 = math.log(abs(s)), ds / s
                X3 = d2s / s - X2**2
                self.corr.append((I, mu, math.copysign(1.0, s0), (eta0, X1, X2, X3), terms))

    def _alpha(self, I, mu, s0, fit):
        """Coefficients a0..a4 of the corrected s part for nucleus value s0
        (a torch scalar, so that they can be differentiated in s0)."""
        eta0, X1, X2, X3 = fit
        rc = self.rc
        a0 = torch.log(torch.abs(s0))
        a1 = -float(self.Z[I]) * (eta0 + s0) / s0
        M = torch.tensor([[rc**2, rc**3, rc**4],
                          [2 * rc, 3 * rc**2, 4 * rc**3],
                          [2.0, 6 * rc, 12 * rc**2]], dtype=torch.float64)
        rhs = torch.stack([X1 - a0 - a1 * rc, X2 - a1, torch.zeros_like(a0) + X3])
        a234 = torch.linalg.solve(M, rhs)
        return [a0, a1, a234[0], a234[1], a234[2]]

    def uncorrected(self, r: torch.Tensor):
        chi = gto_basis(r, self.R, self.sc, self.sl, self.se)
        return chi @ self.C

    def __call__(self, r: torch.Tensor, s0=None):
        """r: [B, N, 3] -> phi [B, N, n_mo].  s0 [n_nuc, n_mo] (optional,
        may require grad) replaces the nucleus values of the corrected
        pairs; which pairs are corrected is fixed at set-up."""
        phi = self.uncorrected(r)
        if not self.corr:
            return phi
        s0 = self.s0 if s0 is None else s0
        cols = [phi[..., mu] for mu in range(self.n_mo)]
        for I, mu, sgn, fit, terms in self.corr:
            alpha = self._alpha(I, mu, s0[I, mu], fit)
            rho = torch.sqrt(((r - self.R[I]) ** 2).sum(-1))
            inside = rho < self.rc
            rho_c = torch.where(inside, rho, torch.full_like(rho, self.rc))
            p = sum(alpha[k] * rho_c**k for k in range(5))
            new = sgn * torch.exp(p) - self._s_radial(terms, rho_c)
            cols[mu] = cols[mu] + torch.where(inside, new, torch.zeros_like(new))
        return torch.stack(cols, -1)
