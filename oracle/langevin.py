"""Langevin Monte Carlo sampling of |psi|^2 (oracle; test infrastructure).

Methods, "Ansatz optimization": electron configurations are sampled with the
Langevin (drift-diffusion) Monte Carlo of Umrigar, Nightingale and Runge
(J. Chem. Phys. 99, 2865 (1993)), simplified: instead of their radial step
proposal, the step length is clipped so that it stays shorter than the
distance to the nearest nucleus, which can then never be overshot.  Table 2:
target acceptance 57 %, 50 discarded steps, 1 decorrelation step,
resampling every 100 iterations.

One step, for all electrons of a walker at once:
  drift    d_i(r) = tau grad_i ln|psi|(r), rescaled to length
           min(|d_i|, dist_i) with dist_i = min_I |r_i - R_I|
  proposal r' = m(r) + sqrt(tau) xi,  m(r) = r + d(r),  xi ~ N(0, 1)
  accept   u < A,  ln A = 2 (ln|psi(r')| - ln|psi(r)|)
                        - (|r - m(r')|^2 - |r' - m(r)|^2) / (2 tau)
           (Metropolis-Hastings with the Gaussian proposal densities in both
           directions, so |psi|^2 is the stationary distribution)
  tau      after each step, tau <- tau exp(k (a - a*)) with a the batch
           acceptance, a* the target and k the adaptation rate

Readings (listed in the design notes): the clipping acts on the drift part
of each electron's step; moves are all-electron; the adaptation rule is the
multiplicative one above.  The random numbers are those of the Metropolis
step (Philox4x32-10, counter (walker, step, call, 0); normals by Box-Muller,
acceptance uniform from call 0xFFFFFFFF).

Pinned by: the stationary variance of a Gaussian |psi|^2 (the unadjusted
drift-diffusion chain is biased by 25 % at the tested step), the mean radius
3/2 bohr of the hydrogen ground state with clipping active, and the clipping
bound on a constructed configuration (tests).
"""

import math

import torch


def clipped_drift(r, grad, nuc, tau):
    """d_i = tau grad_i, each electron's vector rescaled to at most its
    distance to the nearest nucleus.  r, grad [B, N, 3]; nuc [Nn, 3]."""
    d = tau * grad
    if nuc.shape[0] == 0:
        return d
    dist = torch.cdist(r.reshape(-1, 3), nuc).min(dim=1).values.reshape(r.shape[0], r.shape[1])
    norm = torch.linalg.norm(d, dim=-1)
    scale = torch.where(norm > dist, dist / torch.where(norm > 0, norm, torch.ones_like(norm)),
                        torch.ones_like(norm))
    return d * scale[..., None]


def langevin_step(logpsi_grad, r, la, g, nuc, tau, xi, u):
    """One step.  logpsi_grad(r) -> (ln|psi| [B], grad [B, N, 3]); (la, g)
    are those at r; xi [B, N*3] normals, u [B] uniforms.  Returns
    (r, la, g, accepted [B])."""
    r = torch.as_tensor(r, dtype=torch.float64)
    B = r.shape[0]
    xi = torch.as_tensor(xi, dtype=torch.float64).reshape(r.shape)
    m = r + clipped_drift(r, g, nuc, tau)
    rp = m + math.sqrt(tau) * xi
    lap, gp = logpsi_grad(rp)
    mp = rp + clipped_drift(rp, gp, nuc, tau)
    qf = ((rp - m) ** 2).reshape(B, -1).sum(-1)
    qb = ((r - mp) ** 2).reshape(B, -1).sum(-1)
    log_a = 2.0 * (lap - la) - (qb - qf) / (2.0 * tau)
    acc = torch.as_tensor(u, dtype=torch.float64) < torch.exp(log_a)
    r_new = torch.where(acc[:, None, None], rp, r)
    la_new = torch.where(acc, lap, la)
    g_new = torch.where(acc[:, None, None], gp, g)
    return r_new, la_new, g_new, acc


def adapt_tau(tau, acceptance, target=0.57, rate=1.0):
    return tau * math.exp(rate * (acceptance - target))


def langevin_run(logpsi_grad, r, nuc, tau, randoms, n_steps, target=0.57, rate=1.0):
    """n_steps steps; randoms(k) -> (xi, u) for step k.  Returns
    (r, acceptance per step, tau used per step, final tau)."""
    r = torch.as_tensor(r, dtype=torch.float64)
    la, g = logpsi_grad(r)
    accs, taus = [], []
    for k in range(n_steps):
        xi, u = randoms(k)
        r, la, g, acc = langevin_step(logpsi_grad, r, la, g, nuc, tau, xi, u)
        a = float(acc.double().mean())
        accs.append(a)
        taus.append(tau)
        tau = adapt_tau(tau, a, target, rate)
    return r, accs, taus, tau


def oracle_logpsi_grad(oracle):
    """(ln|psi|, d ln|psi| / d r) of the ansatz by one autograd pass."""
    def f(r):
        x = torch.as_tensor(r, dtype=torch.float64).detach().clone().requires_grad_(True)
        lp, _ = oracle.log_psi(x)
        (g,) = torch.autograd.grad(lp.sum(), x)
        return lp.detach(), g.detach()
    return f
