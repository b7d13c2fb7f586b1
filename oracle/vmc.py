"""VMC update pieces around the hot path (oracle; test infrastructure).

  clip_local_energy   smooth clipping of E_loc (Methods, "Ansatz
                      optimization": logarithmic growth outside a window of q
                      times the mean deviation from the batch median)
  energy_gradient     Hermitian gradient estimator, eq. "trainig":
                      grad L = 2 E[(E_loc - L) grad_theta ln|psi|]
  adamw_step          AdamW (decoupled weight decay) with lr decay
                      lr_t = lr0 / (1 + t / t0) (Table 2)
  metropolis_step     all-electron Gaussian Metropolis move on |psi|^2
  philox4x32_10       the counter-based generator of Salmon et al. (SC'11),
                      used by the serving step to draw proposals

Readings (listed in the design notes): median of an even batch is the mean of
the two middle values; clip(E) = m + sgn(E - m) w (1 + ln(|E - m| / w)) for
|E - m| > w with w = q mean|E - m|; beta = (0.9, 0.999), eps = 1e-8, weight
decay 0.01; proposals r' = r + sigma xi over all electrons, accepted when
u < exp(2 (ln|psi'| - ln|psi|)).

Parity pins: Philox against the published known-answer vectors; the
proposal normals against Box-Muller values evaluated in 40-digit arithmetic
from the Philox words; the Metropolis step against the exact moments of
|psi|^2 for a Gaussian (variance 1/(4a)) and for hydrogen (<r> = 3/2), with
a planted exp(Delta) acceptance shown to fail those checks; AdamW against
torch.optim.AdamW; clipping by continuity and fixed points; the gradient
estimator against finite differences of the surrogate loss (tests).
"""

import math

import numpy as np
import torch


def batch_median(e: torch.Tensor):
    s, _ = torch.sort(e)
    B = s.shape[0]
    if B % 2:
        return s[B // 2]
    return 0.5 * (s[B // 2 - 1] + s[B // 2])


def clip_local_energy(e: torch.Tensor, q: float = 5.0):
    e = torch.as_tensor(e, dtype=torch.float64)
    m = batch_median(e)
    w = q * torch.abs(e - m).mean()
    dev = torch.abs(e - m)
    if float(w) == 0.0:
        return e.clone()
    clipped = m + torch.sign(e - m) * w * (1.0 + torch.log(torch.clamp(dev / w, min=1.0)))
    return torch.where(dev <= w, e, clipped)


def energy_gradient(oracle, r, eloc, q: float = 5.0):
    """Returns (grad_theta [n_params], L, clipped E_loc) for one batch."""
    ec = clip_local_energy(eloc, q)
    L = ec.mean()
    B = ec.shape[0]
    ct = 2.0 / B * (ec - L)
    return oracle.param_grad_logabs(r, ct), L, ec


def adamw_step(theta, grad, m, v, t, lr0=0.01, t0=200.0, beta1=0.9, beta2=0.999,
               eps=1e-8, wd=0.01):
    """One AdamW update at step t (t = 0 for the first update).  Returns new
    (theta, m, v)."""
    lr = lr0 / (1.0 + t / t0)
    m = beta1 * m + (1 - beta1) * grad
    v = beta2 * v + (1 - beta2) * grad * grad
    mh = m / (1 - beta1 ** (t + 1))
    vh = v / (1 - beta2 ** (t + 1))
    theta = theta * (1 - lr * wd) - lr * mh / (torch.sqrt(vh) + eps)
    return theta, m, v


# --- Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) ----------------------
_M0, _M1 = 0xD2511F53, 0xCD9E8D57
_W0, _W1 = 0x9E3779B9, 0xBB67AE85
_MASK = 0xFFFFFFFF


def philox4x32_10(ctr, key):
    """ctr: 4 uint32, key: 2 uint32 -> 4 uint32 (pure Python)."""
    c0, c1, c2, c3 = (int(x) & _MASK for x in ctr)
    k0, k1 = (int(x) & _MASK for x in key)
    for rnd in range(10):
        p0 = _M0 * c0
        p1 = _M1 * c2
        hi0, lo0 = p0 >> 32, p0 & _MASK
        hi1, lo1 = p1 >> 32, p1 & _MASK
        c0, c1, c2, c3 = (hi1 ^ c1 ^ k0) & _MASK, lo1, (hi0 ^ c3 ^ k1) & _MASK, lo0
        k0, k1 = (k0 + _W0) & _MASK, (k1 + _W1) & _MASK
    return c0, c1, c2, c3


def u53(a, b):
    """Uniform double in (0, 1) from two 32-bit words."""
    return ((a >> 5) * 67108864.0 + (b >> 6) + 0.5) * (1.0 / 9007199254740992.0)


ACCEPT_CALL = 0xFFFFFFFF


def metropolis_randoms(seed: int, step: int, n_walkers: int, n_coord: int):
    """Proposal normals xi [B, n_coord] and acceptance uniforms u [B] for one
    serving step.  Counter = (walker, step, call, 0), key = seed (lo, hi).
    Call j gives two uniforms -> Box-Muller pair (xi_2j, xi_2j+1); the
    acceptance uniform uses call 0xFFFFFFFF."""
    key = (seed & _MASK, (seed >> 32) & _MASK)
    xi = np.empty((n_walkers, n_coord))
    u = np.empty(n_walkers)
    n_calls = (n_coord + 1) // 2
    for w in range(n_walkers):
        for j in range(n_calls):
            x = philox4x32_10((w, step, j, 0), key)
            u1, u2 = u53(x[0], x[1]), u53(x[2], x[3])
            rad = math.sqrt(-2.0 * math.log(u1))
            xi[w, 2 * j] = rad * math.cos(2 * math.pi * u2)
            if 2 * j + 1 < n_coord:
                xi[w, 2 * j + 1] = rad * math.sin(2 * math.pi * u2)
        x = philox4x32_10((w, step, ACCEPT_CALL, 0), key)
        u[w] = u53(x[0], x[1])
    return xi, u


def metropolis_step(oracle, r, logabs, xi, u, sigma=0.3):
    """Returns (r_new, logabs_new, accepted [B] bool)."""
    r = torch.as_tensor(r, dtype=torch.float64)
    B = r.shape[0]
    prop = r + sigma * torch.as_tensor(xi, dtype=torch.float64).reshape(r.shape)
    with torch.no_grad():
        lp_new, _ = oracle.log_psi(prop)
    acc = torch.as_tensor(u, dtype=torch.float64) < torch.exp(2.0 * (lp_new - torch.as_tensor(logabs)))
    r_new = torch.where(acc[:, None, None], prop, r)
    l_new = torch.where(acc, lp_new, torch.as_tensor(logabs, dtype=torch.float64))
    return r_new, l_new, acc
