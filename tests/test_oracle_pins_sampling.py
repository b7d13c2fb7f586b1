"""Pins of the oracle's sampling pieces and of the nuclear cusp on every
nucleus of the H10 chain.

  - The Metropolis step (Methods, "Ansatz optimization": walkers sample
    |psi|^2) reproduces exact moments of |psi|^2 for two wavefunctions with
    known densities, and the same chains with the acceptance rule
    u < exp(ln|psi'| - ln|psi|) (exp(Delta) instead of exp(2 Delta)), a
    mistake planted in the oracle here, land on the moments of |psi|
    instead and fail the check.
  - The proposal normals equal Box-Muller values evaluated in 40-digit
    arithmetic from the Philox output words (tests/golden/box_muller_values.txt).
  - The e-n cusp (Methods, "Cusp conditions") at all ten nuclei of H10,
    including the consequence of the one (nucleus, MO) pair the correction
    rule leaves out.
"""

import os

import numpy as np
import pytest
import torch

from oracle import Oracle
from oracle.vmc import metropolis_randoms, metropolis_step
from synth import make_config

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


class _Toy:
    """ln|psi| provider for metropolis_step: psi = exp(logpsi(r))."""

    def __init__(self, logpsi):
        self.logpsi = logpsi

    def log_psi(self, r):
        lp = self.logpsi(torch.as_tensor(r, dtype=torch.float64))
        return lp, torch.ones_like(lp)


def _gauss(a):
    return lambda r: -a * (r ** 2).sum((1, 2))


def _hydrogen(r):
    return -torch.linalg.norm(r, dim=-1).sum(-1)


def _chain(toy, B, n_steps, sigma, seed):
    g = torch.Generator().manual_seed(seed)
    r = torch.randn(B, 1, 3, generator=g, dtype=torch.float64)
    lp, _ = toy.log_psi(r)
    accepted = []
    for _ in range(n_steps):
        xi = torch.randn(B, 3, generator=g, dtype=torch.float64)
        u = torch.rand(B, generator=g, dtype=torch.float64)
        r, lp, acc = metropolis_step(toy, r, lp, xi, u, sigma=sigma)
        accepted.append(float(acc.double().mean()))
    return r, accepted


def _halved(toy):
    """The planted mistake: a chain that accepts with exp(Delta) is the
    correct chain for psi^(1/2), i.e. for ln|psi| halved."""
    return _Toy(lambda r: 0.5 * toy.logpsi(r))


def test_metropolis_samples_gaussian_density():
    """|psi|^2 = exp(-2 a r^2): every coordinate has variance 1/(4a)."""
    a = 0.5
    toy = _Toy(_gauss(a))
    r, acc = _chain(toy, 4000, 150, 1.0, 5)
    var = float((r ** 2).mean())
    assert abs(var - 1 / (4 * a)) < 0.025, var
    assert 0.2 < np.mean(acc[-50:]) < 0.9
    # the exp(Delta) rule samples |psi| = exp(-a r^2): variance 1/(2a)
    r_bad, _ = _chain(_halved(toy), 4000, 150, 1.0, 5)
    var_bad = float((r_bad ** 2).mean())
    assert abs(var_bad - 1 / (2 * a)) < 0.05, var_bad
    assert abs(var_bad - 1 / (4 * a)) > 0.3


def test_metropolis_samples_hydrogen_density():
    """Hydrogen ground state psi = exp(-r): <r> = 3/2 bohr under |psi|^2
    (and 3 bohr under |psi|, what the exp(Delta) rule would sample)."""
    toy = _Toy(_hydrogen)
    r, _ = _chain(toy, 4000, 200, 0.8, 7)
    mean_r = float(torch.linalg.norm(r, dim=-1).mean())
    assert abs(mean_r - 1.5) < 0.05, mean_r
    r_bad, _ = _chain(_halved(toy), 4000, 200, 0.8, 7)
    mean_bad = float(torch.linalg.norm(r_bad, dim=-1).mean())
    assert abs(mean_bad - 3.0) < 0.12, mean_bad
    assert abs(mean_bad - 1.5) > 1.0


def test_metropolis_step_acceptance_rule_on_fixed_draws():
    """One step with hand-chosen uniforms: ln|psi'| - ln|psi| = -0.25 gives
    the acceptance probability exp(-0.5) = 0.6065; u just below and just above
    it decide."""
    toy = _Toy(lambda r: -(r[:, 0, 0]))  # ln|psi| = -x
    r = torch.zeros(2, 1, 3, dtype=torch.float64)
    lp, _ = toy.log_psi(r)
    xi = torch.tensor([[0.25, 0.0, 0.0], [0.25, 0.0, 0.0]], dtype=torch.float64)
    p = float(np.exp(-0.5))
    u = torch.tensor([p - 1e-9, p + 1e-9], dtype=torch.float64)
    r_new, lp_new, acc = metropolis_step(toy, r, lp, xi, u, sigma=1.0)
    assert acc.tolist() == [True, False]
    assert float(r_new[0, 0, 0]) == 0.25 and float(r_new[1, 0, 0]) == 0.0
    assert float(lp_new[0]) == -0.25 and float(lp_new[1]) == 0.0


def _box_muller_rows():
    with open(os.path.join(GOLDEN, "box_muller_values.txt")) as fh:
        rows = [l.split() for l in fh if l.strip() and not l.startswith("#")]
    assert len(rows) == 2
    return rows


def test_metropolis_normals_hand_evaluated_box_muller():
    """The proposal normals of two fixed counters equal the Box-Muller pair
    of the counter's uniforms evaluated in 40-digit arithmetic; call j fills
    coordinates 2j (cosine) and 2j + 1 (sine)."""
    for row in _box_muller_rows():
        seed, w, step, call = int(row[0], 16), int(row[1]), int(row[2]), int(row[3])
        xi0, xi1 = float(row[8]), float(row[9])
        xi, _ = metropolis_randoms(seed, step, w + 1, 2 * call + 2)
        assert abs(xi[w, 2 * call] - xi0) < 4e-15 * max(1.0, abs(xi0))
        assert abs(xi[w, 2 * call + 1] - xi1) < 4e-15 * max(1.0, abs(xi1))


def test_box_muller_words_are_the_published_vector():
    """The first row's Philox words are the published known-answer output
    for counter 0 and key 0."""
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) as fh:
        kat = [l.split() for l in fh if l.strip() and not l.startswith("#")][0]
    assert _box_muller_rows()[0][4:8] == kat[6:10]


# ------------------------------------------------ e-n cusp on H10 ---------
def _cusp_slopes(o, w, nuclei, electrons, ts=(2e-6, 1e-6)):
    """Per (nucleus I, electron e): the Richardson-extrapolated direction
    average of u . grad_e ln|psi| with electron e at R_I + t u, and the
    largest relative change of E_loc between the two distances.  One batched
    oracle call."""
    R = w.system.nuc_xyz
    dirs = np.concatenate([np.eye(3), -np.eye(3)])
    keys = [(I, e, t) for I in nuclei for e in electrons for t in ts]
    rs = np.repeat(w.walkers[:1], 6 * len(keys), 0)
    for k, (I, e, t) in enumerate(keys):
        rs[6 * k:6 * k + 6, e] = R[I] + t * dirs
    out = o.evaluate(rs)
    grad, eloc = out["grad"].numpy(), out["eloc"].numpy()
    res = {}
    for k0 in range(0, len(keys), len(ts)):
        I, e, _ = keys[k0]
        slopes, el = [], []
        for k in range(k0, k0 + len(ts)):
            g = grad[6 * k:6 * k + 6, e]
            slopes.append(np.mean(np.einsum("uc,uc->u", g, dirs)))
            el.append(eloc[6 * k:6 * k + 6])
        s0 = (slopes[1] * ts[0] - slopes[0] * ts[1]) / (ts[0] - ts[1])
        res[(I, e)] = (s0, float(np.max(np.abs(el[1] - el[0]) / (1 + np.abs(el[1])))))
    return res


def _uncorrected_pairs(o, system):
    on = {(I, mu) for I, mu, *_ in o.orbitals.corr}
    return [(I, mu) for I in range(system.n_nuc) for mu in range(system.n_mo) if (I, mu) not in on]


def _drop_dets(system, keep):
    import dataclasses
    return dataclasses.replace(system, det_up=system.det_up[keep], det_down=system.det_down[keep],
                               ci=system.ci[keep])


def test_p5_nuclear_cusp_every_h10_nucleus():
    """Every nucleus of the H10 chain, for an up and a down electron: slope
    -> -Z and E_loc finite, once the one determinant that occupies the
    orbital left uncorrected at nucleus 1 (MO 6, whose on-centre s part
    changes sign inside r_cusp; it is occupied only in the down block of
    determinant 5) is removed from the expansion."""
    w = make_config(3, n_walkers=2)
    o = Oracle(w.system, w.net, w.params)
    assert _uncorrected_pairs(o, w.system) == [(1, 6)]
    keep = [p for p in range(w.system.n_det)
            if 6 not in w.system.det_up[p] and 6 not in w.system.det_down[p]]
    assert keep == [p for p in range(w.system.n_det) if p != 5]
    o2 = Oracle(_drop_dets(w.system, keep), w.net, w.params)
    res = _cusp_slopes(o2, w, range(w.system.n_nuc), (0, w.system.n_up))
    for (I, e), (s0, de) in res.items():
        assert abs(s0 + w.system.charge[I]) < 1e-3 * w.system.charge[I], (I, e, s0)
        assert de < 1e-2, (I, e, de)


def test_p5_consequence_of_the_uncorrected_pair():
    """With the full expansion the cusp holds at every nucleus for the up
    electron and at the nine other nuclei for the down electron; at nucleus 1
    the down electron sees determinant 5, which occupies the uncorrected MO:
    the slope misses -Z and E_loc diverges like 1/t there (the behaviour the
    correction removes)."""
    w = make_config(3, n_walkers=2)
    o = Oracle(w.system, w.net, w.params)
    res = _cusp_slopes(o, w, range(w.system.n_nuc), (0, w.system.n_up))
    for (I, e), (s0, de) in res.items():
        if (I, e) == (1, w.system.n_up):
            assert abs(s0 + 1.0) > 1e-2, s0
            assert de > 0.1, de
        else:
            assert abs(s0 + 1.0) < 1e-3, (I, e, s0)
            assert de < 1e-2, (I, e, de)
