"""Neural Jastrow factor and backflow (oracle; test infrastructure).

SchNet-style electron embeddings with three message channels (same-spin
electrons +, opposite-spin electrons -, nuclei n), per-channel filter
networks w, a shared h and per-channel receiving networks g, trainable
nuclear embeddings Y shared across iterations, and cuspless distance
features (Methods, "PauliNet extension of SchNet"; Results, "Robust deep
Jastrow factor and backflow").

Readings taken where the paper is silent (each listed in the design notes):
  * q_k = k / (K - 1) spans [0, 1] (endpoints included), r_c = 10 bohr;
  * activation = shifted softplus ssp(x) = ln(e^x / 2 + 1 / 2) between
    layers, none after the last layer; h and g are single Linear layers;
  * w: Linear(K, D_z) -> ssp -> Linear(D_z, D_z);
    eta, kappa: Linear(D_x, D_x) -> ssp -> Linear(D_x, D_x) -> ssp ->
    Linear(D_x, out);
  * one initial embedding x0 for all electrons;
  * backflow f = 1 + kappa(x_i), so that a network with small weights is a
    perturbation of the Hartree-Fock baseline.

Flat parameter blob (Linear is y = x W + b with W stored [in][out]
row-major), in this order:
  x0[D_x], Y[N_nuc][D_z];
  per layer: for c in (+, -, n): w1W[K][D_z] w1b[D_z] w2W[D_z][D_z] w2b[D_z];
             hW[D_x][D_z] hb[D_z];
             for c in (+, -, n): gW[D_z][D_x] gb[D_x];
  eta:   W1[D_x][D_x] b1 W2[D_x][D_x] b2 W3[D_x][1] b3;
  kappa: W1[D_x][D_x] b1 W2[D_x][D_x] b2 W3[D_x][M] b3.

Parity pins:
  features       pinned: e_k(0) = e_k'(0) = 0 and e_k''(0) closed form.
  network        pinned only by structure: permutation invariance of J and
                 equivariance of f, rotation/translation invariance,
                 cusplessness at coalescence, a constant-filter special case
                 with a hand-derivable value, and finite differences.  The
                 values of a seeded network have no external reference
                 ("parity unpinned" beyond those properties).
"""

import math

import torch
import torch.nn.functional as F

from .hamiltonian import nuclear_distances, pair_distances


def ssp(x):
    """Shifted softplus, ln(e^x/2 + 1/2)."""
    return F.softplus(x) - math.log(2.0)


def distance_features(d: torch.Tensor, K: int, r_c: float):
    """e_k(d) = d^2 exp(-d - (d - mu_k)^2 / sigma_k^2), mu_k = r_c q_k^2,
    sigma_k = (1 + r_c q_k) / 7 (Methods, featurisation).  d: [...] ->
    [..., K]."""
    q = torch.linspace(0.0, 1.0, K, dtype=torch.float64) if K > 1 else torch.zeros(1, dtype=torch.float64)
    mu = r_c * q**2
    sigma = (1.0 + r_c * q) / 7.0
    d = d[..., None]
    return d**2 * torch.exp(-d - (d - mu) ** 2 / sigma**2)


class Params:
    """Named views into the flat parameter blob (see module docstring)."""

    def __init__(self, flat: torch.Tensor, n_nuc: int, n_mo: int, net):
        self.flat = flat
        K, X, Z, L = net.n_feat, net.dim_x, net.dim_z, net.n_layers
        self.off = 0

        def take(*shape):
            n = 1
            for s in shape:
                n *= s
            t = flat[self.off:self.off + n].reshape(*shape)
            self.off += n
            return t

        self.x0 = take(X)
        self.Y = take(n_nuc, Z)
        self.layers = []
        for _ in range(L):
            lay = {"w": {}, "g": {}}
            for c in "+-n":
                lay["w"][c] = (take(K, Z), take(Z), take(Z, Z), take(Z))
            lay["h"] = (take(X, Z), take(Z))
            for c in "+-n":
                lay["g"][c] = (take(Z, X), take(X))
            self.layers.append(lay)
        self.eta = (take(X, X), take(X), take(X, X), take(X), take(X, 1), take(1))
        self.kappa = (take(X, X), take(X), take(X, X), take(X), take(X, n_mo), take(n_mo))
        if self.off != flat.numel():
            raise ValueError(f"parameter blob has {flat.numel()} entries, layout needs {self.off}")


def _filter(e, W1, b1, W2, b2):
    return ssp(e @ W1 + b1) @ W2 + b2


def _mlp3(x, W1, b1, W2, b2, W3, b3):
    return ssp(ssp(x @ W1 + b1) @ W2 + b2) @ W3 + b3


def schnet(r, R, n_up, p: Params, net):
    """Electron embeddings x_i^(L) after L interaction iterations."""
    B, N, _ = r.shape
    e_ee = distance_features(pair_distances(r), net.n_feat, net.feat_cutoff)  # [B,N,N,K]
    e_en = distance_features(nuclear_distances(r, R), net.n_feat, net.feat_cutoff)  # [B,N,Nn,K]
    spin = torch.tensor([0] * n_up + [1] * (N - n_up))
    same = (spin[:, None] == spin[None, :]).to(torch.float64) * (1.0 - torch.eye(N, dtype=torch.float64))
    opp = (spin[:, None] != spin[None, :]).to(torch.float64)
    x = p.x0.expand(B, N, -1)
    for lay in p.layers:
        hW, hb = lay["h"]
        h = x @ hW + hb
        w_p = _filter(e_ee, *lay["w"]["+"])
        w_m = _filter(e_ee, *lay["w"]["-"])
        w_n = _filter(e_en, *lay["w"]["n"])
        z_p = torch.einsum("bijz,ij,bjz->biz", w_p, same, h)
        z_m = torch.einsum("bijz,ij,bjz->biz", w_m, opp, h)
        z_n = torch.einsum("biIz,Iz->biz", w_n, p.Y)
        upd = 0
        for c, z in (("+", z_p), ("-", z_m), ("n", z_n)):
            gW, gb = lay["g"][c]
            upd = upd + z @ gW + gb
        x = x + upd
    return x


def jastrow_backflow(r, R, n_up, p: Params, net):
    """J = eta(sum_i x_i^(L)) and f_i = 1 + kappa(x_i^(L)) (Results, eq. for
    J and f).  Returns J [B] and f [B, N, M]."""
    x = schnet(r, R, n_up, p, net)
    J = _mlp3(x.sum(1), *p.eta)[..., 0]
    f = 1.0 + _mlp3(x, *p.kappa)
    return J, f
