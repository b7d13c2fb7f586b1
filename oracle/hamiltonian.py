"""Coulomb potential and electronic cusp factor (oracle; test infrastructure).

Parity pins:
  coulomb_potential   pinned: hydrogen-like closed forms (exact E_loc tests)
                      and a two-charge hand value in the tests.
  electronic_cusp     pinned: e-e cusp test (averaged slope of ln|psi| -> 1/2
                      for opposite spins, bounded E_loc) in the tests.
"""

import torch


def pair_distances(r: torch.Tensor):
    """|r_i - r_j| for all ordered pairs, with 1 on the diagonal so that the
    (masked-out) self pairs stay differentiable.  r: [B, N, 3]."""
    B, N, _ = r.shape
    diff = r[:, :, None, :] - r[:, None, :, :]
    eye = torch.eye(N, dtype=r.dtype)
    return torch.sqrt((diff**2).sum(-1) + eye)


def nuclear_distances(r: torch.Tensor, R: torch.Tensor):
    """|r_i - R_I|, [B, N, N_nuc]."""
    return torch.sqrt(((r[:, :, None, :] - R[None, None, :, :]) ** 2).sum(-1))


def coulomb_potential(r: torch.Tensor, R: torch.Tensor, Z: torch.Tensor):
    """Potential part of the electronic Hamiltonian (Methods, "Ansatz
    optimization": E_loc = H psi / psi): electron-electron repulsion minus
    electron-nucleus attraction plus the constant nuclear repulsion (the
    energies of Table 1 are total energies)."""
    B, N, _ = r.shape
    d_ee = pair_distances(r)
    iu = torch.triu_indices(N, N, offset=1)
    v_ee = (1.0 / d_ee[:, iu[0], iu[1]]).sum(-1) if N > 1 else r.new_zeros(B)
    d_en = nuclear_distances(r, R)
    v_en = -(Z[None, None, :] / d_en).sum((-1, -2))
    n_nuc = R.shape[0]
    v_nn = r.new_zeros(())
    for I in range(n_nuc):
        for J in range(I + 1, n_nuc):
            v_nn = v_nn + Z[I] * Z[J] / torch.linalg.norm(R[I] - R[J])
    return v_ee + v_en + v_nn


def electronic_cusp(r: torch.Tensor, n_up: int):
    """gamma(r) = sum_{i<j} -c_ij / (1 + |r_i - r_j|)  (Methods, "Cusp
    conditions").  The paper says c_ij is 1/2 or 1/4 depending on the spins;
    the reading here (Kato's conditions) is 1/2 for opposite spins and 1/4
    for same spins."""
    B, N, _ = r.shape
    if N < 2:
        return r.new_zeros(B)
    d = pair_distances(r)
    spin = torch.tensor([0] * n_up + [1] * (N - n_up))
    same = spin[:, None] == spin[None, :]
    c = torch.where(same, torch.tensor(0.25, dtype=r.dtype), torch.tensor(0.5, dtype=r.dtype))
    iu = torch.triu_indices(N, N, offset=1)
    return (-c[iu[0], iu[1]] / (1.0 + d[:, iu[0], iu[1]])).sum(-1)
