"""Synthetic PauliNet workloads (seeded, numpy PCG64).

The paper evaluates H2, LiH, Be, B and H10 with PySCF 6-311G orbitals and a
CASSCF determinant selection (Methods, "Computational details").  Neither
PySCF nor basis-set files are available, so every workload here is a seeded
synthetic analogue with the same structure: primitive s/p Gaussians with
log-uniform exponents, Gaussian-random MO coefficients, an aufbau reference
determinant plus seeded single/double excitations with random CI weights, and
network parameters drawn from N(0, 0.1^2).

Walkers: electron k is assigned to a nucleus by listing every nucleus Z_I times
(nuclei in order) and alternating spins up/down along that list; its position
is drawn from N(R_assigned, sigma^2 I).
"""

from __future__ import annotations

import dataclasses
import itertools
import math
from typing import List, Optional

import numpy as np

CONFIG_NAMES = {
    1: "H2",
    2: "Ne-like",
    3: "H10",
    4: "serving",
    5: "P2-like 30e diatomic",
    6: "Z5 atom (3 up, 2 down)",
    7: "H7 chain (4 up, 3 down)",
}


@dataclasses.dataclass
class System:
    """Molecule, one-electron basis, MOs and determinant expansion."""

    nuc_xyz: np.ndarray  # [n_nuc, 3] bohr
    charge: np.ndarray  # [n_nuc]
    n_up: int
    n_down: int
    shell_center: np.ndarray  # [n_shell] int32
    shell_l: np.ndarray  # [n_shell] int32, 0 = s, 1 = p
    shell_exp: np.ndarray  # [n_shell] float64, one primitive per shell
    mo_coeff: np.ndarray  # [n_basis, n_mo]
    det_up: np.ndarray  # [n_det, n_up] int32
    det_down: np.ndarray  # [n_det, n_down] int32
    ci: np.ndarray  # [n_det]
    cusp_radius: float = 0.1
    cusp_nuc_value: Optional[np.ndarray] = None  # [n_nuc, n_mo] or None

    @property
    def n_elec(self) -> int:
        return self.n_up + self.n_down

    @property
    def n_nuc(self) -> int:
        return int(self.nuc_xyz.shape[0])

    @property
    def n_basis(self) -> int:
        return int(sum(2 * int(l) + 1 for l in self.shell_l))

    @property
    def n_mo(self) -> int:
        return int(self.mo_coeff.shape[1])

    @property
    def n_det(self) -> int:
        return int(self.ci.shape[0])


@dataclasses.dataclass
class NetShape:
    n_feat: int  # K, dimension of the distance features
    feat_cutoff: float  # r_c
    dim_x: int  # D_x
    dim_z: int  # D_z
    n_layers: int  # L
    flags: int = 0  # ansatz variant: 1 = no Jastrow factor, 2 = no backflow


@dataclasses.dataclass
class Workload:
    name: str
    system: System
    net: NetShape
    params: np.ndarray  # flat float64 parameter blob
    walkers: np.ndarray  # [B, N, 3] float64
    precision: str  # nominal precision the workload is quoted in
    seed: int


def param_count(n_nuc: int, n_mo: int, net: NetShape) -> int:
    """Size of the flat parameter blob (sizes only; no arithmetic of the method)."""
    K, X, Z, L = net.n_feat, net.dim_x, net.dim_z, net.n_layers
    filt = K * Z + Z + Z * Z + Z
    layer = 3 * filt + (X * Z + Z) + 3 * (Z * X + X)
    mlp3 = lambda out: X * X + X + X * X + X + X * out + out  # noqa: E731
    return X + n_nuc * Z + L * layer + mlp3(1) + mlp3(n_mo)


def _shells_for(n_nuc_s: List[int], n_nuc_p: List[int], rng) -> tuple:
    centers, ls, exps = [], [], []
    for I, (ns, np_) in enumerate(zip(n_nuc_s, n_nuc_p)):
        for _ in range(ns):
            centers.append(I)
            ls.append(0)
            exps.append(math.exp(rng.uniform(math.log(0.1), math.log(10.0))))
        for _ in range(np_):
            centers.append(I)
            ls.append(1)
            exps.append(math.exp(rng.uniform(math.log(0.1), math.log(10.0))))
    return (
        np.asarray(centers, np.int32),
        np.asarray(ls, np.int32),
        np.asarray(exps, np.float64),
    )


def _spin_candidates(n_occ: int, n_orb: int, max_exc: int):
    """Occupation lists reachable from the aufbau list by <= max_exc
    excitations from the top min(2, n_occ) occupied into the next
    min(8, n_orb - n_occ) virtual orbitals.  Returns {level: [tuple,...]}."""
    ref = tuple(range(n_occ))
    occ_win = list(range(max(0, n_occ - min(2, n_occ)), n_occ))
    vir_win = list(range(n_occ, n_occ + max(0, min(8, n_orb - n_occ))))
    out = {0: [ref]}
    for lvl in range(1, max_exc + 1):
        out[lvl] = []
        for holes in itertools.combinations(occ_win, lvl):
            for parts in itertools.combinations(vir_win, lvl):
                occ = sorted((set(ref) - set(holes)) | set(parts))
                out[lvl].append(tuple(occ))
    return out


def _determinants(n_up, n_down, n_basis, n_det, rng):
    """Aufbau determinant first, then distinct seeded single/double
    excitations (total excitation level 1 or 2 over both spins)."""
    cu = _spin_candidates(n_up, n_basis, 2)
    cd = _spin_candidates(n_down, n_basis, 2)
    cands = []
    for lu in (0, 1, 2):
        for ld in (0, 1, 2):
            if 1 <= lu + ld <= 2:
                for a in cu.get(lu, []):
                    for b in cd.get(ld, []):
                        cands.append((a, b))
    order = rng.permutation(len(cands)) if cands else []
    dets = [(cu[0][0], cd[0][0])]
    for k in order:
        if len(dets) >= n_det:
            break
        dets.append(cands[k])
    P = len(dets)
    det_up = np.asarray([d[0] for d in dets], np.int32).reshape(P, n_up)
    det_down = np.asarray([d[1] for d in dets], np.int32).reshape(P, n_down)
    ci = np.empty(P, np.float64)
    ci[0] = 1.0
    if P > 1:
        ci[1:] = rng.uniform(-0.3, 0.3, size=P - 1)
    used = [0]
    if n_up:
        used.append(int(det_up.max()) + 1)
    if n_down:
        used.append(int(det_down.max()) + 1)
    return det_up, det_down, ci, max(used)


def _assign(charge: np.ndarray, n_up: int, n_down: int):
    """Electron -> nucleus assignment: nuclei listed Z_I times, spins
    alternate along that list (up, down, up, ...)."""
    slots = []
    for I, Z in enumerate(charge):
        slots += [I] * int(round(Z))
    ups = slots[0::2]
    downs = slots[1::2]
    # fix up counts for odd totals / non-neutral requests
    while len(ups) < n_up:
        ups.append(slots[len(ups) % len(slots)])
    while len(downs) < n_down:
        downs.append(slots[len(downs) % len(slots)])
    return np.asarray(ups[:n_up] + downs[:n_down], np.int64)


def make_walkers(system: System, n_walkers: int, sigma: float, rng) -> np.ndarray:
    a = _assign(system.charge, system.n_up, system.n_down)
    centers = system.nuc_xyz[a]  # [N,3]
    r = centers[None] + sigma * rng.standard_normal((n_walkers, system.n_elec, 3))
    return r.astype(np.float64)


def make_system_workload(
    name,
    nuc_xyz,
    charge,
    n_up,
    n_down,
    n_s,
    n_p,
    n_det,
    net: NetShape,
    n_walkers,
    sigma,
    seed,
    precision="fp64",
    cusp_radius=0.1,
) -> Workload:
    rng = np.random.default_rng(seed)
    nuc_xyz = np.asarray(nuc_xyz, np.float64).reshape(-1, 3)
    charge = np.asarray(charge, np.float64)
    sc, sl, se = _shells_for(n_s, n_p, rng)
    n_basis = int(sum(2 * int(l) + 1 for l in sl))
    det_up, det_down, ci, m_used = _determinants(n_up, n_down, n_basis, n_det, rng)
    mo = rng.standard_normal((n_basis, m_used))
    system = System(
        nuc_xyz=nuc_xyz,
        charge=charge,
        n_up=n_up,
        n_down=n_down,
        shell_center=sc,
        shell_l=sl,
        shell_exp=se,
        mo_coeff=mo,
        det_up=det_up,
        det_down=det_down,
        ci=ci,
        cusp_radius=cusp_radius,
        cusp_nuc_value=None,
    )
    n_par = param_count(system.n_nuc, system.n_mo, net)
    params = 0.1 * rng.standard_normal(n_par)
    walkers = make_walkers(system, n_walkers, sigma, rng)
    return Workload(name, system, net, params, walkers, precision, seed)


def make_config(idx: int, n_walkers: Optional[int] = None) -> Workload:
    """Workloads 1, 2, 3 and 5 (4 is the serving stream, see make_serving_jobs),
    and the unequal-spin parity cases 6 and 7."""
    seed = 1000 + idx
    if idx == 1:
        net = NetShape(16, 10.0, 32, 16, 2)
        return make_system_workload(
            "H2", [[0, 0, -0.7], [0, 0, 0.7]], [1, 1], 1, 1, [4, 4], [0, 0], 1,
            net, n_walkers or 512, 1.0, seed, "fp64")
    if idx == 2:
        net = NetShape(32, 10.0, 64, 32, 3)
        return make_system_workload(
            "Ne-like", [[0, 0, 0]], [10], 5, 5, [8], [6], 16,
            net, n_walkers or 4096, 1.5, seed, "fp64|fp32-net")
    if idx == 3:
        net = NetShape(32, 10.0, 64, 32, 3)
        z = (np.arange(10) - 4.5) * 1.8
        xyz = np.stack([np.zeros(10), np.zeros(10), z], 1)
        return make_system_workload(
            "H10", xyz, [1] * 10, 5, 5, [4] * 10, [0] * 10, 16,
            net, n_walkers or 8192, 1.0, seed, "bf16-net")
    if idx == 5:
        net = NetShape(32, 10.0, 128, 64, 4)
        return make_system_workload(
            "30e diatomic", [[0, 0, -2.0], [0, 0, 2.0]], [15, 15], 15, 15,
            [10, 10], [8, 8], 64, net, n_walkers or 16384, 1.0, seed, "bf16-net")
    # parity cases with unequal spin blocks, shaped like members of the
    # serving stream (an odd-Z atom and an odd hydrogen chain)
    if idx == 6:
        net = NetShape(32, 10.0, 64, 32, 3)
        return make_system_workload(
            "Z5 atom", [[0, 0, 0]], [5], 3, 2, [8], [6], 12,
            net, n_walkers or 2048, 1.0, seed, "fp64|fp32-net")
    if idx == 7:
        net = NetShape(32, 10.0, 64, 32, 3)
        z = (np.arange(7) - 3.0) * 1.8
        xyz = np.stack([np.zeros(7), np.zeros(7), z], 1)
        return make_system_workload(
            "H7", xyz, [1] * 7, 4, 3, [4] * 7, [0] * 7, 9,
            net, n_walkers or 2048, 1.0, seed, "fp64|fp32-net")
    raise ValueError(f"no system workload {idx}")


@dataclasses.dataclass
class ServingJob:
    job_id: int
    arrival_s: float
    n_steps: int
    workload: Workload


def make_serving_jobs(n_jobs: int = 64, seed: int = 1004, mean_gap_s: float = 0.25,
                      n_steps: int = 100, walker_scale: float = 1.0) -> List[ServingJob]:
    """The serving stream: H-chains (2..16 atoms, spacing 1.4..3.0 bohr along z)
    or single neutral atoms (Z = 2..18), 50/50; 1..32 determinants; 1024..8192
    walkers (multiples of 256); Poisson arrivals."""
    rng = np.random.default_rng(seed)
    net = NetShape(32, 10.0, 64, 32, 3)
    jobs = []
    t = 0.0
    for j in range(n_jobs):
        t += rng.exponential(mean_gap_s)
        if rng.uniform() < 0.5:
            n_at = int(rng.integers(2, 17))
            gap = float(rng.uniform(1.4, 3.0))
            z = (np.arange(n_at) - (n_at - 1) / 2) * gap
            xyz = np.stack([np.zeros(n_at), np.zeros(n_at), z], 1)
            charge = [1] * n_at
            n_s, n_p = [4] * n_at, [0] * n_at
            name = f"H{n_at}"
        else:
            Z = int(rng.integers(2, 19))
            xyz = [[0.0, 0.0, 0.0]]
            charge = [Z]
            n_s, n_p = ([8], [6]) if Z <= 10 else ([10], [8])
            name = f"Z{Z}"
        N = int(sum(charge))
        n_up = (N + 1) // 2
        n_down = N - n_up
        n_det = int(rng.integers(1, 33))
        walkers = int(rng.integers(1024, 8193)) // 256 * 256
        walkers = max(256, int(walkers * walker_scale) // 256 * 256) if walker_scale != 1.0 else walkers
        sub_seed = int(rng.integers(0, 2**31 - 1))
        wl = make_system_workload(name, xyz, charge, n_up, n_down, n_s, n_p, n_det, net,
                                  walkers, 1.0, sub_seed, "fp64|fp32-net")
        jobs.append(ServingJob(j, t, n_steps, wl))
    return jobs
