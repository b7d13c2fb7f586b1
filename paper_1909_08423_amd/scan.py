"""One-dimensional scans of the wavefunction (the paper's Fig. 4 shows psi
and E_loc of LiH as one electron moves along a line while the others stay
fixed).

`line_scan` places one electron of a reference configuration at n points
p(t) = start + t (end - start), t = 0 .. 1, and evaluates the whole batch
with one pn_eval call: ln|psi|, sign, the gradient, the Laplacian and E_loc
at every point.  Building the batch is input preparation (one broadcast copy
of the walker and the points of the line); every step of the evaluation runs
in the library's kernels.
"""

from __future__ import annotations

from . import _lib


def line_walkers(walker, electron: int, start, end, n_points: int):
    """[n_points, N, 3] float64 device tensor: `walker` ([N, 3]) with electron
    `electron` moved to start + t (end - start), t = k / (n_points - 1)."""
    import torch
    w = torch.as_tensor(walker, dtype=torch.float64)
    dev = w.device if w.is_cuda else torch.device("cuda")
    w = w.to(dev)
    a = torch.as_tensor(start, dtype=torch.float64, device=dev)
    b = torch.as_tensor(end, dtype=torch.float64, device=dev)
    t = torch.linspace(0.0, 1.0, n_points, dtype=torch.float64, device=dev)
    r = w.unsqueeze(0).repeat(n_points, 1, 1)
    r[:, electron, :] = a + t[:, None] * (b - a)
    return r.contiguous(), t


def line_scan(ctx, params, walker, electron: int, start, end, n_points: int, prec=_lib.PN_PREC_FP64, ws=None):
    """ln|psi|, sign, grad, lap and E_loc along the line (dict of device
    tensors, plus "t" and the walkers "r")."""
    r, t = line_walkers(walker, electron, start, end, n_points)
    out = ctx.eval(r, params, prec, ws=ws)
    out["t"] = t
    out["r"] = r
    return out
