"""The allocation-free entry point pn_eval_noalloc (static device workspace)
against pn_eval, through the C ABI: two calls in a row, the second with a
smaller batch, in FP64 and in the FP32-network form.  The walker tiles
differ between the two entry points but every walker is computed by the
same kernels, so the outputs agree bit for bit (the FP64 parity bar,
|d| <= 1e-6 relative, is asserted as well)."""

import numpy as np
import pytest
import torch

from gpu_util import announce, parity_ratios
from synth import make_config

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pn():
    import paper_1909_08423_amd as pn
    assert torch.cuda.is_available(), "no ROCm device"
    pn.load_library()
    return pn


@pytest.mark.parametrize("idx,prec,sizes", [(2, "fp64", (700, 300)), (5, "fp32", (160, 48)), (7, "fp32", (900, 5))])
def test_noalloc_matches_eval(pn, idx, prec, sizes):
    w = make_config(idx, n_walkers=max(sizes))
    ctx = pn.PauliNetContext(w.system, w.net)
    p = pn._lib.PRECISIONS[prec]
    th = torch.tensor(w.params, dtype=torch.float64, device="cuda")
    for B in sizes:
        announce(f"pn_eval_noalloc vs pn_eval, workload {idx}, {prec}, B={B}")
        r = torch.tensor(w.walkers[:B], dtype=torch.float64, device="cuda")
        a = ctx.eval_noalloc(r, th, p)
        b = ctx.eval(r, th, p)
        torch.cuda.synchronize()
        a = {k: v.cpu().numpy() for k, v in a.items()}
        b = {k: v.cpu().numpy() for k, v in b.items()}
        rat = parity_ratios(a, b)
        for k, v in rat.items():
            assert v.max() <= 1e-6, (k, v.max())
        for k in a:
            np.testing.assert_array_equal(a[k], b[k])
