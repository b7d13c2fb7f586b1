"""The one-dimensional scan workload (the paper's Fig. 4: psi and E_loc as
one electron moves along a line): the scan through pn_eval against the FP64
oracle at every point, on H2 along the bond axis through both nuclei (so
the line crosses the cusp-correction radius of each)."""

import numpy as np
import pytest
import torch

from gpu_util import announce, parity_ratios, summarize
from synth import make_config

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pn():
    import paper_1909_08423_amd as pn
    assert torch.cuda.is_available(), "no ROCm device"
    pn.load_library()
    return pn


def test_line_scan_matches_oracle(pn):
    from oracle import Oracle
    from paper_1909_08423_amd.scan import line_scan
    w = make_config(1, n_walkers=2)
    ctx = pn.PauliNetContext(w.system, w.net)
    th = torch.tensor(w.params, dtype=torch.float64, device="cuda")
    # 201 points from z = -2.5 to z = 2.5 (nuclei at +-0.7; the step puts
    # points inside the 0.1 bohr cusp radius without landing on a nucleus)
    announce("line scan, H2, 201 points")
    out = line_scan(ctx, th, w.walkers[0], 0, [0.013, -0.011, -2.5], [0.013, -0.011, 2.5], 201)
    torch.cuda.synchronize()
    got = {k: v.cpu().numpy() for k, v in out.items()}
    ref = {k: v.numpy() for k, v in Oracle(w.system, w.net, w.params).evaluate(got["r"]).items()}
    np.testing.assert_array_equal(got["sign"], ref["sign"])
    rat = parity_ratios(got, ref)
    for k, v in rat.items():
        assert v.max() <= 1e-6, f"{k}: {summarize(rat)}"
    z = got["r"][:, 0, 2]
    near = np.min(np.abs(np.abs(z) - 0.7))
    assert near < 0.1  # the line passes inside a cusp radius
    assert np.all(np.isfinite(got["eloc"]))
