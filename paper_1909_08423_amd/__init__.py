"""MI355X (gfx950) PauliNet walker evaluation.

The compute path is the HIP library libpaulinet.so (built in-tree by
paper_1909_08423_amd.build); this package only marshals arguments to its C
ABI.  Importing works without a GPU; every call that launches work needs the
library and a ROCm device and raises if either is missing.
"""

from ._lib import (  # noqa: F401
    PLAN_EVAL,
    PLAN_FULL_ADJOINT,
    PLAN_VALUE_ADJOINT,
    PLAN_VALUE_ONLY,
    PN_OUT_ADJOINT,
    PN_OUT_ALL,
    PN_OUT_ELOC,
    PN_OUT_GRAD,
    PN_OUT_LAP,
    PN_OUT_LOGABS,
    PN_PREC_FP64,
    PN_PREC_NET_BF16,
    PN_PREC_NET_FP32,
    PauliNetContext,
    PauliNetError,
    library_path,
    langevin_run,
    load_library,
    job_bytes,
    paulinet_eval,
    serve_step,
    vmc_step,
    vmc_workspace_bytes,
)
