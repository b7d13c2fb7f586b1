"""ctypes binding of the C ABI declared in include/paulinet.h.

Argument marshalling only: tensors are passed by device pointer, the HIP
stream is torch's current stream, and every step of the computation runs in
the library's kernels.  There is no fallback: a missing library or device is
an error.
"""

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libpaulinet.so")

PN_PREC_FP64 = 0
PN_PREC_NET_FP32 = 1
PN_PREC_NET_BF16 = 2
PRECISIONS = {"fp64": PN_PREC_FP64, "fp32": PN_PREC_NET_FP32, "bf16": PN_PREC_NET_BF16}

_c_dp = ctypes.POINTER(ctypes.c_double)
_c_ip = ctypes.POINTER(ctypes.c_int32)


class pn_system_desc(ctypes.Structure):
    _fields_ = [
        ("n_nuc", ctypes.c_int32),
        ("nuc_xyz", _c_dp),
        ("charge", _c_dp),
        ("n_up", ctypes.c_int32),
        ("n_down", ctypes.c_int32),
        ("n_shell", ctypes.c_int32),
        ("shell_center", _c_ip),
        ("shell_l", _c_ip),
        ("shell_exp", _c_dp),
        ("n_mo", ctypes.c_int32),
        ("mo_coeff", _c_dp),
        ("n_det", ctypes.c_int32),
        ("det_up", _c_ip),
        ("det_down", _c_ip),
        ("ci", _c_dp),
        ("cusp_radius", ctypes.c_double),
        ("cusp_nuc_value", _c_dp),
    ]


class pn_net_desc(ctypes.Structure):
    _fields_ = [
        ("n_feat", ctypes.c_int32),
        ("feat_cutoff", ctypes.c_double),
        ("dim_x", ctypes.c_int32),
        ("dim_z", ctypes.c_int32),
        ("n_layers", ctypes.c_int32),
        ("flags", ctypes.c_int32),
    ]


class pn_plan_info(ctypes.Structure):
    _fields_ = [("tile_walkers", ctypes.c_int64), ("chunk_coords", ctypes.c_int32), ("n_chunks", ctypes.c_int32),
                ("lowrank", ctypes.c_int32), ("reserved", ctypes.c_int32), ("workspace_bytes", ctypes.c_size_t)]


PN_DET_DIRECT = 4
PN_OUT_LOGABS, PN_OUT_GRAD, PN_OUT_LAP, PN_OUT_ELOC, PN_OUT_ADJOINT = 1, 2, 4, 8, 16
PN_OUT_ALL = 31
PLAN_EVAL, PLAN_VALUE_ADJOINT, PLAN_FULL_ADJOINT, PLAN_VALUE_ONLY = 0, 1, 2, 3


class pn_param_entry(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("offset", ctypes.c_int64), ("ndim", ctypes.c_int32),
                ("shape", ctypes.c_int32 * 2)]


class pn_langevin_hparams(ctypes.Structure):
    _fields_ = [("target_accept", ctypes.c_double), ("adapt_rate", ctypes.c_double)]


class pn_vmc_hparams(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in
                ("sigma", "lr0", "t0", "clip_q", "beta1", "beta2", "eps", "weight_decay")]


class pn_vmc_job(ctypes.Structure):
    _fields_ = [
        ("n_walkers", ctypes.c_int64),
        ("r", ctypes.c_void_p),
        ("params", ctypes.c_void_p),
        ("adam_m", ctypes.c_void_p),
        ("adam_v", ctypes.c_void_p),
        ("eloc", ctypes.c_void_p),
        ("stats", ctypes.c_void_p),
        ("seed", ctypes.c_uint64),
        ("step", ctypes.c_int64),
    ]


class pn_job_slot(ctypes.Structure):
    _fields_ = [("ctx", ctypes.c_void_p), ("job", pn_vmc_job), ("ws", ctypes.c_void_p), ("ws_bytes", ctypes.c_size_t)]


DEFAULT_HPARAMS = dict(sigma=0.3, lr0=0.01, t0=200.0, clip_q=5.0, beta1=0.9, beta2=0.999, eps=1e-8,
                       weight_decay=0.01)


class PauliNetError(RuntimeError):
    pass


_lib = None


def library_path():
    return _LIB_PATH


def load_library():
    """Load libpaulinet.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise PauliNetError(
            f"{_LIB_PATH} is missing: build it with `python -m paper_1909_08423_amd.build`")
    lib = ctypes.CDLL(_LIB_PATH)
    vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
    lib.pn_ctx_create.argtypes = [ctypes.POINTER(pn_system_desc), ctypes.POINTER(pn_net_desc),
                                  ctypes.POINTER(vp)]
    lib.pn_ctx_create.restype = i32
    lib.pn_ctx_destroy.argtypes = [vp]
    lib.pn_ctx_destroy.restype = None
    lib.pn_param_count.argtypes = [vp]
    lib.pn_param_count.restype = i64
    lib.pn_workspace_bytes.argtypes = [vp, i64, i32, ctypes.c_uint32, ctypes.POINTER(ctypes.c_size_t)]
    lib.pn_workspace_bytes.restype = i32
    lib.pn_eval.argtypes = [vp, vp, i64, vp, vp, i32, vp, vp, vp, vp, vp, vp, ctypes.c_size_t]
    lib.pn_eval.restype = i32
    lib.pn_param_layout.argtypes = [vp, ctypes.POINTER(pn_param_entry), i32, ctypes.POINTER(i32)]
    lib.pn_param_layout.restype = i32
    lib.pn_eval_backward_cusp.argtypes = [vp, vp, i64, vp, vp, i32, vp, vp, vp, ctypes.c_size_t]
    lib.pn_eval_backward_cusp.restype = i32
    lib.pn_workspace_bytes_full.argtypes = [vp, i64, i32, ctypes.POINTER(ctypes.c_size_t)]
    lib.pn_workspace_bytes_full.restype = i32
    lib.pn_eval_backward.argtypes = [vp, vp, i64, vp, vp, i32, vp, vp, vp, vp, vp, vp, ctypes.c_size_t]
    lib.pn_eval_backward.restype = i32
    lib.pn_stage_timing.argtypes = [vp, i32]
    lib.pn_stage_timing.restype = i32
    lib.pn_stage_times.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64), i32]
    lib.pn_stage_times.restype = i32
    lib.pn_langevin_workspace_bytes.argtypes = [vp, i64, i32, ctypes.POINTER(ctypes.c_size_t)]
    lib.pn_langevin_workspace_bytes.restype = i32
    lib.pn_langevin_run.argtypes = [vp, vp, i64, vp, vp, i32, ctypes.POINTER(pn_langevin_hparams), vp, i32,
                                    ctypes.c_uint64, i64, vp, vp, ctypes.c_size_t]
    lib.pn_langevin_run.restype = i32
    lib.pn_vmc_workspace_bytes.argtypes = [vp, i64, i32, ctypes.POINTER(ctypes.c_size_t)]
    lib.pn_vmc_workspace_bytes.restype = i32
    lib.pn_vmc_step.argtypes = [vp, vp, ctypes.POINTER(pn_vmc_job), i32, ctypes.POINTER(pn_vmc_hparams), vp,
                                ctypes.c_size_t]
    lib.pn_vmc_step.restype = i32
    lib.pn_eval_noalloc.argtypes = [vp, vp, i64, vp, vp, i32, vp, vp, vp, vp, vp]
    lib.pn_eval_noalloc.restype = i32
    lib.pn_job_bytes.argtypes = [vp, i64, i32, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t)]
    lib.pn_job_bytes.restype = i32
    lib.pn_serve_step.argtypes = [vp, ctypes.POINTER(pn_job_slot), i32, i32, ctypes.POINTER(pn_vmc_hparams)]
    lib.pn_serve_step.restype = i32
    lib.pn_eval_plan.argtypes = [vp, i64, i32, i32, ctypes.POINTER(pn_plan_info)]
    lib.pn_eval_plan.restype = i32
    lib.pn_status_string.argtypes = [i32]
    lib.pn_status_string.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _check(status, what):
    if status != 0:
        msg = load_library().pn_status_string(status).decode()
        raise PauliNetError(f"{what} failed: {msg} (status {status})")


def _ptr(t):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


class PauliNetContext:
    """One system + network shape.  Arrays of the description are copied to
    the device at construction; parameters and walkers are passed per call."""

    def __init__(self, system, net):
        lib = load_library()
        self._keep = []

        def arr(a, dt):
            a = np.ascontiguousarray(np.asarray(a, dtype=dt))
            self._keep.append(a)
            return a.ctypes.data_as(_c_dp if dt == np.float64 else _c_ip)

        s = pn_system_desc()
        s.n_nuc = int(system.nuc_xyz.shape[0])
        s.nuc_xyz = arr(system.nuc_xyz, np.float64)
        s.charge = arr(system.charge, np.float64)
        s.n_up, s.n_down = int(system.n_up), int(system.n_down)
        s.n_shell = int(len(system.shell_l))
        s.shell_center = arr(system.shell_center, np.int32)
        s.shell_l = arr(system.shell_l, np.int32)
        s.shell_exp = arr(system.shell_exp, np.float64)
        s.n_mo = int(system.mo_coeff.shape[1])
        s.mo_coeff = arr(system.mo_coeff, np.float64)
        s.n_det = int(system.ci.shape[0])
        s.det_up = arr(np.asarray(system.det_up).reshape(-1), np.int32)
        s.det_down = arr(np.asarray(system.det_down).reshape(-1), np.int32)
        s.ci = arr(system.ci, np.float64)
        s.cusp_radius = float(system.cusp_radius)
        s.cusp_nuc_value = (arr(system.cusp_nuc_value, np.float64)
                            if system.cusp_nuc_value is not None else _c_dp())
        n = pn_net_desc()
        n.n_feat, n.feat_cutoff = int(net.n_feat), float(net.feat_cutoff)
        n.dim_x, n.dim_z, n.n_layers = int(net.dim_x), int(net.dim_z), int(net.n_layers)
        n.flags = int(getattr(net, "flags", 0))
        out = ctypes.c_void_p()
        _check(lib.pn_ctx_create(ctypes.byref(s), ctypes.byref(n), ctypes.byref(out)), "pn_ctx_create")
        self._ctx = out
        self._lib = lib
        self.n_elec = s.n_up + s.n_down
        self.n_nuc, self.n_mo = int(s.n_nuc), int(s.n_mo)
        self._ws = {}

    def close(self):
        if getattr(self, "_ctx", None):
            self._lib.pn_ctx_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    STAGES = ("convert", "geometry_orbitals", "filters", "net_value", "slater_value", "net_tangent",
              "slater_tangent", "finalize")

    def stage_timing(self, enable=True):
        _check(self._lib.pn_stage_timing(self._ctx, int(bool(enable))), "pn_stage_timing")

    def stage_times(self):
        """{stage: (total ms, launches)} since timing was enabled."""
        n = len(self.STAGES)
        ms = (ctypes.c_double * n)()
        cnt = (ctypes.c_int64 * n)()
        _check(self._lib.pn_stage_times(self._ctx, ms, cnt, n), "pn_stage_times")
        return {k: (ms[i], cnt[i]) for i, k in enumerate(self.STAGES)}

    @property
    def param_count(self):
        return int(self._lib.pn_param_count(self._ctx))

    def param_layout(self):
        """[(name, offset, shape)] of the parameter blob, in blob order."""
        n = ctypes.c_int32()
        self._lib.pn_param_layout(self._ctx, None, 0, ctypes.byref(n))
        arr = (pn_param_entry * n.value)()
        _check(self._lib.pn_param_layout(self._ctx, arr, n.value, ctypes.byref(n)), "pn_param_layout")
        return [(e.name.decode(), int(e.offset), tuple(int(e.shape[k]) for k in range(e.ndim))) for e in arr]

    def plan(self, n_walkers, prec=PN_PREC_FP64, kind=PLAN_EVAL):
        """How the library carries out a call: tile, tangent chunk, number of
        chunks, determinant path, workspace bytes."""
        info = pn_plan_info()
        _check(self._lib.pn_eval_plan(self._ctx, int(n_walkers), int(prec), int(kind), ctypes.byref(info)),
               "pn_eval_plan")
        return {"tile_walkers": int(info.tile_walkers), "chunk_coords": int(info.chunk_coords),
                "n_chunks": int(info.n_chunks), "lowrank": bool(info.lowrank),
                "workspace_bytes": int(info.workspace_bytes)}

    def workspace_bytes(self, n_walkers, prec=PN_PREC_FP64, full=False, out_mask=PN_OUT_ALL):
        """Workspace bytes for pn_eval calls producing the outputs in out_mask
        (PN_OUT_*) and the value-path adjoint; full=True also covers the full
        adjoint."""
        b = ctypes.c_size_t()
        if full:
            st = self._lib.pn_workspace_bytes_full(self._ctx, int(n_walkers), int(prec), ctypes.byref(b))
        else:
            st = self._lib.pn_workspace_bytes(self._ctx, int(n_walkers), int(prec), int(out_mask), ctypes.byref(b))
        _check(st, "pn_workspace_bytes")
        return int(b.value)

    def workspace(self, n_walkers, prec, device, full=False, out_mask=PN_OUT_ALL):
        import torch
        need = self.workspace_bytes(n_walkers, prec, full, out_mask)
        key = (str(device),)
        ws = self._ws.get(key)
        if ws is None or ws.numel() < need:
            ws = torch.empty(need, dtype=torch.uint8, device=device)
            self._ws[key] = ws
        return ws

    @staticmethod
    def _stream():
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)

    def eval(self, r, params, prec=PN_PREC_FP64, want_derivs=True, out=None, ws=None):
        """r: [B, N, 3] float64 CUDA tensor; params: [n_params] float64 CUDA
        tensor.  Returns dict logabs, sign (and grad, lap, eloc)."""
        import torch
        if not (r.is_cuda and params.is_cuda):
            raise PauliNetError("pn_eval needs device tensors")
        if r.dtype != torch.float64 or params.dtype != torch.float64:
            raise PauliNetError("r and params must be float64")
        r = r.contiguous()
        params = params.contiguous()
        B = int(r.shape[0])
        if r.shape[1] != self.n_elec or r.shape[2] != 3:
            raise PauliNetError(f"r must be [B, {self.n_elec}, 3]")
        if params.numel() != self.param_count:
            raise PauliNetError(f"params must have {self.param_count} entries")
        dev = r.device
        if out is None:
            out = {"logabs": torch.empty(B, dtype=torch.float64, device=dev),
                   "sign": torch.empty(B, dtype=torch.float64, device=dev)}
            if want_derivs:
                out["grad"] = torch.empty(B, self.n_elec, 3, dtype=torch.float64, device=dev)
                out["lap"] = torch.empty(B, dtype=torch.float64, device=dev)
                out["eloc"] = torch.empty(B, dtype=torch.float64, device=dev)
        if ws is None:
            derivs = any(out.get(k) is not None for k in ("grad", "lap", "eloc"))
            ws = self.workspace(B, prec, dev, out_mask=PN_OUT_ALL if derivs else PN_OUT_LOGABS)
        st = self._lib.pn_eval(self._ctx, self._stream(), B, _ptr(r), _ptr(params), int(prec),
                               _ptr(out["logabs"]), _ptr(out["sign"]), _ptr(out.get("grad")),
                               _ptr(out.get("lap")), _ptr(out.get("eloc")), _ptr(ws), ws.numel())
        _check(st, "pn_eval")
        return out

    def eval_noalloc(self, r, params, prec=PN_PREC_FP64, out=None):
        """pn_eval_noalloc: as eval, with the library's static workspace."""
        import torch
        r = r.contiguous()
        params = params.contiguous()
        B = int(r.shape[0])
        if out is None:
            dev = r.device
            out = {k: torch.empty(B, dtype=torch.float64, device=dev) for k in ("logabs", "sign", "lap", "eloc")}
            out["grad"] = torch.empty(B, self.n_elec, 3, dtype=torch.float64, device=dev)
        st = self._lib.pn_eval_noalloc(self._ctx, self._stream(), B, _ptr(r), _ptr(params), int(prec),
                                       _ptr(out["logabs"]), _ptr(out["sign"]), _ptr(out.get("grad")),
                                       _ptr(out.get("lap")), _ptr(out.get("eloc")))
        _check(st, "pn_eval_noalloc")
        return out

    def eval_backward(self, r, params, ct_logabs=None, prec=PN_PREC_FP64, grad_params=None, ws=None,
                      ct_grad=None, ct_lap=None, ct_eloc=None):
        """grad_params += sum_w [ct_logabs d ln|psi| + ct_grad . d grad + ct_lap d lap
        + ct_eloc d E_loc] / d params (each cotangent may be None = zero)."""
        import torch
        r = r.contiguous()
        params = params.contiguous()
        B = int(r.shape[0])

        def prep(t, shape):
            if t is None:
                return None
            t = t.to(torch.float64).contiguous()
            if tuple(t.shape) != shape:
                raise PauliNetError(f"cotangent of shape {tuple(t.shape)}, expected {shape}")
            return t
        ct_logabs = prep(ct_logabs, (B,))
        ct_grad = prep(ct_grad, (B, self.n_elec, 3))
        ct_lap = prep(ct_lap, (B,))
        ct_eloc = prep(ct_eloc, (B,))
        full = ct_grad is not None or ct_lap is not None or ct_eloc is not None
        if grad_params is None:
            grad_params = torch.zeros(self.param_count, dtype=torch.float64, device=r.device)
        if ws is None:
            ws = self.workspace(B, prec, r.device, full)
        st = self._lib.pn_eval_backward(self._ctx, self._stream(), B, _ptr(r), _ptr(params), int(prec),
                                        _ptr(ct_logabs), _ptr(ct_grad), _ptr(ct_lap), _ptr(ct_eloc),
                                        _ptr(grad_params), _ptr(ws), ws.numel())
        _check(st, "pn_eval_backward")
        return grad_params


def _cusp_grad(self, r, params, ct_logabs, prec=PN_PREC_FP64, grad_cusp=None, ws=None):
    """grad_cusp[I, mu] += sum_w ct_logabs[w] d ln|psi_w| / d s0[I, mu] (the
    orbital values at the nuclei of the cusp correction)."""
    import torch
    r = r.contiguous()
    params = params.contiguous()
    ct_logabs = ct_logabs.to(torch.float64).contiguous()
    B = int(r.shape[0])
    if grad_cusp is None:
        grad_cusp = torch.zeros(self.n_nuc, self.n_mo, dtype=torch.float64, device=r.device)
    if ws is None:
        ws = self.workspace(B, prec, r.device)
    _check(self._lib.pn_eval_backward_cusp(self._ctx, self._stream(), B, _ptr(r), _ptr(params), int(prec),
                                           _ptr(ct_logabs), _ptr(grad_cusp), _ptr(ws), ws.numel()),
           "pn_eval_backward_cusp")
    return grad_cusp


PauliNetContext.eval_backward_cusp = _cusp_grad


def _autograd_function():
    import torch

    class PauliNetEval(torch.autograd.Function):
        """(ln|psi|, sign, grad, lap, E_loc) = f(params) for fixed walkers;
        the backward is the library's hand-written adjoint (pn_eval_backward
        with the output cotangents, the Laplacian's second-order terms
        included)."""

        @staticmethod
        def forward(fctx, params, r, pnctx, prec):
            out = pnctx.eval(r.detach(), params.detach(), prec)
            fctx.save_for_backward(params, r)
            fctx.pnctx, fctx.prec = pnctx, prec
            fctx.mark_non_differentiable(out["sign"])
            # outputs the loss does not use arrive as None, so that a loss on
            # ln|psi| alone runs the value-path adjoint (the estimator's case)
            fctx.set_materialize_grads(False)
            return out["logabs"], out["sign"], out["grad"], out["lap"], out["eloc"]

        @staticmethod
        def backward(fctx, g_logabs, g_sign, g_grad, g_lap, g_eloc):
            params, r = fctx.saved_tensors
            if g_logabs is None and g_grad is None and g_lap is None and g_eloc is None:
                return None, None, None, None
            gp = fctx.pnctx.eval_backward(r.detach(), params.detach(), g_logabs, fctx.prec, ct_grad=g_grad,
                                          ct_lap=g_lap, ct_eloc=g_eloc)
            return gp.to(params.dtype), None, None, None

    return PauliNetEval


_PNE = None


def paulinet_eval(pnctx, r, params, prec=PN_PREC_FP64):
    """Differentiable evaluation: returns (logabs, sign, grad, lap, eloc);
    gradients flow to `params` (float64 device tensor) through the library's
    adjoint.  Walker positions are inputs only (their derivatives are the
    `grad` and `lap` outputs themselves)."""
    global _PNE
    if _PNE is None:
        _PNE = _autograd_function()
    return _PNE.apply(params, r, pnctx, prec)


def vmc_workspace_bytes(ctx, n_walkers, prec):
    b = ctypes.c_size_t()
    _check(ctx._lib.pn_vmc_workspace_bytes(ctx._ctx, int(n_walkers), int(prec), ctypes.byref(b)),
           "pn_vmc_workspace_bytes")
    return int(b.value)


def job_bytes(ctx, n_walkers, prec):
    """(resident, scratch) device bytes of a serving job (pn_job_bytes)."""
    res, scr = ctypes.c_size_t(), ctypes.c_size_t()
    _check(ctx._lib.pn_job_bytes(ctx._ctx, int(n_walkers), int(prec), ctypes.byref(res), ctypes.byref(scr)),
           "pn_job_bytes")
    return int(res.value), int(scr.value)


def _job_struct(state):
    import torch
    j = pn_vmc_job()
    j.n_walkers = int(state["r"].shape[0])
    for k in ("r", "params", "adam_m", "adam_v", "eloc", "stats"):
        t = state[k]
        if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
            raise PauliNetError(f"{k} must be a contiguous float64 device tensor")
        setattr(j, k, t.data_ptr())
    j.seed = int(state["seed"]) & 0xFFFFFFFFFFFFFFFF
    j.step = int(state["step"])
    return j


def serve_step(states, prec, hparams=None, stream=None):
    """One VMC step of every job in `states` (each a dict as for vmc_step,
    with its PauliNetContext under "ctx") as one pn_serve_step launch
    sequence on `stream`.  The caller advances each state's "step"."""
    import torch
    if not states:
        return
    hp = dict(DEFAULT_HPARAMS)
    hp.update(hparams or {})
    h = pn_vmc_hparams(**hp)
    arr = (pn_job_slot * len(states))()
    for k, st in enumerate(states):
        arr[k].ctx = st["ctx"]._ctx
        arr[k].job = _job_struct(st)
        arr[k].ws = st["ws"].data_ptr()
        arr[k].ws_bytes = st["ws"].numel()
    s = stream if stream is not None else torch.cuda.current_stream()
    lib = states[0]["ctx"]._lib
    _check(lib.pn_serve_step(ctypes.c_void_p(s.cuda_stream), arr, len(states), int(prec), ctypes.byref(h)),
           "pn_serve_step")


def vmc_step(ctx, state, prec, hparams=None, stream=None):
    """One VMC step of a job on `stream` (torch stream; default current).
    `state` holds device tensors r, params, adam_m, adam_v, eloc, stats, ws
    and ints seed, step; the tensors are updated in place."""
    import torch
    hp = dict(DEFAULT_HPARAMS)
    hp.update(hparams or {})
    h = pn_vmc_hparams(**hp)
    j = _job_struct(state)
    st = stream if stream is not None else torch.cuda.current_stream()
    ws = state["ws"]
    _check(ctx._lib.pn_vmc_step(ctx._ctx, ctypes.c_void_p(st.cuda_stream), ctypes.byref(j), int(prec),
                                ctypes.byref(h), ctypes.c_void_p(ws.data_ptr()), ws.numel()), "pn_vmc_step")


def langevin_run(ctx, r, params, prec, tau, n_steps, seed, step0=0, target_accept=0.57, adapt_rate=1.0,
                 ws=None, stream=None):
    """n_steps Langevin steps on r ([B, N, 3] float64 device tensor, updated
    in place); tau: [1] float64 device tensor (updated).  Returns the
    [n_steps, 2] device tensor of (acceptance, tau used)."""
    import torch
    for name, t in (("r", r), ("params", params), ("tau", tau)):
        if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
            raise PauliNetError(f"{name} must be a contiguous float64 device tensor")
    B = int(r.shape[0])
    if ws is None:
        b = ctypes.c_size_t()
        _check(ctx._lib.pn_langevin_workspace_bytes(ctx._ctx, B, int(prec), ctypes.byref(b)),
               "pn_langevin_workspace_bytes")
        ws = torch.empty(int(b.value), dtype=torch.uint8, device=r.device)
    stats = torch.empty(max(int(n_steps), 1), 2, dtype=torch.float64, device=r.device)
    hp = pn_langevin_hparams(float(target_accept), float(adapt_rate))
    s = ctypes.c_void_p((stream or torch.cuda.current_stream()).cuda_stream)
    _check(ctx._lib.pn_langevin_run(ctx._ctx, s, B, _ptr(r), _ptr(params), int(prec), ctypes.byref(hp), _ptr(tau),
                                    int(n_steps), ctypes.c_uint64(int(seed)), int(step0), _ptr(stats), _ptr(ws),
                                    ws.numel()), "pn_langevin_run")
    return stats[:n_steps]
