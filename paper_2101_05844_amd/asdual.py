"""Python binding of libasdual (ctypes; argument marshalling only).

Every computation runs in the HIP library; this module passes device
pointers of torch tensors and the current HIP stream.  It refuses to work
without the built library (no fallback of any kind).

Function names follow the C ABI in include/asdual.h.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Dict, List, Optional, Sequence

import numpy as np
import torch  # must be imported before the library so both share one HIP runtime

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libasdual.so")

ASD_MAX_LAYERS = 16
ASD_MAX_MASKS = 8
ASD_LAYER_DENSE, ASD_LAYER_CONV2D = 0, 1
ASD_RULE_ADAM, ASD_RULE_SUPERGRADIENT = 0, 1
ASD_PREC_FP32, ASD_PREC_FP64, ASD_PREC_MIXED, ASD_PREC_BF16, ASD_PREC_BF16_ALL = 0, 1, 2, 3, 4
ASD_PHASE_BIGM, ASD_PHASE_AS = 0, 1
ASD_DOMAIN_BOX, ASD_DOMAIN_L2 = 0, 1
(ASD_F_ALPHA, ASD_F_BETA0, ASD_F_BETA1, ASD_F_ALPHA_M, ASD_F_ALPHA_V, ASD_F_BETA0_M, ASD_F_BETA0_V,
 ASD_F_BETA1_M, ASD_F_BETA1_V, ASD_F_MASK_BETA, ASD_F_MASK_M, ASD_F_MASK_V, ASD_F_MASK_LI,
 ASD_F_MASK_UI, ASD_F_MASK_Z, ASD_F_MASK_XPREV) = range(16)

STATUS = {0: "ASD_OK", 1: "ASD_EINVAL", 2: "ASD_ENOMEM", 3: "ASD_EDEVICE", 4: "ASD_EUNSUPPORTED"}


class AsdError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class LayerDesc(C.Structure):
    _fields_ = [("kind", C.c_int32), ("in_c", C.c_int32), ("in_h", C.c_int32), ("in_w", C.c_int32),
                ("out_c", C.c_int32), ("out_h", C.c_int32), ("out_w", C.c_int32),
                ("kernel", C.c_int32), ("stride", C.c_int32), ("pad", C.c_int32),
                ("W", C.c_void_p), ("b", C.c_void_p)]


class Params(C.Structure):
    _fields_ = [("bigm_iters", C.c_int32), ("as_iters", C.c_int32), ("add_every", C.c_int32),
                ("add_count", C.c_int32), ("max_masks", C.c_int32), ("rule", C.c_int32),
                ("bigm_lr0", C.c_double), ("bigm_lr1", C.c_double), ("as_lr0", C.c_double),
                ("as_lr1", C.c_double), ("adam_beta1", C.c_double), ("adam_beta2", C.c_double),
                ("adam_eps", C.c_double), ("precision", C.c_int32)]


class SPParams(C.Structure):
    _fields_ = [("iters", C.c_int32), ("gamma0", C.c_double), ("init_steps", C.c_int32),
                ("init_lr0", C.c_double), ("init_lr1", C.c_double), ("cap_alpha", C.c_double),
                ("cap_beta", C.c_double), ("lds_staging", C.c_int32)]


ASD_SP_X, ASD_SP_XBAR, ASD_SP_ALPHA, ASD_SP_ZETA1, ASD_SP_ZETA3, ASD_SP_ZETA4 = 0, 1, 2, 3, 4, 5
ASD_SP_MU_ALPHA, ASD_SP_MU_BETA, ASD_SP_Z, ASD_SP_ZETA2 = 6, 7, 8, 9


class Batch(C.Structure):
    _fields_ = [("S", C.c_int32), ("l0", C.c_void_p), ("u0", C.c_void_p),
                ("lhat", C.POINTER(C.c_void_p)), ("uhat", C.POINTER(C.c_void_p)), ("c", C.c_void_p)]


class Counts(C.Structure):
    _fields_ = [("n_masks", C.c_int32), ("step", C.c_int32), ("mask_step", C.c_int32 * ASD_MAX_MASKS)]


class KernelTime(C.Structure):
    _fields_ = [("role", C.c_int32), ("layer", C.c_int32), ("launches", C.c_int32),
                ("total_ms", C.c_double)]


ASD_K_BACKWARD, ASD_K_FORWARD, ASD_K_MASK, ASD_K_FINAL, ASD_K_OTHER = range(5)
ROLE_NAMES = {0: "backward", 1: "forward", 2: "mask", 3: "final", 4: "other", 5: "grad_weight",
              6: "grad_bias", 7: "grad_box", 8: "forward_pass", 9: "backward_pair"}
ASD_PROFILE_OFF, ASD_PROFILE_LAUNCHES, ASD_PROFILE_KERNELS = 0, 1, 2


class Tuning(C.Structure):
    _fields_ = [("ksplit", C.c_int32 * 16), ("fwd_mfma", C.c_int32 * 16), ("bwd_cb", C.c_int32 * 16),
                ("bwd_pos", C.c_int32 * 16), ("bwd_nt", C.c_int32 * 16), ("fwd_kw", C.c_int32 * 16),
                ("bwd_kw", C.c_int32 * 16)]


class EvalOut(C.Structure):
    _fields_ = [("obj", C.c_void_p),
                ("xstar", C.c_void_p * ASD_MAX_LAYERS),
                ("zstar", C.c_void_p * ASD_MAX_LAYERS),
                ("grad_alpha", C.c_void_p * ASD_MAX_LAYERS),
                ("grad_beta0", C.c_void_p * ASD_MAX_LAYERS),
                ("grad_beta1", C.c_void_p * ASD_MAX_LAYERS),
                ("grad_mask", (C.c_void_p * ASD_MAX_MASKS) * ASD_MAX_LAYERS),
                ("f", C.c_void_p * ASD_MAX_LAYERS),
                ("g", C.c_void_p * ASD_MAX_LAYERS),
                ("path", C.c_int32)]


ASD_EVAL_GENERAL, ASD_EVAL_ITERATION = 0, 1


_lib = None

EXPORTED = ["asd_net_create", "asd_net_destroy", "asd_params_default", "asd_plan_workspace_size",
            "asd_plan_create", "asd_plan_destroy", "asd_init", "asd_run", "asd_bound", "asd_solve",
            "asd_state_get", "asd_state_set", "asd_state_get_counts", "asd_state_set_counts",
            "asd_eval", "asd_oracle", "asd_bound_grad", "asd_set_budgets", "asd_solve_group", "asd_solve_graph", "asd_check_finite",
            "asd_plan_autotune", "asd_plan_get_tuning", "asd_plan_set_tuning", "asd_interval_bounds", "asd_profile_enable", "asd_profile_read",
            "asd_solve_static", "asd_intermediate_workspace_size", "asd_intermediate_bounds", "asd_set_input_domain",
            "asd_sp_params_default", "asd_sp_workspace_size", "asd_sp_init", "asd_sp_run", "asd_sp_bound",
            "asd_sp_solve", "asd_sp_read",
            "asd_last_error", "asd_abi_version"]


def lib():
    """Loads libasdual.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2101_05844_amd.build` "
                           "(there is no fallback implementation)")
    L = C.CDLL(LIB_PATH)
    vp, i32 = C.c_void_p, C.c_int32
    L.asd_net_create.argtypes = [C.POINTER(LayerDesc), i32, C.POINTER(vp)]
    L.asd_net_destroy.argtypes = [vp]
    L.asd_net_destroy.restype = None
    L.asd_params_default.argtypes = [C.POINTER(Params)]
    L.asd_params_default.restype = None
    L.asd_plan_workspace_size.argtypes = [vp, i32, C.POINTER(Params), C.POINTER(C.c_size_t)]
    L.asd_plan_create.argtypes = [vp, i32, C.POINTER(Params), vp, C.c_size_t, vp, C.POINTER(vp)]
    L.asd_plan_destroy.argtypes = [vp]
    L.asd_plan_destroy.restype = None
    L.asd_init.argtypes = [vp, C.POINTER(Batch), vp]
    L.asd_run.argtypes = [vp, i32, i32, i32, vp]
    L.asd_bound.argtypes = [vp, vp, vp, vp]
    L.asd_solve.argtypes = [vp, C.POINTER(Batch), vp, vp, vp]
    L.asd_solve_static.argtypes = [vp, C.POINTER(Params), C.POINTER(Batch), vp, vp, vp]
    L.asd_state_get.argtypes = [vp, i32, i32, i32, vp, vp]
    L.asd_state_set.argtypes = [vp, i32, i32, i32, vp, vp]
    L.asd_state_get_counts.argtypes = [vp, C.POINTER(Counts)]
    L.asd_state_set_counts.argtypes = [vp, C.POINTER(Counts), i32, vp]
    L.asd_eval.argtypes = [vp, C.POINTER(EvalOut), vp]
    L.asd_oracle.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp]
    L.asd_bound_grad.argtypes = [vp, vp, C.POINTER(vp), C.POINTER(vp), vp, vp, i32, vp]
    L.asd_set_budgets.argtypes = [vp, C.POINTER(i32), vp]
    L.asd_set_input_domain.argtypes = [vp, i32, vp, vp, vp]
    L.asd_solve_graph.argtypes = [vp, C.POINTER(Batch), vp, vp]
    L.asd_check_finite.argtypes = [vp, vp, vp, vp]
    L.asd_plan_autotune.argtypes = [vp, i32, i32, vp]
    L.asd_plan_get_tuning.argtypes = [vp, C.POINTER(Tuning)]
    L.asd_plan_set_tuning.argtypes = [vp, C.POINTER(Tuning)]
    L.asd_solve_group.argtypes = [C.POINTER(vp), C.POINTER(C.POINTER(Batch)), C.POINTER(vp), i32, C.POINTER(vp)]
    L.asd_interval_bounds.argtypes = [vp, i32, vp, vp, C.POINTER(vp), C.POINTER(vp), vp]
    L.asd_intermediate_workspace_size.argtypes = [vp, i32, C.POINTER(Params), C.POINTER(C.c_size_t)]
    L.asd_intermediate_bounds.argtypes = [vp, i32, C.POINTER(Params), vp, vp, C.POINTER(vp), C.POINTER(vp), vp,
                                          C.c_size_t, vp]
    L.asd_sp_params_default.argtypes = [C.POINTER(SPParams)]
    L.asd_sp_params_default.restype = None
    L.asd_sp_workspace_size.argtypes = [vp, C.POINTER(C.c_size_t)]
    L.asd_sp_init.argtypes = [vp, C.POINTER(SPParams), vp, C.c_size_t, vp]
    L.asd_sp_run.argtypes = [vp, i32, i32, vp]
    L.asd_sp_bound.argtypes = [vp, vp, vp]
    L.asd_sp_solve.argtypes = [vp, C.POINTER(SPParams), vp, C.c_size_t, vp, vp]
    L.asd_sp_read.argtypes = [vp, i32, i32, vp, vp]
    L.asd_profile_enable.argtypes = [vp, i32]
    L.asd_profile_read.argtypes = [vp, C.POINTER(KernelTime), i32, C.POINTER(i32)]
    L.asd_last_error.argtypes = []
    L.asd_last_error.restype = C.c_char_p
    L.asd_abi_version.argtypes = []
    L.asd_abi_version.restype = i32
    for name in EXPORTED:
        if name not in ("asd_net_destroy", "asd_params_default", "asd_plan_destroy", "asd_last_error",
                        "asd_abi_version", "asd_sp_params_default"):
            getattr(L, name).restype = i32
    _lib = L
    return L


def _check(status: int):
    if status != 0:
        raise AsdError(status, lib().asd_last_error().decode())


def _stream(stream=None) -> int:
    s = torch.cuda.current_stream() if stream is None else stream
    return s.cuda_stream


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    assert t.is_cuda and t.is_contiguous(), "device tensors must be contiguous CUDA/HIP tensors"
    return t.data_ptr()


# ----------------------------------------------------------------------------
# Thin wrappers with the C names
# ----------------------------------------------------------------------------


def asd_params_default() -> Params:
    p = Params()
    lib().asd_params_default(C.byref(p))
    return p


def asd_sp_params_default() -> SPParams:
    p = SPParams()
    lib().asd_sp_params_default(C.byref(p))
    return p


def params_from_schedule(s, precision: int = ASD_PREC_FP32) -> Params:
    p = asd_params_default()
    p.precision = precision
    p.bigm_iters, p.as_iters = s.bigm_iters, s.as_iters
    p.add_every, p.add_count, p.max_masks = s.add_every, s.add_count, s.max_masks
    p.bigm_lr0, p.bigm_lr1 = s.bigm_lr
    p.as_lr0, p.as_lr1 = s.as_lr
    p.adam_beta1, p.adam_beta2, p.adam_eps = s.adam_beta1, s.adam_beta2, s.adam_eps
    return p


class Net:
    """Device copy of a network's FP32 weights plus the library's net handle."""

    def __init__(self, layers, device="cuda"):
        self.layers = layers
        self.W = [torch.as_tensor(np.ascontiguousarray(L.W), device=device) for L in layers]
        self.b = [torch.as_tensor(np.ascontiguousarray(L.b), device=device) for L in layers]
        descs = (LayerDesc * len(layers))()
        for i, L in enumerate(layers):
            d = descs[i]
            sp = L.spec
            if L.kind == "dense":
                d.kind, d.in_c, d.in_h, d.in_w = ASD_LAYER_DENSE, sp.n_in, 1, 1
                d.out_c, d.out_h, d.out_w = sp.n_out, 1, 1
                d.kernel, d.stride, d.pad = 1, 1, 0
            else:
                d.kind, d.in_c, d.in_h, d.in_w = ASD_LAYER_CONV2D, sp.c_in, sp.h_in, sp.w_in
                d.out_c, d.out_h, d.out_w = sp.c_out, sp.h_out, sp.w_out
                d.kernel, d.stride, d.pad = sp.k, sp.stride, sp.pad
            d.W, d.b = self.W[i].data_ptr(), self.b[i].data_ptr()
        h = C.c_void_p()
        _check(lib().asd_net_create(descs, len(layers), C.byref(h)))
        self.handle = h
        self.n = len(layers)
        self.sizes = [layers[0].n_in] + [L.n_out for L in layers]

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.asd_net_destroy(self.handle)
            self.handle = None

    def interval_bounds(self, l0: torch.Tensor, u0: torch.Tensor, stream=None):
        """asd_interval_bounds: pre-activation bounds of layers 1..n."""
        S = l0.shape[0]
        lh = [torch.empty(S, n, device=l0.device, dtype=torch.float32) for n in self.sizes[1:]]
        uh = [torch.empty_like(t) for t in lh]
        lp = (C.c_void_p * self.n)(*[t.data_ptr() for t in lh])
        up = (C.c_void_p * self.n)(*[t.data_ptr() for t in uh])
        _check(lib().asd_interval_bounds(self.handle, S, _ptr(l0), _ptr(u0), lp, up, _stream(stream)))
        return lh, uh

    def intermediate_bounds(self, l0: torch.Tensor, u0: torch.Tensor, params: Params, stream=None):
        """asd_intermediate_bounds: pre-activation bounds of the ReLU layers
        1..n-1 for D boxes l0, u0 [D][n_0] (float32, device), each layer k >= 2
        from the solver on its sub-network; the workspace is a torch tensor
        held for the call."""
        D = l0.shape[0]
        nbytes = C.c_size_t()
        _check(lib().asd_intermediate_workspace_size(self.handle, D, C.byref(params), C.byref(nbytes)))
        ws = torch.empty(nbytes.value + 256, dtype=torch.uint8, device=l0.device)
        lh = [torch.empty(D, n, device=l0.device, dtype=torch.float32) for n in self.sizes[1:-1]]
        uh = [torch.empty_like(t) for t in lh]
        lp = (C.c_void_p * max(1, len(lh)))(*[t.data_ptr() for t in lh])
        up = (C.c_void_p * max(1, len(uh)))(*[t.data_ptr() for t in uh])
        _check(lib().asd_intermediate_bounds(self.handle, D, C.byref(params), _ptr(l0), _ptr(u0), lp, up,
                                             ws.data_ptr(), nbytes.value + 256, _stream(stream)))
        # the workspace must outlive the queued kernels
        (torch.cuda.current_stream() if stream is None else stream).synchronize()
        return lh, uh


class Plan:
    """A plan for S subproblems with its workspace (a torch uint8 tensor)."""

    def __init__(self, net: Net, S: int, params: Params, stream=None):
        self.net, self.S, self.params = net, S, params
        self.dtype = torch.float64 if params.precision == ASD_PREC_FP64 else torch.float32
        nbytes = C.c_size_t()
        _check(lib().asd_plan_workspace_size(net.handle, S, C.byref(params), C.byref(nbytes)))
        self.workspace = torch.empty(nbytes.value + 256, dtype=torch.uint8, device="cuda")
        base = self.workspace.data_ptr()
        aligned = (base + 255) // 256 * 256
        h = C.c_void_p()
        _check(lib().asd_plan_create(net.handle, S, C.byref(params), aligned, nbytes.value,
                                     _stream(stream), C.byref(h)))
        self.handle = h
        self._keep = None
        # bumped by every call that changes the plan's duals, masks or batch
        # (a backward pass of BoundFunction checks that its solve's state is
        # still the plan's)
        self.generation = 0

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.asd_plan_destroy(self.handle)
            self.handle = None

    # -- batch ---------------------------------------------------------------
    def init(self, l0, u0, lhat: Sequence[torch.Tensor], uhat: Sequence[torch.Tensor], c, stream=None):
        """asd_init.  All tensors float32 on the device, [S][n] row-major."""
        self.generation += 1
        lh = (C.c_void_p * max(1, len(lhat)))(*[_ptr(t) for t in lhat])
        uh = (C.c_void_p * max(1, len(uhat)))(*[_ptr(t) for t in uhat])
        b = Batch(self.S, _ptr(l0), _ptr(u0), C.cast(lh, C.POINTER(C.c_void_p)),
                  C.cast(uh, C.POINTER(C.c_void_p)), _ptr(c))
        self._keep = (l0, u0, list(lhat), list(uhat), c)
        _check(lib().asd_init(self.handle, C.byref(b), _stream(stream)))

    def run(self, phase: int, t_begin: int, n_iters: int, stream=None):
        self.generation += 1
        _check(lib().asd_run(self.handle, phase, t_begin, n_iters, _stream(stream)))

    def bound(self, want_x0: bool = False, stream=None):
        out = torch.empty(self.S, dtype=torch.float64, device="cuda")
        x0 = torch.empty(self.S, self.net.sizes[0], dtype=torch.float32, device="cuda") if want_x0 else None
        _check(lib().asd_bound(self.handle, out.data_ptr(), _ptr(x0), _stream(stream)))
        return (out, x0) if want_x0 else out

    def set_budgets(self, budgets: Optional[Sequence[int]], stream=None):
        """asd_set_budgets: per-subproblem Active Set budgets (non-increasing), or None."""
        if budgets is None:
            _check(lib().asd_set_budgets(self.handle, None, _stream(stream)))
            self.budgets = None
            return
        arr = (C.c_int32 * self.S)(*[int(b) for b in budgets])
        _check(lib().asd_set_budgets(self.handle, arr, _stream(stream)))
        self.budgets = [int(b) for b in budgets]

    def set_input_domain(self, domain: int, centre: Optional[torch.Tensor] = None,
                         radius: Optional[torch.Tensor] = None, stream=None):
        """asd_set_input_domain: ASD_DOMAIN_BOX, or ASD_DOMAIN_L2 with centres
        [S][n_0] and radii [S] (float32, device; the batches' l0, u0 must be
        the balls' box hulls)."""
        self.generation += 1
        _check(lib().asd_set_input_domain(self.handle, domain, _ptr(centre), _ptr(radius), _stream(stream)))

    # -- Saddle Point (Sec. 5) from the plan's current duals ------------------
    def sp_init(self, sp: SPParams, stream=None):
        """asd_sp_init with a workspace owned by this object (kept until the
        next sp_init)."""
        nbytes = C.c_size_t()
        _check(lib().asd_sp_workspace_size(self.handle, C.byref(nbytes)))
        self._sp_ws = torch.empty(nbytes.value + 256, dtype=torch.uint8, device="cuda")
        aligned = (self._sp_ws.data_ptr() + 255) // 256 * 256
        self._sp = sp
        _check(lib().asd_sp_init(self.handle, C.byref(sp), aligned, nbytes.value, _stream(stream)))

    def sp_run(self, t_begin: int, n_iters: int, stream=None):
        _check(lib().asd_sp_run(self.handle, t_begin, n_iters, _stream(stream)))

    def sp_bound(self, stream=None) -> torch.Tensor:
        out = torch.empty(self.S, dtype=torch.float64, device="cuda")
        _check(lib().asd_sp_bound(self.handle, out.data_ptr(), _stream(stream)))
        return out

    def sp_solve(self, sp: SPParams, stream=None) -> torch.Tensor:
        """Saddle Point (AS-SP after Active Set iterations) from the current
        duals: set-up, sp.iters iterations and the bound."""
        self.sp_init(sp, stream)
        self.sp_run(0, sp.iters, stream)
        return self.sp_bound(stream)

    def sp_read(self, field: int, k: int, stream=None) -> torch.Tensor:
        n = self.net.sizes[k - 1] if field == ASD_SP_ZETA2 else self.net.sizes[k]
        out = torch.empty(self.S, n, dtype=self.dtype, device="cuda")
        _check(lib().asd_sp_read(self.handle, field, k, out.data_ptr(), _stream(stream)))
        return out

    def autotune(self, ktune: int = 2, reps: int = 5, stream=None):
        """asd_plan_autotune (after init); returns the chosen tuning."""
        _check(lib().asd_plan_autotune(self.handle, ktune, reps, _stream(stream)))
        return self.tuning()

    def tuning(self) -> Dict:
        t = Tuning()
        _check(lib().asd_plan_get_tuning(self.handle, C.byref(t)))
        n = self.net.n
        return {f: list(getattr(t, f))[:n] for f in ("ksplit", "fwd_mfma", "bwd_cb", "bwd_pos", "bwd_nt", "fwd_kw", "bwd_kw")}

    def set_tuning(self, d: Dict):
        t = Tuning()
        _check(lib().asd_plan_get_tuning(self.handle, C.byref(t)))
        for f, vals in d.items():
            arr = getattr(t, f)
            for i, v in enumerate(vals):
                arr[i] = int(v)
        _check(lib().asd_plan_set_tuning(self.handle, C.byref(t)))

    def as_iters(self) -> int:
        b = getattr(self, "budgets", None)
        return b[0] if b else self.params.as_iters

    def solve(self, l0, u0, lhat, uhat, c, want_x0: bool = False, stream=None):
        self.init(l0, u0, lhat, uhat, c, stream)
        self.run(ASD_PHASE_BIGM, 0, self.params.bigm_iters, stream)
        self.run(ASD_PHASE_AS, 0, self.as_iters(), stream)
        return self.bound(want_x0, stream)

    def check_finite(self, lb: torch.Tensor, stream=None) -> torch.Tensor:
        """asd_check_finite: int32 flags [S] (bit 0: bound not finite, bit 1: a multiplier not
        finite, bit 2: invalid inputs loaded by asd_init)."""
        lb = lb.to(device="cuda", dtype=torch.float64).contiguous()
        flags = torch.empty(self.S, dtype=torch.int32, device="cuda")
        _check(lib().asd_check_finite(self.handle, lb.data_ptr(), flags.data_ptr(), _stream(stream)))
        return flags

    def solve_graph(self, l0, u0, lhat, uhat, c, stream=None):
        """asd_solve_graph: asd_solve with the iterations replayed from a HIP graph."""
        self.generation += 1
        lh = (C.c_void_p * max(1, len(lhat)))(*[_ptr(t) for t in lhat])
        uh = (C.c_void_p * max(1, len(uhat)))(*[_ptr(t) for t in uhat])
        b = Batch(self.S, _ptr(l0), _ptr(u0), C.cast(lh, C.POINTER(C.c_void_p)),
                  C.cast(uh, C.POINTER(C.c_void_p)), _ptr(c))
        self._keep = (l0, u0, list(lhat), list(uhat), c)
        out = torch.empty(self.S, dtype=torch.float64, device="cuda")
        # a graph is captured from a stream of its own (not the default stream)
        cur = torch.cuda.current_stream() if stream is None else stream
        if getattr(self, "_graph_stream", None) is None:
            self._graph_stream = torch.cuda.Stream()
        gs = self._graph_stream
        gs.wait_stream(cur)
        _check(lib().asd_solve_graph(self.handle, C.byref(b), out.data_ptr(), gs.cuda_stream))
        cur.wait_stream(gs)
        return out

    # -- state ---------------------------------------------------------------
    def _n(self, field, k):
        return self.net.sizes[k - 1] if field == ASD_F_MASK_XPREV else self.net.sizes[k]

    def get(self, field: int, k: int, q: int = 0, stream=None) -> torch.Tensor:
        dst = torch.empty(self.S, self._n(field, k), dtype=self.dtype, device="cuda")
        _check(lib().asd_state_get(self.handle, field, k, q, dst.data_ptr(), _stream(stream)))
        return dst

    def set(self, field: int, k: int, src: torch.Tensor, q: int = 0, stream=None):
        self.generation += 1
        src = src.to(device="cuda", dtype=self.dtype).contiguous()
        assert tuple(src.shape) == (self.S, self._n(field, k))
        _check(lib().asd_state_set(self.handle, field, k, q, src.data_ptr(), _stream(stream)))
        torch.cuda.current_stream().synchronize() if stream is None else stream.synchronize()

    def counts(self) -> Counts:
        c = Counts()
        _check(lib().asd_state_get_counts(self.handle, C.byref(c)))
        return c

    def set_counts(self, n_masks: int, step: int, mask_step: Sequence[int], recompute: bool = True,
                   stream=None):
        self.generation += 1
        c = Counts()
        c.n_masks, c.step = n_masks, step
        for q, v in enumerate(mask_step):
            c.mask_step[q] = v
        _check(lib().asd_state_set_counts(self.handle, C.byref(c), int(recompute), _stream(stream)))

    # -- evaluation ----------------------------------------------------------
    def eval(self, path: int = ASD_EVAL_GENERAL, stream=None) -> Dict:
        """asd_eval at the current duals: objective (general path only), x*,
        z*, f, g and the supergradient, through the general kernels or the
        iteration kernels (path ASD_EVAL_ITERATION)."""
        n, S, sizes = self.net.n, self.S, self.net.sizes
        K = self.counts().n_masks
        out = EvalOut()
        out.path = path
        E = lambda k: torch.empty(S, sizes[k], device="cuda", dtype=self.dtype)
        want_obj = path == ASD_EVAL_GENERAL or self.params.precision == ASD_PREC_FP64
        res = {"obj": torch.empty(S, dtype=torch.float64, device="cuda") if want_obj else None,
               "f": [E(k) for k in range(n)],
               "g": [None] + [E(k) for k in range(1, n)],
               "x": [E(k) for k in range(n)],
               "z": [None] + [E(k) for k in range(1, n)],
               "ga": [None] + [E(k) for k in range(1, n)],
               "gb0": [None] + [E(k) for k in range(1, n)],
               "gb1": [None] + [E(k) for k in range(1, n)],
               "gm": [None] + [[E(k) for _ in range(K)] for k in range(1, n)]}
        out.obj = res["obj"].data_ptr() if want_obj else None
        for k in range(n):
            out.xstar[k] = res["x"][k].data_ptr()
            out.f[k] = res["f"][k].data_ptr()
            if k >= 1:
                out.g[k] = res["g"][k].data_ptr()
                out.zstar[k] = res["z"][k].data_ptr()
                out.grad_alpha[k] = res["ga"][k].data_ptr()
                out.grad_beta0[k] = res["gb0"][k].data_ptr()
                out.grad_beta1[k] = res["gb1"][k].data_ptr()
                for q in range(K):
                    out.grad_mask[k][q] = res["gm"][k][q].data_ptr()
        _check(lib().asd_eval(self.handle, C.byref(out), _stream(stream)))
        return res

    def bound_grad(self, g: torch.Tensor, weights: bool = True, box: bool = True, reuse: bool = False,
                   stream=None):
        """asd_bound_grad: gradient of sum_s g[s] d_B(s) at the current duals.

        Returns (dW, db, dl0, du0): dW[k], db[k] float64 tensors shaped like
        layer k+1's weight and bias (None when weights is False), dl0, du0
        [S][n_0] float64 (None when box is False).  reuse: take the minimiser
        of the last asd_bound if the plan's state is unchanged since (the
        weights and the batch must not have been changed in place)."""
        n = self.net.n
        g = g.to(device="cuda", dtype=torch.float64).contiguous()
        assert tuple(g.shape) == (self.S,)
        dW = [torch.empty(tuple(W.shape), dtype=torch.float64, device="cuda") for W in self.net.W] \
            if weights else None
        db = [torch.empty(tuple(b.shape), dtype=torch.float64, device="cuda") for b in self.net.b] \
            if weights else None
        dl0 = torch.empty(self.S, self.net.sizes[0], dtype=torch.float64, device="cuda") if box else None
        du0 = torch.empty_like(dl0) if box else None
        pw = (C.c_void_p * n)(*[t.data_ptr() for t in dW]) if weights else None
        pb = (C.c_void_p * n)(*[t.data_ptr() for t in db]) if weights else None
        _check(lib().asd_bound_grad(self.handle, g.data_ptr(),
                                    C.cast(pw, C.POINTER(C.c_void_p)) if pw is not None else None,
                                    C.cast(pb, C.POINTER(C.c_void_p)) if pb is not None else None,
                                    _ptr(dl0), _ptr(du0), int(reuse), _stream(stream)))
        return dW, db, dl0, du0

    def profile(self, mode):
        """asd_profile_enable: HIP-event pairs around every launch of this plan
        (mode ASD_PROFILE_LAUNCHES, or True: the launches as a solve runs them;
        ASD_PROFILE_KERNELS: every kernel alone; False / 0: off)."""
        _check(lib().asd_profile_enable(self.handle, int(mode)))

    def profile_read(self):
        """asd_profile_read: {(role, layer): (launches, total_ms)}."""
        cap = 256
        arr = (KernelTime * cap)()
        n = C.c_int32()
        _check(lib().asd_profile_read(self.handle, arr, cap, C.byref(n)))
        return {(ROLE_NAMES[arr[i].role], arr[i].layer): (arr[i].launches, arr[i].total_ms)
                for i in range(min(n.value, cap))}

    def oracle(self, k: int, x_prev: torch.Tensor, z: torch.Tensor, stream=None):
        """asd_oracle: explicit mask bits over each neuron's receptive field, LI, UI."""
        L = self.net.layers[k - 1]
        fan = L.spec.n_in if L.kind == "dense" else L.spec.c_in * L.spec.k * L.spec.k
        nw = (fan + 31) // 32
        n = self.net.sizes[k]
        bits = torch.empty(self.S, n, nw, dtype=torch.int32, device="cuda")
        LI = torch.empty(self.S, n, device="cuda", dtype=self.dtype)
        UI = torch.empty(self.S, n, device="cuda", dtype=self.dtype)
        x_prev = x_prev.to(self.dtype).contiguous()
        z = z.to(self.dtype).contiguous()
        _check(lib().asd_oracle(self.handle, k, _ptr(x_prev), _ptr(z),
                                bits.data_ptr(), LI.data_ptr(), UI.data_ptr(), _stream(stream)))
        return bits, LI, UI, fan


def unpack_bits(bits: np.ndarray, fan: int) -> np.ndarray:
    """[..., nw] uint32 words -> [..., fan] bool (bit t of word w = entry 32 w + t)."""
    b = np.asarray(bits).astype(np.uint32)
    shifts = np.arange(32, dtype=np.uint32)
    out = ((b[..., :, None] >> shifts) & 1).astype(bool)
    return out.reshape(*b.shape[:-1], -1)[..., :fan]


def solve_group(plans: Sequence["Plan"], batches, streams=None):
    """asd_solve_group: batches[i] = (l0, u0, lhat, uhat, c) for plans[i];
    each plan on its own stream (new streams at default priority unless
    given).  Returns the bounds [S_i] per plan (float64 tensors)."""
    n = len(plans)
    if streams is None:
        streams = [torch.cuda.Stream() for _ in range(n)]
    cur = torch.cuda.current_stream()
    for s_ in streams:
        s_.wait_stream(cur)
    keep, bs = [], []
    for P, (l0, u0, lhat, uhat, c) in zip(plans, batches):
        lh = (C.c_void_p * max(1, len(lhat)))(*[_ptr(t) for t in lhat])
        uh = (C.c_void_p * max(1, len(uhat)))(*[_ptr(t) for t in uhat])
        b = Batch(P.S, _ptr(l0), _ptr(u0), C.cast(lh, C.POINTER(C.c_void_p)), C.cast(uh, C.POINTER(C.c_void_p)),
                  _ptr(c))
        keep.append((lh, uh, l0, u0, lhat, uhat, c))
        P._keep = (l0, u0, list(lhat), list(uhat), c)
        bs.append(b)
    outs = [torch.empty(P.S, dtype=torch.float64, device="cuda") for P in plans]
    parr = (C.c_void_p * n)(*[P.handle.value for P in plans])
    barr = (C.POINTER(Batch) * n)(*[C.pointer(b) for b in bs])
    oarr = (C.c_void_p * n)(*[o.data_ptr() for o in outs])
    sarr = (C.c_void_p * n)(*[s_.cuda_stream for s_ in streams])
    for P in plans:
        P.generation += 1
    _check(lib().asd_solve_group(parr, barr, oarr, n, sarr))
    for s_ in streams:
        cur.wait_stream(s_)
    return outs


def solve_static(net: "Net", params: Params, l0, u0, lhat, uhat, c, want_x0: bool = False, stream=None):
    """asd_solve_static: a whole solve over the library's static workspace
    (no plan, no workspace allocation); returns the bounds [S] (and x*_0)."""
    S = l0.shape[0]
    lh = (C.c_void_p * max(1, len(lhat)))(*[_ptr(t) for t in lhat])
    uh = (C.c_void_p * max(1, len(uhat)))(*[_ptr(t) for t in uhat])
    b = Batch(S, _ptr(l0), _ptr(u0), C.cast(lh, C.POINTER(C.c_void_p)), C.cast(uh, C.POINTER(C.c_void_p)), _ptr(c))
    out = torch.empty(S, dtype=torch.float64, device="cuda")
    x0 = torch.empty(S, net.sizes[0], dtype=torch.float32, device="cuda") if want_x0 else None
    _check(lib().asd_solve_static(net.handle, C.byref(params), C.byref(b), out.data_ptr(), _ptr(x0),
                                  _stream(stream)))
    return (out, x0) if want_x0 else out


class BoundFunction(torch.autograd.Function):
    """Solves the batch and returns the FP64 bounds [S]; the backward pass is
    the gradient of the bound at the final duals and active sets (Danskin,
    asd_bound_grad) with respect to the net's weights and biases and the
    input box, the pre-activation bounds held fixed.

    Usage: BoundFunction.apply(plan, l0, u0, lhat, uhat, c, *plan.net.W, *plan.net.b)
    with lhat/uhat tuples; set requires_grad on the tensors whose gradient is
    wanted (the net's W/b tensors are the ones the library reads)."""

    @staticmethod
    def forward(ctx, plan, l0, u0, lhat, uhat, c, *params):
        ctx.plan = plan
        ctx.n = plan.net.n
        lb = plan.solve(l0, u0, list(lhat), list(uhat), c)
        ctx.generation = plan.generation
        return lb

    @staticmethod
    def backward(ctx, glb):
        plan = ctx.plan
        if plan.generation != ctx.generation:
            raise RuntimeError("BoundFunction.backward: the plan's duals or batch changed after this forward "
                               "pass (another solve, run, init or state_set on the same plan); the gradient "
                               "would belong to a different solve.  Give each forward pass its own plan, or "
                               "run the backward pass before reusing the plan.")
        need_w = any(ctx.needs_input_grad[6:])
        need_box = ctx.needs_input_grad[1] or ctx.needs_input_grad[2]
        # the forward pass ended with asd_bound on this plan; autograd runs
        # the backward pass before any optimiser step touches the weights
        dW, db, dl0, du0 = plan.bound_grad(glb, weights=need_w, box=need_box, reuse=True)
        n = ctx.n
        gw = [None] * n if dW is None else [t.to(torch.float32) for t in dW]
        gb = [None] * n if db is None else [t.to(torch.float32) for t in db]
        gl = dl0.to(torch.float32) if dl0 is not None else None
        gu = du0.to(torch.float32) if du0 is not None else None
        return (None, gl, gu, None, None, None, *gw, *gb)
