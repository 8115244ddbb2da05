"""ctypes binding of liblqmg (include/lqmg.h).

Argument marshalling only: every step of the computation runs in the HIP
library.  Device memory comes from torch tensors on the current HIP device;
the context issues its work on the stream given at creation (default: torch's
current stream).  The library must be built (``paper_1509_06865_amd.build``);
there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, fields

import torch

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "lib", "liblqmg.so")
_lib = None

LQ_OK, LQ_WARN_NOCONV = 0, 1
PREC_FP64, PREC_MIXED = 0, 1
SMOOTH_SAP, SMOOTH_GMRES = 0, 1
EXPORTED = ["lq_params_default", "lq_create", "lq_destroy", "lq_last_error", "q_apply", "q_apply_c64",
            "mg_setup", "mg_solve_shifted", "rqi_lowmodes", "mg_info", "mg_get_interp", "mg_get_coarse",
            "mg_restrict", "mg_prolong", "mg_coarse_apply", "mg_smooth", "mg_cycle", "lq_inner_products",
            "lq_kernel_timer_start", "lq_kernel_timer_read", "lq_herm_eigh", "lq_coarse_variant", "lq_ptc_forward", "lq_mod_relu", "lq_ptc_backward",
            "lq_mod_relu_backward", "lq_proj_loss", "lq_adam_step", "lq_inner_products_noalloc", "mg_info2",
            "mg_get_level2", "lma_low", "lma_high", "lq_timeslice_products", "lanczos_lowmodes",
            "lq_clover", "lq_ptc_forward_bf16", "lq_ptc_backward_bf16"]

# kernel classes of lq_kernel_timer_start
KT_WILSON, KT_SAP, KT_RESTRICT, KT_PROLONG, KT_COARSE, KT_GRAM, KT_COMBINE = range(7)


class LQError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"liblqmg error {code}: {msg}")
        self.code = code


class _Params(C.Structure):
    _fields_ = [("precision", C.c_int), ("smoother", C.c_int), ("pre", C.c_int), ("post", C.c_int),
                ("sap_mr", C.c_int), ("gmres_smooth_m", C.c_int), ("coarse_m", C.c_int),
                ("coarse_restarts", C.c_int), ("coarse_tol", C.c_double), ("fgmres_m", C.c_int),
                ("fgmres_restarts", C.c_int), ("n_init", C.c_int), ("n_setup", C.c_int),
                ("rqi_block", C.c_int), ("rqi_max_sweeps", C.c_int), ("rqi_solve_tol", C.c_double),
                ("rayleigh_ritz", C.c_int), ("rqi_guard", C.c_int), ("rqi_solve_restarts", C.c_int),
                ("rqi_deflate", C.c_int), ("rqi_start_passes", C.c_int), ("graphs", C.c_int),
                ("coarse_bf16", C.c_int), ("coarse2_m", C.c_int), ("coarse2_restarts", C.c_int),
                ("coarse2_tol", C.c_double), ("smooth1_m", C.c_int), ("post1", C.c_int),
                ("rqi_stall_restarts", C.c_int), ("rqi_stall_eps", C.c_double)]


class _SolveStats(C.Structure):
    _fields_ = [("iters", C.c_int * 16), ("relres", C.c_double * 16), ("coarse_iters", C.c_int)]


class _RQIStats(C.Structure):
    _fields_ = [("sweeps", C.c_int), ("solves", C.c_int), ("fgmres_iters", C.c_int), ("p_rebuilds", C.c_int),
                ("t_solve", C.c_double), ("t_ortho", C.c_double), ("t_rebuild", C.c_double),
                ("t_rq", C.c_double)]


@dataclass
class MGParams:
    """Mirror of lq_mg_params; None fields keep the library default."""
    precision: int | None = None
    smoother: int | None = None
    pre: int | None = None
    post: int | None = None
    sap_mr: int | None = None
    gmres_smooth_m: int | None = None
    coarse_m: int | None = None
    coarse_restarts: int | None = None
    coarse_tol: float | None = None
    fgmres_m: int | None = None
    fgmres_restarts: int | None = None
    n_init: int | None = None
    n_setup: int | None = None
    rqi_block: int | None = None
    rqi_max_sweeps: int | None = None
    rqi_solve_tol: float | None = None
    rayleigh_ritz: int | None = None
    rqi_guard: int | None = None
    rqi_solve_restarts: int | None = None
    rqi_deflate: int | None = None
    rqi_start_passes: int | None = None
    graphs: int | None = None
    coarse_bf16: int | None = None
    coarse2_m: int | None = None
    coarse2_restarts: int | None = None
    coarse2_tol: float | None = None
    smooth1_m: int | None = None
    post1: int | None = None
    rqi_stall_restarts: int | None = None
    rqi_stall_eps: float | None = None

    def to_c(self, lib) -> _Params:
        p = _Params()
        lib.lq_params_default(C.byref(p))
        for f in fields(self):
            v = getattr(self, f.name)
            if v is not None:
                setattr(p, f.name, v)
        return p


def library_path() -> str:
    return _LIB_PATH


def load():
    """Load liblqmg.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise ImportError(f"{_LIB_PATH} is missing: run `python -m paper_1509_06865_amd.build` first")
    lib = C.CDLL(_LIB_PATH)
    vp, i, d = C.c_void_p, C.c_int, C.c_double
    ip, dp = C.POINTER(C.c_int), C.POINTER(C.c_double)
    sig = {
        "lq_params_default": (i, [C.POINTER(_Params)]),
        "lq_create": (i, [C.POINTER(vp), ip, i, vp]),
        "lq_destroy": (i, [vp]),
        "lq_last_error": (C.c_char_p, [vp]),
        "q_apply": (i, [vp, vp, d, vp, vp, i]),
        "q_apply_c64": (i, [vp, vp, d, vp, vp, i]),
        "mg_setup": (i, [vp, vp, d, i, ip, ip, vp, C.POINTER(_Params)]),
        "mg_info2": (i, [vp, ip, ip]),
        "lma_low": (i, [vp, vp, d, i, vp, dp, dp, d, dp, dp, ip]),
        "lma_high": (i, [vp, vp, d, i, vp, dp, dp, d, i, vp, d, dp]),
        "lq_timeslice_products": (i, [vp, i, vp, i, vp, vp]),
        "lanczos_lowmodes": (i, [vp, vp, d, i, i, i, d, i, vp, dp, vp, dp, ip]),
        "lq_clover": (i, [vp, vp, d]),
        "lq_ptc_forward_bf16": (i, [vp, vp, i, vp, i, vp, vp]),
        "mg_get_level2": (i, [vp, vp, vp]),
        "mg_solve_shifted": (i, [vp, i, dp, vp, vp, d, C.POINTER(_SolveStats)]),
        "rqi_lowmodes": (i, [vp, i, d, dp, vp, dp, vp, i, C.POINTER(_RQIStats)]),
        "mg_info": (i, [vp, ip, ip]),
        "mg_get_interp": (i, [vp, vp]),
        "mg_get_coarse": (i, [vp, vp]),
        "mg_restrict": (i, [vp, i, vp, vp]),
        "mg_prolong": (i, [vp, i, vp, vp]),
        "mg_coarse_apply": (i, [vp, i, dp, vp, vp]),
        "mg_smooth": (i, [vp, i, dp, vp, vp, i]),
        "mg_cycle": (i, [vp, i, dp, vp, vp]),
        "lq_inner_products": (i, [vp, i, vp, i, vp, C.c_longlong, vp]),
        "lq_inner_products_noalloc": (i, [vp, i, vp, i, vp, C.c_longlong, vp]),
        "lq_kernel_timer_start": (i, [i]),
        "lq_kernel_timer_read": (i, [C.POINTER(C.c_longlong), dp, dp]),
        "lq_herm_eigh": (i, [i, vp, vp, vp]),
        "lq_coarse_variant": (i, [i]),
        "lq_ptc_forward": (i, [vp, vp, i, vp, i, vp, vp]),
        "lq_mod_relu": (i, [vp, i, vp, vp, vp]),
        "lq_ptc_backward": (i, [vp, vp, i, vp, i, vp, vp, vp, vp]),
        "lq_ptc_backward_bf16": (i, [vp, vp, i, vp, i, vp, vp, vp, vp]),
        "lq_mod_relu_backward": (i, [vp, i, vp, vp, vp, vp, vp]),
        "lq_proj_loss": (i, [vp, ip, i, vp, i, vp, dp, vp]),
        "lq_adam_step": (i, [vp, C.c_longlong, vp, vp, vp, vp, d, d, d, d, i]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _ptr(t: torch.Tensor | None):
    if t is None:
        return None
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return C.c_void_p(t.data_ptr())


def _need(t: torch.Tensor, name: str, shape, dtype) -> None:
    """Reject a tensor the library would read out of bounds or misinterpret:
    the C side cannot check sizes."""
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be on the HIP device")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")


def _dbl(vals):
    arr = (C.c_double * len(vals))(*[float(v) for v in vals])
    return arr


class Context:
    """One lattice (dims = (X, Y, Z, T), t_bc = -1 antiperiodic / +1 periodic)."""

    def __init__(self, dims, t_bc: int = -1, stream: torch.cuda.Stream | None = None):
        self.lib = load()
        self.dims = tuple(int(d) for d in dims)
        self.V = self.dims[0] * self.dims[1] * self.dims[2] * self.dims[3]
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = C.c_void_p()
        dims_c = (C.c_int * 4)(*self.dims)
        rc = self.lib.lq_create(C.byref(h), dims_c, int(t_bc), C.c_void_p(self.stream.cuda_stream))
        if rc != 0:
            raise LQError(rc, "lq_create failed")
        self.h = h
        self.nv = None
        self.n_agg = None

    def close(self):
        if getattr(self, "h", None):
            self.lib.lq_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, allow_warn=False):
        if rc < 0 or (rc > 0 and not allow_warn):
            raise LQError(rc, self.lib.lq_last_error(self.h).decode())
        return rc

    # -- Q ----------------------------------------------------------------------
    def clover(self, U: torch.Tensor | None, csw: float):
        """Set the clover term built from U (device [4, 9, V] complex128) with
        coefficient csw for every later operator application; csw = 0 removes
        it.  Drops the hierarchy (call mg_setup afterwards)."""
        if U is not None:
            _need(U, "U", (4, 9, self.V), torch.complex128)
        self._check(self.lib.lq_clover(self.h, _ptr(U) if U is not None else None, float(csw)))

    def q_apply(self, U: torch.Tensor, m0: float, x: torch.Tensor, out: torch.Tensor | None = None):
        n = x.shape[0] if x.dim() == 3 else 1
        y = torch.empty_like(x) if out is None else out
        if x.dtype == torch.complex128:
            self._check(self.lib.q_apply(self.h, _ptr(U), float(m0), _ptr(x), _ptr(y), n))
        elif x.dtype == torch.complex64:
            self._check(self.lib.q_apply_c64(self.h, _ptr(U), float(m0), _ptr(x), _ptr(y), n))
        else:
            raise TypeError("x must be complex64 or complex128")
        return y

    def ptc_forward(self, U: torch.Tensor, phi: torch.Tensor, W: torch.Tensor):
        """One parallel-transport convolution (complex128): phi [c_in, 12, V],
        W [c_out, c_in, 81, 4, 4] -> [c_out, 12, V]."""
        c_in, c_out = int(phi.shape[0]), int(W.shape[0])
        self._net_args(U, phi, W, c_in, c_out)
        out = torch.empty((c_out,) + tuple(phi.shape[1:]), dtype=phi.dtype, device=phi.device)
        self._check(self.lib.lq_ptc_forward(self.h, _ptr(U), c_in, _ptr(phi), c_out, _ptr(W.contiguous()),
                                            _ptr(out)))
        return out

    def ptc_forward_bf16(self, U: torch.Tensor, phi: torch.Tensor, W: torch.Tensor):
        """The same layer on the bfloat16 matrix cores (FP32 accumulation), c_in, c_out <= 24."""
        c_in, c_out = int(phi.shape[0]), int(W.shape[0])
        self._net_args(U, phi, W, c_in, c_out)
        out = torch.empty((c_out,) + tuple(phi.shape[1:]), dtype=phi.dtype, device=phi.device)
        self._check(self.lib.lq_ptc_forward_bf16(self.h, _ptr(U), c_in, _ptr(phi), c_out, _ptr(W.contiguous()),
                                                 _ptr(out)))
        return out

    def ptc_backward(self, U: torch.Tensor, phi: torch.Tensor, W: torch.Tensor, g_out: torch.Tensor):
        """Gradients (same form as g_out = dL/dRe out + i dL/dIm out) of a real
        loss with respect to phi and W through one layer."""
        c_in, c_out = int(phi.shape[0]), int(W.shape[0])
        self._net_args(U, phi, W, c_in, c_out)
        _need(g_out, "g_out", (c_out, 12, self.V), torch.complex128)
        g_in = torch.empty_like(phi)
        g_W = torch.empty_like(W)
        self._check(self.lib.lq_ptc_backward(self.h, _ptr(U), c_in, _ptr(phi), c_out, _ptr(W.contiguous()),
                                             _ptr(g_out.contiguous()), _ptr(g_in), _ptr(g_W)))
        return g_in, g_W

    def ptc_backward_bf16(self, U: torch.Tensor, phi: torch.Tensor, W: torch.Tensor, g_out: torch.Tensor,
                          need_in: bool = True, need_W: bool = True):
        """The same gradients on the bfloat16 matrix cores (FP32 accumulation),
        c_in, c_out <= 24; a gradient not asked for is returned as None."""
        c_in, c_out = int(phi.shape[0]), int(W.shape[0])
        self._net_args(U, phi, W, c_in, c_out)
        _need(g_out, "g_out", (c_out, 12, self.V), torch.complex128)
        g_in = torch.empty_like(phi) if need_in else None
        g_W = torch.empty_like(W) if need_W else None
        self._check(self.lib.lq_ptc_backward_bf16(self.h, _ptr(U), c_in, _ptr(phi), c_out, _ptr(W.contiguous()),
                                                  _ptr(g_out.contiguous()), _ptr(g_in), _ptr(g_W)))
        return g_in, g_W

    def _net_args(self, U, phi, W, c_in, c_out):
        _need(U, "U", (4, 9, self.V), torch.complex128)
        _need(phi, "phi", (c_in, 12, self.V), torch.complex128)
        _need(W, "W", (c_out, c_in, 81, 4, 4), torch.complex128)

    def mod_relu(self, phi: torch.Tensor, b: torch.Tensor):
        """The network's nonlinearity: phi [C, 12, V] complex128, b [C] float64 (device)."""
        _need(phi, "phi", (int(phi.shape[0]), 12, self.V), torch.complex128)
        out = torch.empty_like(phi)
        bb = b.to(device=phi.device, dtype=torch.float64).contiguous()
        _need(bb, "b", (int(phi.shape[0]),), torch.float64)
        self._check(self.lib.lq_mod_relu(self.h, int(phi.shape[0]), _ptr(phi), _ptr(bb), _ptr(out)))
        return out

    def mod_relu_backward(self, phi: torch.Tensor, b: torch.Tensor, g_out: torch.Tensor):
        """Gradients through the nonlinearity: (g_phi, g_b)."""
        C_ = int(phi.shape[0])
        _need(phi, "phi", (C_, 12, self.V), torch.complex128)
        _need(g_out, "g_out", (C_, 12, self.V), torch.complex128)
        bb = b.to(device=phi.device, dtype=torch.float64).contiguous()
        _need(bb, "b", (C_,), torch.float64)
        g_phi = torch.empty_like(phi)
        g_b = torch.empty_like(bb)
        self._check(self.lib.lq_mod_relu_backward(self.h, int(phi.shape[0]), _ptr(phi), _ptr(bb),
                                                  _ptr(g_out.contiguous()), _ptr(g_phi), _ptr(g_b)))
        return g_phi, g_b

    def _forward_keep(self, U, phi0, weights, biases, bf16=False):
        inputs, pre = [], []
        phi = phi0
        layer_fn = self.ptc_forward_bf16 if bf16 else self.ptc_forward
        for layer, W in enumerate(weights):
            inputs.append(phi)
            phi = layer_fn(U, phi, W)
            if layer < len(weights) - 1:
                pre.append(phi)
                phi = self.mod_relu(phi, biases[layer])
        return phi, inputs, pre

    def lcnn_backward(self, U: torch.Tensor, phi0: torch.Tensor, weights, biases, g_out: torch.Tensor,
                      kept=None, bf16: bool = False):
        """Gradients of a real loss with respect to every weight and bias of the
        network, given g_out for its output: the forward is rerun (or its kept
        intermediates used) to have each layer's input, then the library's
        backward calls run in reverse order (the layers' on the bfloat16
        matrix cores with bf16)."""
        _, inputs, pre = kept if kept is not None else self._forward_keep(U, phi0, weights, biases, bf16)
        layer_bwd = self.ptc_backward_bf16 if bf16 else self.ptc_backward
        g = g_out
        gW, gb = [None] * len(weights), [None] * len(biases)
        for layer in range(len(weights) - 1, -1, -1):
            if layer < len(weights) - 1:
                g, gb[layer] = self.mod_relu_backward(pre[layer], biases[layer], g)
            g, gW[layer] = layer_bwd(U, inputs[layer], weights[layer], g)
        return gW, gb

    def proj_loss(self, X: torch.Tensor, u: torch.Tensor, agg, grad: bool = True):
        """The network's training loss for outputs X [n_out, 12, V] and targets
        u [K, 12, V] over aggregates agg; returns (loss, dL/dX or None)."""
        _need(X, "X", (int(X.shape[0]), 12, self.V), torch.complex128)
        _need(u, "u", (int(u.shape[0]), 12, self.V), torch.complex128)
        a = (C.c_int * 4)(*agg)
        loss = C.c_double()
        g = torch.empty_like(X) if grad else None
        self._check(self.lib.lq_proj_loss(self.h, a, int(X.shape[0]), _ptr(X.contiguous()), int(u.shape[0]),
                                          _ptr(u.contiguous()), C.byref(loss), _ptr(g)))
        return loss.value, g

    def adam_step(self, p: torch.Tensor, g: torch.Tensor, m: torch.Tensor, v: torch.Tensor, lr: float,
                  betas=(0.9, 0.999), eps: float = 1e-8, t: int = 1):
        """One Adam step in place on p (real or complex; complex as real and
        imaginary parts); m, v are real tensors of p's real view."""
        pr = torch.view_as_real(p) if p.is_complex() else p
        gr = torch.view_as_real(g) if g.is_complex() else g
        for name, arr in (("g", gr), ("m", m), ("v", v)):
            _need(arr, name, tuple(pr.shape), torch.float64)
        if pr.dtype != torch.float64 or pr.device.type != "cuda":
            raise TypeError("p must be a float64 or complex128 tensor on the HIP device")
        self._check(self.lib.lq_adam_step(self.h, pr.numel(), _ptr(pr), _ptr(gr.contiguous()), _ptr(m), _ptr(v),
                                          float(lr), float(betas[0]), float(betas[1]), float(eps), int(t)))

    def lcnn_train_step(self, U, phi0, weights, biases, u, agg, state, lr, t, bf16: bool = False):
        """One training step of the network on the device: forward, loss over
        the aggregates, backward, Adam (step t) on every weight and bias in
        place.  state: the Adam moments, a list of (m, v) per parameter
        (weights then biases).  bf16: the layers' forward and backward on the
        bfloat16 matrix cores (weights, moments and the update stay FP64).
        Returns the loss before the update."""
        out, inputs, pre = self._forward_keep(U, phi0, weights, biases, bf16)
        loss, gX = self.proj_loss(out, u, agg)
        gW, gb = self.lcnn_backward(U, phi0, weights, biases, gX, kept=(out, inputs, pre), bf16=bf16)
        for p, g, (m, v) in zip(list(weights) + list(biases), gW + gb, state):
            self.adam_step(p, g, m, v, lr, t=t)
        return loss

    def lcnn_forward(self, U: torch.Tensor, phi0: torch.Tensor, weights, biases, bf16: bool = False):
        """The learned setup's network on the device: the layers and the
        nonlinearities in turn (each a library call); bf16 runs the layers on
        the bfloat16 matrix cores (inference; widths up to 24)."""
        phi = phi0
        layer_fn = self.ptc_forward_bf16 if bf16 else self.ptc_forward
        for layer, W in enumerate(weights):
            phi = layer_fn(U, phi, W)
            if layer < len(weights) - 1:
                phi = self.mod_relu(phi, biases[layer])
        return phi

    # -- multigrid ------------------------------------------------------------------
    def mg_setup(self, U, m0, agg, tv0, params: MGParams | None = None, agg2=None, nv2=None):
        """Two levels (aggregates agg, Nv = tv0.shape[0] test vectors), or three
        with agg2 (blocks of the lattice of aggregates) and nv2 level-2 vectors."""
        p = (params or MGParams()).to_c(self.lib)
        n_levels = 2 if agg2 is None else 3
        aggs = [list(agg)] + ([list(agg2)] if agg2 is not None else [])
        agg_c = ((C.c_int * 4) * len(aggs))(*[(C.c_int * 4)(*[int(a) for a in row]) for row in aggs])
        nvs = [int(tv0.shape[0])] + ([int(nv2)] if agg2 is not None else [])
        nv_c = (C.c_int * len(nvs))(*nvs)
        self._check(self.lib.mg_setup(self.h, _ptr(U), float(m0), n_levels, nv_c,
                                      C.cast(agg_c, C.POINTER(C.c_int)), _ptr(tv0), C.byref(p)))
        nv, na = C.c_int(), C.c_int()
        self._check(self.lib.mg_info(self.h, C.byref(nv), C.byref(na)))
        self.nv, self.n_agg = nv.value, na.value
        self.n_levels = n_levels
        self.nv2 = self.n_agg2 = None
        if n_levels == 3:
            self._check(self.lib.mg_info2(self.h, C.byref(nv), C.byref(na)))
            self.nv2, self.n_agg2 = nv.value, na.value

    def get_level2(self):
        """(P2 [Nv2, nA, 2 Nv], Q_c2 [nA2, 5, 2 Nv2, 2 Nv2]) of a three-level hierarchy (complex128)."""
        P2 = torch.empty((self.nv2, self.n_agg, 2 * self.nv), dtype=torch.complex128, device="cuda")
        Qc2 = torch.empty((self.n_agg2, 5, 2 * self.nv2, 2 * self.nv2), dtype=torch.complex128, device="cuda")
        self._check(self.lib.mg_get_level2(self.h, _ptr(P2), _ptr(Qc2)))
        return P2, Qc2

    def mg_solve_shifted(self, sigma, rhs, tol, out=None):
        n = rhs.shape[0]
        x = torch.empty_like(rhs) if out is None else out
        st = _SolveStats()
        rc = self._check(self.lib.mg_solve_shifted(self.h, n, _dbl(sigma), _ptr(rhs), _ptr(x), float(tol),
                                                   C.byref(st)), allow_warn=True)
        info = {"iters": list(st.iters)[:n], "relres": list(st.relres)[:n], "coarse_iters": st.coarse_iters,
                "converged": rc == 0}
        return x, info

    def rqi_lowmodes(self, n_eig, tol, V0=None, out=None):
        dev = torch.device("cuda", torch.cuda.current_device())
        V = torch.empty((n_eig, 12, self.V), dtype=torch.complex128, device=dev) if out is None else out
        lam = (C.c_double * n_eig)()
        res = (C.c_double * n_eig)()
        st = _RQIStats()
        n_v0 = 0 if V0 is None else int(V0.shape[0])
        rc = self._check(self.lib.rqi_lowmodes(self.h, int(n_eig), float(tol), lam, _ptr(V), res, _ptr(V0), n_v0,
                                               C.byref(st)), allow_warn=True)
        info = {f[0]: getattr(st, f[0]) for f in _RQIStats._fields_}
        info["converged"] = rc == 0
        return list(lam), V, list(res), info

    def get_interp(self):
        P = torch.empty((self.nv, 12, self.V), dtype=torch.complex128, device="cuda")
        self._check(self.lib.mg_get_interp(self.h, _ptr(P)))
        return P

    def get_coarse(self):
        n2 = 2 * self.nv
        Qc = torch.empty((self.n_agg, 5, n2, n2), dtype=torch.complex128, device="cuda")
        self._check(self.lib.mg_get_coarse(self.h, _ptr(Qc)))
        return Qc

    def restrict(self, f):
        c = torch.empty((f.shape[0], self.n_agg, 2 * self.nv), dtype=torch.complex128, device=f.device)
        self._check(self.lib.mg_restrict(self.h, f.shape[0], _ptr(f), _ptr(c)))
        return c

    def prolong(self, c):
        f = torch.empty((c.shape[0], 12, self.V), dtype=torch.complex128, device=c.device)
        self._check(self.lib.mg_prolong(self.h, c.shape[0], _ptr(c), _ptr(f)))
        return f

    def coarse_apply(self, sigma, x):
        y = torch.empty_like(x)
        self._check(self.lib.mg_coarse_apply(self.h, x.shape[0], _dbl(sigma), _ptr(x), _ptr(y)))
        return y

    def smooth(self, sigma, r, steps):
        z = torch.empty_like(r)
        self._check(self.lib.mg_smooth(self.h, r.shape[0], _dbl(sigma), _ptr(r), _ptr(z), int(steps)))
        return z

    def inner_products(self, E, W):
        """<E_i, W_k> for device complex128 tensors E [nb, ...] and W [nw, ...]."""
        import numpy as np
        nb, nw = E.shape[0], W.shape[0]
        n = E[0].numel()
        out = np.empty((nb, nw), dtype=np.complex128)
        self._check(self.lib.lq_inner_products(self.h, nb, _ptr(E), nw, _ptr(W), n,
                                               C.c_void_p(out.ctypes.data)))
        return out

    def inner_products_noalloc(self, E, W):
        """As inner_products, through the entry point that allocates no device
        memory (its partial sums live in the library's fixed scratch array)."""
        import numpy as np
        nb, nw = E.shape[0], W.shape[0]
        n = E[0].numel()
        out = np.empty((nb, nw), dtype=np.complex128)
        self._check(self.lib.lq_inner_products_noalloc(self.h, nb, _ptr(E), nw, _ptr(W), n,
                                                       C.c_void_p(out.ctypes.data)))
        return out

    # -- approximate low-mode averaging (sec. 3.2, 3.3) ---------------------------
    def lma_low(self, U, m0, V, lam, eps, cutoff):
        """Low-mode loop and connected correlator per timeslice from approximate
        eigenpairs (V device [n, 12, V] complex128): (loop_low [T], conn_low [T], n_kept)."""
        import numpy as np
        n, T = int(V.shape[0]), self.dims[3]
        _need(V, "V", (n, 12, self.V), torch.complex128)
        lo = np.zeros(2 * T)
        co = np.zeros(2 * T)
        kept = C.c_int()
        self._check(self.lib.lma_low(self.h, _ptr(U), float(m0), n, _ptr(V), _dbl(lam), _dbl(eps), float(cutoff),
                                     lo.ctypes.data_as(C.POINTER(C.c_double)),
                                     co.ctypes.data_as(C.POINTER(C.c_double)), C.byref(kept)))
        return lo[0::2] + 1j * lo[1::2], co[0::2] + 1j * co[1::2], kept.value

    def lma_high(self, U, m0, V, lam, eps, cutoff, eta, tol=1e-10):
        """High-mode loop samples [n_noise, T] for noise fields eta (device [n_noise, 12, V])."""
        import numpy as np
        T = self.dims[3]
        n = 0 if V is None else int(V.shape[0])
        if n:
            _need(V, "V", (n, 12, self.V), torch.complex128)
        _need(eta, "eta", (int(eta.shape[0]), 12, self.V), torch.complex128)
        out = np.zeros((int(eta.shape[0]), 2 * T))
        self._check(self.lib.lma_high(self.h, _ptr(U), float(m0), n, _ptr(V) if n else None,
                                      _dbl(lam) if n else None, _dbl(eps) if n else None, float(cutoff),
                                      int(eta.shape[0]), _ptr(eta), float(tol),
                                      out.ctypes.data_as(C.POINTER(C.c_double))))
        return out[:, 0::2] + 1j * out[:, 1::2]

    def timeslice_products(self, E, W):
        """[T, nb, nw] per-timeslice inner products <E_i, W_k> (device complex128 fields)."""
        import numpy as np
        nb, nw, T = int(E.shape[0]), int(W.shape[0]), self.dims[3]
        out = np.empty((T, nb, nw), dtype=np.complex128)
        self._check(self.lib.lq_timeslice_products(self.h, nb, _ptr(E), nw, _ptr(W), C.c_void_p(out.ctypes.data)))
        return out

    # -- restarted Krylov eigensolver (the comparison of sec. 2.2) -------------------
    def lanczos_lowmodes(self, U, m0, n_eig, v0, tol=1e-10, n_kv=100, n_guard=4, max_restarts=1000):
        """The n_eig lowest-|lambda| eigenpairs of Q by restarted Lanczos on Q^2 (no multigrid).
        v0: device start vector [12, V] complex128.  Returns (lambda, V [n_eig, 12, V] device,
        residuals, {"restarts", "q2_products", "converged"})."""
        import numpy as np
        _need(v0, "v0", (12, self.V), torch.complex128)
        lam = np.zeros(n_eig)
        res = np.zeros(n_eig)
        Vout = torch.empty((n_eig, 12, self.V), dtype=torch.complex128, device=v0.device)
        info = (C.c_int * 3)()
        self._check(self.lib.lanczos_lowmodes(self.h, _ptr(U), float(m0), int(n_eig), int(n_guard), int(n_kv),
                                              float(tol), int(max_restarts), _ptr(v0),
                                              lam.ctypes.data_as(C.POINTER(C.c_double)), _ptr(Vout),
                                              res.ctypes.data_as(C.POINTER(C.c_double)), info))
        return lam, Vout, res, {"restarts": info[0], "q2_products": info[1], "converged": bool(info[2])}

    def cycle(self, sigma, r):
        z = torch.empty_like(r)
        self._check(self.lib.mg_cycle(self.h, r.shape[0], _dbl(sigma), _ptr(r), _ptr(z)))
        return z


def kernel_timer_start(kind: int):
    """Time every launch of one kernel class from now on (-1: off)."""
    rc = load().lq_kernel_timer_start(int(kind))
    if rc != 0:
        raise LQError(rc, "lq_kernel_timer_start: unknown kernel class")


def kernel_timer_read():
    """(launches, total device ms, total algorithmic bytes) since the last start."""
    n, ms, by = C.c_longlong(), C.c_double(), C.c_double()
    rc = load().lq_kernel_timer_read(C.byref(n), C.byref(ms), C.byref(by))
    if rc != 0:
        raise LQError(rc, "lq_kernel_timer_read failed")
    return n.value, ms.value, by.value


def coarse_variant(v: int) -> None:
    """Force coarse-apply kernel v (0..7; 6 = matrix cores in FP32, 7 = matrix cores on bfloat16 operands) for
    every shape, or -1 for the tuned choice."""
    rc = load().lq_coarse_variant(int(v))
    if rc != 0:
        raise LQError(rc, f"lq_coarse_variant({v}) failed")


def herm_eigh(A):
    """Eigenvalues (ascending) and eigenvectors (columns) of a host Hermitian
    complex matrix through the library's dense helper."""
    import numpy as np
    A = np.ascontiguousarray(A, dtype=np.complex128)
    n = A.shape[0]
    w = np.empty(n)
    V = np.empty((n, n), dtype=np.complex128)
    rc = load().lq_herm_eigh(n, C.c_void_p(A.ctypes.data), C.c_void_p(w.ctypes.data), C.c_void_p(V.ctypes.data))
    if rc != 0:
        raise LQError(rc, "lq_herm_eigh failed")
    return w, V
