"""Thin Python binding of libvp (include/vp.h): argument marshalling only.

Every step of an evaluation runs in the library's HIP kernels; this module
only converts arrays and tensors to the pointers and sizes the C ABI takes.
PyTorch provides device memory and streams.  If libvp.so is missing the
import of the library fails loudly: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np
import torch  # loaded first: libvp then shares torch's HIP runtime

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libvp.so")

VP_OK, VP_EINVAL, VP_ENOMEM, VP_EDEVICE, VP_EUNSUPPORTED, VP_EINTERNAL = range(6)
VP_FP64, VP_FP32_BULK = 0, 1
VP_FLAG_AUTOTUNE = 1
VP_FLAG_ONE_STREAM = 2
VP_FLAG_AUTOTUNE_LEAF = 8
KERNELS = {"laplace": 0, "yukawa": 1}
M2L_MODES = {"auto": 0, "fp64": 1, "fp32": 2, "split": 3, "fp64_scaled": 4, "fp32_scaled": 5}
P2P_MODES = {"auto": 0, "pairwise": 1, "tables": 2}
ARR = {
    "src_perm": 0, "tgt_perm": 1, "box": 2, "level_begin": 3,
    "U_ptr": 4, "U_idx": 5, "V_ptr": 6, "V_idx": 7, "W_ptr": 8, "W_idx": 9,
    "X_ptr": 10, "X_idx": 11, "multipole": 12, "local": 13, "src_keys": 14, "tgt_keys": 15,
}
_ARR_DTYPE = {0: np.int32, 1: np.int32, 2: np.int32, 3: np.int32, 4: np.int32, 5: np.int32,
              6: np.int32, 7: np.int32, 8: np.int32, 9: np.int32, 10: np.int32, 11: np.int32,
              12: np.float64, 13: np.float64, 14: np.int64, 15: np.int64}

# Every entry point declared in include/vp.h.
EXPORTS = ("vp_default_options", "vp_plan", "vp_plan_oversampled", "vp_eval", "vp_eval_adjoint", "vp_eval_grad_targets",
           "vp_eval_noalloc", "vp_set_stream", "vp_destroy", "vp_last_error", "vp_get_info", "vp_get_array",
           "vp_set_timing", "vp_get_timing", "vp_correction_blocks")
STAGES = ("charge", "p2m", "m2m", "m2l", "p2l", "l2l", "p2p", "far", "finish", "tables", "corr", "coarse", "p2m_pat", "m2p")


class VPError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"libvp status {status}: {msg}")
        self.status = status


class Options(ctypes.Structure):
    _fields_ = [("order", ctypes.c_int32), ("max_leaf", ctypes.c_int32), ("nbatch", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("m2l_mode", ctypes.c_int32), ("p2p_mode", ctypes.c_int32),
                ("max_level", ctypes.c_int32), ("flags", ctypes.c_int32), ("root", ctypes.c_double * 3),
                ("stream", ctypes.c_void_p), ("kernel", ctypes.c_int32), ("m2l_waves", ctypes.c_int32),
                ("lam", ctypes.c_double), ("table_waves", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class Oversampling(ctypes.Structure):
    _fields_ = [("p", ctypes.c_int32), ("q", ctypes.c_int32), ("nbox", ctypes.c_int64), ("n_in", ctypes.c_int64),
                ("in_start", ctypes.c_void_p), ("out_start", ctypes.c_void_p)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("m", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("nbatch", ctypes.c_int32), ("order", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("m2l_mode", ctypes.c_int32), ("p2p_mode_used", ctypes.c_int32), ("max_leaf", ctypes.c_int32),
                ("nbox", ctypes.c_int32), ("nleaf", ctypes.c_int32), ("nlevels", ctypes.c_int32),
                ("self_targets", ctypes.c_int32), ("list_len", ctypes.c_int64 * 4),
                ("table_leaves", ctypes.c_int64), ("near_pairs", ctypes.c_int64),
                ("workspace_bytes", ctypes.c_int64), ("m2l_translations", ctypes.c_int64),
                ("m2l_tile_ops", ctypes.c_int64), ("table_tile_ops", ctypes.c_int64),
                ("m2l_coarse_translations", ctypes.c_int64), ("m2l_coarse_tile_ops", ctypes.c_int64),
                ("split_level", ctypes.c_int32), ("corr_cells", ctypes.c_int32),
                ("corr_shared_cells", ctypes.c_int32), ("corr_values_read", ctypes.c_int64),
                ("corr_groups", ctypes.c_int32), ("corr_one_block", ctypes.c_int32),
                ("root", ctypes.c_double * 3), ("table_pairs", ctypes.c_int64),
                ("noalloc_bytes", ctypes.c_int64), ("n_in", ctypes.c_int64),
                ("os_p", ctypes.c_int32), ("os_q", ctypes.c_int32), ("kernel", ctypes.c_int32),
                ("table_pattern", ctypes.c_int32), ("lam", ctypes.c_double), ("tuned", ctypes.c_int32),
                ("m2l_waves", ctypes.c_int32), ("table_waves", ctypes.c_int32), ("one_stream", ctypes.c_int32),
                ("tune_ms", ctypes.c_double), ("l2p_from_parents", ctypes.c_int32), ("corr_folded", ctypes.c_int32)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["list_len"] = list(self.list_len)
        d["root"] = list(self.root)
        return d


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libvp.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"libvp.so not found at {path}: run __graft_entry__.build() first "
                          "(there is no CPU fallback)")
    lib = ctypes.CDLL(path)
    vp = ctypes.c_void_p
    dp = ctypes.c_void_p
    lib.vp_default_options.argtypes = [ctypes.POINTER(Options)]
    lib.vp_default_options.restype = None
    lib.vp_plan.argtypes = [dp, dp, dp, ctypes.c_int64, dp, dp, ctypes.c_int64, dp, dp, dp,
                            ctypes.POINTER(Options), ctypes.POINTER(vp)]
    lib.vp_plan.restype = ctypes.c_int
    lib.vp_plan_oversampled.argtypes = [dp, dp, dp, ctypes.c_int64, dp, dp, ctypes.c_int64, dp, dp, dp,
                                        ctypes.POINTER(Oversampling), ctypes.POINTER(Options), ctypes.POINTER(vp)]
    lib.vp_plan_oversampled.restype = ctypes.c_int
    for name in ("vp_eval", "vp_eval_adjoint", "vp_eval_grad_targets", "vp_eval_noalloc"):
        fn = getattr(lib, name)
        fn.argtypes = [vp, dp, dp]
        fn.restype = ctypes.c_int
    lib.vp_set_stream.argtypes = [vp, ctypes.c_void_p]
    lib.vp_set_stream.restype = ctypes.c_int
    lib.vp_destroy.argtypes = [vp]
    lib.vp_destroy.restype = ctypes.c_int
    lib.vp_last_error.argtypes = [vp]
    lib.vp_last_error.restype = ctypes.c_char_p
    lib.vp_get_info.argtypes = [vp, ctypes.POINTER(PlanInfo)]
    lib.vp_get_info.restype = ctypes.c_int
    lib.vp_get_array.argtypes = [vp, ctypes.c_int32, ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)]
    lib.vp_get_array.restype = ctypes.c_int
    lib.vp_set_timing.argtypes = [vp, ctypes.c_int32]
    lib.vp_set_timing.restype = ctypes.c_int
    lib.vp_get_timing.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]
    lib.vp_get_timing.restype = ctypes.c_int
    lib.vp_correction_blocks.argtypes = [ctypes.c_int32, ctypes.c_int32, dp, dp, dp, ctypes.c_int64, dp, dp,
                                         ctypes.c_void_p]
    lib.vp_correction_blocks.restype = ctypes.c_int
    _lib = lib
    return lib


def default_options() -> Options:
    o = Options()
    load_library().vp_default_options(ctypes.byref(o))
    return o


def _host(a, dtype):
    if a is None:
        return None
    if isinstance(a, torch.Tensor):
        a = a.detach().cpu().numpy()
    return np.ascontiguousarray(a, dtype=dtype)


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _current_stream():
    if torch.cuda.is_available():
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return ctypes.c_void_p(0)


class Plan:
    """A static-geometry plan: nodes, weights, targets and correction matrix.

    Targets default to the nodes.  Evaluations take and return float64
    device tensors [nbatch, n] / [nbatch, m] in the caller's order.

    oversampling=dict(p=, q=, in_start=, out_start=, n_in=) builds an
    oversampled plan (vp_plan_oversampled): the nodes x, y, w are the q x q
    sources of every box, the densities are [nbatch, n_in] values at the
    p x p nodes, and the correction columns index those values.
    """

    def __init__(self, x, y, w, tx=None, ty=None, rowptr=None, col=None, val=None, *, order: int = 30,
                 max_leaf: int = 64, nbatch: int = 1, precision: str = "fp64", m2l_mode: str = "auto",
                 p2p_mode: str = "auto", root=None, max_level: int = 0, autotune: bool = False,
                 one_stream: bool = False, oversampling: Optional[dict] = None, kernel: str = "laplace",
                 lam: float = 0.0, autotune_leaf: bool = False, m2l_waves: int = 0, table_waves: int = 0,
                 stream=None):
        lib = load_library()
        self._lib = lib
        self._h = ctypes.c_void_p()
        x = _host(x, np.float64)
        y = _host(y, np.float64)
        w = _host(w, np.float64)
        tx = _host(tx, np.float64)
        ty = _host(ty, np.float64)
        rowptr = _host(rowptr, np.int64)
        col = _host(col, np.int32)
        val = _host(val, np.float64)
        n = x.shape[0]
        m = n if tx is None else tx.shape[0]
        o = default_options()
        o.order = order
        o.max_leaf = max_leaf
        o.nbatch = nbatch
        o.precision = {"fp64": VP_FP64, "fp32": VP_FP32_BULK}[precision]
        o.m2l_mode = M2L_MODES[m2l_mode]
        o.p2p_mode = P2P_MODES[p2p_mode]
        o.max_level = max_level
        o.flags = ((VP_FLAG_AUTOTUNE if autotune else 0) | (VP_FLAG_ONE_STREAM if one_stream else 0)
                   | (VP_FLAG_AUTOTUNE_LEAF if autotune_leaf else 0))
        o.m2l_waves = m2l_waves
        o.table_waves = table_waves
        if root is not None:
            o.root[0], o.root[1], o.root[2] = root
        o.kernel = KERNELS[kernel]
        o.lam = lam
        o.stream = _current_stream() if stream is None else ctypes.c_void_p(stream)
        if oversampling is None:
            st = lib.vp_plan(_ptr(x), _ptr(y), _ptr(w), n, _ptr(tx), _ptr(ty), m, _ptr(rowptr), _ptr(col),
                             _ptr(val), ctypes.byref(o), ctypes.byref(self._h))
            n_in = n
        else:
            ins = _host(oversampling["in_start"], np.int64)
            outs = _host(oversampling["out_start"], np.int64)
            n_in = int(oversampling["n_in"])
            os_ = Oversampling(int(oversampling["p"]), int(oversampling["q"]), ins.shape[0], n_in,
                               ins.ctypes.data, outs.ctypes.data)
            st = lib.vp_plan_oversampled(_ptr(x), _ptr(y), _ptr(w), n, _ptr(tx), _ptr(ty), m, _ptr(rowptr),
                                         _ptr(col), _ptr(val), ctypes.byref(os_), ctypes.byref(o),
                                         ctypes.byref(self._h))
        if st != VP_OK:
            raise VPError(st, lib.vp_last_error(None).decode())
        # n: the length of the density rows (the density values of an oversampled plan)
        self.n, self.m, self.nbatch = n_in, m, nbatch
        self.n_src = n
        self.precision = precision
        self.order = order

    # -- helpers -------------------------------------------------------------
    def _check(self, st):
        if st != VP_OK:
            raise VPError(st, self._lib.vp_last_error(self._h).decode())

    def _dev(self, t: torch.Tensor, length: int, name: str) -> torch.Tensor:
        if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
            raise TypeError(f"{name} must be a CUDA (HIP) tensor")
        if t.dtype != torch.float64:
            raise TypeError(f"{name} must be float64")
        if t.dim() == 1:
            t = t.unsqueeze(0)
        if t.shape != (self.nbatch, length):
            raise ValueError(f"{name} must have shape ({self.nbatch}, {length}), got {tuple(t.shape)}")
        return t.contiguous()

    def set_stream(self, stream=None):
        s = _current_stream() if stream is None else ctypes.c_void_p(stream)
        self._check(self._lib.vp_set_stream(self._h, s))

    # -- evaluations ---------------------------------------------------------
    def eval(self, f: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """u = V f + C f at the targets: [nbatch, m]."""
        f = self._dev(f, self.n, "f")
        if out is None:
            out = torch.empty((self.nbatch, self.m), dtype=torch.float64, device=f.device)
        self._check(self._lib.vp_eval(self._h, ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(out.data_ptr())))
        return out

    def eval_noalloc(self, f: torch.Tensor, out: torch.Tensor) -> torch.Tensor:
        """vp_eval_noalloc: as eval, with the workspace in the library's static
        device array (the caller provides the output)."""
        f = self._dev(f, self.n, "f")
        out = self._dev(out, self.m, "out")
        self._check(self._lib.vp_eval_noalloc(self._h, ctypes.c_void_p(f.data_ptr()),
                                              ctypes.c_void_p(out.data_ptr())))
        return out

    def eval_adjoint(self, g: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """df = (V + C)^T g at the nodes: [nbatch, n]."""
        g = self._dev(g, self.m, "g")
        if out is None:
            out = torch.empty((self.nbatch, self.n), dtype=torch.float64, device=g.device)
        self._check(self._lib.vp_eval_adjoint(self._h, ctypes.c_void_p(g.data_ptr()),
                                              ctypes.c_void_p(out.data_ptr())))
        return out

    def eval_grad_targets(self, f: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """Target gradient of the smooth sum: [nbatch, 2, m]."""
        f = self._dev(f, self.n, "f")
        if out is None:
            out = torch.empty((self.nbatch, 2, self.m), dtype=torch.float64, device=f.device)
        self._check(self._lib.vp_eval_grad_targets(self._h, ctypes.c_void_p(f.data_ptr()),
                                                   ctypes.c_void_p(out.data_ptr())))
        return out

    # -- introspection -------------------------------------------------------
    def info(self) -> dict:
        inf = PlanInfo()
        self._check(self._lib.vp_get_info(self._h, ctypes.byref(inf)))
        return inf.as_dict()

    def get_array(self, name: str) -> np.ndarray:
        which = ARR[name]
        cnt = ctypes.c_int64()
        self._check(self._lib.vp_get_array(self._h, which, None, ctypes.byref(cnt)))
        out = np.empty(cnt.value, dtype=_ARR_DTYPE[which])
        self._check(self._lib.vp_get_array(self._h, which, out.ctypes.data_as(ctypes.c_void_p), ctypes.byref(cnt)))
        return out

    def set_timing(self, enable: bool = True):
        """Enable (and clear) or disable per-stage HIP-event timing."""
        self._check(self._lib.vp_set_timing(self._h, 1 if enable else 0))

    def timing(self) -> dict:
        """Summed milliseconds per stage and the number of timed evaluations."""
        ms = (ctypes.c_double * len(STAGES))()
        cnt = ctypes.c_int64()
        self._check(self._lib.vp_get_timing(self._h, ms, ctypes.byref(cnt)))
        return {"evals": cnt.value, "ms": dict(zip(STAGES, list(ms)))}

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            self._lib.vp_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ----------------------------------------------------------------------------
# autograd
# ----------------------------------------------------------------------------
class VolumePotential(torch.autograd.Function):
    """u = (V + C) f with dL/df = (V + C)^T dL/du (vp_eval / vp_eval_adjoint)."""

    @staticmethod
    def forward(ctx, f, plan: Plan):
        ctx.plan = plan
        return plan.eval(f.detach())

    @staticmethod
    def backward(ctx, g):
        return ctx.plan.eval_adjoint(g.contiguous()), None


class TargetPotential(torch.autograd.Function):
    """u(t) = V f at the plan's targets, differentiable in the targets and f.

    targets is the [2, m] tensor the plan was built from; its gradient is
    sum_b g_b[i] grad_t V_b(t_i) (vp_eval_grad_targets), the density gradient
    is the adjoint.  Moving targets requires a new plan.
    """

    @staticmethod
    def forward(ctx, targets, f, plan: Plan):
        ctx.plan = plan
        ctx.save_for_backward(f.detach())
        return plan.eval(f.detach())

    @staticmethod
    def backward(ctx, g):
        (f,) = ctx.saved_tensors
        plan = ctx.plan
        gt = None
        if ctx.needs_input_grad[0]:
            grad = plan.eval_grad_targets(f)  # [nbatch, 2, m]
            gt = (grad * g.unsqueeze(1)).sum(0)
        gf = plan.eval_adjoint(g.contiguous()) if ctx.needs_input_grad[1] else None
        return gt, gf, None


CELL_SHAPES = {"box": 0, "triangle": 1}


def correction_blocks(shape: str, p: int, ref_x, ref_y, wref, maps: torch.Tensor,
                      out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Own-cell singular correction blocks on the device (vp_correction_blocks).

    shape: "box" (N = p^2 nodes) or "triangle" (N = p(p+1)/2); ref_x, ref_y,
    wref: the node pattern and its smooth weights in reference coordinates
    (host arrays); maps: float64 device tensor [ncell, 6] of (o_x, o_y, A_00,
    A_01, A_10, A_11).  Returns the float64 device tensor [ncell, N, N]."""
    lib = load_library()
    rx, ry, rw = _host(ref_x, np.float64), _host(ref_y, np.float64), _host(wref, np.float64)
    N = rx.shape[0]
    if maps.dtype != torch.float64 or not maps.is_cuda or maps.dim() != 2 or maps.shape[1] != 6:
        raise ValueError("maps must be a float64 device tensor [ncell, 6]")
    maps = maps.contiguous()
    ncell = maps.shape[0]
    if out is None:
        out = torch.empty((ncell, N, N), dtype=torch.float64, device=maps.device)
    st = lib.vp_correction_blocks(CELL_SHAPES[shape], p, _ptr(rx), _ptr(ry), _ptr(rw), ncell,
                                  ctypes.c_void_p(maps.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                  _current_stream())
    if st != VP_OK:
        raise VPError(st, lib.vp_last_error(None).decode())
    return out


def volume_potential(f: torch.Tensor, plan: Plan) -> torch.Tensor:
    return VolumePotential.apply(f, plan)


def target_potential(targets: torch.Tensor, f: torch.Tensor, plan: Plan) -> torch.Tensor:
    return TargetPotential.apply(targets, f, plan)
