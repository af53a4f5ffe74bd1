"""Python binding of the SLOS C ABI (include/slos.h): argument marshalling only.

Every step of the computation runs in the HIP library; torch provides device
memory and the stream.  The library is loaded from this package directory and
a missing or unloadable library raises -- there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libslos.so")

SLOS_OK = 0
SLOS_C64 = 0x1
SLOS_C128 = 0x2
SLOS_COMPENSATED = 0x100
SLOS_COMP_KNUTH = 0x800
SLOS_COMP_FP64 = 0x1000
SLOS_KEEP_LAYERS = 0x200
SLOS_HOST_ONLY = 0x400
MAX_MODES = 255
MAX_PHOTONS = 32

ERRORS = {
    -1: "INVALID_ARG", -2: "SIZE_OVERFLOW", -3: "OOM", -4: "DTYPE",
    -5: "HIP_ERROR", -6: "NOT_KEPT", -7: "NO_DEVICE",
}


class SlosError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class Options(ctypes.Structure):
    _fields_ = [("leaf_max", ctypes.c_int32), ("comp_from_layer", ctypes.c_int32),
                ("block_threads", ctypes.c_int32), ("grid_blocks", ctypes.c_int32),
                ("outputs_per_lane", ctypes.c_int32), ("xcd_chunk", ctypes.c_int32),
                ("ticket_leaves", ctypes.c_int32), ("max_batch", ctypes.c_int32),
                ("wide_descriptors", ctypes.c_int32), ("leaf_order", ctypes.c_int32),
                ("low_block_max", ctypes.c_int32)]


_lib = None


class SourceParams(ctypes.Structure):
    _fields_ = [("emission_probability", ctypes.c_double),
                ("multiphoton_component", ctypes.c_double),
                ("indistinguishability", ctypes.c_double)]


def lib():
    """The loaded libslos.so (raises if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_2204_00602_amd.build` (needs hipcc)")
    L = ctypes.CDLL(LIB_PATH)
    i32p = ctypes.POINTER(ctypes.c_int32)
    i64p = ctypes.POINTER(ctypes.c_int64)
    vp = ctypes.c_void_p
    L.slos_fock_count.argtypes = [ctypes.c_int, ctypes.c_int, i64p]
    L.slos_fock_rank.argtypes = [ctypes.c_int, ctypes.c_int, i32p, i64p]
    L.slos_fock_unrank.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int64, i32p]
    L.slos_plan.argtypes = [ctypes.c_int, ctypes.c_int, i32p, ctypes.c_int, ctypes.POINTER(vp)]
    L.slos_plan_ex.argtypes = [ctypes.c_int, ctypes.c_int, i32p, ctypes.c_int,
                               ctypes.POINTER(Options), ctypes.POINTER(vp)]
    L.slos_plan_destroy.argtypes = [vp]
    L.slos_plan_destroy.restype = None
    L.slos_num_outputs.argtypes = [vp]
    L.slos_num_outputs.restype = ctypes.c_int64
    L.slos_rank.argtypes = [vp, i32p, i64p]
    L.slos_unrank.argtypes = [vp, ctypes.c_int64, i32p]
    L.slos_plan_info.argtypes = [vp, ctypes.c_int, i64p, i64p]
    L.slos_plan_leaf.argtypes = [vp, ctypes.c_int, ctypes.c_int64, i64p, i32p, i32p, i32p]
    L.slos_amplitudes.argtypes = [vp, vp, vp, vp, vp]
    L.slos_probs.argtypes = [vp, vp, vp, vp, vp]
    L.slos_amplitudes_noalloc.argtypes = [vp, vp, vp, vp, vp]
    L.slos_backward.argtypes = [vp, vp, vp, vp, vp]
    L.slos_amplitudes_many.argtypes = [vp, ctypes.c_int, vp, vp, vp, vp]
    L.slos_probs_many.argtypes = [vp, ctypes.c_int, vp, vp, vp, vp]
    L.slos_backward_many.argtypes = [vp, ctypes.c_int, vp, vp, vp, vp]
    L.slos_sq_loss_grad_many.argtypes = [vp, ctypes.c_int, vp, vp, ctypes.c_int64, vp, vp, vp, vp]
    L.slos_output_scales.argtypes = [vp, vp, ctypes.c_int64, vp]
    L.slos_sq_loss_backward_many.argtypes = [vp, ctypes.c_int, vp, vp, vp, vp, ctypes.c_int64, vp, vp, vp, vp]
    L.slos_cdf.argtypes = [vp, vp, vp]
    L.slos_select.argtypes = [vp, vp, i32p, ctypes.c_int64, vp, vp]
    L.slos_marginals.argtypes = [vp, vp, vp, vp]
    L.slos_sample.argtypes = [vp, vp, vp, ctypes.c_int64, vp, vp]
    L.slos_postselect.argtypes = [vp, vp, i32p, ctypes.c_int, i32p, i32p, vp, vp, vp, ctypes.c_int64, vp, vp]
    L.slos_mesh_unitary.argtypes = [ctypes.c_int, ctypes.c_int, vp, vp, ctypes.c_int, vp]
    L.slos_mesh_backward.argtypes = [ctypes.c_int, ctypes.c_int, vp, vp, vp, ctypes.c_int, vp]
    L.slos_batch_plan.argtypes = [ctypes.c_int, i32p, i32p, ctypes.c_int, ctypes.POINTER(Options),
                                  ctypes.POINTER(vp)]
    L.slos_batch_destroy.argtypes = [vp]
    L.slos_batch_destroy.restype = None
    L.slos_batch_offsets.argtypes = [vp, i64p, i64p]
    L.slos_batch_amplitudes.argtypes = [vp, vp, vp, vp, vp]
    L.slos_batch_capture.argtypes = [vp, vp, vp, vp]
    L.slos_batch_replay.argtypes = [vp, vp]
    L.slos_source_plan.argtypes = [ctypes.c_int, i32p, ctypes.POINTER(SourceParams), ctypes.c_int,
                                   ctypes.POINTER(Options), ctypes.POINTER(vp)]
    L.slos_source_destroy.argtypes = [vp]
    L.slos_source_destroy.restype = None
    L.slos_source_num_outputs.argtypes = [vp]
    L.slos_source_num_outputs.restype = ctypes.c_int64
    L.slos_source_info.argtypes = [vp, i64p, ctypes.POINTER(ctypes.c_double)]
    L.slos_source_probs.argtypes = [vp, vp, vp, vp]
    L.slos_source_postselect.argtypes = [vp, vp, i32p, ctypes.c_int, i32p, i32p, ctypes.c_int,
                                         ctypes.POINTER(ctypes.c_double), vp]
    L.slos_plan_capture.argtypes = [vp, ctypes.c_int, ctypes.c_int, vp, vp, vp]
    L.slos_plan_replay.argtypes = [vp, vp]
    L.slos_plan_set_timing.argtypes = [vp, ctypes.c_int]
    L.slos_plan_layer_ms.argtypes = [vp, ctypes.POINTER(ctypes.c_float), ctypes.c_int]
    L.slos_last_error.argtypes = []
    L.slos_last_error.restype = ctypes.c_char_p
    for name in ("slos_fock_count", "slos_fock_rank", "slos_fock_unrank", "slos_rank", "slos_unrank", "slos_plan",
                 "slos_plan_ex", "slos_plan_info", "slos_plan_leaf", "slos_amplitudes", "slos_amplitudes_noalloc",
                 "slos_probs", "slos_cdf", "slos_marginals", "slos_sample", "slos_postselect", "slos_select", "slos_amplitudes_many",
                 "slos_probs_many", "slos_backward_many", "slos_sq_loss_grad_many", "slos_output_scales",
                 "slos_sq_loss_backward_many", "slos_plan_set_timing", "slos_plan_layer_ms", "slos_backward",
                 "slos_mesh_unitary", "slos_mesh_backward", "slos_batch_plan", "slos_batch_offsets",
                 "slos_batch_amplitudes", "slos_batch_capture", "slos_batch_replay", "slos_source_plan",
                 "slos_source_info", "slos_source_probs", "slos_source_postselect", "slos_plan_capture",
                 "slos_plan_replay"):
        getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def _check(rc: int):
    if rc != SLOS_OK:
        raise SlosError(rc, lib().slos_last_error().decode(errors="replace"))


def _state_arr(state, m=None):
    a = np.ascontiguousarray(np.asarray(state, dtype=np.int32).reshape(-1))
    if m is not None and a.size != m:
        raise ValueError(f"state has {a.size} modes, expected {m}")
    return a


def fock_count(m: int, n: int) -> int:
    out = ctypes.c_int64()
    _check(lib().slos_fock_count(m, n, ctypes.byref(out)))
    return out.value


def fock_rank(state) -> int:
    s = _state_arr(state)
    out = ctypes.c_int64()
    _check(lib().slos_fock_rank(s.size, int(s.sum()), s.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                ctypes.byref(out)))
    return out.value


def fock_unrank(m: int, n: int, rank: int) -> np.ndarray:
    s = np.zeros(m, dtype=np.int32)
    _check(lib().slos_fock_unrank(m, n, int(rank), s.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))
    return s


def _stream_ptr(stream) -> int:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream)


class Plan:
    """Compile-once plan for (m, input_state, dtype); run for many U.

    Mirrors the paper's `backend(U).compile(input_state)` then `all_prob`
    usage (Appendix B.6) with the output order fixed to colex rank.
    """

    def __init__(self, input_state: Sequence[int], dtype: str = "c64", compensated=False,
                 keep_layers: bool = False, host_only: bool = False,
                 options: Optional[dict] = None):
        """compensated: False, True (biased-FMA error recovery), "knuth"
        (two-product + Knuth two-sum) or "fp64" (terms widened to FP64 and
        summed with FP64 FMAs); complex64 only."""
        self.input_state = _state_arr(input_state)
        self.m = int(self.input_state.size)
        self.n = int(self.input_state.sum())
        if dtype not in ("c64", "c128"):
            raise ValueError("dtype must be 'c64' or 'c128'")
        self.dtype = dtype
        flags = SLOS_C64 if dtype == "c64" else SLOS_C128
        if compensated:
            flags |= SLOS_COMPENSATED
            if compensated == "knuth":
                flags |= SLOS_COMP_KNUTH
            elif compensated == "fp64":
                flags |= SLOS_COMP_FP64
            elif compensated is not True:
                raise ValueError("compensated must be False, True, 'knuth' or 'fp64'")
        if keep_layers:
            flags |= SLOS_KEEP_LAYERS
        if host_only:
            flags |= SLOS_HOST_ONLY
        self.flags = flags
        self.host_only = host_only
        opts = Options()
        for k, v in (options or {}).items():
            setattr(opts, k, int(v))
        self.options = dict(options or {})
        handle = ctypes.c_void_p()
        self._lib = lib()
        _check(self._lib.slos_plan_ex(self.m, self.n,
                                      self.input_state.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                      flags, ctypes.byref(opts), ctypes.byref(handle)))
        self._h = handle
        self.num_outputs = int(self._lib.slos_num_outputs(handle))

    def close(self):
        if getattr(self, "_h", None):
            self._lib.slos_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- inspection -----------------------------------------------------
    def layer_info(self, k: int):
        ns, nl = ctypes.c_int64(), ctypes.c_int64()
        _check(self._lib.slos_plan_info(self._h, k, ctypes.byref(ns), ctypes.byref(nl)))
        return ns.value, nl.value

    def leaf(self, k: int, idx: int):
        ob = ctypes.c_int64()
        q, K = ctypes.c_int32(), ctypes.c_int32()
        hm = (ctypes.c_int32 * MAX_PHOTONS)()
        _check(self._lib.slos_plan_leaf(self._h, k, idx, ctypes.byref(ob), ctypes.byref(q),
                                        ctypes.byref(K), hm))
        return ob.value, q.value, K.value, [hm[i] for i in range(k - K.value)]

    # ---- timing -------------------------------------------------------------
    def set_timing(self, on: bool = True):
        """Record HIP events around every layer launch of later calls."""
        _check(self._lib.slos_plan_set_timing(self._h, 1 if on else 0))

    def layer_ms(self):
        """Per-layer kernel durations (ms) of the last call; last entry = FP64 sum."""
        buf = (ctypes.c_float * (self.n + 1))()
        _check(self._lib.slos_plan_layer_ms(self._h, buf, self.n + 1))
        return [buf[i] for i in range(self.n + 1)]

    # ---- device calls -----------------------------------------------------
    def _complex_dtype(self):
        import torch
        return torch.complex64 if self.dtype == "c64" else torch.complex128

    def _check_U(self, U):
        import torch
        if not isinstance(U, torch.Tensor) or U.device.type != "cuda":
            raise TypeError("U must be a CUDA (HIP) torch tensor")
        if U.dtype != self._complex_dtype():
            raise TypeError(f"U must be {self._complex_dtype()} for a {self.dtype} plan")
        if tuple(U.shape) != (self.m, self.m) or not U.is_contiguous():
            raise ValueError(f"U must be a contiguous {self.m}x{self.m} tensor")

    def amplitudes(self, U, out=None, sum_p=None, stream=None):
        """out[rank(S)] = a(S) for all S; returns out (and fills sum_p[0] = sum P if given)."""
        import torch
        self._check_U(U)
        self.forward_count = getattr(self, "forward_count", 0) + 1
        if out is None:
            out = torch.empty(self.num_outputs, dtype=self._complex_dtype(), device=U.device)
        elif out.dtype != self._complex_dtype() or out.numel() != self.num_outputs or not out.is_contiguous():
            raise ValueError("out has the wrong dtype, size or layout")
        sp = None
        if sum_p is not None:
            if sum_p.dtype != torch.float64 or sum_p.device != U.device:
                raise TypeError("sum_p must be a float64 tensor on the same device")
            sp = sum_p.data_ptr()
        _check(self._lib.slos_amplitudes(self._h, U.data_ptr(), out.data_ptr(), sp, _stream_ptr(stream)))
        return out

    def probs(self, U, out=None, sum_p=None, stream=None):
        """out[rank(S)] = P(S) (float32 for c64, float64 for c128)."""
        import torch
        self._check_U(U)
        self.forward_count = getattr(self, "forward_count", 0) + 1
        rdt = torch.float32 if self.dtype == "c64" else torch.float64
        if out is None:
            out = torch.empty(self.num_outputs, dtype=rdt, device=U.device)
        elif out.dtype != rdt or out.numel() != self.num_outputs or not out.is_contiguous():
            raise ValueError("out has the wrong dtype, size or layout")
        sp = None
        if sum_p is not None:
            if sum_p.dtype != torch.float64 or sum_p.device != U.device:
                raise TypeError("sum_p must be a float64 tensor on the same device")
            sp = sum_p.data_ptr()
        _check(self._lib.slos_probs(self._h, U.data_ptr(), out.data_ptr(), sp, _stream_ptr(stream)))
        return out

    def _check_many(self, U):
        import torch
        if not isinstance(U, torch.Tensor) or U.device.type != "cuda" or U.dtype != self._complex_dtype():
            raise TypeError(f"U must be a {self._complex_dtype()} CUDA (HIP) tensor")
        if U.dim() != 3 or tuple(U.shape[1:]) != (self.m, self.m) or not U.is_contiguous():
            raise ValueError(f"U must be a contiguous batch x {self.m} x {self.m} tensor")
        b = U.shape[0]
        if b < 1 or b > self.options.get("max_batch", 1):
            raise ValueError(f"batch {b} outside [1, max_batch]")
        return b

    def amplitudes_many(self, U, out=None, sum_p=None, stream=None):
        """a(S) for a batch of unitaries (batch x m x m): out is batch x M."""
        import torch
        b = self._check_many(U)
        self.forward_count = getattr(self, "forward_count", 0) + 1
        if out is None:
            out = torch.empty((b, self.num_outputs), dtype=self._complex_dtype(), device=U.device)
        elif out.dtype != self._complex_dtype() or out.numel() != b * self.num_outputs or not out.is_contiguous():
            raise ValueError("out has the wrong dtype, size or layout")
        if sum_p is not None and (sum_p.dtype != torch.float64 or sum_p.numel() != b):
            raise TypeError("sum_p must be a float64 tensor with one entry per instance")
        _check(self._lib.slos_amplitudes_many(self._h, b, U.data_ptr(), out.data_ptr(),
                                              None if sum_p is None else sum_p.data_ptr(), _stream_ptr(stream)))
        return out

    def capture(self, U, out, sum_p=None, probs=False):
        """Record one forward pass on these buffers into a HIP graph owned by the
        plan (amplitudes, or P with probs=True; U is m x m or batch x m x m).
        Nothing runs now; replay() launches the graph."""
        import torch
        if U.dim() == 3:
            b = self._check_many(U)
        else:
            self._check_U(U)
            b = 1
        if probs:
            want = torch.float32 if self.dtype == "c64" else torch.float64
        else:
            want = self._complex_dtype()
        if out.dtype != want or out.numel() != b * self.num_outputs or not out.is_contiguous() \
                or out.device != U.device:
            raise ValueError("out has the wrong dtype, size, layout or device")
        if sum_p is not None and (sum_p.dtype != torch.float64 or sum_p.numel() < b or sum_p.device != U.device):
            raise TypeError("sum_p must be a float64 tensor with one entry per instance")
        self._bound = (U, out, sum_p)  # the graph keeps raw pointers: keep the tensors alive
        _check(self._lib.slos_plan_capture(self._h, b, 1 if probs else 0, U.data_ptr(), out.data_ptr(),
                                           None if sum_p is None else sum_p.data_ptr()))

    def replay(self, stream=None):
        """Launch the captured forward pass on a stream."""
        self.forward_count = getattr(self, "forward_count", 0) + 1
        _check(self._lib.slos_plan_replay(self._h, _stream_ptr(stream)))

    def backward_many(self, U, grad_a, grad_U=None, stream=None):
        """Gradients with respect to each U of a batch (see backward)."""
        import torch
        b = self._check_many(U)
        if not (self.flags & SLOS_KEEP_LAYERS):
            raise SlosError(-6, "plan was built without keep_layers=True")
        if grad_a.dtype != self._complex_dtype() or grad_a.numel() != b * self.num_outputs:
            raise ValueError("grad_a has the wrong dtype or size")
        grad_a = grad_a.contiguous()
        if grad_U is None:
            grad_U = torch.empty_like(U)
        _check(self._lib.slos_backward_many(self._h, b, U.data_ptr(), grad_a.data_ptr(), grad_U.data_ptr(),
                                            _stream_ptr(stream)))
        return grad_U

    def sq_loss_grad_many(self, a, ranks, p_target, grad_a=None, loss=None, stream=None):
        """grad_a = 4 (|a|^2 - p_target) a at the target ranks, 0 elsewhere, and
        the per-instance FP64 loss sum_t (|a(ranks[t])|^2 - p_target[:, t])^2
        (slos_sq_loss_grad_many).  a: batch x M; ranks: int64 device tensor;
        p_target: batch x len(ranks) FP64.  Returns (grad_a, loss)."""
        import torch
        if a.dtype != self._complex_dtype() or a.numel() % self.num_outputs or not a.is_contiguous():
            raise ValueError("a must be a contiguous batch x M tensor of the plan's type")
        b = a.numel() // self.num_outputs
        ranks = torch.as_tensor(ranks, dtype=torch.int64, device=a.device).contiguous()
        p_target = torch.as_tensor(p_target, dtype=torch.float64, device=a.device).contiguous()
        if p_target.numel() != b * ranks.numel():
            raise ValueError("p_target needs batch x len(ranks) values")
        if grad_a is None:
            grad_a = torch.empty_like(a)
        elif grad_a.dtype != a.dtype or grad_a.numel() != a.numel() or not grad_a.is_contiguous():
            raise ValueError("grad_a has the wrong dtype, size or layout")
        if loss is None:
            loss = torch.empty(b, dtype=torch.float64, device=a.device)
        elif loss.dtype != torch.float64 or loss.numel() != b:
            raise ValueError("loss must be a float64 tensor with one entry per instance")
        _check(self._lib.slos_sq_loss_grad_many(self._h, b, a.data_ptr(), ranks.data_ptr(), ranks.numel(),
                                                p_target.data_ptr(), grad_a.data_ptr(), loss.data_ptr(),
                                                _stream_ptr(stream)))
        return grad_a, loss

    def output_scales(self, ranks):
        """c_S of the outputs at `ranks` (host int64 array): a(S) = c_S A_n[S]
        (slos_output_scales).  Returns a float64 numpy array."""
        r = np.ascontiguousarray(np.asarray(ranks, dtype=np.int64).reshape(-1))
        out = np.empty(r.size, dtype=np.float64)
        _check(self._lib.slos_output_scales(self._h, r.ctypes.data if r.size else None, r.size,
                                            out.ctypes.data if r.size else None))
        return out

    def sq_loss_backward_many(self, U, a, ranks, scales, p_target, grad_U=None, loss=None, stream=None):
        """The squared-error loss on the target ranks and its gradient with
        respect to each U of the batch in one call (slos_sq_loss_backward_many):
        the same results as sq_loss_grad_many followed by backward_many.
        scales: device FP64 values of output_scales(ranks).  Returns (grad_U, loss)."""
        import torch
        b = self._check_many(U)
        if not (self.flags & SLOS_KEEP_LAYERS):
            raise SlosError(-6, "plan was built without keep_layers=True")
        if a.dtype != self._complex_dtype() or a.numel() != b * self.num_outputs or not a.is_contiguous():
            raise ValueError("a must be a contiguous batch x M tensor of the plan's type")
        ranks = torch.as_tensor(ranks, dtype=torch.int64, device=a.device).contiguous()
        scales = torch.as_tensor(scales, dtype=torch.float64, device=a.device).contiguous()
        p_target = torch.as_tensor(p_target, dtype=torch.float64, device=a.device).contiguous()
        if scales.numel() != ranks.numel():
            raise ValueError("scales needs one value per rank")
        if p_target.numel() != b * ranks.numel():
            raise ValueError("p_target needs batch x len(ranks) values")
        if grad_U is None:
            grad_U = torch.empty_like(U)
        if loss is None:
            loss = torch.empty(b, dtype=torch.float64, device=a.device)
        elif loss.dtype != torch.float64 or loss.numel() != b:
            raise ValueError("loss must be a float64 tensor with one entry per instance")
        _check(self._lib.slos_sq_loss_backward_many(self._h, b, U.data_ptr(), a.data_ptr(), ranks.data_ptr(),
                                                    scales.data_ptr(), ranks.numel(), p_target.data_ptr(),
                                                    grad_U.data_ptr(), loss.data_ptr(), _stream_ptr(stream)))
        return grad_U, loss

    def backward(self, U, grad_a, grad_U=None, stream=None):
        """Gradient with respect to U of a real loss, given its gradient with
        respect to the amplitudes (both in the PyTorch complex convention).
        Uses the layers kept by the last forward call on this plan."""
        import torch
        self._check_U(U)
        if not (self.flags & SLOS_KEEP_LAYERS):
            raise SlosError(-6, "plan was built without keep_layers=True")
        if grad_a.dtype != self._complex_dtype() or grad_a.numel() != self.num_outputs:
            raise ValueError("grad_a has the wrong dtype or size")
        grad_a = grad_a.contiguous()
        if grad_U is None:
            grad_U = torch.empty_like(U)
        _check(self._lib.slos_backward(self._h, U.data_ptr(), grad_a.data_ptr(), grad_U.data_ptr(),
                                       _stream_ptr(stream)))
        return grad_U

    def select(self, U, targets, out=None, stream=None):
        """a(S) for the given output states only (count x m), via the
        recurrence restricted to t <= S; returns a device tensor of count."""
        import torch
        self._check_U(U)
        t = np.ascontiguousarray(np.asarray(targets, dtype=np.int32).reshape(-1, self.m))
        if out is None:
            out = torch.empty(t.shape[0], dtype=self._complex_dtype(), device=U.device)
        elif out.dtype != self._complex_dtype() or out.numel() != t.shape[0] or not out.is_contiguous():
            raise ValueError("out has the wrong dtype, size or layout")
        _check(self._lib.slos_select(self._h, U.data_ptr(), t.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                     t.shape[0], out.data_ptr(), _stream_ptr(stream)))
        return out

    # ---- weak simulation ----------------------------------------------------
    def _check_probs(self, probs):
        import torch
        rdt = torch.float32 if self.dtype == "c64" else torch.float64
        if probs.dtype != rdt or probs.numel() != self.num_outputs or probs.device.type != "cuda" \
                or not probs.is_contiguous():
            raise ValueError(f"probs must be a contiguous {rdt} device tensor of {self.num_outputs} values")

    def cdf(self, probs, stream=None):
        """Build the plan's cumulative table for `probs` (see slos_cdf)."""
        self._check_probs(probs)
        _check(self._lib.slos_cdf(self._h, probs.data_ptr(), _stream_ptr(stream)))

    def marginals(self, probs, stream=None):
        """P(K) for K = 1..m (Eq. eqpk) as an FP64 device tensor; call cdf(probs) first."""
        import torch
        self._check_probs(probs)
        pk = torch.empty(self.m, dtype=torch.float64, device=probs.device)
        _check(self._lib.slos_marginals(self._h, probs.data_ptr(), pk.data_ptr(), _stream_ptr(stream)))
        return pk

    def sample(self, probs, r, stream=None):
        """Colex ranks of the outputs drawn for uniforms r (FP64 device tensor); call cdf(probs) first."""
        import torch
        self._check_probs(probs)
        if r.dtype != torch.float64 or r.device.type != "cuda" or not r.is_contiguous():
            raise ValueError("r must be a contiguous float64 device tensor")
        ranks = torch.empty(r.numel(), dtype=torch.int64, device=r.device)
        _check(self._lib.slos_sample(self._h, probs.data_ptr(), r.data_ptr(), r.numel(), ranks.data_ptr(),
                                     _stream_ptr(stream)))
        return ranks

    def postselect(self, probs, group_of_mode, count_min, count_max, masked=False, ranks=None, stream=None):
        """Keep the outputs whose mode groups hold count_min[g]..count_max[g]
        photons (see slos_postselect).  Returns (kept_sum, masked P or None,
        conditional table for `ranks` or None) as device tensors."""
        import torch
        self._check_probs(probs)
        gm = np.ascontiguousarray(np.asarray(group_of_mode, dtype=np.int32).reshape(-1))
        lo = np.ascontiguousarray(np.asarray(count_min, dtype=np.int32).reshape(-1))
        hi = np.ascontiguousarray(np.asarray(count_max, dtype=np.int32).reshape(-1))
        if gm.size != self.m or lo.size != hi.size:
            raise ValueError("group_of_mode needs m entries and count_min/count_max one per group")
        i32p = ctypes.POINTER(ctypes.c_int32)
        kept = torch.zeros(1, dtype=torch.float64, device=probs.device)
        out = torch.empty_like(probs) if masked else None
        table = None
        rptr, nr = None, 0
        if ranks is not None:
            ranks = torch.as_tensor(ranks, dtype=torch.int64, device=probs.device).contiguous()
            table = torch.empty(ranks.numel(), dtype=torch.float64, device=probs.device)
            rptr, nr = ranks.data_ptr(), ranks.numel()
        _check(self._lib.slos_postselect(self._h, probs.data_ptr(), gm.ctypes.data_as(i32p), int(lo.size),
                                         lo.ctypes.data_as(i32p), hi.ctypes.data_as(i32p), kept.data_ptr(),
                                         None if out is None else out.data_ptr(), rptr, nr,
                                         None if table is None else table.data_ptr(), _stream_ptr(stream)))
        return kept, out, table

    def rank(self, state) -> int:
        """Index of a(state) in this plan's outputs (slos_rank)."""
        s = _state_arr(state, self.m)
        r = ctypes.c_int64(0)
        _check(self._lib.slos_rank(self._h, s.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), ctypes.byref(r)))
        return int(r.value)

    def unrank(self, r: int) -> np.ndarray:
        """Output state at index r of this plan's outputs (slos_unrank)."""
        s = np.zeros(self.m, np.int32)
        _check(self._lib.slos_unrank(self._h, int(r), s.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))
        return s


class Batch:
    """Many independent (U, input state) instances of uneven size, computed by
    one kernel launch (optionally replayed from a captured HIP graph).

    U and the amplitudes are packed: instance i's U starts at element
    u_offsets[i] (row-major m_i x m_i), its amplitudes at out_offsets[i].
    """

    def __init__(self, input_states, dtype: str = "c64", options: Optional[dict] = None):
        states = [np.ascontiguousarray(np.asarray(s, dtype=np.int32).reshape(-1)) for s in input_states]
        self.count = len(states)
        self.ms = np.array([s.size for s in states], dtype=np.int32)
        self.ns = np.array([int(s.sum()) for s in states], dtype=np.int32)
        flat = np.ascontiguousarray(np.concatenate(states)) if states else np.zeros(0, np.int32)
        if dtype not in ("c64", "c128"):
            raise ValueError("dtype must be 'c64' or 'c128'")
        self.dtype = dtype
        opts = Options()
        for k, v in (options or {}).items():
            setattr(opts, k, int(v))
        self._lib = lib()
        h = ctypes.c_void_p()
        i32p = ctypes.POINTER(ctypes.c_int32)
        _check(self._lib.slos_batch_plan(self.count, self.ms.ctypes.data_as(i32p), flat.ctypes.data_as(i32p),
                                         SLOS_C64 if dtype == "c64" else SLOS_C128, ctypes.byref(opts),
                                         ctypes.byref(h)))
        self._h = h
        self.u_offsets = np.zeros(self.count + 1, dtype=np.int64)
        self.out_offsets = np.zeros(self.count + 1, dtype=np.int64)
        i64p = ctypes.POINTER(ctypes.c_int64)
        _check(self._lib.slos_batch_offsets(h, self.u_offsets.ctypes.data_as(i64p),
                                            self.out_offsets.ctypes.data_as(i64p)))
        self.total_outputs = int(self.out_offsets[-1])
        self.total_u = int(self.u_offsets[-1])

    def close(self):
        if getattr(self, "_h", None):
            self._lib.slos_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _cdt(self):
        import torch
        return torch.complex64 if self.dtype == "c64" else torch.complex128

    def pack_u(self, Us):
        """Pack a list of m_i x m_i arrays/tensors into one device tensor."""
        import torch
        parts = [torch.as_tensor(np.asarray(u) if not isinstance(u, torch.Tensor) else u).reshape(-1) for u in Us]
        return torch.cat(parts).to(self._cdt()).cuda().contiguous()

    def _check(self, U, out, sum_p):
        import torch
        if U.dtype != self._cdt() or U.numel() != self.total_u or U.device.type != "cuda":
            raise ValueError("U must be the packed device tensor of the batch")
        if out.dtype != self._cdt() or out.numel() != self.total_outputs:
            raise ValueError("out has the wrong dtype or size")
        if sum_p is not None and (sum_p.dtype != torch.float64 or sum_p.numel() != self.count):
            raise ValueError("sum_p must be a float64 tensor with one entry per instance")

    def amplitudes(self, U, out=None, sum_p=None, stream=None):
        import torch
        if out is None:
            out = torch.empty(self.total_outputs, dtype=self._cdt(), device=U.device)
        self._check(U, out, sum_p)
        _check(self._lib.slos_batch_amplitudes(self._h, U.data_ptr(), out.data_ptr(),
                                               None if sum_p is None else sum_p.data_ptr(), _stream_ptr(stream)))
        return out

    def capture(self, U, out, sum_p=None):
        """Record the batch launch on these buffers into a HIP graph."""
        self._check(U, out, sum_p)
        self._bound = (U, out, sum_p)  # the graph keeps raw pointers: keep the tensors alive
        _check(self._lib.slos_batch_capture(self._h, U.data_ptr(), out.data_ptr(),
                                            None if sum_p is None else sum_p.data_ptr()))

    def replay(self, stream=None):
        _check(self._lib.slos_batch_replay(self._h, _stream_ptr(stream)))

    def output(self, out, i):
        return out[int(self.out_offsets[i]):int(self.out_offsets[i + 1])]


class Source:
    """Output distribution of an imperfect single-photon source behind an input
    state (slos_source_plan): photon numbers 0..nmax, each in colex order, one
    after the other (`offsets[k]` .. `offsets[k+1]`), FP64."""

    def __init__(self, input_state: Sequence[int], emission_probability: float = 1.0,
                 multiphoton_component: float = 0.0, indistinguishability: float = 1.0,
                 nmax: int = -1, options: Optional[dict] = None):
        self.input_state = _state_arr(input_state)
        self.m = int(self.input_state.size)
        self.n = int(self.input_state.sum())
        sp = SourceParams(float(emission_probability), float(multiphoton_component), float(indistinguishability))
        opts = Options()
        for k, v in (options or {}).items():
            setattr(opts, k, int(v))
        self._lib = lib()
        h = ctypes.c_void_p()
        _check(self._lib.slos_source_plan(self.m, self.input_state.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                          ctypes.byref(sp), int(nmax), ctypes.byref(opts), ctypes.byref(h)))
        self._h = h
        self.num_outputs = int(self._lib.slos_source_num_outputs(h))
        off = np.zeros(2 * self.n + 18, dtype=np.int64)
        em = np.zeros(3, dtype=np.float64)
        _check(self._lib.slos_source_info(h, off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                          em.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        self.nmax = int(np.flatnonzero(off[1:] == self.num_outputs)[0])
        self.offsets = off[: self.nmax + 2].copy()
        self.emission = tuple(float(v) for v in em)

    def close(self):
        if getattr(self, "_h", None):
            self._lib.slos_source_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def probs(self, U, out=None, stream=None):
        """Mixture probabilities for U (complex128 m x m on the device)."""
        import torch
        if not (isinstance(U, torch.Tensor) and U.is_cuda and U.dtype == torch.complex128
                and tuple(U.shape) == (self.m, self.m) and U.is_contiguous()):
            raise ValueError(f"U must be a contiguous complex128 CUDA tensor of shape ({self.m}, {self.m})")
        if out is None:
            out = torch.empty(self.num_outputs, dtype=torch.float64, device=U.device)
        elif not (out.is_cuda and out.dtype == torch.float64 and out.numel() == self.num_outputs
                  and out.is_contiguous()):
            raise ValueError("out must be a contiguous float64 CUDA tensor of num_outputs elements")
        _check(self._lib.slos_source_probs(self._h, U.data_ptr(), out.data_ptr(), _stream_ptr(stream)))
        return out

    def split(self, probs):
        """Views of `probs` per photon number k = 0..nmax."""
        return [probs[self.offsets[k]:self.offsets[k + 1]] for k in range(self.nmax + 1)]

    def postselect(self, probs, group_of_mode=None, count_min=(), count_max=(), min_modes: int = 0, stream=None):
        """Per photon number: (total, physical, kept), a (nmax + 1) x 3 array
        (see slos_source_postselect)."""
        import torch
        if not (isinstance(probs, torch.Tensor) and probs.is_cuda and probs.dtype == torch.float64
                and probs.numel() == self.num_outputs):
            raise ValueError("probs must be the float64 CUDA output of probs()")
        i32p = ctypes.POINTER(ctypes.c_int32)
        lo = np.ascontiguousarray(np.asarray(count_min, dtype=np.int32).reshape(-1))
        hi = np.ascontiguousarray(np.asarray(count_max, dtype=np.int32).reshape(-1))
        if lo.size != hi.size:
            raise ValueError("count_min and count_max need one entry per group")
        gm = None
        if group_of_mode is not None:
            gm = np.ascontiguousarray(np.asarray(group_of_mode, dtype=np.int32).reshape(-1))
            if gm.size != self.m:
                raise ValueError("group_of_mode needs m entries")
        res = np.zeros(3 * (self.nmax + 1), dtype=np.float64)
        _check(self._lib.slos_source_postselect(self._h, probs.data_ptr(),
                                                None if gm is None else gm.ctypes.data_as(i32p), int(lo.size),
                                                lo.ctypes.data_as(i32p), hi.ctypes.data_as(i32p), int(min_modes),
                                                res.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                                _stream_ptr(stream)))
        return res.reshape(self.nmax + 1, 3)


def mesh_mzi_count(m: int) -> int:
    return m * (m - 1) // 2


def mesh_unitary(phases, m: int, dtype: str = "c128", stream=None, out=None):
    """U (batch x m x m) of the rectangular MZI mesh for FP64 phases (batch x m(m-1))."""
    import torch
    if phases.dtype != torch.float64 or phases.device.type != "cuda":
        raise TypeError("phases must be a float64 CUDA tensor")
    phases = phases.contiguous()
    batch = phases.shape[0] if phases.dim() == 2 else 1
    if phases.numel() != batch * 2 * mesh_mzi_count(m):
        raise ValueError("phases must hold 2 * m(m-1)/2 values per batch entry")
    cdt = torch.complex64 if dtype == "c64" else torch.complex128
    if out is None:
        U = torch.empty((batch, m, m), dtype=cdt, device=phases.device)
    elif out.dtype != cdt or out.numel() != batch * m * m or not out.is_contiguous():
        raise ValueError("out has the wrong dtype, size or layout")
    else:
        U = out
    _check(lib().slos_mesh_unitary(m, batch, phases.data_ptr(), U.data_ptr(),
                                   SLOS_C64 if dtype == "c64" else SLOS_C128, _stream_ptr(stream)))
    return U


def mesh_backward(phases, grad_U, stream=None, out=None):
    """dL/dphases (batch x m(m-1), FP64) from grad_U (batch x m x m, PyTorch convention)."""
    import torch
    phases = phases.contiguous()
    grad_U = grad_U.contiguous()
    batch, m = grad_U.shape[0], grad_U.shape[-1]
    dt = SLOS_C64 if grad_U.dtype == torch.complex64 else SLOS_C128
    if out is None:
        g = torch.empty((batch, 2 * mesh_mzi_count(m)), dtype=torch.float64, device=phases.device)
    elif out.dtype != torch.float64 or out.numel() != batch * 2 * mesh_mzi_count(m) or not out.is_contiguous():
        raise ValueError("out has the wrong dtype, size or layout")
    else:
        g = out
    _check(lib().slos_mesh_backward(m, batch, phases.data_ptr(), grad_U.data_ptr(), g.data_ptr(), dt,
                                    _stream_ptr(stream)))
    return g


def algorithmic_bytes(m: int, n: int, elem_bytes: int, last_write_bytes: Optional[int] = None) -> int:
    """Bytes the recurrence must move: every layer A_0..A_{n-1} read once, A_1..A_n written once."""
    import math
    N = [math.comb(m + k - 1, k) for k in range(n + 1)]
    lw = elem_bytes if last_write_bytes is None else last_write_bytes
    return elem_bytes * sum(N[:n]) + elem_bytes * sum(N[1:n]) + lw * N[n]
