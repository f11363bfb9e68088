"""Python binding of the gfx950 batched fitness evaluator (libgpeval.so).

Argument marshalling only: every step of scoring runs in the HIP library.
PyTorch provides device memory and streams.  If the library has not been
built, every entry point raises -- there is no CPU fallback.

Entry points mirror ``include/gpeval.h``:
    gp_eval(...)       score a population held in device tensors
    gp_validate(...)   host-side structural check of a population
    evaluate(...)      convenience: numpy in, upload, gp_eval, numpy out
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
#: the in-tree build; GPEVAL_LIB may point at another build of the same source
LIB_PATH = os.environ.get("GPEVAL_LIB") or os.path.join(_PKG, "libgpeval.so")

GP_OK, GP_E_INVALID_ARG, GP_E_BAD_PROGRAM, GP_E_TOO_LARGE, GP_E_NO_MEMORY, GP_E_HIP = \
    0, -1, -2, -3, -4, -5
GP_ALL_OPS = (1 << 12) - 1

_lib = None


class GPError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("gpeval error %d: %s" % (code, msg))
        self.code = code


def lib():
    """The loaded HIP library (raises if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libgpeval.so is not built; run __graft_entry__.build() "
                               "(or python -m paper_2607_06731_amd._build)")
        L = ctypes.CDLL(LIB_PATH)
        vp, i64, i32, u32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint32
        L.gp_last_error.restype = ctypes.c_char_p
        L.gp_last_error.argtypes = []
        L.gp_version.restype = ctypes.c_int
        L.gp_validate.argtypes = [vp, vp, i64, i64, i32, u32, vp, vp, vp]
        L.gp_validate.restype = ctypes.c_int
        L.gp_eval.argtypes = [vp, vp, i64, i64, vp, i64, vp, i32, i64, vp, i64,
                              ctypes.c_double, u32, vp, vp, vp]
        L.gp_eval.restype = ctypes.c_int
        L.gp_predict.argtypes = [vp, vp, i64, i64, vp, i64, vp, i32, i64, i64, u32, vp, i64,
                                 vp, vp]
        L.gp_predict.restype = ctypes.c_int
        L.gp_release_workspaces.argtypes = []
        L.gp_release_workspaces.restype = None
        L.gp_timing_enable.argtypes = [ctypes.c_int]
        L.gp_timing_enable.restype = ctypes.c_int
        L.gp_timing_reset.argtypes = []
        L.gp_timing_reset.restype = ctypes.c_int
        L.gp_timing_read.argtypes = [vp, vp]
        L.gp_timing_read.restype = ctypes.c_int
        _lib = L
    return _lib


def _check(rc):
    if rc != GP_OK:
        raise GPError(rc, lib().gp_last_error().decode())
    return rc


TIMING_PHASES = ("prepare", "eval_d8", "eval_d16", "eval_d32", "reduce", "total")


def timing_enable(on=True):
    _check(lib().gp_timing_enable(1 if on else 0))


def timing_reset():
    _check(lib().gp_timing_reset())


def timing_read():
    """Accumulated per-phase milliseconds of timed gp_eval calls."""
    ms = (ctypes.c_double * len(TIMING_PHASES))()
    n = ctypes.c_int64(0)
    _check(lib().gp_timing_read(ms, ctypes.byref(n)))
    return dict(zip(TIMING_PHASES, list(ms))), n.value


def _np_ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def gp_validate(nodes, offsets, n_consts, n_vars, allowed_op_mask=0):
    """Host check; returns (status int32[P], max_depth int32[P], first_bad)."""
    nodes = np.ascontiguousarray(nodes, dtype=np.uint32)
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    P = offsets.size - 1
    status = np.zeros(P, np.int32)
    maxd = np.zeros(P, np.int32)
    first = ctypes.c_int64(-1)
    rc = lib().gp_validate(_np_ptr(nodes), _np_ptr(offsets), P, int(n_consts), int(n_vars),
                           int(allowed_op_mask), _np_ptr(status), _np_ptr(maxd),
                           ctypes.byref(first))
    if rc not in (GP_OK, GP_E_BAD_PROGRAM):
        _check(rc)
    return status, maxd, first.value


def _dev_ptr(t, dtype, name):
    import torch
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a device tensor" % name)
    if t.dtype != dtype:
        raise TypeError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    return ctypes.c_void_p(t.data_ptr()) if t.numel() else None


def _stream_handle(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def gp_eval(nodes, offsets, consts, X, y, tax_on_length, out_fitness,
            out_status=None, allowed_op_mask=0, ld_x=None, n_cases=None, stream=None):
    """Score the population held in device tensors (asynchronous on stream).

    nodes uint32[N], offsets int64[P+1], consts float32[C], X float32
    [n_vars, ld_x] (variable major), y float32[>= n_cases], out_fitness
    float64[P], out_status int32[P] or None.
    """
    import torch
    P = offsets.numel() - 1
    if out_fitness.numel() != P:
        raise ValueError("out_fitness must have n_programs entries")
    if X.dim() != 2:
        raise ValueError("X must be 2-D [n_vars, ld_x]")
    n_vars = X.shape[0]
    ld = X.shape[1] if ld_x is None else int(ld_x)
    n = y.numel() if n_cases is None else int(n_cases)
    rc = lib().gp_eval(_dev_ptr(nodes, torch.uint32, "nodes"), _dev_ptr(offsets, torch.int64, "offsets"),
                       P, nodes.numel(), _dev_ptr(consts, torch.float32, "consts"), consts.numel(),
                       _dev_ptr(X, torch.float32, "X"), n_vars, ld,
                       _dev_ptr(y, torch.float32, "y"), n, float(tax_on_length),
                       int(allowed_op_mask), _dev_ptr(out_fitness, torch.float64, "out_fitness"),
                       _dev_ptr(out_status, torch.int32, "out_status"), _stream_handle(stream))
    _check(rc)
    return out_fitness


def gp_predict(nodes, offsets, consts, X, out, out_status=None, allowed_op_mask=0,
               n_cases=None, stream=None):
    """Per-case outputs into out float32[P, ld_out] (device tensors)."""
    import torch
    P = offsets.numel() - 1
    if X.dim() != 2:
        raise ValueError("X must be 2-D [n_vars, ld_x]")
    n = X.shape[1] if n_cases is None else int(n_cases)
    if out.dim() != 2 or out.shape[0] != P or out.stride(1) != 1:
        raise ValueError("out must be [n_programs, ld_out] with unit column stride")
    rc = lib().gp_predict(_dev_ptr(nodes, torch.uint32, "nodes"),
                          _dev_ptr(offsets, torch.int64, "offsets"), P, nodes.numel(),
                          _dev_ptr(consts, torch.float32, "consts"), consts.numel(),
                          _dev_ptr(X, torch.float32, "X"), X.shape[0], X.shape[1], n,
                          int(allowed_op_mask), ctypes.c_void_p(out.data_ptr()), out.stride(0),
                          _dev_ptr(out_status, torch.int32, "out_status"), _stream_handle(stream))
    _check(rc)
    return out


def predict(nodes, offsets, consts, X, allowed_op_mask=0, device="cuda"):
    """numpy in, numpy out: per-case outputs float32[P, n_cases]."""
    import torch
    pop = DevicePopulation(nodes, offsets, consts, device)
    Xn = np.ascontiguousarray(X, np.float32)
    if Xn.ndim == 1:
        Xn = Xn.reshape(1, -1)
    Xd = torch.from_numpy(Xn).to(device)
    out = torch.empty((pop.n_programs, Xn.shape[1]), dtype=torch.float32, device=device)
    gp_predict(pop.nodes, pop.offsets, pop.consts, Xd, out, allowed_op_mask=allowed_op_mask)
    torch.cuda.synchronize()
    return out.cpu().numpy()


class DevicePopulation:
    """A population uploaded once (programs go to the device once per
    generation, one aggregate per program comes back)."""

    def __init__(self, nodes, offsets, consts, device="cuda"):
        import torch
        self.nodes = torch.from_numpy(np.ascontiguousarray(nodes, np.uint32)).to(device)
        self.offsets = torch.from_numpy(np.ascontiguousarray(offsets, np.int64)).to(device)
        c = np.ascontiguousarray(consts, np.float32)
        self.consts = torch.from_numpy(c).to(device)
        self.n_programs = self.offsets.numel() - 1


class DeviceDataset:
    """Fitness cases resident on the device (uploaded once, reused)."""

    def __init__(self, X, y, device="cuda"):
        import torch
        X = np.ascontiguousarray(X, np.float32)
        if X.ndim == 1:
            X = X.reshape(1, -1)
        self.X = torch.from_numpy(X).to(device)
        self.y = torch.from_numpy(np.ascontiguousarray(y, np.float32)).to(device)
        self.n_vars = X.shape[0]
        self.n_cases = self.y.numel()


def evaluate(nodes, offsets, consts, X, y, tax_on_length=0.0, allowed_op_mask=0,
             return_status=False, device="cuda"):
    """numpy in, numpy out: upload, score, download (synchronizes)."""
    import torch
    pop = DevicePopulation(nodes, offsets, consts, device)
    data = DeviceDataset(X, y, device)
    out = torch.empty(pop.n_programs, dtype=torch.float64, device=device)
    st = torch.empty(pop.n_programs, dtype=torch.int32, device=device) if return_status else None
    gp_eval(pop.nodes, pop.offsets, pop.consts, data.X, data.y, tax_on_length, out, st,
            allowed_op_mask)
    torch.cuda.synchronize()
    if return_status:
        return out.cpu().numpy(), st.cpu().numpy()
    return out.cpu().numpy()
