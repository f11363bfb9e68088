"""Python binding of the gfx950 batched fitness evaluator (libgpeval.so).

Argument marshalling only: every step of scoring runs in the HIP library.
PyTorch provides device memory and streams.  If the library has not been
built, every entry point raises -- there is no CPU fallback.

Entry points mirror ``include/gpeval.h``:
    gp_eval(...)          score a population held in device tensors
    gp_eval_batched(...)  score several requests, each on its own dataset
    gp_predict(...)       per-case outputs of every program
    Plan                  a captured (hipGraph) evaluation, optionally autotuned
    gp_validate(...)      host-side structural check of a population
    evaluate(...)         convenience: numpy in, upload, gp_eval, numpy out
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
GP_E_CANCELLED = -6
GP_N_OPS = 28
GP_ALL_OPS = (1 << GP_N_OPS) - 1
GP_BASE_OPS = (1 << 12) - 1       # LOAD..ABS, the benchmark set
GP_NOALLOC_WORKSPACE_BYTES = 64 << 20   # the fixed workspace of gp_eval_noalloc
GP_PROG_BAD_PAIR = 10

_lib = None


class GPProblem(ctypes.Structure):
    """struct gp_problem of include/gpeval.h"""
    _fields_ = [("nodes", ctypes.c_void_p), ("offsets", ctypes.c_void_p),
                ("n_programs", ctypes.c_int64), ("n_nodes", ctypes.c_int64),
                ("consts", ctypes.c_void_p), ("n_consts", ctypes.c_int64),
                ("X", ctypes.c_void_p), ("n_vars", ctypes.c_int32), ("ld_x", ctypes.c_int64),
                ("y", ctypes.c_void_p), ("n_cases", ctypes.c_int64),
                ("tax_on_length", ctypes.c_double), ("allowed_op_mask", ctypes.c_uint32),
                ("out_fitness", ctypes.c_void_p), ("out_status", ctypes.c_void_p)]


class GPDataset(ctypes.Structure):
    """struct gp_dataset of include/gpeval.h"""
    _fields_ = [("X", ctypes.c_void_p), ("y", ctypes.c_void_p), ("ld_x", ctypes.c_int64),
                ("n_cases", ctypes.c_int64), ("tax_on_length", ctypes.c_double),
                ("n_vars", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class GPRequest(ctypes.Structure):
    """struct gp_request of include/gpeval.h"""
    _fields_ = [("nodes", ctypes.c_void_p), ("offsets", ctypes.c_void_p),
                ("consts", ctypes.c_void_p), ("n_programs", ctypes.c_int64),
                ("n_nodes", ctypes.c_int64), ("n_consts", ctypes.c_int64),
                ("out_fitness", ctypes.c_void_p), ("out_status", ctypes.c_void_p),
                ("dataset", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class GPTuning(ctypes.Structure):
    """struct gp_tuning of include/gpeval.h"""
    _fields_ = [("programs_per_item", ctypes.c_int32), ("wg_per_cu", ctypes.c_int32),
                ("concurrent_classes", ctypes.c_int32), ("tile_lds_bytes", ctypes.c_int32),
                ("max_tiles", ctypes.c_int32)]


class GPServerConfig(ctypes.Structure):
    """struct gp_server_config of include/gpeval.h"""
    _fields_ = [("device_budget_bytes", ctypes.c_int64), ("pinned_bytes", ctypes.c_int64),
                ("chunk_node_evals", ctypes.c_int64), ("batch_node_evals", ctypes.c_int64),
                ("n_streams", ctypes.c_int32), ("max_batch_chunks", ctypes.c_int32),
                ("one_launch_per_request", ctypes.c_int32), ("allowed_op_mask", ctypes.c_uint32)]


class GPServerStats(ctypes.Structure):
    """struct gp_server_stats of include/gpeval.h"""
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("failed", ctypes.c_int64), ("launches", ctypes.c_int64),
                ("chunks_launched", ctypes.c_int64), ("node_evals", ctypes.c_double),
                ("latency_p50_ms", ctypes.c_double), ("latency_p99_ms", ctypes.c_double),
                ("latency_max_ms", ctypes.c_double), ("latency_mean_ms", ctypes.c_double),
                ("busy_ms", ctypes.c_double), ("wall_ms", ctypes.c_double),
                ("device_bytes_in_use", ctypes.c_int64), ("device_bytes_peak", ctypes.c_int64),
                ("waiting", ctypes.c_int32), ("in_flight", ctypes.c_int32),
                ("cancelled", ctypes.c_int64), ("retried", ctypes.c_int64)]


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
        L.gp_eval_noalloc.argtypes = L.gp_eval.argtypes
        L.gp_eval_noalloc.restype = ctypes.c_int
        L.gp_eval_correlation.argtypes = [vp, vp, i64, i64, vp, i64, vp, i32, i64, vp, i64,
                                          ctypes.c_double, u32, vp, vp, vp]
        L.gp_eval_correlation.restype = ctypes.c_int
        L.gp_eval_reward.argtypes = [vp, vp, i64, i64, vp, i64, vp, i32, i64, vp, i64,
                                     ctypes.c_double, i32, u32, vp, vp, vp]
        L.gp_eval_reward.restype = ctypes.c_int
        L.gp_mc_rank.argtypes = [vp, i64, i32, ctypes.c_uint64, i32, vp, vp, vp, vp]
        L.gp_mc_rank.restype = ctypes.c_int
        L.gp_eval_batched.argtypes = [vp, i32, vp, i32, i64, i64, i32, i64, u32, vp]
        L.gp_eval_batched.restype = ctypes.c_int
        L.gp_predict.argtypes = [vp, vp, i64, i64, vp, i64, vp, i32, i64, i64, u32, vp, i64,
                                 vp, vp]
        L.gp_predict.restype = ctypes.c_int
        L.gp_plan_create.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(GPProblem),
                                     ctypes.POINTER(GPTuning), ctypes.c_int, vp]
        L.gp_plan_create.restype = ctypes.c_int
        L.gp_plan_launch.argtypes = [vp, vp]
        L.gp_plan_launch.restype = ctypes.c_int
        L.gp_plan_update.argtypes = [vp, ctypes.POINTER(GPProblem)]
        L.gp_plan_update.restype = ctypes.c_int
        L.gp_plan_get_tuning.argtypes = [vp, ctypes.POINTER(GPTuning)]
        L.gp_plan_get_tuning.restype = ctypes.c_int
        L.gp_plan_destroy.argtypes = [vp]
        L.gp_plan_destroy.restype = None
        L.gp_workspace_size.argtypes = [i64, i64, i32, i32, i32, i64,
                                        ctypes.POINTER(ctypes.c_size_t)]
        L.gp_workspace_size.restype = ctypes.c_int
        L.gp_server_create.argtypes = [ctypes.POINTER(ctypes.c_void_p),
                                       ctypes.POINTER(GPServerConfig)]
        L.gp_server_create.restype = ctypes.c_int
        L.gp_server_add_dataset.argtypes = [vp, vp, i32, i64, vp, i64, ctypes.c_double,
                                            ctypes.POINTER(ctypes.c_int32)]
        L.gp_server_add_dataset.restype = ctypes.c_int
        L.gp_server_remove_dataset.argtypes = [vp, i32]
        L.gp_server_remove_dataset.restype = ctypes.c_int
        L.gp_server_submit.argtypes = [vp, i32, vp, i64, vp, i64, vp, i64, vp, vp,
                                       ctypes.POINTER(ctypes.c_int64)]
        L.gp_server_submit.restype = ctypes.c_int
        L.gp_server_poll.argtypes = [vp, ctypes.c_double, vp, vp, i32,
                                     ctypes.POINTER(ctypes.c_int32)]
        L.gp_server_poll.restype = ctypes.c_int
        L.gp_server_wait.argtypes = [vp, i64, ctypes.c_double, ctypes.POINTER(ctypes.c_int32),
                                     ctypes.POINTER(ctypes.c_int32)]
        L.gp_server_wait.restype = ctypes.c_int
        L.gp_server_cancel.argtypes = [vp, i64]
        L.gp_server_cancel.restype = ctypes.c_int
        L.gp_server_get_stats.argtypes = [vp, ctypes.POINTER(GPServerStats)]
        L.gp_server_get_stats.restype = ctypes.c_int
        L.gp_server_reset_stats.argtypes = [vp]
        L.gp_server_reset_stats.restype = ctypes.c_int
        L.gp_server_destroy.argtypes = [vp]
        L.gp_server_destroy.restype = None
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
    return _eval_call(lib().gp_eval, nodes, offsets, consts, X, y, tax_on_length, out_fitness,
                      out_status, allowed_op_mask, ld_x, n_cases, stream)


def gp_eval_noalloc(nodes, offsets, consts, X, y, tax_on_length, out_fitness,
                    out_status=None, allowed_op_mask=0, ld_x=None, n_cases=None, stream=None):
    """gp_eval on the library's fixed device workspace (no allocation);
    arguments and results as gp_eval."""
    return _eval_call(lib().gp_eval_noalloc, nodes, offsets, consts, X, y, tax_on_length,
                      out_fitness, out_status, allowed_op_mask, ld_x, n_cases, stream)


def _eval_call(fn, nodes, offsets, consts, X, y, tax_on_length, out_fitness, out_status,
               allowed_op_mask, ld_x, n_cases, stream):
    import torch
    P = offsets.numel() - 1
    if out_fitness.numel() != P:
        raise ValueError("out_fitness must have n_programs entries")
    if X.dim() != 2:
        raise ValueError("X must be 2-D [n_vars, ld_x]")
    n_vars = X.shape[0]
    ld = X.shape[1] if ld_x is None else int(ld_x)
    n = y.numel() if n_cases is None else int(n_cases)
    rc = fn(_dev_ptr(nodes, torch.uint32, "nodes"), _dev_ptr(offsets, torch.int64, "offsets"),
            P, nodes.numel(), _dev_ptr(consts, torch.float32, "consts"), consts.numel(),
            _dev_ptr(X, torch.float32, "X"), n_vars, ld,
            _dev_ptr(y, torch.float32, "y"), n, float(tax_on_length),
            int(allowed_op_mask), _dev_ptr(out_fitness, torch.float64, "out_fitness"),
            _dev_ptr(out_status, torch.int32, "out_status"), _stream_handle(stream))
    _check(rc)
    return out_fitness


def gp_eval_correlation(nodes, offsets, consts, X, y, max_score, out_score,
                        out_status=None, allowed_op_mask=0, ld_x=None, n_cases=None,
                        stream=None):
    """Correlation score (Eq. 1-2) of the population held in device tensors
    (asynchronous on stream); arguments as gp_eval, max_score = M."""
    import torch
    P = offsets.numel() - 1
    if out_score.numel() != P:
        raise ValueError("out_score must have n_programs entries")
    if X.dim() != 2:
        raise ValueError("X must be 2-D [n_vars, ld_x]")
    n_vars = X.shape[0]
    ld = X.shape[1] if ld_x is None else int(ld_x)
    n = y.numel() if n_cases is None else int(n_cases)
    rc = lib().gp_eval_correlation(
        _dev_ptr(nodes, torch.uint32, "nodes"), _dev_ptr(offsets, torch.int64, "offsets"),
        P, nodes.numel(), _dev_ptr(consts, torch.float32, "consts"), consts.numel(),
        _dev_ptr(X, torch.float32, "X"), n_vars, ld, _dev_ptr(y, torch.float32, "y"), n,
        float(max_score), int(allowed_op_mask), _dev_ptr(out_score, torch.float64, "out_score"),
        _dev_ptr(out_status, torch.int32, "out_status"), _stream_handle(stream))
    _check(rc)
    return out_score


def gp_eval_reward(nodes, offsets, consts, X, y, max_score, power, out_reward,
                   out_status=None, allowed_op_mask=0, ld_x=None, n_cases=None, stream=None):
    """Integer point-to-point reward (Eq. 5; power 1, 2, 3 or 8) of the
    population held in device tensors (asynchronous on stream); arguments
    as gp_eval, max_score = M."""
    import torch
    P = offsets.numel() - 1
    if out_reward.numel() != P:
        raise ValueError("out_reward must have n_programs entries")
    if X.dim() != 2:
        raise ValueError("X must be 2-D [n_vars, ld_x]")
    n_vars = X.shape[0]
    ld = X.shape[1] if ld_x is None else int(ld_x)
    n = y.numel() if n_cases is None else int(n_cases)
    rc = lib().gp_eval_reward(
        _dev_ptr(nodes, torch.uint32, "nodes"), _dev_ptr(offsets, torch.int64, "offsets"),
        P, nodes.numel(), _dev_ptr(consts, torch.float32, "consts"), consts.numel(),
        _dev_ptr(X, torch.float32, "X"), n_vars, ld, _dev_ptr(y, torch.float32, "y"), n,
        float(max_score), int(power), int(allowed_op_mask),
        _dev_ptr(out_reward, torch.float64, "out_reward"),
        _dev_ptr(out_status, torch.int32, "out_status"), _stream_handle(stream))
    _check(rc)
    return out_reward


def gp_mc_rank(fitness, higher_is_better, seed, out_band, out_children=None,
               out_sample_keys=None, sample_size=100, stream=None):
    """Monte-Carlo ranking of a device float64 fitness tensor (asynchronous):
    percentile bands into out_band (int32), Table 2's expected children
    into out_children (float32, optional), the sorted sample keys into
    out_sample_keys (float64[sample_size], optional)."""
    import torch
    n = fitness.numel()
    if out_band.numel() != n:
        raise ValueError("out_band must have one entry per individual")
    rc = lib().gp_mc_rank(_dev_ptr(fitness, torch.float64, "fitness"), n,
                          1 if higher_is_better else 0, int(seed) & ((1 << 64) - 1),
                          int(sample_size), _dev_ptr(out_band, torch.int32, "out_band"),
                          _dev_ptr(out_children, torch.float32, "out_children"),
                          _dev_ptr(out_sample_keys, torch.float64, "out_sample_keys"),
                          _stream_handle(stream))
    _check(rc)
    return out_band


def table_tensor(entries, device="cuda"):
    """Pack ctypes structures into a device byte tensor (the dataset and
    request tables of gp_eval_batched)."""
    import torch
    if not entries:
        return torch.zeros(0, dtype=torch.uint8, device=device)
    raw = b"".join(bytes(e) for e in entries)
    host = torch.frombuffer(bytearray(raw), dtype=torch.uint8)
    return host.to(device)


def dataset_entry(data, tax_on_length=0.0):
    """GPDataset for a resident dataset (X [n_vars, ld], y [n_cases])."""
    import torch
    return GPDataset(_dev_ptr(data.X, torch.float32, "X"), _dev_ptr(data.y, torch.float32, "y"),
                     data.X.shape[1], data.n_cases, float(tax_on_length), data.n_vars, 0)


def request_entry(pop, dataset, out_fitness, out_status=None):
    """GPRequest for a resident population scored against table entry
    `dataset`, writing into out_fitness (float64[P]) / out_status."""
    import torch
    if out_fitness.numel() < pop.n_programs:
        raise ValueError("out_fitness holds fewer than n_programs values")
    if out_status is not None and out_status.numel() < pop.n_programs:
        raise ValueError("out_status holds fewer than n_programs values")
    return GPRequest(_dev_ptr(pop.nodes, torch.uint32, "nodes"),
                     _dev_ptr(pop.offsets, torch.int64, "offsets"),
                     _dev_ptr(pop.consts, torch.float32, "consts"), pop.n_programs,
                     pop.nodes.numel(), pop.consts.numel(),
                     _dev_ptr(out_fitness, torch.float64, "out_fitness"),
                     _dev_ptr(out_status, torch.int32, "out_status"), int(dataset), 0)


def gp_eval_batched(requests, datasets, total_programs, total_nodes, max_n_vars, max_n_cases,
                    allowed_op_mask=0, stream=None):
    """Score many requests in one launch.  requests / datasets: uint8 device
    tensors holding packed GPRequest / GPDataset entries (see table_tensor);
    the totals and bounds are the host's view of those tables."""
    import torch
    n_req = requests.numel() // ctypes.sizeof(GPRequest)
    n_ds = datasets.numel() // ctypes.sizeof(GPDataset)
    rc = lib().gp_eval_batched(_dev_ptr(requests, torch.uint8, "requests"), n_req,
                               _dev_ptr(datasets, torch.uint8, "datasets"), n_ds,
                               int(total_programs), int(total_nodes), int(max_n_vars),
                               int(max_n_cases), int(allowed_op_mask), _stream_handle(stream))
    _check(rc)


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


def _problem(pop, data, tax, out, status, allowed_op_mask):
    import torch
    return GPProblem(_dev_ptr(pop.nodes, torch.uint32, "nodes"),
                     _dev_ptr(pop.offsets, torch.int64, "offsets"), pop.n_programs,
                     pop.nodes.numel(), _dev_ptr(pop.consts, torch.float32, "consts"),
                     pop.consts.numel(), _dev_ptr(data.X, torch.float32, "X"), data.n_vars,
                     data.X.shape[1], _dev_ptr(data.y, torch.float32, "y"), data.n_cases,
                     float(tax), int(allowed_op_mask), _dev_ptr(out, torch.float64, "out"),
                     _dev_ptr(status, torch.int32, "status"))


class Plan:
    """A captured evaluation (hipGraph) of one population shape; relaunch it
    after rewriting the population/data tensors in place."""

    def __init__(self, pop, data, tax_on_length, out, status=None, allowed_op_mask=0,
                 tuning=None, autotune=False, stream=None):
        self._keep = (pop, data, out, status)
        pb = _problem(pop, data, tax_on_length, out, status, allowed_op_mask)
        tu = None
        if tuning is not None:
            tu = GPTuning(int(tuning.get("programs_per_item", 0)), int(tuning.get("wg_per_cu", 0)),
                          int(tuning.get("concurrent_classes", 0)),
                          int(tuning.get("tile_lds_bytes", 0)), int(tuning.get("max_tiles", 0)))
        h = ctypes.c_void_p()
        _check(lib().gp_plan_create(ctypes.byref(h), ctypes.byref(pb),
                                    ctypes.byref(tu) if tu is not None else None,
                                    1 if autotune else 0, _stream_handle(stream)))
        self._h = h

    def launch(self, stream=None):
        _check(lib().gp_plan_launch(self._h, _stream_handle(stream)))

    def update(self, pop, data, tax_on_length, out, status=None, allowed_op_mask=0):
        self._keep = (pop, data, out, status)
        pb = _problem(pop, data, tax_on_length, out, status, allowed_op_mask)
        _check(lib().gp_plan_update(self._h, ctypes.byref(pb)))

    @property
    def tuning(self):
        t = GPTuning()
        _check(lib().gp_plan_get_tuning(self._h, ctypes.byref(t)))
        return {"programs_per_item": t.programs_per_item, "wg_per_cu": t.wg_per_cu,
                "concurrent_classes": t.concurrent_classes, "tile_lds_bytes": t.tile_lds_bytes,
                "max_tiles": t.max_tiles}

    def close(self):
        if getattr(self, "_h", None):
            lib().gp_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


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


def evaluate_correlation(nodes, offsets, consts, X, y, max_score=1e4, allowed_op_mask=0,
                         return_status=False, device="cuda"):
    """numpy in, numpy out: upload, correlation score, download (synchronizes)."""
    import torch
    pop = DevicePopulation(nodes, offsets, consts, device)
    data = DeviceDataset(X, y, device)
    out = torch.empty(pop.n_programs, dtype=torch.float64, device=device)
    st = torch.empty(pop.n_programs, dtype=torch.int32, device=device) if return_status else None
    gp_eval_correlation(pop.nodes, pop.offsets, pop.consts, data.X, data.y, max_score, out, st,
                        allowed_op_mask)
    torch.cuda.synchronize()
    if return_status:
        return out.cpu().numpy(), st.cpu().numpy()
    return out.cpu().numpy()


def evaluate_reward(nodes, offsets, consts, X, y, max_score=1e4, power=1, allowed_op_mask=0,
                    return_status=False, device="cuda"):
    """numpy in, numpy out: upload, integer reward, download (synchronizes)."""
    import torch
    pop = DevicePopulation(nodes, offsets, consts, device)
    data = DeviceDataset(X, y, device)
    out = torch.empty(pop.n_programs, dtype=torch.float64, device=device)
    st = torch.empty(pop.n_programs, dtype=torch.int32, device=device) if return_status else None
    gp_eval_reward(pop.nodes, pop.offsets, pop.consts, data.X, data.y, max_score, power, out,
                   st, allowed_op_mask)
    torch.cuda.synchronize()
    if return_status:
        return out.cpu().numpy(), st.cpu().numpy()
    return out.cpu().numpy()


def workspace_size(n_programs, n_nodes, n_requests=1, n_datasets=1, max_n_vars=1,
                   max_n_cases=1):
    """gp_workspace_size: device bytes one call of this shape may hold."""
    b = ctypes.c_size_t()
    _check(lib().gp_workspace_size(int(n_programs), int(n_nodes), int(n_requests),
                                   int(n_datasets), int(max_n_vars), int(max_n_cases),
                                   ctypes.byref(b)))
    return b.value


class Server:
    """gp_server: resident datasets, admission by device budget, chunking and
    continuous batching on the library's scheduler thread.  Requests take
    host (numpy) arrays; this wrapper keeps them alive until their ticket
    completes and returns the result arrays."""

    def __init__(self, device_budget_bytes=0, pinned_bytes=0, chunk_node_evals=0,
                 batch_node_evals=0, n_streams=0, max_batch_chunks=0,
                 one_launch_per_request=False, allowed_op_mask=0):
        cfg = GPServerConfig(int(device_budget_bytes), int(pinned_bytes), int(chunk_node_evals),
                             int(batch_node_evals), int(n_streams), int(max_batch_chunks),
                             1 if one_launch_per_request else 0, int(allowed_op_mask))
        h = ctypes.c_void_p()
        _check(lib().gp_server_create(ctypes.byref(h), ctypes.byref(cfg)))
        self._h = h
        self._pending = {}          # ticket -> (arrays kept alive, fitness, status)

    def add_dataset(self, X, y, tax_on_length=0.0):
        X = np.ascontiguousarray(X, np.float32)
        if X.ndim == 1:
            X = X.reshape(1, -1)
        y = np.ascontiguousarray(y, np.float32)
        i = ctypes.c_int32()
        _check(lib().gp_server_add_dataset(self._h, X.ctypes.data, X.shape[0], X.shape[1],
                                           y.ctypes.data, y.size, float(tax_on_length),
                                           ctypes.byref(i)))
        return i.value

    def remove_dataset(self, dataset_id):
        _check(lib().gp_server_remove_dataset(self._h, int(dataset_id)))

    def submit(self, dataset_id, nodes, offsets, consts):
        nodes = np.ascontiguousarray(nodes, np.uint32)
        offsets = np.ascontiguousarray(offsets, np.int64)
        consts = np.ascontiguousarray(consts, np.float32)
        P = offsets.size - 1
        # written by the server only when the request completes with GP_OK
        fit = np.full(P, -1.0, np.float64)
        st = np.full(P, -1, np.int32)
        t = ctypes.c_int64()
        _check(lib().gp_server_submit(self._h, int(dataset_id),
                                      nodes.ctypes.data if nodes.size else None, nodes.size,
                                      offsets.ctypes.data, P,
                                      consts.ctypes.data if consts.size else None, consts.size,
                                      fit.ctypes.data, st.ctypes.data, ctypes.byref(t)))
        self._pending[t.value] = ((nodes, offsets, consts), fit, st)
        return t.value

    def poll(self, timeout_ms=0.0, max_n=256):
        """Completed requests: list of (ticket, result code, fitness, status)."""
        tk = np.empty(max_n, np.int64)
        rc = np.empty(max_n, np.int32)
        n = ctypes.c_int32()
        _check(lib().gp_server_poll(self._h, float(timeout_ms), tk.ctypes.data, rc.ctypes.data,
                                    max_n, ctypes.byref(n)))
        out = []
        for i in range(n.value):
            _, fit, st = self._pending.pop(int(tk[i]))
            out.append((int(tk[i]), int(rc[i]), fit, st))
        return out

    def wait(self, ticket, timeout_ms=-1.0):
        """(result code, fitness, status) of one ticket, or None on timeout."""
        done, res = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().gp_server_wait(self._h, int(ticket), float(timeout_ms), ctypes.byref(done),
                                    ctypes.byref(res)))
        if not done.value:
            return None
        _, fit, st = self._pending.pop(int(ticket))
        return res.value, fit, st

    def cancel(self, ticket):
        """Cancels a pending request (it completes with GP_E_CANCELLED)."""
        _check(lib().gp_server_cancel(self._h, int(ticket)))

    def stats(self):
        s = GPServerStats()
        _check(lib().gp_server_get_stats(self._h, ctypes.byref(s)))
        return {k: getattr(s, k) for k, _ in GPServerStats._fields_}

    def reset_stats(self):
        _check(lib().gp_server_reset_stats(self._h))

    def close(self):
        if getattr(self, "_h", None):
            lib().gp_server_destroy(self._h)
            self._h = None
            self._pending.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
