"""Thin ctypes binding of libcentra.so (include/centra.h).

Argument marshalling only: every step of the hot path runs in the HIP
kernels of the library.  Device buffers are torch tensors on a HIP device
(PyTorch provides device memory and streams, nothing else).  If the library
has not been built this module raises; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcentra.so")

CENTRA_OK = 0
CENTRA_NOT_CERTIFIED = 1
CENTRA_STOPPED = 2
CENTRA_EINVAL = -1
CENTRA_ENOMEM = -2
CENTRA_EHIP = -3
CENTRA_ENOSPC = -4
CENTRA_ENOTSUP = -5

CENTRA_SCHEDULE_GEOMETRIC = 0
CENTRA_SCHEDULE_ADAPTIVE = 1
CENTRA_SCHEDULE_FIXED = 2
CENTRA_SPACE_SHORTEST_PATHS = 0
CENTRA_SPACE_TRIANGLES = 1
CENTRA_SPACE_KPATHS = 2
CENTRA_SPACE_PATHS_BIDIR = 3
CENTRA_METHOD_CENTRA = 0
CENTRA_METHOD_HEDGE_P = 1
CENTRA_MAX_KAPPA = 16

_c = ctypes
_vp = _c.c_void_p


class CentraError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"centra error {code}: {msg}")
        self.code = code


class Csr(_c.Structure):
    _fields_ = [("n", _c.c_uint32), ("directed", _c.c_uint32), ("n_arcs", _c.c_uint64),
                ("row_ptr", _vp), ("col_idx", _vp), ("rrow_ptr", _vp), ("rcol_idx", _vp)]


class BoundOut(_c.Structure):
    _fields_ = [("c_hat", _c.c_double), ("amcera", _c.c_double), ("wimpy", _c.c_double),
                ("xi", _c.c_double), ("nu", _c.c_double), ("rtilde", _c.c_double),
                ("r", _c.c_double), ("eta", _c.c_double), ("certified", _c.c_int)]


class VcOut(_c.Structure):
    _fields_ = [("d1", _c.c_uint32), ("dk_lemma", _c.c_uint64), ("dk_union", _c.c_uint64), ("dk", _c.c_uint64)]


class Params(_c.Structure):
    _fields_ = [("k", _c.c_uint32), ("t", _c.c_uint32), ("eps", _c.c_double), ("delta", _c.c_double),
                ("seed", _c.c_uint64), ("instance", _c.c_uint32), ("m_init", _c.c_uint64),
                ("m_max", _c.c_uint64), ("growth_num", _c.c_uint32), ("growth_den", _c.c_uint32),
                ("schedule", _c.c_uint32), ("space", _c.c_uint32), ("kappa", _c.c_uint32),
                ("method", _c.c_uint32)]


class Result(_c.Structure):
    _fields_ = [("n_picked", _c.c_uint32), ("iterations", _c.c_uint32), ("certified", _c.c_int),
                ("coverage", _c.c_uint64), ("m_final", _c.c_uint64),
                ("c_hat", _c.c_double), ("amcera", _c.c_double), ("wimpy", _c.c_double),
                ("xi", _c.c_double), ("nu", _c.c_double), ("rtilde", _c.c_double), ("r", _c.c_double),
                ("eta", _c.c_double), ("ms_sample", _c.c_double), ("ms_cover", _c.c_double),
                ("ms_mcera", _c.c_double), ("ms_total", _c.c_double)]


class Iteration(_c.Structure):
    _fields_ = [("i", _c.c_uint32), ("m", _c.c_uint64), ("coverage", _c.c_uint64), ("sum_topk", _c.c_int64),
                ("deg_topk", _c.c_uint64), ("b_max", _c.c_uint32), ("delta_i", _c.c_double),
                ("amcera", _c.c_double), ("wimpy", _c.c_double), ("xi", _c.c_double), ("nu", _c.c_double),
                ("rtilde", _c.c_double), ("r", _c.c_double), ("eta", _c.c_double), ("certified", _c.c_int),
                ("ms_sample", _c.c_double), ("ms_cover", _c.c_double), ("ms_mcera", _c.c_double),
                ("arcs", _c.c_uint64), ("nodes", _c.c_uint64)]


CENTRA_CHECKPOINT_VERSION = 1


class Checkpoint(_c.Structure):
    _fields_ = [("version", _c.c_uint32), ("i", _c.c_uint32), ("graph_hash", _c.c_uint64),
                ("params_hash", _c.c_uint64), ("m_i", _c.c_uint64), ("m_next", _c.c_uint64),
                ("entries", _c.c_uint64)]

    def to_dict(self) -> dict:
        return {f: int(getattr(self, f)) for f, _ in self._fields_}

    @classmethod
    def from_dict(cls, d: dict) -> "Checkpoint":
        return cls(**{f: int(d[f]) for f, _ in cls._fields_})


class SamplerStats(_c.Structure):
    _fields_ = [("launches", _c.c_uint64), ("kernel_ms", _c.c_double), ("samples", _c.c_uint64),
                ("arcs", _c.c_uint64), ("nodes", _c.c_uint64), ("hyperedge_nodes", _c.c_uint64),
                ("lds_bitmap", _c.c_uint32), ("slots", _c.c_uint32), ("wide", _c.c_uint64),
                ("wide_ms", _c.c_double), ("wide_arcs", _c.c_uint64)]


class PoolParams(_c.Structure):
    _fields_ = [("seed", _c.c_uint64), ("instance", _c.c_uint32), ("t", _c.c_uint32), ("m_init", _c.c_uint64),
                ("m_max", _c.c_uint64), ("growth_num", _c.c_uint32), ("growth_den", _c.c_uint32)]


class QueryInfo(_c.Structure):
    _fields_ = [("arrival_s", _c.c_double), ("admitted_s", _c.c_double), ("finished_s", _c.c_double),
                ("pool", _c.c_uint32)]


class EngineStats(_c.Structure):
    _fields_ = [("ticks", _c.c_uint64), ("sampler_launches", _c.c_uint64), ("samples", _c.c_uint64),
                ("greedy_runs", _c.c_uint64), ("greedy_launches", _c.c_uint64), ("graph_replays", _c.c_uint64), ("graphs_captured", _c.c_uint64),
                ("ms_sample", _c.c_double), ("ms_levels", _c.c_double), ("ms_greedy", _c.c_double),
                ("ms_select", _c.c_double), ("peak_bytes", _c.c_uint64), ("peak_active", _c.c_uint32),
                ("tuned_block", _c.c_uint32)]


class ExtendArgs(_c.Structure):
    _fields_ = [("n", _c.c_uint32), ("k", _c.c_uint32), ("m_prev", _c.c_uint64), ("m", _c.c_uint64),
                ("he_off", _vp), ("he_nodes", _vp), ("he_cap", _c.c_uint64),
                ("picks", _vp), ("cov_cum", _vp), ("n_picked", _vp),
                ("t", _c.c_uint32), ("instance", _c.c_uint32), ("seed", _c.c_uint64),
                ("topk_sum", _vp), ("deg_topk_sum", _vp), ("b_max", _vp), ("R_out", _vp)]


CENTRA_ENGINE_NO_GRAPHS = 1
CENTRA_ENGINE_NO_TUNE = 2
CENTRA_ENGINE_NO_CACHE = 4


# name -> (restype, argtypes); the names and order are those of centra.h
SIGNATURES = {
    "centra_abi_version": (_c.c_uint32, []),
    "centra_create": (_c.c_int, [_c.c_int, _c.c_size_t, _c.POINTER(_vp)]),
    "centra_destroy": (None, [_vp]),
    "centra_last_error": (_c.c_char_p, [_vp]),
    "centra_context_log": (_c.c_char_p, [_vp]),
    "centra_graph_prepare": (_c.c_int, [_vp, _c.POINTER(Csr), _c.c_uint32, _c.POINTER(_vp), _vp]),
    "centra_graph_release": (None, [_vp]),
    "centra_graph_info": (_c.c_int, [_vp, _c.POINTER(_c.c_uint32), _c.POINTER(_c.c_uint32)]),
    "centra_graph_hash": (_c.c_int, [_vp, _c.POINTER(_c.c_uint64)]),
    "centra_sample_paths": (_c.c_int, [_vp, _vp, _c.c_uint64, _c.c_uint32, _c.c_uint64, _c.c_uint32, _vp, _vp,
                                       _c.c_uint64, _c.POINTER(_c.c_uint64), _vp, _vp, _vp]),
    "centra_sample_paths_bidir": (_c.c_int, [_vp, _vp, _c.c_uint64, _c.c_uint32, _c.c_uint64, _c.c_uint32, _vp,
                                             _vp, _c.c_uint64, _c.POINTER(_c.c_uint64), _vp, _vp, _vp]),
    "centra_greedy_cover": (_c.c_int, [_vp, _c.c_uint32, _c.c_uint64, _vp, _vp, _c.c_uint32, _vp, _vp, _vp, _vp]),
    "centra_greedy_cover_noalloc": (_c.c_int, [_c.c_uint32, _c.c_uint64, _vp, _vp, _c.c_uint32, _vp, _vp, _vp, _vp]),
    "centra_mcera": (_c.c_int, [_vp, _c.c_uint32, _c.c_uint64, _vp, _vp, _c.c_uint64, _c.c_uint32, _c.c_uint32,
                                _c.c_uint32, _vp, _vp, _vp, _vp, _vp]),
    "centra_sample_paths_append": (_c.c_int, [_vp, _vp, _c.c_uint64, _c.c_uint32, _c.c_uint64, _c.c_uint32, _vp,
                                              _vp, _c.c_uint64, _vp, _vp]),
    "centra_extend": (_c.c_int, [_vp, _c.POINTER(ExtendArgs), _vp]),
    "centra_reserve": (_c.c_int, [_vp, _vp, _c.c_uint32, _c.c_uint32, _c.c_uint64, _c.c_uint64, _c.c_uint32,
                                  _c.c_uint32, _vp]),
    "centra_check": (_c.c_int, [_vp, _vp]),
    "centra_sampler_stats_get": (_c.c_int, [_vp, _c.POINTER(SamplerStats), _c.c_int]),
    "centra_triangle_count": (_c.c_int, [_vp, _vp, _c.POINTER(_c.c_uint64), _vp]),
    "centra_sample_triangles": (_c.c_int, [_vp, _vp, _c.c_uint64, _c.c_uint32, _c.c_uint64, _c.c_uint32, _vp, _vp,
                                           _vp]),
    "centra_sample_kpaths": (_c.c_int, [_vp, _vp, _c.c_uint32, _c.c_uint64, _c.c_uint32, _c.c_uint64, _c.c_uint32,
                                        _vp, _vp, _vp]),
    "centra_bound": (_c.c_int, [_c.c_uint64, _c.c_uint64, _c.c_int64, _c.c_uint32, _c.c_uint64, _c.c_uint32,
                                _c.c_double, _c.c_double, _c.POINTER(BoundOut)]),
    "centra_hedge_bound": (_c.c_int, [_c.c_uint64, _c.c_uint64, _c.c_uint64, _c.c_uint32, _c.c_double, _c.c_double,
                                      _c.POINTER(BoundOut)]),
    "centra_vc_dims": (_c.c_int, [_c.c_uint64, _c.c_uint32, _c.c_uint64, _c.POINTER(VcOut)]),
    "centra_progressive": (_c.c_int, [_vp, _vp, _c.POINTER(Params), _vp, _c.POINTER(Result),
                                      _c.POINTER(Iteration), _c.c_uint32, _vp]),
    "centra_params_hash": (_c.c_int, [_c.POINTER(Params), _c.POINTER(_c.c_uint64)]),
    "centra_progressive_resumable": (_c.c_int, [_vp, _vp, _c.POINTER(Params), _c.POINTER(Checkpoint),
                                                _c.POINTER(Checkpoint), _c.c_uint32, _vp, _c.POINTER(Result),
                                                _c.POINTER(Iteration), _c.c_uint32, _vp]),
    "centra_engine_create": (_c.c_int, [_vp, _c.c_size_t, _c.c_uint32, _c.POINTER(_vp)]),
    "centra_engine_destroy": (None, [_vp]),
    "centra_engine_add_pool": (_c.c_int, [_vp, _vp, _c.POINTER(PoolParams), _c.POINTER(_c.c_uint32)]),
    "centra_engine_prefill": (_c.c_int, [_vp, _c.c_uint32, _c.c_uint64, _vp]),
    "centra_engine_submit": (_c.c_int, [_vp, _c.c_uint32, _c.c_uint32, _c.c_uint32, _c.c_double, _c.c_double,
                                        _c.c_double, _c.POINTER(_c.c_uint32)]),
    "centra_engine_run": (_c.c_int, [_vp, _c.c_int, _vp]),
    "centra_engine_result": (_c.c_int, [_vp, _c.c_uint32, _vp, _c.POINTER(Result), _c.POINTER(QueryInfo)]),
    "centra_engine_stats_get": (_c.c_int, [_vp, _c.POINTER(EngineStats)]),
    "centra_engine_log": (_c.c_char_p, [_vp]),
}

_lib = None


def lib():
    """The loaded libcentra.so; raises if it was not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build the HIP library first "
                              "(python -c 'import __graft_entry__ as g; g.build()')")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _ptr(x):
    """Device (or host numpy) pointer of a buffer, or None."""
    if x is None:
        return None
    if isinstance(x, np.ndarray):
        return x.ctypes.data
    if x.device.type != "cuda":
        raise ValueError("expected a tensor on a HIP device")
    if not x.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return x.data_ptr()


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _check(rc: int, ctx=None):
    if rc < 0:
        raise CentraError(rc, centra_last_error(ctx))
    return rc


def _dtype_check(t, dtype, name):
    if t is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")


# ---------------------------------------------------------------------------
def centra_abi_version() -> int:
    return lib().centra_abi_version()


def centra_create(device: int = 0, hbm_budget_bytes: int = 0):
    out = _vp()
    _check(lib().centra_create(device, hbm_budget_bytes, ctypes.byref(out)))
    return out


def centra_destroy(ctx) -> None:
    lib().centra_destroy(ctx)


def centra_last_error(ctx=None) -> str:
    s = lib().centra_last_error(ctx)
    return s.decode() if s else ""


def centra_context_log(ctx) -> str:
    s = lib().centra_context_log(ctx)
    return s.decode() if s else ""


def centra_graph_prepare(ctx, row_ptr, col_idx, rrow_ptr=None, rcol_idx=None, count_bits_override: int = 0,
                         stream=None):
    """Prepares a CSR graph held in device tensors (uint32 / torch.int32 views)."""
    import torch
    for name, t in (("row_ptr", row_ptr), ("col_idx", col_idx), ("rrow_ptr", rrow_ptr), ("rcol_idx", rcol_idx)):
        _dtype_check(t, torch.int32, name)
    directed = rrow_ptr is not None
    csr = Csr(row_ptr.numel() - 1, 1 if directed else 0, col_idx.numel(), _ptr(row_ptr), _ptr(col_idx),
              _ptr(rrow_ptr), _ptr(rcol_idx))
    out = _vp()
    _check(lib().centra_graph_prepare(ctx, ctypes.byref(csr), count_bits_override, ctypes.byref(out),
                                      _stream(stream)), ctx)
    return out


def centra_graph_release(g) -> None:
    lib().centra_graph_release(g)


def centra_graph_info(g):
    a, b = ctypes.c_uint32(), ctypes.c_uint32()
    _check(lib().centra_graph_info(g, ctypes.byref(a), ctypes.byref(b)))
    return a.value, b.value


def centra_sample_paths(ctx, g, seed: int, instance: int, first_sample: int, count: int, he_off, he_nodes,
                        he_cap: int | None = None, st_out=None, dist_out=None, stream=None):
    """Returns (rc, he_needed).  rc may be CENTRA_ENOSPC (no exception)."""
    import torch
    _dtype_check(he_off, torch.int64, "he_off")
    _dtype_check(he_nodes, torch.int32, "he_nodes")
    if he_cap is None:
        he_cap = he_nodes.numel() if he_nodes is not None else 0
    need = ctypes.c_uint64()
    rc = lib().centra_sample_paths(ctx, g, seed, instance, first_sample, count, _ptr(he_off), _ptr(he_nodes),
                                   he_cap, ctypes.byref(need), _ptr(st_out), _ptr(dist_out), _stream(stream))
    if rc != CENTRA_ENOSPC:
        _check(rc, ctx)
    return rc, need.value


def centra_sample_paths_bidir(ctx, g, seed: int, instance: int, first_sample: int, count: int, he_off, he_nodes,
                              he_cap: int | None = None, st_out=None, dist_out=None, stream=None):
    """Returns (rc, he_needed).  rc may be CENTRA_ENOSPC (no exception)."""
    import torch
    _dtype_check(he_off, torch.int64, "he_off")
    _dtype_check(he_nodes, torch.int32, "he_nodes")
    if he_cap is None:
        he_cap = he_nodes.numel() if he_nodes is not None else 0
    need = ctypes.c_uint64()
    rc = lib().centra_sample_paths_bidir(ctx, g, seed, instance, first_sample, count, _ptr(he_off), _ptr(he_nodes),
                                         he_cap, ctypes.byref(need), _ptr(st_out), _ptr(dist_out), _stream(stream))
    if rc != CENTRA_ENOSPC:
        _check(rc, ctx)
    return rc, need.value


def centra_greedy_cover(ctx, n: int, he_off, he_nodes, k: int, picks, cov_cum, n_picked, stream=None) -> int:
    m = he_off.numel() - 1
    return _check(lib().centra_greedy_cover(ctx, n, m, _ptr(he_off), _ptr(he_nodes), k, _ptr(picks),
                                            _ptr(cov_cum), _ptr(n_picked), _stream(stream)), ctx)


def centra_greedy_cover_noalloc(n: int, he_off, he_nodes, k: int, picks, cov_cum, n_picked, stream=None) -> int:
    m = he_off.numel() - 1
    return _check(lib().centra_greedy_cover_noalloc(n, m, _ptr(he_off), _ptr(he_nodes), k, _ptr(picks),
                                                    _ptr(cov_cum), _ptr(n_picked), _stream(stream)))


def centra_mcera(ctx, n: int, he_off, he_nodes, seed: int, instance: int, t: int, k: int, topk_sum, deg_topk,
                 b_max, R_out=None, stream=None) -> int:
    m = he_off.numel() - 1
    return _check(lib().centra_mcera(ctx, n, m, _ptr(he_off), _ptr(he_nodes), seed, instance, t, k,
                                     _ptr(topk_sum), _ptr(deg_topk), _ptr(b_max), _ptr(R_out), _stream(stream)),
                  ctx)


def centra_sample_paths_append(ctx, g, seed: int, instance: int, first_sample: int, count: int, he_off, he_nodes,
                               he_cap: int | None = None, he_total=None, stream=None) -> int:
    """Stream-ordered: he_off is the store's offset array from the first new
    sample on (a slice store_off[m_before:]); nothing is synchronised."""
    import torch
    _dtype_check(he_off, torch.int64, "he_off")
    _dtype_check(he_nodes, torch.int32, "he_nodes")
    if he_cap is None:
        he_cap = he_nodes.numel() if he_nodes is not None else 0
    return _check(lib().centra_sample_paths_append(ctx, g, seed, instance, first_sample, count, _ptr(he_off),
                                                   _ptr(he_nodes), he_cap, _ptr(he_total), _stream(stream)), ctx)


def centra_extend(ctx, n: int, k: int, m_prev: int, m: int, he_off, he_nodes, he_cap: int | None = None,
                  picks=None, cov_cum=None, n_picked=None, t: int = 0, seed: int = 0, instance: int = 0,
                  topk_sum=None, deg_topk=None, b_max=None, R_out=None, stream=None) -> int:
    """Stream-ordered greedy + AMCERA on samples [0, m) of a growing store."""
    if he_cap is None:
        he_cap = he_nodes.numel() if he_nodes is not None else 0
    a = ExtendArgs(n=n, k=k, m_prev=m_prev, m=m, he_off=_ptr(he_off), he_nodes=_ptr(he_nodes), he_cap=he_cap,
                   picks=_ptr(picks), cov_cum=_ptr(cov_cum), n_picked=_ptr(n_picked), t=t, instance=instance,
                   seed=seed, topk_sum=_ptr(topk_sum), deg_topk_sum=_ptr(deg_topk), b_max=_ptr(b_max),
                   R_out=_ptr(R_out))
    return _check(lib().centra_extend(ctx, ctypes.byref(a), _stream(stream)), ctx)


def centra_reserve(ctx, g, n: int, batch: int, m_max: int, he_cap: int, k: int, t: int, stream=None) -> int:
    return _check(lib().centra_reserve(ctx, g, n, batch, m_max, he_cap, k, t, _stream(stream)), ctx)


def centra_check(ctx, stream=None) -> int:
    """Returns CENTRA_OK or CENTRA_ENOSPC; raises on other device-side errors."""
    rc = lib().centra_check(ctx, _stream(stream))
    if rc != CENTRA_ENOSPC:
        _check(rc, ctx)
    return rc


def centra_sampler_stats_get(ctx, reset: bool = False) -> SamplerStats:
    out = SamplerStats()
    _check(lib().centra_sampler_stats_get(ctx, ctypes.byref(out), 1 if reset else 0), ctx)
    return out


def centra_bound(m: int, cov: int, sum_topk: int, t: int, deg_topk: int, b_max: int, eps: float,
                 delta_i: float) -> BoundOut:
    out = BoundOut()
    _check(lib().centra_bound(m, cov, sum_topk, t, deg_topk, b_max, eps, delta_i, ctypes.byref(out)))
    return out


def centra_hedge_bound(m: int, cov: int, n: int, k: int, eps: float, delta_i: float) -> BoundOut:
    out = BoundOut()
    _check(lib().centra_hedge_bound(m, cov, n, k, eps, delta_i, ctypes.byref(out)))
    return out


def centra_vc_dims(b: int, k: int, n: int) -> VcOut:
    out = VcOut()
    _check(lib().centra_vc_dims(b, k, n, ctypes.byref(out)))
    return out


def centra_progressive(ctx, g, k: int, t: int, eps: float, delta: float, seed: int, instance: int, m_init: int,
                       m_max: int, growth_num: int = 2, growth_den: int = 1, log_cap: int = 64, stream=None,
                       schedule: int = CENTRA_SCHEDULE_GEOMETRIC, space: int = CENTRA_SPACE_SHORTEST_PATHS,
                       kappa: int = 0, method: int = 0):
    """Returns (rc, picks np.uint32[n_picked], Result, [Iteration])."""
    p = Params(k, t, eps, delta, seed, instance, m_init, m_max, growth_num, growth_den, schedule, space, kappa,
               method)
    picks = np.zeros(max(1, k), dtype=np.uint32)
    res = Result()
    log = (Iteration * max(1, log_cap))()
    rc = _check(lib().centra_progressive(ctx, g, ctypes.byref(p), picks.ctypes.data, ctypes.byref(res), log,
                                         log_cap, _stream(stream)), ctx)
    return rc, picks[: res.n_picked].copy(), res, list(log)[: min(res.iterations, log_cap)]


def centra_params_hash(p: Params) -> int:
    out = ctypes.c_uint64()
    _check(lib().centra_params_hash(ctypes.byref(p), ctypes.byref(out)))
    return out.value


def centra_graph_hash(g) -> int:
    out = ctypes.c_uint64()
    _check(lib().centra_graph_hash(g, ctypes.byref(out)))
    return out.value


def centra_progressive_resumable(ctx, g, p: Params, resume: Checkpoint | None = None, stop_after: int = 0,
                                 log_cap: int = 64, stream=None):
    """Returns (rc, picks np.uint32[n_picked], Result, {i: Iteration} of the
    iterations this call ran, Checkpoint or None).  rc is CENTRA_OK,
    CENTRA_NOT_CERTIFIED or CENTRA_STOPPED."""
    picks = np.zeros(max(1, p.k), dtype=np.uint32)
    res = Result()
    log = (Iteration * max(1, log_cap))()
    ck = Checkpoint()
    rc = _check(lib().centra_progressive_resumable(ctx, g, ctypes.byref(p),
                                                   ctypes.byref(resume) if resume is not None else None,
                                                   ctypes.byref(ck), stop_after, picks.ctypes.data,
                                                   ctypes.byref(res), log, log_cap, _stream(stream)), ctx)
    first = resume.i + 1 if resume is not None else 1
    its = {i: log[i - 1] for i in range(first, min(res.iterations, log_cap) + 1)}
    return rc, picks[: res.n_picked].copy(), res, its, (ck if ck.version else None)


# ---------------------------------------------------------------------------
class DeviceGraph:
    """A CSR graph uploaded to device tensors and prepared by the library."""

    def __init__(self, ctx, graph, device="cuda", count_bits_override: int = 0):
        import torch
        self.n = graph.n
        self.directed = graph.directed

        def up(a):
            return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint32).view(np.int32)).to(device)

        self.row_ptr = up(graph.row_ptr)
        self.col_idx = up(graph.col_idx)
        self.rrow_ptr = up(graph.rrow_ptr) if graph.directed else None
        self.rcol_idx = up(graph.rcol_idx) if graph.directed else None
        self.handle = centra_graph_prepare(ctx, self.row_ptr, self.col_idx, self.rrow_ptr, self.rcol_idx,
                                           count_bits_override)

    def info(self):
        return centra_graph_info(self.handle)

    def hash(self) -> int:
        return centra_graph_hash(self.handle)

    def release(self):
        if self.handle:
            centra_graph_release(self.handle)
            self.handle = None


def centra_triangle_count(ctx, g, stream=None) -> int:
    T = ctypes.c_uint64()
    _check(lib().centra_triangle_count(ctx, g, ctypes.byref(T), _stream(stream)), ctx)
    return T.value


def centra_sample_triangles(ctx, g, seed: int, instance: int, first: int, count: int, he_off, he_nodes, stream=None):
    import torch
    _dtype_check(he_off, torch.int64, "he_off")
    _dtype_check(he_nodes, torch.int32, "he_nodes")
    _check(lib().centra_sample_triangles(ctx, g, seed, instance, first, count, _ptr(he_off), _ptr(he_nodes),
                                         _stream(stream)), ctx)


def sample_triangles(ctx, dg, seed: int, instance: int, first: int, count: int, device="cuda"):
    """Samples triangles [first, first+count) into fresh device tensors:
    (he_off int64[count+1], he_nodes int32[3 count])."""
    import torch
    he_off = torch.empty(count + 1, dtype=torch.int64, device=device)
    he_nodes = torch.empty(max(1, 3 * count), dtype=torch.int32, device=device)
    centra_sample_triangles(ctx, dg.handle, seed, instance, first, count, he_off, he_nodes)
    return he_off, he_nodes[: 3 * count]


def centra_sample_kpaths(ctx, g, kappa: int, seed: int, instance: int, first: int, count: int, he_off, he_nodes,
                         stream=None):
    import torch
    _dtype_check(he_off, torch.int64, "he_off")
    _dtype_check(he_nodes, torch.int32, "he_nodes")
    if he_nodes.numel() < count * kappa:
        raise ValueError("he_nodes must hold count * kappa entries")
    _check(lib().centra_sample_kpaths(ctx, g, kappa, seed, instance, first, count, _ptr(he_off), _ptr(he_nodes),
                                      _stream(stream)), ctx)


def sample_kpaths(ctx, dg, kappa: int, seed: int, instance: int, first: int, count: int, device="cuda"):
    """Samples kappa-paths [first, first+count) into fresh device tensors:
    (he_off int64[count+1], he_nodes int32[he_off[count]])."""
    import torch
    he_off = torch.empty(count + 1, dtype=torch.int64, device=device)
    he_nodes = torch.empty(max(1, count * max(1, kappa)), dtype=torch.int32, device=device)
    centra_sample_kpaths(ctx, dg.handle, kappa, seed, instance, first, count, he_off, he_nodes)
    return he_off, he_nodes[: int(he_off[count].item())]


def sample_paths(ctx, dg: DeviceGraph, seed: int, instance: int, first: int, count: int, with_st: bool = False,
                 device="cuda", bidir: bool = False):
    """Samples [first, first+count) into fresh device tensors (the balanced
    bidirectional sampler if bidir).
    Returns (he_off int64[count+1], he_nodes int32[I]) (+ (st, dist) if with_st)."""
    import torch
    call = centra_sample_paths_bidir if bidir else centra_sample_paths
    he_off = torch.empty(count + 1, dtype=torch.int64, device=device)
    cap = max(16, count * 8)
    st = torch.empty(2 * max(1, count), dtype=torch.int32, device=device) if with_st else None
    dist = torch.empty(max(1, count), dtype=torch.int32, device=device) if with_st else None
    he_nodes = torch.empty(cap, dtype=torch.int32, device=device)
    rc, need = call(ctx, dg.handle, seed, instance, first, count, he_off, he_nodes, cap, st, dist)
    if rc == CENTRA_ENOSPC:
        he_nodes = torch.empty(max(1, need), dtype=torch.int32, device=device)
        rc, need = call(ctx, dg.handle, seed, instance, first, count, he_off, he_nodes, need, st, dist)
    out = (he_off, he_nodes[:need])
    if with_st:
        out = out + (st, dist)
    return out


# ---------------------------------------------------------------------------
class Engine:
    """The batching and serving engine (centra_engine_*): pools of resident
    samples and queries run together, tick by tick."""

    def __init__(self, ctx, hbm_budget_bytes: int = 0, flags: int = 0):
        self.ctx = ctx
        out = _vp()
        _check(lib().centra_engine_create(ctx, hbm_budget_bytes, flags, ctypes.byref(out)), ctx)
        self.handle = out
        self.ks = []

    def add_pool(self, graph_handle, seed: int, instance: int, t: int, m_init: int, m_max: int,
                 growth_num: int = 2, growth_den: int = 1) -> int:
        p = PoolParams(seed, instance, t, m_init, m_max, growth_num, growth_den)
        pid = ctypes.c_uint32()
        _check(lib().centra_engine_add_pool(self.handle, graph_handle, ctypes.byref(p), ctypes.byref(pid)), self.ctx)
        return pid.value

    def prefill(self, pool: int, m: int, stream=None) -> None:
        _check(lib().centra_engine_prefill(self.handle, pool, m, _stream(stream)), self.ctx)

    def submit(self, pool: int, k: int, t: int, eps: float, delta: float, arrival_s: float = 0.0) -> int:
        q = ctypes.c_uint32()
        _check(lib().centra_engine_submit(self.handle, pool, k, t, eps, delta, arrival_s, ctypes.byref(q)), self.ctx)
        while len(self.ks) <= q.value:
            self.ks.append(0)
        self.ks[q.value] = k
        return q.value

    def run(self, realtime: bool = False, stream=None) -> None:
        _check(lib().centra_engine_run(self.handle, 1 if realtime else 0, _stream(stream)), self.ctx)

    def result(self, qid: int):
        """Returns (rc, picks np.uint32[n_picked], Result, QueryInfo)."""
        picks = np.zeros(max(1, self.ks[qid]), dtype=np.uint32)
        res, info = Result(), QueryInfo()
        rc = lib().centra_engine_result(self.handle, qid, picks.ctypes.data, ctypes.byref(res), ctypes.byref(info))
        if rc < 0:
            raise CentraError(rc, centra_last_error(self.ctx))
        return rc, picks[: res.n_picked].copy(), res, info

    def stats(self) -> EngineStats:
        out = EngineStats()
        _check(lib().centra_engine_stats_get(self.handle, ctypes.byref(out)), self.ctx)
        return out

    def log(self) -> str:
        s = lib().centra_engine_log(self.handle)
        return s.decode() if s else ""

    def destroy(self) -> None:
        if self.handle:
            lib().centra_engine_destroy(self.handle)
            self.handle = None
