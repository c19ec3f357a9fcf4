"""Python surface of librd: the same entry points as include/rd.h, taking torch
tensors for device memory and torch streams for ordering.  Marshalling only."""
from __future__ import annotations

import ctypes

import numpy as np

from . import _lib
from ._lib import FP64, PERSISTENT, RdModel, RdOptions, RdRequestInfo


class RdError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"librd error {code} ({_lib.ERRORS.get(code, '?')}): {msg}")
        self.code = code


def _check(ret: int) -> int:
    if ret < 0:
        raise RdError(int(ret), _lib.last_error())
    return int(ret)


def _model(kind: int, m: int, params):
    p = np.ascontiguousarray(np.asarray(params, dtype=np.float64).ravel())
    mdl = RdModel(int(kind), int(m), p.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), p.size)
    return mdl, p


def make_options(precision=FP64, schedule=PERSISTENT, tol_transform=1, max_steps=100000,
                 newton_max=7, fixed_steps=0, h0=0.0, h_min=0.0, variant=0,
                 use_graph=False, order=1, jacobian=0, h_cells_ptr=None,
                 session_streams=0) -> RdOptions:
    o = RdOptions()
    o.session_streams = int(session_streams)
    o.order = int(order)
    o.jacobian = int(jacobian)
    o.h_cells = h_cells_ptr
    o.precision, o.schedule, o.tol_transform = int(precision), int(schedule), int(tol_transform)
    o.max_steps, o.newton_max, o.fixed_steps = int(max_steps), int(newton_max), int(fixed_steps)
    o.h0, o.h_min, o.variant, o.use_graph = float(h0), float(h_min), int(variant), int(use_graph)
    return o


def _check_states(states):
    import torch
    if not isinstance(states, torch.Tensor) or states.dtype != torch.float64 or \
            not states.is_cuda or states.dim() != 2 or not states.is_contiguous():
        raise ValueError("states must be a contiguous float64 CUDA tensor of shape [m, n]")


def _check_stats(stats, n):
    import torch
    if stats is None:
        return None
    if not isinstance(stats, torch.Tensor) or stats.dtype != torch.int32 or not stats.is_cuda \
            or tuple(stats.shape) != (_lib.NSTATS, n) or not stats.is_contiguous():
        raise ValueError(f"stats must be a contiguous int32 CUDA tensor of shape [9, {n}]")
    return stats.data_ptr()


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def reaction_step(states, dt, rtol, atol, kind, params, *, stats=None, stream=None,
                  async_=False, h_cells=None, **opts) -> int:
    """Advance every cell (column) of ``states`` [m, n] float64 (device) over
    [0, dt] in place.  Returns the number of cells with a nonzero status
    (0 when async_).  Keyword options as in rd_options (precision, schedule,
    tol_transform, max_steps, newton_max, fixed_steps, h0, h_min, variant,
    use_graph, order, jacobian).  ``h_cells``: optional float64 CUDA tensor [n],
    the per-cell warm-start step size, read and updated in place."""
    import torch
    lib = _lib.load()
    _check_states(states)
    m, n = int(states.shape[0]), int(states.shape[1])
    sp = _check_stats(stats, n)
    hp = None
    if h_cells is not None:
        if not isinstance(h_cells, torch.Tensor) or h_cells.dtype != torch.float64 or \
                not h_cells.is_cuda or tuple(h_cells.shape) != (n,) or not h_cells.is_contiguous():
            raise ValueError(f"h_cells must be a contiguous float64 CUDA tensor of shape [{n}]")
        hp = h_cells.data_ptr()
    mdl, keep = _model(kind, m, params)
    o = make_options(h_cells_ptr=hp, **opts)
    ret = lib.rd_reaction_step_ex(ctypes.c_void_p(states.data_ptr()), n, m, float(dt),
                                  float(rtol), float(atol), ctypes.byref(mdl), ctypes.byref(o),
                                  ctypes.c_void_p(sp) if sp else None, _stream_handle(stream),
                                  1 if async_ else 0)
    del keep
    return _check(ret)


def _grid(shape, h, diff):
    """rd_grid for a uniform grid of `shape` = (nx, ny) or (nx, ny, nz)."""
    d = np.ascontiguousarray(diff, dtype=np.float64)
    dims = tuple(int(v) for v in shape)
    if len(dims) not in (2, 3):
        raise ValueError("shape must be (nx, ny) or (nx, ny, nz)")
    nz = dims[2] if len(dims) == 3 else 1
    g = _lib.RdGrid(len(dims), dims[0], dims[1], nz, float(h),
                    d.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return g, d


def diffusion_step(states, shape, h, diff, dt, *, stages=0, stream=None) -> int:
    """D_dt on the uniform grid (cell c = x + nx (y + ny z)) in place: RKC
    stabilised explicit steps for dU/dt = eps_i Lap_h U with zero-flux
    boundaries.  Returns the stage count used."""
    lib = _lib.load()
    _check_states(states)
    m, n = int(states.shape[0]), int(states.shape[1])
    if int(np.prod(shape)) != n or len(diff) != m:
        raise ValueError("grid shape / diff do not match states")
    g, keep = _grid(shape, h, diff)
    r = lib.rd_diffusion_step(ctypes.c_void_p(states.data_ptr()), m, ctypes.byref(g), float(dt),
                              int(stages), _stream_handle(stream))
    del keep
    return _check(r)


def strang_step(states, shape, h, diff, dt, rtol, atol, kind, params, *, stats=None,
                stream=None, **opts) -> int:
    """U <- R_{dt/2} D_dt R_{dt/2} U in place (paper §2.1).  stats: optional int32
    CUDA tensor [2, 9, n] (counters of the two reaction halves).  Returns the
    summed failed-cell counts of the two halves."""
    import torch
    lib = _lib.load()
    _check_states(states)
    m, n = int(states.shape[0]), int(states.shape[1])
    if int(np.prod(shape)) != n or len(diff) != m:
        raise ValueError("grid shape / diff do not match states")
    sp = None
    if stats is not None:
        if not isinstance(stats, torch.Tensor) or stats.dtype != torch.int32 or not stats.is_cuda \
                or tuple(stats.shape) != (2, _lib.NSTATS, n) or not stats.is_contiguous():
            raise ValueError(f"stats must be a contiguous int32 CUDA tensor of shape [2, 9, {n}]")
        sp = stats.data_ptr()
    g, keep = _grid(shape, h, diff)
    mdl, keep2 = _model(kind, m, params)
    o = make_options(**opts)
    r = lib.rd_strang_step(ctypes.c_void_p(states.data_ptr()), m, ctypes.byref(g), float(dt),
                           float(rtol), float(atol), ctypes.byref(mdl), ctypes.byref(o),
                           ctypes.c_void_p(sp) if sp else None, _stream_handle(stream))
    del keep, keep2
    return _check(r)


def _mra_params(dim, levels, eps, scale, m, refine=False):
    sc = None if scale is None else np.ascontiguousarray(scale, dtype=np.float64)
    if sc is not None and sc.size != m:
        raise ValueError("scale needs one value per species")
    p = _lib.RdMraParams(int(dim), int(levels), float(eps),
                         None if sc is None else sc.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                         1 if refine else 0)
    return p, sc


def mra_leaves(fine, dim, levels, eps, *, scale=None, refine=False, stream=None):
    """Leaf set of the graded multiresolution tree of `fine` ([m, 2^(dim levels)]
    float64 CUDA tensor, x fastest).  Returns (keys int64 CUDA tensor holding
    the uint64 node keys in Morton order, values [m, n_leaves] CUDA tensor,
    per-level leaf counts as a list).  refine: nodes with significant details
    get children too."""
    import torch
    lib = _lib.load()
    _check_states(fine)
    m = int(fine.shape[0])
    if int(fine.shape[1]) != 1 << (dim * levels):
        raise ValueError("fine must hold 2^(dim*levels) cells per species")
    p, keep = _mra_params(dim, levels, eps, scale, m, refine)
    sh = _stream_handle(stream)
    n = _check(lib.rd_mra_leaves(ctypes.c_void_p(fine.data_ptr()), m, ctypes.byref(p), None, None, 0,
                                 None, sh))
    keys = torch.empty(n, dtype=torch.int64, device=fine.device)
    vals = torch.empty((m, n), dtype=torch.float64, device=fine.device)
    counts = (ctypes.c_int64 * (levels + 1))()
    n2 = _check(lib.rd_mra_leaves(ctypes.c_void_p(fine.data_ptr()), m, ctypes.byref(p),
                                  ctypes.c_void_p(keys.data_ptr()), ctypes.c_void_p(vals.data_ptr()),
                                  n, counts, sh))
    del keep
    if n2 != n:
        raise RuntimeError("leaf count changed between calls")
    return keys, vals, list(counts)


def mra_reconstruct(keys, values, dim, levels, *, scale=None, stream=None):
    """Finest-level field ([m, 2^(dim levels)], x fastest) from a leaf set."""
    import torch
    lib = _lib.load()
    _check_states(values)
    m, n = int(values.shape[0]), int(values.shape[1])
    if keys.dtype != torch.int64 or not keys.is_cuda or tuple(keys.shape) != (n,):
        raise ValueError("keys must be an int64 CUDA tensor of n_leaves entries")
    p, keep = _mra_params(dim, levels, 0.0, scale, m)
    out = torch.empty((m, 1 << (dim * levels)), dtype=torch.float64, device=values.device)
    _check(lib.rd_mra_reconstruct(ctypes.c_void_p(keys.data_ptr()), ctypes.c_void_p(values.data_ptr()),
                                  n, m, ctypes.byref(p), ctypes.c_void_p(out.data_ptr()),
                                  _stream_handle(stream)))
    del keep
    return out


def mra_adapt(keys, values, dim, levels, eps, *, scale=None, refine=True, stream=None):
    """Leaf set adapted to the values of a leaf set (refinement and
    coarsening): returns (keys, values, per-level counts) as mra_leaves."""
    import torch
    lib = _lib.load()
    _check_states(values)
    m, n = int(values.shape[0]), int(values.shape[1])
    if keys.dtype != torch.int64 or not keys.is_cuda or tuple(keys.shape) != (n,):
        raise ValueError("keys must be an int64 CUDA tensor of n_leaves entries")
    p, keep = _mra_params(dim, levels, eps, scale, m, refine)
    sh = _stream_handle(stream)
    kp, vp = ctypes.c_void_p(keys.data_ptr()), ctypes.c_void_p(values.data_ptr())
    nn = _check(lib.rd_mra_adapt(kp, vp, n, m, ctypes.byref(p), None, None, 0, None, sh))
    okeys = torch.empty(nn, dtype=torch.int64, device=values.device)
    ovals = torch.empty((m, nn), dtype=torch.float64, device=values.device)
    counts = (ctypes.c_int64 * (levels + 1))()
    n2 = _check(lib.rd_mra_adapt(kp, vp, n, m, ctypes.byref(p), ctypes.c_void_p(okeys.data_ptr()),
                                 ctypes.c_void_p(ovals.data_ptr()), nn, counts, sh))
    del keep
    if n2 != nn:
        raise RuntimeError("leaf count changed between calls")
    return okeys, ovals, list(counts)


def last_kernel_ms() -> float:
    """Duration of this thread's last reaction-step kernel (HIP events on its
    launch stream), in ms; negative if unavailable."""
    return float(_lib.load().rd_last_kernel_ms())


def variant_count(kind, m, precision=FP64, schedule=PERSISTENT) -> int:
    return int(_lib.load().rd_variant_count(kind, m, precision, schedule))


def variant_name(kind, m, precision=FP64, schedule=PERSISTENT, variant=0) -> str | None:
    r = _lib.load().rd_variant_name(kind, m, precision, schedule, variant)
    return r.decode() if r else None


def variant_lanes(kind, m, precision=FP64, schedule=PERSISTENT, variant=0) -> int:
    """Lanes per cell of a kernel variant (1 or 16)."""
    return _check(_lib.load().rd_variant_lanes(kind, m, precision, schedule, variant))


def set_default_variant(kind, m, precision, schedule, variant) -> None:
    _check(_lib.load().rd_set_default_variant(kind, m, precision, schedule, variant))


def persistent_grid(kind, m, precision=FP64, variant=0, n_cells=1 << 30) -> int:
    return _check(_lib.load().rd_persistent_grid(kind, m, precision, variant, n_cells))


def request_bytes(n_cells, m, with_stats=False) -> int:
    return int(_lib.load().rd_request_bytes(n_cells, m, 1 if with_stats else 0))


class Session:
    """Serving session (rd_session_*): requests of any size and model are
    admitted into an HBM arena of ``budget_bytes`` and run concurrently."""

    def __init__(self, budget_bytes: int, device: int = 0, n_streams: int = 0, **opts):
        lib = _lib.load()
        self._h = ctypes.c_void_p()
        o = make_options(session_streams=n_streams, **opts)
        _check(lib.rd_session_create(ctypes.byref(self._h), int(device), int(budget_bytes),
                                     ctypes.byref(o)))
        self._keep = {}

    def submit(self, states, dt, rtol, atol, kind, params, stats=None, stream=None) -> int:
        """Queue a request; the session reads ``states`` after the work already
        enqueued on ``stream`` (default: torch's current stream)."""
        lib = _lib.load()
        _check_states(states)
        m, n = int(states.shape[0]), int(states.shape[1])
        sp = _check_stats(stats, n)
        mdl, keep = _model(kind, m, params)
        rid = ctypes.c_uint64()
        _check(lib.rd_submit_ex(self._h, ctypes.c_void_p(states.data_ptr()), n, m, float(dt),
                                float(rtol), float(atol), ctypes.byref(mdl),
                                ctypes.c_void_p(sp) if sp else None, _stream_handle(stream),
                                ctypes.byref(rid)))
        del keep
        self._keep[rid.value] = (states, stats)
        return rid.value

    def poll(self, rid: int):
        info = RdRequestInfo()
        r = _check(_lib.load().rd_poll(self._h, ctypes.c_uint64(rid), ctypes.byref(info)))
        if r == 0:
            self._keep.pop(rid, None)
            return info
        return None

    def wait(self, rid: int) -> RdRequestInfo:
        info = RdRequestInfo()
        _check(_lib.load().rd_wait(self._h, ctypes.c_uint64(rid), ctypes.byref(info)))
        self._keep.pop(rid, None)
        return info

    def close(self):
        if self._h:
            _check(_lib.load().rd_session_destroy(self._h))
            self._h = ctypes.c_void_p()
            self._keep.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
