"""ctypes binding of the CPU FP64 Radau5 oracle.

TEST INFRASTRUCTURE ONLY: imported by the tests, by ``__graft_entry__.smoke``
and by the CPU-baseline leg of ``bench.py``.  The product package never imports
it, and it imports nothing from the product package.

The oracle integrates, for every cell independently, du/dt = f(u) over one
reaction substep with Radau5 (Descombes et al. §2.1; Hairer & Wanner, Solving
ODEs II, §IV.8), solving the untransformed 3m x 3m stage system.  Unknowns are
laid out one array per species (paper §3.2): ``states[i, c]``.
"""
import ctypes
import os

import numpy as np

from .build import LIB, build_oracle

OREGONATOR, KINETICS, NAGUMO, LINEAR, ROBERTSON, BYTECODE = 1, 2, 3, 4, 5, 6
NSTATS = 9
STAT_NAMES = ("status", "nstep", "naccept", "nreject", "nfev", "njac", "ndec",
              "nsol", "nnewt")


class _Model(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("m", ctypes.c_int32),
                ("params", ctypes.POINTER(ctypes.c_double)),
                ("n_params", ctypes.c_int64)]


class _Options(ctypes.Structure):
    _fields_ = [("tol_transform", ctypes.c_int32), ("max_steps", ctypes.c_int32),
                ("newton_max", ctypes.c_int32), ("fixed_steps", ctypes.c_int32),
                ("h0", ctypes.c_double), ("h_min", ctypes.c_double),
                ("jacobian", ctypes.c_int32), ("pad_", ctypes.c_int32),
                ("h_cells", ctypes.POINTER(ctypes.c_double))]


_lib = None


def load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB):
        build_oracle()
    _lib = bind(ctypes.CDLL(LIB))
    return _lib


def bind(lib):
    """Declare the argument and result types of the oracle's entry points on
    a loaded library (also used by the tests for separately built copies)."""
    lib.rdo_reaction_step.restype = ctypes.c_int64
    lib.rdo_reaction_step.argtypes = [
        ctypes.POINTER(ctypes.c_double), ctypes.c_int64, ctypes.c_int32,
        ctypes.c_double, ctypes.c_double, ctypes.c_double,
        ctypes.POINTER(_Model), ctypes.POINTER(_Options),
        ctypes.POINTER(ctypes.c_int32), ctypes.c_int32]
    lib.rdo_single_step.restype = ctypes.c_int32
    lib.rdo_single_step.argtypes = [
        ctypes.POINTER(ctypes.c_double), ctypes.c_int32, ctypes.c_double,
        ctypes.c_double, ctypes.c_double, ctypes.c_int32, ctypes.c_int32,
        ctypes.POINTER(_Model), ctypes.POINTER(ctypes.c_double),
        ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int32)]
    lib.rdo_model_eval.restype = ctypes.c_int32
    lib.rdo_model_eval.argtypes = [ctypes.POINTER(_Model), ctypes.POINTER(ctypes.c_double),
                                   ctypes.POINTER(ctypes.c_double),
                                   ctypes.POINTER(ctypes.c_double)]
    lib.rdo_start_values.restype = ctypes.c_int32
    lib.rdo_start_values.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.c_int32,
                                     ctypes.c_double, ctypes.c_double,
                                     ctypes.POINTER(ctypes.c_double)]
    lib.rdo_constants.restype = None
    lib.rdo_constants.argtypes = [ctypes.POINTER(ctypes.c_double)]
    return lib


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _model(kind, m, params):
    p = np.ascontiguousarray(params, dtype=np.float64).ravel()
    mdl = _Model(int(kind), int(m), _dptr(p), p.size)
    return mdl, p  # keep p alive


def _options(tol_transform=1, max_steps=100000, newton_max=7, fixed_steps=0,
             h0=0.0, h_min=0.0, jacobian=0, h_cells=None):
    hp = _dptr(h_cells) if h_cells is not None else None
    return _Options(int(tol_transform), int(max_steps), int(newton_max),
                    int(fixed_steps), float(h0), float(h_min), int(jacobian), 0, hp)


def reaction_step(states, dt, rtol, atol, kind, params, nthreads=0, h_cells=None, **opts):
    """Integrate every column of ``states`` ([m, n] float64) over [0, dt].

    Returns ``(y, stats, ret)``: the new states (a copy), the [9, n] int32
    counters, and the library's return value (number of failed cells, or a
    negative call-level error).  ``h_cells`` (float64 [n], optional) is the
    per-cell warm-start step size, updated in place.
    """
    lib = load()
    y = np.array(states, dtype=np.float64, order="C", copy=True)
    if y.ndim != 2:
        raise ValueError("states must be [m, n]")
    m, n = y.shape
    stats = np.zeros((NSTATS, n), dtype=np.int32)
    mdl, keep = _model(kind, m, params)
    if h_cells is not None:
        if not (isinstance(h_cells, np.ndarray) and h_cells.dtype == np.float64
                and h_cells.flags.c_contiguous and h_cells.shape == (n,)):
            raise ValueError("h_cells must be a contiguous float64 array of n values")
    o = _options(h_cells=h_cells, **opts)
    ret = lib.rdo_reaction_step(
        _dptr(y), n, m, float(dt), float(rtol), float(atol), ctypes.byref(mdl),
        ctypes.byref(o), stats.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
        int(nthreads))
    del keep
    return y, stats, int(ret)


def single_step(y0, h, rtol, atol, kind, params, tol_transform=1, newton_max=7):
    """One Radau IIA step (test hook). Returns (y1, (err1, err2), k_used, failed)."""
    lib = load()
    y0 = np.ascontiguousarray(y0, dtype=np.float64)
    m = y0.size
    y1 = np.zeros(m)
    err = np.zeros(2)
    info = np.zeros(2, dtype=np.int32)
    mdl, keep = _model(kind, m, params)
    rc = lib.rdo_single_step(_dptr(y0), m, float(h), float(rtol), float(atol),
                             int(tol_transform), int(newton_max),
                             ctypes.byref(mdl), _dptr(y1), _dptr(err),
                             info.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    del keep
    if rc != 0:
        raise ValueError(f"rdo_single_step returned {rc}")
    return y1, (float(err[0]), float(err[1])), int(info[0]), bool(info[1])


def start_values(zold, h, h_old):
    """Newton start values of the next step (test hook): ``zold`` [3, m] are
    the stage increments of the last accepted step of size ``h_old``; returns
    the [3, m] increments of the collocation cubic continued over a step h."""
    lib = load()
    zold = np.ascontiguousarray(zold, dtype=np.float64)
    if zold.ndim != 2 or zold.shape[0] != 3:
        raise ValueError("zold must be [3, m]")
    m = zold.shape[1]
    z = np.zeros((3, m))
    rc = lib.rdo_start_values(_dptr(zold), m, float(h), float(h_old), _dptr(z))
    if rc != 0:
        raise ValueError(f"rdo_start_values returned {rc}")
    return z


def model_eval(kind, params, y, m=None):
    """f(y) and the Jacobian J(y) ([m, m]) as the oracle's model code computes
    them (bytecode models: forward differences)."""
    lib = load()
    y = np.ascontiguousarray(y, dtype=np.float64)
    m = y.size if m is None else m
    f = np.zeros(m)
    J = np.zeros((m, m))
    mdl, keep = _model(kind, m, params)
    rc = lib.rdo_model_eval(ctypes.byref(mdl), _dptr(y), _dptr(f), _dptr(J))
    del keep
    if rc != 0:
        raise ValueError(f"rdo_model_eval returned {rc}")
    return f, J


def constants():
    """The method constants the oracle uses: dict c, A, gamma_hat, d."""
    lib = load()
    out = np.zeros(16)
    lib.rdo_constants(_dptr(out))
    return {"c": out[0:3].copy(), "A": out[3:12].reshape(3, 3).copy(),
            "gamma_hat": float(out[12]), "d": out[13:16].copy()}
