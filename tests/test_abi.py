"""The C-ABI library loads on the host and exports every symbol include/rd.h
declares; host-side validation paths (no GPU compute)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "rd.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(rd_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_1506_04651_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("librd.so not built (run __graft_entry__.build())")
    return _lib.load()


def test_every_declared_symbol_is_exported(lib):
    from paper_1506_04651_amd import _lib
    names = declared_symbols()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
        assert n in _lib.SIGNATURES, f"{n} has no Python binding"


def test_default_options(lib):
    from paper_1506_04651_amd import _lib
    o = _lib.default_options()
    assert (o.precision, o.schedule, o.tol_transform, o.max_steps, o.newton_max,
            o.fixed_steps, o.h0, o.h_min, o.variant, o.use_graph) == (0, 0, 1, 100000, 7, 0,
                                                                       0.0, 0.0, 0, 0)
    assert (o.order, o.jacobian, o.h_cells, o.session_streams) == (1, 0, None, 0)


def test_request_bytes(lib):
    assert lib.rd_request_bytes(0, 3, 0) == 0
    assert lib.rd_request_bytes(1000, 3, 0) == 24064  # 24000 rounded up to 256
    assert lib.rd_request_bytes(1000, 3, 1) == 24064 + 36096
    # from 8192 cells on, the claim-order scratch of the persistent launch
    # (an int32 position and a byte per cell, plus bucket counters) is counted
    n = 100000
    b = lib.rd_request_bytes(n, 3, 0)
    assert b >= 2400000 + 4 * n + n
    assert b - (2400000 + 4 * n + n) < 64 * 1024


def test_variants_listed(lib):
    import paper_1506_04651_amd as rd
    for prec in (rd.FP64, rd.MIXED):
        for sched in (rd.PERSISTENT, rd.ONE_LAUNCH):
            n = rd.variant_count(rd.OREGONATOR, 3, prec, sched)
            assert n >= 1
            for v in range(1, n + 1):
                assert rd.variant_name(rd.OREGONATOR, 3, prec, sched, v)
    with pytest.raises(rd.RdError):
        rd.set_default_variant(rd.OREGONATOR, 3, rd.FP64, rd.PERSISTENT, 999)


def test_group_variant_sets(lib):
    """Kinetics and linear models with 5..8 species share the 8-column kernel
    set, with 9..16 the 16-column set; ids and names agree across each set."""
    import paper_1506_04651_amd as rd
    for kind in (rd.KINETICS, rd.LINEAR):
        for prec in (rd.FP64, rd.MIXED):
            n8 = [rd.variant_count(kind, m, prec, rd.PERSISTENT) for m in (5, 6, 7, 8)]
            n16 = [rd.variant_count(kind, m, prec, rd.PERSISTENT) for m in (9, 12, 16)]
            assert len(set(n8)) == 1 and n8[0] >= 1 and len(set(n16)) == 1 and n16[0] >= 1
            assert all(".g16c8." in rd.variant_name(kind, 6, prec, rd.PERSISTENT, v)
                       for v in range(1, n8[0] + 1))
            assert all(".g16." in rd.variant_name(kind, 10, prec, rd.PERSISTENT, v)
                       for v in range(1, n16[0] + 1))
            assert rd.variant_name(kind, 7, prec, rd.ONE_LAUNCH, 1).startswith(
                ("kinetics.g16c8", "linear.g16c8"))


def test_validation_before_device_use(lib):
    """Invalid calls return RD_EINVAL from host-side checks; empty batches
    return 0 without touching a device."""
    from paper_1506_04651_amd import _lib
    p = (ctypes.c_double * 4)(1e-2, 1e-5, 1.6, 2e-3)
    good = _lib.RdModel(1, 3, ctypes.cast(p, ctypes.POINTER(ctypes.c_double)), 4)
    bad_kind = _lib.RdModel(9, 3, ctypes.cast(p, ctypes.POINTER(ctypes.c_double)), 4)
    short = _lib.RdModel(1, 3, ctypes.cast(p, ctypes.POINTER(ctypes.c_double)), 2)
    call = lib.rd_reaction_step_ex
    assert call(None, 0, 3, 0.1, 1e-5, 1e-5, ctypes.byref(good), None, None, None, 0) == 0
    dummy = ctypes.c_void_p(1)
    for args in [(dummy, 10, 3, 0.0, 1e-5, 1e-5, good), (dummy, 10, 3, float("nan"), 1e-5, 1e-5, good),
                 (dummy, 10, 3, 0.1, 0.0, 1e-5, good), (dummy, 10, 3, 0.1, 1e-5, -1.0, good),
                 (dummy, -1, 3, 0.1, 1e-5, 1e-5, good), (dummy, 10, 2, 0.1, 1e-5, 1e-5, good),
                 (dummy, 10, 3, 0.1, 1e-5, 1e-5, bad_kind), (dummy, 10, 3, 0.1, 1e-5, 1e-5, short),
                 (None, 10, 3, 0.1, 1e-5, 1e-5, good)]:
        st, n, m, dt, rt, at, md = args
        assert call(st, n, m, dt, rt, at, ctypes.byref(md), None, None, None, 0) == -1, args
        assert lib.rd_last_error()
    o = _lib.default_options()
    o.precision = 1
    o.fixed_steps = 3
    assert call(dummy, 10, 3, 0.1, 1e-5, 1e-5, ctypes.byref(good), ctypes.byref(o), None, None, 0) == -1
    o = _lib.default_options()
    o.newton_max = 0
    assert call(dummy, 10, 3, 0.1, 1e-5, 1e-5, ctypes.byref(good), ctypes.byref(o), None, None, 0) == -1


def _bc_model(prog, m):
    from paper_1506_04651_amd import _lib
    arr = (ctypes.c_double * len(prog))(*prog)
    return _lib.RdModel(6, m, ctypes.cast(arr, ctypes.POINTER(ctypes.c_double)), len(prog)), arr


def test_bytecode_programs_validated_on_the_host(lib):
    """Register programs are checked before any device work: valid programs
    pass (n = 0 does nothing), malformed ones return RD_EINVAL."""
    from paper_1506_04651_amd import _lib
    from paper_1506_04651_amd import workloads as W
    call = lib.rd_reaction_step_ex
    for prog, m in [(W.oregonator_program(), 3), (W.robertson_program(), 3),
                    (W.nagumo_program(2.0), 1)]:
        md, keep = _bc_model(list(prog), m)
        assert call(None, 0, m, 0.1, 1e-5, 1e-8, ctypes.byref(md), None, None, None, 0) == 0
    bad = [([1, 0, 10, 0, 0, 0], 1), ([1, 0, 0, 0, 0, 0], 1), ([1, 0, 9, 1, 0, 0], 1),
           ([2, 0, 9, 0, 0, 0, 9, 0, 0, 0], 1), ([1, 0, 1, 5, 0, 0], 1),
           ([2, 0, 1, 1, 2, 0, 9, 0, 1, 0], 1), ([2, 1, 2.0, 1, 1, 0, 0, 9, 0, 1, 0], 1),
           ([1, 0, 9, 0, 70, 0], 1), ([1, 0, 9, 0, 0.5, 0], 1), ([1, 0, 9, 0, 0], 1),
           ([1, 0, 9, 0, 0, 0], 17)]
    for prog, m in bad:
        md, keep = _bc_model(prog, m)
        assert call(None, 0, m, 0.1, 1e-5, 1e-8, ctypes.byref(md), None, None, None, 0) == -1, prog
    # a jacobian mode other than analytic / finite differences is invalid;
    # finite differences are provided for the kinetics model on the group
    # kernels, not for the linear test model
    p = (ctypes.c_double * 4)(1e-2, 1e-5, 1.6, 2e-3)
    good = _lib.RdModel(1, 3, ctypes.cast(p, ctypes.POINTER(ctypes.c_double)), 4)
    o = _lib.default_options()
    o.jacobian = 2
    assert call(None, 0, 3, 0.1, 1e-5, 1e-8, ctypes.byref(good), ctypes.byref(o), None, None, 0) == -1
    o.jacobian = 1
    assert call(None, 0, 3, 0.1, 1e-5, 1e-8, ctypes.byref(good), ctypes.byref(o), None, None, 0) == 0
    K = (ctypes.c_double * 512)(*([0.0] * 512))
    kin = _lib.RdModel(2, 16, ctypes.cast(K, ctypes.POINTER(ctypes.c_double)), 512)
    assert call(None, 0, 16, 0.1, 1e-5, 1e-8, ctypes.byref(kin), ctypes.byref(o), None, None, 0) == 0
    lin = _lib.RdModel(4, 16, ctypes.cast(K, ctypes.POINTER(ctypes.c_double)), 256)
    assert call(None, 0, 16, 0.1, 1e-5, 1e-8, ctypes.byref(lin), ctypes.byref(o), None, None, 0) == -1
    # a 16-species register program is accepted
    from tests.bytecode_models import kinetics_program, sparse_kinetics
    import numpy as np
    Kc, Gc = sparse_kinetics(16, 1)
    md, keep = _bc_model(list(kinetics_program(Kc, Gc)), 16)
    assert call(None, 0, 16, 0.1, 1e-5, 1e-8, ctypes.byref(md), None, None, None, 0) == 0


def test_diffusion_and_strang_validation(lib):
    """Malformed grids and steps are rejected before any device work."""
    from paper_1506_04651_amd import _lib
    eps = (ctypes.c_double * 3)(2.5e-3, 2.5e-3, 1.5e-3)
    epsp = ctypes.cast(eps, ctypes.POINTER(ctypes.c_double))
    dummy = ctypes.c_void_p(1)
    bad_grids = [_lib.RdGrid(1, 8, 8, 1, 0.1, epsp), _lib.RdGrid(2, 8, 8, 2, 0.1, epsp),
                 _lib.RdGrid(3, 0, 8, 8, 0.1, epsp), _lib.RdGrid(2, 8, 8, 1, 0.0, epsp),
                 _lib.RdGrid(2, 8, 8, 1, float("nan"), epsp), _lib.RdGrid(2, 8, 8, 1, 0.1, None)]
    for g in bad_grids:
        assert lib.rd_diffusion_step(dummy, 3, ctypes.byref(g), 1e-3, 0, None) == -1
    g = _lib.RdGrid(2, 8, 8, 1, 0.1, epsp)
    assert lib.rd_diffusion_step(dummy, 3, ctypes.byref(g), 0.0, 0, None) == -1
    assert lib.rd_diffusion_step(dummy, 3, ctypes.byref(g), 1e-3, -1, None) == -1
    assert lib.rd_diffusion_step(None, 3, ctypes.byref(g), 1e-3, 0, None) == -1
    neg = (ctypes.c_double * 3)(2.5e-3, -1.0, 1.5e-3)
    g2 = _lib.RdGrid(2, 8, 8, 1, 0.1, ctypes.cast(neg, ctypes.POINTER(ctypes.c_double)))
    assert lib.rd_diffusion_step(dummy, 3, ctypes.byref(g2), 1e-3, 0, None) == -1
    p = (ctypes.c_double * 4)(1e-2, 1e-5, 1.6, 2e-3)
    md = _lib.RdModel(1, 3, ctypes.cast(p, ctypes.POINTER(ctypes.c_double)), 4)
    assert lib.rd_strang_step(dummy, 3, ctypes.byref(bad_grids[0]), 1e-3, 1e-5, 1e-8,
                              ctypes.byref(md), None, None, None) == -1
    o = _lib.default_options()
    o.h_cells = 1
    assert lib.rd_strang_step(dummy, 3, ctypes.byref(g), 1e-3, 1e-5, 1e-8,
                              ctypes.byref(md), ctypes.byref(o), None, None) == -1


def test_mra_validation(lib):
    """Malformed multiresolution calls are rejected before any device work."""
    from paper_1506_04651_amd import _lib
    dummy = ctypes.c_void_p(1)
    sc = (ctypes.c_double * 2)(1.0, 0.0)
    bad = [_lib.RdMraParams(1, 5, 1e-3, None, 0), _lib.RdMraParams(2, 0, 1e-3, None, 0),
           _lib.RdMraParams(3, 11, 1e-3, None, 0), _lib.RdMraParams(2, 5, -1.0, None, 0),
           _lib.RdMraParams(2, 5, float("nan"), None, 0),
           _lib.RdMraParams(2, 5, 1e-3, ctypes.cast(sc, ctypes.POINTER(ctypes.c_double)), 1)]
    for p in bad:
        assert lib.rd_mra_leaves(dummy, 2, ctypes.byref(p), None, None, 0, None, None) == -1
        assert lib.rd_mra_reconstruct(dummy, dummy, 10, 2, ctypes.byref(p), dummy, None) == -1
        assert lib.rd_mra_adapt(dummy, dummy, 10, 2, ctypes.byref(p), None, None, 0, None, None) == -1
    good = _lib.RdMraParams(2, 5, 1e-3, None, 1)
    assert lib.rd_mra_leaves(None, 2, ctypes.byref(good), None, None, 0, None, None) == -1
    assert lib.rd_mra_leaves(dummy, 2, ctypes.byref(good), None, None, -1, None, None) == -1
    assert lib.rd_mra_leaves(dummy, 0, ctypes.byref(good), None, None, 0, None, None) == -1
    assert lib.rd_mra_adapt(None, dummy, 10, 2, ctypes.byref(good), None, None, 0, None, None) == -1
    assert lib.rd_mra_adapt(dummy, None, 10, 2, ctypes.byref(good), None, None, 0, None, None) == -1
    assert lib.rd_mra_adapt(dummy, dummy, 0, 2, ctypes.byref(good), None, None, 0, None, None) == -1
    assert lib.rd_mra_adapt(dummy, dummy, 10, 2, ctypes.byref(good), None, None, -1, None, None) == -1
    assert lib.rd_mra_reconstruct(dummy, dummy, 10, 2, ctypes.byref(good), None, None) == -1


def test_product_path_does_not_reference_the_oracle():
    pkg = os.path.join(ROOT, "paper_1506_04651_amd")
    for dp, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".h")):
                txt = open(os.path.join(dp, f)).read()
                assert "import oracle" not in txt and "from oracle" not in txt, f
                assert "rdo_" not in txt and "liboracle" not in txt, f


def test_variant_lanes_per_cell(lib):
    """The variant table's lanes per cell: one lane for the one-lane kernels,
    16 for the 16-lane-group kernels, both offered for kinetics with m <= 4."""
    import paper_1506_04651_amd as rd
    assert rd.variant_lanes(rd.OREGONATOR, 3, rd.FP64, rd.PERSISTENT, 1) == 1
    assert rd.variant_lanes(rd.KINETICS, 16, rd.FP64, rd.PERSISTENT, 1) == 16
    for m in (1, 2, 3, 4):
        for prec in (rd.FP64, rd.MIXED):
            n = rd.variant_count(rd.KINETICS, m, prec, rd.PERSISTENT)
            lanes = {rd.variant_lanes(rd.KINETICS, m, prec, rd.PERSISTENT, v) for v in range(1, n + 1)}
            assert lanes == {1, 16}, (m, prec, lanes)
    with pytest.raises(rd.RdError):
        rd.variant_lanes(rd.OREGONATOR, 3, rd.FP64, rd.PERSISTENT, 999)
