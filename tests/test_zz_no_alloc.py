"""rd_reaction_step_noalloc through the C ABI: calls in a row with different
sizes, precisions and models, each bitwise equal (states and per-cell
counters) to rd_reaction_step_ex on the same inputs; the device's free memory
does not change across the allocation-free calls; requests above the fixed
scratch are refused without touching the states."""
import ctypes

import numpy as np
import pytest

from paper_1506_04651_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def rd():
    import paper_1506_04651_amd as rd
    rd.load()
    assert torch.cuda.is_available()
    return rd


def noalloc(rd, u, w, stats=None, **opts):
    from paper_1506_04651_amd import _lib
    from paper_1506_04651_amd.api import _model, make_options
    lib = _lib.load()
    m, n = int(u.shape[0]), int(u.shape[1])
    mdl, keep = _model(w.kind, m, w.params)
    o = make_options(**opts)
    r = lib.rd_reaction_step_noalloc(ctypes.c_void_p(u.data_ptr()), n, m, float(w.dt),
                                     float(w.rtol), float(w.atol), ctypes.byref(mdl),
                                     ctypes.byref(o),
                                     ctypes.c_void_p(stats.data_ptr()) if stats is not None else None,
                                     ctypes.c_void_p(torch.cuda.current_stream().cuda_stream), 0)
    del keep
    return int(r)


CASES = [
    # (name, workload factory, options): the largest accepted batch first,
    # then smaller ones
    ("3d max size fp64", lambda: W.oregonator_3d(), dict(precision=0)),
    ("2d subset mixed", lambda: W.oregonator_2d().subset(np.arange(50000)), dict(precision=1)),
    ("kinetics m16 small", lambda: W.kinetics16(n=3000), dict(precision=0)),
    ("1d below the claim-order size, one launch", lambda: W.oregonator_1d(n=4000),
     dict(precision=0, schedule=1)),
]


def test_noalloc_equals_allocating_entry_point(rd):
    from paper_1506_04651_amd import _lib
    lib = _lib.load()
    assert lib.rd_noalloc_scratch_bytes() >= 5 * 4194304
    works = [(name, f(), o) for name, f, o in CASES]
    assert works[0][1].n == 4194304  # RD_NOALLOC_MAX_CELLS
    # every tensor exists before the calls, so that the free-memory check
    # sees only what the calls themselves might allocate
    bufs = [(torch.empty((w.m, w.n), dtype=torch.float64, device="cuda"),
             torch.zeros((9, w.n), dtype=torch.int32, device="cuda")) for _, w, _ in works]
    src = [torch.tensor(w.states, dtype=torch.float64, device="cuda") for _, w, _ in works]
    torch.cuda.synchronize()
    # two passes over the cases: the first also sees the runtime load each
    # kernel's code object on its first launch; the second must leave the
    # device's free memory unchanged, and repeat the first bitwise
    passes = []
    free = []
    for p in range(2):
        torch.cuda.synchronize()
        free.append(torch.cuda.mem_get_info()[0])
        for (name, w, o), (u, st), x in zip(works, bufs, src):
            print("[case] noalloc pass", p, name, "n", w.n, flush=True)
            u.copy_(x)
            st.zero_()
            r = noalloc(rd, u, w, st, **o)
            assert r == 0, (name, r, _lib.last_error())
        torch.cuda.synchronize()
        passes.append([(u.cpu(), st.cpu()) for u, st in bufs])
    free.append(torch.cuda.mem_get_info()[0])
    assert free[2] == free[1], free
    for (y0, s0), (y1, s1) in zip(*passes):
        assert torch.equal(y0, y1) and torch.equal(s0, s1)
    outs = passes[1]
    del bufs, src
    for (name, w, o), (y, s) in zip(works, outs):
        print("[case] allocating entry point", name, flush=True)
        u = torch.tensor(w.states, dtype=torch.float64, device="cuda")
        st = torch.zeros((9, w.n), dtype=torch.int32, device="cuda")
        r = rd.reaction_step(u, w.dt, w.rtol, w.atol, w.kind, w.params, stats=st, **o)
        torch.cuda.synchronize()
        assert r == 0
        assert torch.equal(u.cpu(), y), name
        assert torch.equal(st.cpu(), s), name


def test_noalloc_refuses_oversize_and_bad_options(rd):
    w = W.oregonator_1d(n=1024)
    n = 4194304 + 1
    u = torch.zeros((3, n), dtype=torch.float64, device="cuda")
    r = noalloc(rd, u, w)
    assert r == -4  # RD_ETOOBIG, before any device work
    assert float(u.abs().max()) == 0.0
    u = torch.tensor(w.states, dtype=torch.float64, device="cuda")
    assert noalloc(rd, u, w, use_graph=True) == -1
    assert noalloc(rd, u[:, :0].contiguous(), w) == 0
