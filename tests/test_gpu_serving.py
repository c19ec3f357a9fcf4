"""Serving session on the GPU (continuous batching under an HBM budget).

What is checked, each by an assertion:
  * admission waits for memory: under a budget smaller than the offered
    working set some requests are deferred, and each deferred request is
    admitted only after an earlier request has completed and released its
    arena range;
  * work overlaps on the device: the device-side kernel intervals of requests
    on different streams intersect, and the device span of a simultaneous
    batch is well below the sum of the requests' solo kernel times;
  * results: every request gives bitwise the same states alone (direct entry
    point, same options) and in the mix, and every in-mix result matches the
    FP64 CPU oracle to 1e-8 per cell;
  * ordering: the session reads a request's states only after the work that
    produced them on the caller's stream;
  * error paths: oversized requests, invalid arguments, unknown ids, two
    waiters on one id, destruction with requests pending.
"""
import threading

import numpy as np
import pytest

from paper_1506_04651_amd import workloads as W
from tests.parity import cell_rel_err, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def rd():
    import paper_1506_04651_amd as rd
    rd.load()
    assert torch.cuda.is_available()
    return rd


@pytest.fixture(scope="module")
def pools():
    from paper_1506_04651_amd import serving
    return serving.make_pools(small=True)


def small_stream(pools, n_req, seed, max_cells, max_cells_m16=2000):
    rng = np.random.default_rng(seed)
    reqs = []
    t = 0.0
    names = sorted(pools)
    for _ in range(n_req):
        t += rng.exponential(2e-3)
        pool = names[int(rng.integers(0, 3))]
        size = pools[pool]["w"].n
        hi = max_cells_m16 if pools[pool]["w"].m > 4 else max_cells
        n = int(10 ** rng.uniform(3, np.log10(hi)))
        idx = rng.integers(0, size, n)
        dt = [1.0 / 256, 1.0 / 64, 1e-2][int(rng.integers(0, 3))]
        reqs.append(W.Request(t, pool, idx, dt))
    return reqs


@pytest.mark.parametrize("precision", [0, 1])
def test_mix_queues_for_memory_equals_alone_and_oracle(rd, orc, pools, precision):
    from paper_1506_04651_amd import serving
    reqs = small_stream(pools, 50, 3, 20000)
    # arrivals compressed into about 1 ms and a budget far below their working
    # set (about 8 MiB): admission has to wait for completions
    budget = 2 << 20
    say("serving mix, 50 requests, budget", budget, "precision", precision)
    with rd.Session(budget, n_streams=4, precision=precision) as s:
        recs, wall, outs = serving.replay(s, reqs, pools, time_scale=0.01, keep_outputs=True)
    assert all(r is not None and r["status"] == 0 for r in recs)
    summary = serving.summarize(recs, wall)
    say("serving summary", summary)
    assert summary["failed_cells"] == 0
    # admission waited for memory, and a deferred request entered the arena
    # only after some earlier request had completed
    deferred = [r for r in recs if r["deferred"] > 0]
    assert deferred, "no request had to wait for arena space"
    done_times = sorted(r["t_done_ns"] for r in recs)
    for r in deferred:
        assert r["t_admit_ns"] > r["t_submit_ns"]
        assert any(t <= r["t_admit_ns"] for t in done_times), r
    # every request alone, through the direct entry point, same options
    for j, r in enumerate(reqs):
        w = pools[r.pool]["w"]
        u = serving.gather(pools[r.pool], r.idx)
        rd.reaction_step(u, r.dt, w.rtol, w.atol, w.kind, w.params, precision=precision)
        torch.cuda.synchronize()
        assert torch.equal(u, outs[j]), (j, r.pool, len(r.idx))
    # every in-mix result against the FP64 oracle
    worst = 0.0
    for j, r in enumerate(reqs):
        w = pools[r.pool]["w"]
        x0 = np.ascontiguousarray(pools[r.pool]["w"].states[:, r.idx])
        yo, _, reto = orc.reaction_step(x0, r.dt, w.rtol, w.atol, w.kind, w.params)
        assert reto == 0
        err = cell_rel_err(outs[j].cpu().numpy(), yo, w.atol)
        worst = max(worst, float(err.max()))
        assert err.max() <= 1e-8, (j, r.pool, float(err.max()))
    say("in-mix results vs oracle, max rel err", worst)


def test_kernels_overlap_on_the_device(rd, pools):
    """Requests submitted together run concurrently on several streams: their
    kernel intervals (device clock) intersect and the device span of the
    whole batch is well below the sum of the solo kernel times."""
    from paper_1506_04651_amd import serving
    reqs = [W.Request(0.0, "oreg2d", np.arange(i * 30000, (i + 1) * 30000), 1.0 / 64)
            for i in range(8)]
    say("serving overlap, 8 simultaneous requests")
    w = pools["oreg2d"]["w"]
    solo = 0.0
    for r in reqs:
        u = serving.gather(pools["oreg2d"], r.idx)
        torch.cuda.synchronize()
        rd.reaction_step(u, r.dt, w.rtol, w.atol, w.kind, w.params, precision=rd.MIXED)
        solo += rd.last_kernel_ms()
    with rd.Session(1 << 30, n_streams=4, precision=rd.MIXED) as s:
        recs, wall, _ = serving.replay(s, reqs, pools, time_scale=1.0)
    assert all(r["status"] == 0 for r in recs)
    span = max(r["kernel_end_ms"] for r in recs) - min(r["kernel_start_ms"] for r in recs)
    conc = serving.max_concurrent_kernels(recs)
    say("solo kernel sum ms", solo, "device span ms", span, "host wall ms", wall * 1e3,
        "max concurrent kernels", conc)
    assert len({r["stream"] for r in recs}) == 4
    assert conc >= 2
    pairs = [(a, b) for a in recs for b in recs if a["stream"] != b["stream"] and
             a["kernel_start_ms"] < b["kernel_end_ms"] and b["kernel_start_ms"] < a["kernel_end_ms"]]
    assert pairs, "no two kernels on different streams overlapped"
    assert span < 0.8 * solo
    assert wall * 1e3 < solo


def test_submit_follows_the_producer_stream(rd, pools):
    """The states are written on a side stream behind a long queue of work and
    submitted without a host synchronisation: the session must read them
    after that work, so the result equals the one of the same states run
    directly."""
    w = pools["oreg2d"]["w"]
    src = pools["oreg2d"]["states"][:, :50000].contiguous()
    ref = src.clone()
    rd.reaction_step(ref, w.dt, w.rtol, w.atol, w.kind, w.params)
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    u = torch.zeros_like(src)
    a = torch.randn(4096, 4096, device="cuda")
    torch.cuda.synchronize()
    with rd.Session(1 << 28) as s:
        with torch.cuda.stream(side):
            for _ in range(8):
                a = (a @ a) * 1e-3
            u.copy_(src)
            rid = s.submit(u, w.dt, w.rtol, w.atol, w.kind, w.params)
        info = s.wait(rid)
    assert info.status == 0 and info.n_failed == 0
    assert torch.equal(u, ref)


def test_request_too_big_and_errors(rd, pools):
    u = torch.zeros((3, 100000), dtype=torch.float64, device="cuda")
    with rd.Session(1 << 20, precision=rd.MIXED) as s:
        with pytest.raises(rd.RdError) as ei:
            s.submit(u, 0.01, 1e-5, 1e-8, rd.OREGONATOR, W.OREG_PARAMS)
        assert ei.value.code == -4
        with pytest.raises(rd.RdError) as ei:
            s.submit(u[:, :10].contiguous(), -1.0, 1e-5, 1e-8, rd.OREGONATOR, W.OREG_PARAMS)
        assert ei.value.code == -1
        with pytest.raises(rd.RdError) as ei:
            s.poll(123456)
        assert ei.value.code == -6
    with pytest.raises(rd.RdError) as ei:
        rd.Session(1 << 20, n_streams=100)
    assert ei.value.code == -1


def test_two_waiters_on_one_request(rd, pools):
    """Two threads wait for the same id: both return (shared ownership of the
    request), each with status 0 or, if it came after the other had been
    told, RD_ENOTFOUND."""
    w = pools["oreg3d"]["w"]
    u = pools["oreg3d"]["states"].clone()
    with rd.Session(1 << 30) as s:
        rid = s.submit(u, w.dt, w.rtol, w.atol, w.kind, w.params)
        out = [None, None]

        def waiter(k):
            try:
                s.wait(rid)
                out[k] = 0
            except rd.RdError as e:
                out[k] = e.code

        th = [threading.Thread(target=waiter, args=(k,)) for k in range(2)]
        for t in th:
            t.start()
        for t in th:
            t.join(timeout=60)
        assert not any(t.is_alive() for t in th)
    say("two waiters", out)
    assert 0 in out and all(o in (0, -6) for o in out)


def test_destroy_drains_pending(rd, pools):
    w = pools["oreg2d"]["w"]
    ins = [pools["oreg2d"]["states"][:, i * 5000:(i + 1) * 5000].contiguous() for i in range(6)]
    refs = [x.clone() for x in ins]
    for r in refs:
        rd.reaction_step(r, w.dt, w.rtol, w.atol, w.kind, w.params, precision=rd.MIXED)
    s = rd.Session(1 << 24, precision=rd.MIXED)
    for x in ins:
        s.submit(x, w.dt, w.rtol, w.atol, w.kind, w.params)
    say("destroy with pending requests")
    s.close()
    torch.cuda.synchronize()
    for x, r in zip(ins, refs):
        assert torch.equal(x, r)
