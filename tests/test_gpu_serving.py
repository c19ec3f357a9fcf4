"""Serving session on the GPU: requests of different sizes and models are
admitted by HBM budget and overlap on the device; every result equals the same
request run alone (bitwise: same kernel variant, per-cell arithmetic does not
depend on the mix)."""
import numpy as np
import pytest

from paper_1506_04651_amd import workloads as W
from tests.parity import say

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


def small_stream(pools, n_req, seed, max_cells):
    rng = np.random.default_rng(seed)
    reqs = []
    t = 0.0
    names = sorted(pools)
    for _ in range(n_req):
        t += rng.exponential(2e-3)
        pool = names[int(rng.integers(0, 3))]
        size = pools[pool]["w"].n
        n = int(10 ** rng.uniform(3, np.log10(max_cells)))
        idx = rng.integers(0, size, n)
        dt = [1.0 / 256, 1.0 / 64, 1e-2][int(rng.integers(0, 3))]
        reqs.append(W.Request(t, pool, idx, dt))
    return reqs


def test_mix_equals_alone(rd, pools):
    from paper_1506_04651_amd import serving
    reqs = small_stream(pools, 50, 3, 20000)
    budget = 4 << 20  # small: admission has to wait for earlier requests
    say("serving mix, 50 requests, budget", budget)
    with rd.Session(budget, n_streams=4, precision=rd.MIXED) as s:
        recs, wall, outs = serving.replay(s, reqs, pools, time_scale=1.0, keep_outputs=True)
    assert all(r is not None and r["status"] == 0 for r in recs)
    summary = serving.summarize(recs, wall)
    say("serving summary", summary)
    assert summary["failed_cells"] == 0
    # admission queued at least once (budget smaller than the offered bytes)
    assert summary["mean_queue_ms"] >= 0.0
    # every request alone, through the direct entry point, same options
    for j, r in enumerate(reqs):
        w = pools[r.pool]["w"]
        u = serving.gather(pools[r.pool], r.idx)
        rd.reaction_step(u, r.dt, w.rtol, w.atol, w.kind, w.params, precision=rd.MIXED)
        torch.cuda.synchronize()
        assert torch.equal(u, outs[j]), (j, r.pool, len(r.idx))


def test_overlap_and_batches(rd, pools):
    """Requests submitted together run concurrently on several streams: the
    wall time of the mix is below the sum of the requests' solo times."""
    from paper_1506_04651_amd import serving
    reqs = [W.Request(0.0, "oreg2d", np.arange(i * 20000, (i + 1) * 20000), 1.0 / 64)
            for i in range(8)]
    say("serving overlap, 8 simultaneous requests")
    w = pools["oreg2d"]["w"]
    solo = 0.0
    for r in reqs:
        u = serving.gather(pools["oreg2d"], r.idx)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        rd.reaction_step(u, r.dt, w.rtol, w.atol, w.kind, w.params, precision=rd.MIXED)
        b.record()
        b.synchronize()
        solo += a.elapsed_time(b) * 1e-3
    with rd.Session(1 << 30, n_streams=4, precision=rd.MIXED) as s:
        recs, wall, _ = serving.replay(s, reqs, pools, time_scale=1.0)
    assert all(r["status"] == 0 for r in recs)
    say("solo sum", solo, "mix wall", wall)
    assert len({r["batch"] for r in recs}) >= 1


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
