"""GPU diffusion step (RKC stabilised explicit, Neumann Laplacian) and Strang
step R_{dt/2} D_dt R_{dt/2} (paper §2.1) against the numpy oracle, and the
paper's complexity statistic (Appendix A) on a BZ field evolved by Strang
steps."""
import numpy as np
import pytest

from oracle import diffusion as D
from paper_1506_04651_amd import complexity as CX
from paper_1506_04651_amd import workloads as W
from tests.parity import compare, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

BZ_DIFF = [2.5e-3, 2.5e-3, 1.5e-3]  # paper §1, model II


@pytest.fixture(scope="module")
def rd():
    import paper_1506_04651_amd as rd
    rd.load()
    assert torch.cuda.is_available()
    return rd


@pytest.mark.parametrize("shape,dt,stages", [((257, 193), 2e-3, 0), ((33, 29, 17), 5e-3, 0),
                                              ((64, 48), 1e-3, 7), ((1, 300), 1e-2, 0)])
def test_diffusion_step_matches_oracle(rd, shape, dt, stages):
    n = int(np.prod(shape))
    h = 1.0 / shape[0]
    rng = np.random.default_rng(n)
    u0 = rng.uniform(0.0, 1.0, (3, n))
    say("diffusion", shape, "dt", dt)
    u = torch.tensor(u0, dtype=torch.float64, device="cuda")
    s = rd.diffusion_step(u, shape, h, BZ_DIFF, dt, stages=stages)
    ref, s_ref = D.diffusion_step(u0, shape, h, BZ_DIFF, dt, stages=stages or None)
    assert s == s_ref and s >= 2
    got = u.cpu().numpy()
    err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
    say("stages", s, "max rel diff", err)
    assert err <= 1e-12
    # zero-flux boundaries conserve every species' total
    assert np.allclose(got.sum(axis=1), u0.sum(axis=1), rtol=1e-12)


@pytest.mark.parametrize("shape,dt", [((64, 48), 1e-3), ((32, 30, 18), 5e-3), ((2, 150), 1e-2)])
def test_two_cells_per_thread_equal_one_cell(rd, shape, dt):
    """With rows of even length and 16-byte aligned vectors the stage kernels
    take two neighbouring cells per thread; the same states placed one double
    off that alignment run the one-cell kernels.  Both give bitwise the same
    result, and the oracle's to 1e-12 (row length 2: the pair is the whole
    row, with no neighbour on either side)."""
    n = int(np.prod(shape))
    h = 1.0 / shape[0]
    rng = np.random.default_rng(n + 1)
    u0 = rng.uniform(0.0, 1.0, (3, n))
    say("diffusion pairs vs single cells", shape, "dt", dt)
    a = torch.tensor(u0, dtype=torch.float64, device="cuda")
    buf = torch.zeros(3 * n + 1, dtype=torch.float64, device="cuda")
    b = buf[1:].view(3, n)
    b.copy_(a)
    assert a.data_ptr() % 16 == 0 and b.data_ptr() % 16 == 8
    sa = rd.diffusion_step(a, shape, h, BZ_DIFF, dt)
    sb = rd.diffusion_step(b, shape, h, BZ_DIFF, dt)
    torch.cuda.synchronize()
    assert sa == sb and sa >= 2
    assert torch.equal(a, b)
    ref, s_ref = D.diffusion_step(u0, shape, h, BZ_DIFF, dt)
    assert s_ref == sa
    err = np.max(np.abs(a.cpu().numpy() - ref)) / np.max(np.abs(ref))
    say("stages", sa, "max rel diff", err)
    assert err <= 1e-12


def test_strang_steps_match_oracle(rd, orc):
    """Three Strang steps on the paper-constant BZ field (96^2), GPU and
    oracle each from the same generated states."""
    N = 96
    shape, h = (N, N), 1.0 / N
    w = W.oregonator_2d_paper(side=N, dt=1e-3)
    say("strang BZ", shape)
    u = torch.tensor(w.states, dtype=torch.float64, device="cuda")
    st = torch.zeros((2, 9, w.n), dtype=torch.int32, device="cuda")
    yo = w.states
    for k in range(3):
        ret = rd.strang_step(u, shape, h, BZ_DIFF, w.dt, w.rtol, w.atol, w.kind, w.params,
                             stats=st)
        yo, (s1, s2), rets, s = D.strang_step(orc, yo, shape, h, BZ_DIFF, w.dt, w.rtol, w.atol,
                                              w.kind, w.params)
        assert ret == 0 and rets == (0, 0)
        stg = st.cpu().numpy()
        rep = compare(u.cpu().numpy(), stg[1], yo, s2, w.atol, label=f"strang step {k}")
        assert np.mean(np.all(stg[0][1:] == s1[1:], axis=0)) >= 0.995
        assert rep["max_err_same_trace"] <= 1e-8
        assert rep["trace_divergent"] <= max(3, int(3e-3 * w.n))
        assert rep["max_err_divergent"] <= 10 * w.rtol


def test_complexity_on_strang_evolved_field(rd):
    """The paper measures complexity on its BZ simulation (Delta t = 1e-3,
    1024^2).  Here the synthetic spiral field is first evolved by Strang
    steps, so that its fronts carry the reaction-diffusion structure, then the
    complexity of one R_{Delta t/2} is taken (counter logic and its parity are
    covered by the tests above)."""
    w = W.oregonator_2d_paper(side=1024, dt=1e-3)
    shape, h = (1024, 1024), 1.0 / 1024
    u = torch.tensor(w.states, dtype=torch.float64, device="cuda")
    nsteps = 40
    say("strang evolution of the 1024^2 BZ field,", nsteps, "steps")
    for _ in range(nsteps):
        assert rd.strang_step(u, shape, h, BZ_DIFF, w.dt, w.rtol, w.atol, w.kind, w.params) == 0
    st = torch.zeros((9, w.n), dtype=torch.int32, device="cuda")
    assert rd.reaction_step(u, w.dt / 2, w.rtol, w.atol, w.kind, w.params, stats=st) == 0
    c = CX.complexity(st.cpu().numpy(), jac_evals=3)
    s = CX.summary(c)
    say("complexity after Strang evolution", s)
    assert s["min"] >= 8 and 0.0 < s["time_share_below_17"] <= 1.0


def test_strang_graph_replay_matches_eager(rd):
    """The whole split step recorded as one graph (both reaction halves with
    their claim-order passes, the diffusion stages, the failure counts): every
    replay, with the program's own eager work in between, gives the eager
    step's states, counters and failure count bitwise; a second states buffer
    records a graph of its own."""
    N = 128
    shape, h = (N, N), 1.0 / N
    w = W.oregonator_2d_paper(side=N, dt=1e-3)
    u0 = torch.tensor(w.states, dtype=torch.float64, device="cuda")
    s = torch.cuda.Stream()
    ref = u0.clone()
    st_ref = torch.zeros((2, 9, w.n), dtype=torch.int32, device="cuda")
    say("strang eager reference", shape)
    with torch.cuda.stream(s):
        r_ref = rd.strang_step(ref, shape, h, BZ_DIFF, w.dt, w.rtol, w.atol, w.kind, w.params,
                               stats=st_ref, stream=s)
    s.synchronize()
    bufs = [torch.empty_like(u0), torch.empty_like(u0)]
    st = torch.zeros_like(st_ref)
    for rep in range(5):
        u = bufs[0] if rep < 4 else bufs[1]
        say("strang graph replay", rep)
        with torch.cuda.stream(s):
            u.copy_(u0)
            st.zero_()
            r = rd.strang_step(u, shape, h, BZ_DIFF, w.dt, w.rtol, w.atol, w.kind, w.params,
                               stats=st, stream=s, use_graph=True)
        s.synchronize()
        assert r == r_ref
        assert torch.equal(u, ref) and torch.equal(st, st_ref)
        torch.cuda.synchronize()
        _ = (u0 * 2.0).sum().item()


def test_strang_graph_small_grid_without_stats(rd):
    """A grid below the claim-order threshold (the counters are then cleared
    by a kernel of their own inside the graph) and no statistics: replays
    equal the eager step."""
    N = 48
    shape, h = (N, N), 1.0 / N
    w = W.oregonator_2d_paper(side=N, dt=1e-3)
    u0 = torch.tensor(w.states, dtype=torch.float64, device="cuda")
    s = torch.cuda.Stream()
    ref = u0.clone()
    with torch.cuda.stream(s):
        r_ref = rd.strang_step(ref, shape, h, BZ_DIFF, w.dt, w.rtol, w.atol, w.kind, w.params,
                               stream=s)
    s.synchronize()
    u = torch.empty_like(u0)
    for rep in range(3):
        say("small strang graph replay", rep)
        with torch.cuda.stream(s):
            u.copy_(u0)
            r = rd.strang_step(u, shape, h, BZ_DIFF, w.dt, w.rtol, w.atol, w.kind, w.params,
                               stream=s, use_graph=True, precision=rd.MIXED)
        s.synchronize()
        assert r == 0
    # mixed-precision replays agree with one another and with an eager mixed step
    ref_m = u0.clone()
    with torch.cuda.stream(s):
        rd.strang_step(ref_m, shape, h, BZ_DIFF, w.dt, w.rtol, w.atol, w.kind, w.params,
                       stream=s, precision=rd.MIXED)
    s.synchronize()
    assert torch.equal(u, ref_m)
    assert r_ref == 0
