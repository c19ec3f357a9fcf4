"""The autotuner on the GPU.

* Every variant of a set is timed on the batch; variants of one engine must
  give bitwise the same states (none is rejected), the fastest becomes the
  default that variant 0 selects, and the default is per kernel set (for the
  16-lane kernels: one set for 5..8 species, one for 9..16).
* The search covers the lanes per cell: for the kinetics model with m = 4 the
  16-lane-group kernels (4 cells per wave) are variants beside the one-lane
  kernels (64 cells per wave); they run other arithmetic and are accepted on
  identical counters and states within 1e-10.
* The search covers the LDS layout of the one-lane engine (lane columns or
  lane rows of the per-lane slots), bitwise equal.
* The tuned default, launched through a captured hipGraph and replayed, is
  checked cell by cell against the CPU oracle on every replay.
Defaults are restored afterwards."""
import numpy as np
import pytest

from paper_1506_04651_amd import workloads as W
from tests.parity import compare, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def rd():
    import paper_1506_04651_amd as rd
    rd.load()
    assert torch.cuda.is_available()
    return rd


@pytest.mark.parametrize("case", ["oregonator_2d", "kinetics_m7"])
def test_autotune_sets_a_valid_default(rd, case):
    from paper_1506_04651_amd import autotune
    if case == "oregonator_2d":
        w = W.oregonator_2d().subset(W.sample_indices(262144, 20000, 9))
    else:
        w = W.kinetics16(n=3000, m=7, seed=5)
    u0 = torch.tensor(w.states, dtype=torch.float64, device="cuda")
    prec, sched = rd.FP64, rd.PERSISTENT
    try:
        res = autotune.tune(u0, w.dt, w.rtol, w.atol, w.kind, w.params, prec, sched, reps=1)
        say(case, "best", res["names"][res["best"]], "of", len(res["ms"]))
        assert not res["rejected"]
        assert len(res["ms"]) == rd.variant_count(w.kind, w.m, prec, sched)
        if case == "oregonator_2d":
            assert any(n.endswith(".aos") for n in res["names"].values())
        # variant 0 now resolves to the tuned one, for every m of the set
        assert rd.variant_name(w.kind, w.m, prec, sched, 0) == res["names"][res["best"]]
        if case == "kinetics_m7":
            assert rd.variant_name(w.kind, 5, prec, sched, 0) == res["names"][res["best"]]
            assert rd.variant_name(w.kind, 12, prec, sched, 0) == rd.variant_name(w.kind, 12, prec, sched, 1)
        u = u0.clone()
        assert rd.reaction_step(u, w.dt, w.rtol, w.atol, w.kind, w.params) == 0
        v = u0.clone()
        assert rd.reaction_step(v, w.dt, w.rtol, w.atol, w.kind, w.params, variant=1) == 0
        assert torch.equal(u, v)
    finally:
        rd.set_default_variant(w.kind, w.m, prec, sched, 1)
    assert rd.variant_name(w.kind, w.m, prec, sched, 0) == rd.variant_name(w.kind, w.m, prec, sched, 1)


@pytest.mark.parametrize("precision", [0, 1])
def test_autotune_searches_lanes_per_cell(rd, orc, precision):
    from paper_1506_04651_amd import autotune
    w = W.kinetics16(n=20000, m=4, seed=21)
    u0 = torch.tensor(w.states, dtype=torch.float64, device="cuda")
    sched = rd.PERSISTENT
    lanes = {v: rd.variant_lanes(w.kind, w.m, precision, sched, v)
             for v in range(1, rd.variant_count(w.kind, w.m, precision, sched) + 1)}
    assert set(lanes.values()) == {1, 16}
    try:
        res = autotune.tune(u0, w.dt, w.rtol, w.atol, w.kind, w.params, precision, sched,
                            reps=2)
        say("kinetics m=4 precision", precision, "lanes", res["lanes"], "ms", res["ms"],
            "rejected", res["rejected"])
        assert set(res["lanes"].values()) == {1, 16}
        # both engines against the oracle
        idx = W.sample_indices(w.n, 2048, 3)
        yo, sto, _ = orc.reaction_step(w.states[:, idx].copy(), w.dt, w.rtol, w.atol, w.kind,
                                       w.params)
        for v, nl in lanes.items():
            u = u0.clone()
            st = torch.zeros((9, w.n), dtype=torch.int32, device="cuda")
            assert rd.reaction_step(u, w.dt, w.rtol, w.atol, w.kind, w.params, stats=st,
                                    precision=precision, variant=v) == 0
            rep = compare(u.cpu().numpy()[:, idx], st.cpu().numpy()[:, idx], yo, sto, w.atol,
                          label=f"kin4 lanes{nl} p{precision}")
            assert rep["max_err"] <= 1e-8 and rep["trace_divergent"] == 0
    finally:
        rd.set_default_variant(w.kind, w.m, precision, sched, 1)


def test_tuned_graph_replays_match_oracle(rd, orc):
    """Tune the 2D field (a seeded 30 000-cell subset), then replay the tuned
    default through one captured hipGraph several times, with eager work
    between replays; every replay's states and counters against the oracle."""
    from paper_1506_04651_amd import autotune
    w = W.oregonator_2d().subset(W.sample_indices(262144, 30000, 17))
    u0 = torch.tensor(w.states, dtype=torch.float64, device="cuda")
    yo, sto, reto = orc.reaction_step(w.states, w.dt, w.rtol, w.atol, w.kind, w.params)
    assert reto == 0
    try:
        res = autotune.tune(u0, w.dt, w.rtol, w.atol, w.kind, w.params, rd.FP64,
                            rd.PERSISTENT, reps=1)
        say("tuned 2d subset:", res["names"][res["best"]])
        s = torch.cuda.Stream()
        u = torch.empty_like(u0)
        st = torch.zeros((9, w.n), dtype=torch.int32, device="cuda")
        for rep in range(3):
            with torch.cuda.stream(s):
                u.copy_(u0)
                st.zero_()
                ret = rd.reaction_step(u, w.dt, w.rtol, w.atol, w.kind, w.params, stats=st,
                                       use_graph=True)
            s.synchronize()
            assert ret == 0
            r = compare(u.cpu().numpy(), st.cpu().numpy(), yo, sto, w.atol,
                        label=f"tuned graph replay {rep}")
            assert r["max_err"] <= 1e-8 and r["trace_divergent"] == 0
            torch.cuda.synchronize()
            _ = (u0 * 2.0).sum().item()
    finally:
        rd.set_default_variant(w.kind, w.m, rd.FP64, rd.PERSISTENT, 1)
