"""The autotuner on the GPU: every variant of the set is timed on the batch,
none is rejected (all give the same states), the fastest becomes the default
that variant 0 selects, and the default is per kernel set (for the 16-lane
kernels: one set for 5..8 species, one for 9..16).  Defaults are restored."""
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
