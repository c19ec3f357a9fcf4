"""GPU multiresolution leaf sets against the MRA oracle: identical keys
(integer parity), identical leaf values and per-level counts, identical
reconstruction; and the adapted-grid pipeline of the paper (leaf set ->
reaction step on the leaves -> reconstruction) on the BZ field."""
import numpy as np
import pytest

from oracle import mra as M
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


def front_field_rowmajor(d, J, m=2, width=0.02, seed=0):
    N = 1 << J
    x = (np.arange(N) + 0.5) / N
    g = np.meshgrid(*([x] * d), indexing="ij")       # g[0] slowest ... g[-1] fastest (= x)
    rng = np.random.default_rng(seed)
    c = rng.uniform(0.35, 0.65, d)
    r = np.sqrt(sum((g[a] - c[a]) ** 2 for a in range(d)))
    u = np.tanh((r - 0.25) / width)
    comps = [u, 0.5 * u * u + 0.1 * g[-1]] + [np.cos(3 * g[0] + k) for k in range(m - 2)]
    return np.vstack([v.ravel() for v in comps[:m]])


@pytest.mark.parametrize("d,J,eps,m", [(2, 8, 1e-3, 2), (2, 8, 3e-2, 2), (2, 6, 0.0, 3),
                                       (3, 5, 1e-3, 2), (2, 7, 1e-3, 1),
                                       # below one 4096-cell brick: the per-cell Morton copies
                                       (2, 5, 1e-3, 2), (3, 3, 0.0, 2)])
def test_leaf_set_parity(rd, d, J, eps, m):
    f = front_field_rowmajor(d, J, m=m, seed=J)
    scale = np.linspace(1.0, 2.0, m)
    say("mra parity d", d, "J", J, "eps", eps, "m", m)
    ft = torch.tensor(f, dtype=torch.float64, device="cuda")
    keys, vals, counts = rd.mra_leaves(ft, d, J, eps, scale=scale)
    ko, vo, co = M.leaves(M.row_major_to_morton(f, d, J), d, J, eps, scale)
    kg = keys.cpu().numpy().view(np.uint64)
    say("leaves", kg.size, "of", 1 << (d * J), "per level", counts)
    assert np.array_equal(kg, ko)
    assert np.array_equal(np.array(counts), co)
    assert np.array_equal(vals.cpu().numpy(), vo)
    rec = rd.mra_reconstruct(keys, vals, d, J).cpu().numpy()
    reco = M.morton_to_row_major(M.reconstruct(ko, vo, d, J), d, J)
    assert np.array_equal(rec, reco)
    if eps == 0.0:
        assert np.array_equal(rec, f)


def test_bz_adapted_grid_pipeline(rd, orc):
    """The paper's use: the reaction step runs on the leaves of the adapted
    grid (§2.2, §3.2).  512^2 BZ field (q = 0.02): leaf set (integer parity
    with the oracle), reaction step on the leaf values, reconstruction."""
    w = W.oregonator_2d_paper(side=512, dt=5e-4)
    d, J, eps = 2, 9, 1e-2  # the generator noise (1e-3) sits above smaller thresholds
    scale = np.max(np.abs(w.states), axis=1)
    ft = torch.tensor(w.states, dtype=torch.float64, device="cuda")
    keys, vals, counts = rd.mra_leaves(ft, d, J, eps, scale=scale)
    ko, vo, co = M.leaves(M.row_major_to_morton(w.states, d, J), d, J, eps, scale)
    assert np.array_equal(keys.cpu().numpy().view(np.uint64), ko)
    n = int(keys.numel())
    say("BZ 512^2 leaves", n, "compression", 1 - n / w.n, "per level", counts)
    assert n < w.n
    st = torch.zeros((9, n), dtype=torch.int32, device="cuda")
    v = vals.contiguous()
    assert rd.reaction_step(v, w.dt, w.rtol, w.atol, w.kind, w.params, stats=st) == 0
    # the same leaf values (from the oracle's leaf set) through the oracle
    yo, sto, ro = orc.reaction_step(vo, w.dt, w.rtol, w.atol, w.kind, w.params)
    assert ro == 0
    err = np.max(np.abs(v.cpu().numpy() - yo) / np.maximum(np.abs(yo), w.atol))
    say("reaction on leaves: max rel err vs oracle", err)
    assert err <= 1e-8
    rec = rd.mra_reconstruct(keys, v, d, J)
    assert rec.shape == ft.shape and torch.isfinite(rec).all()


@pytest.mark.parametrize("d,J,eps", [(2, 8, 1e-3), (3, 5, 1e-3), (2, 7, 3e-2)])
def test_leaf_set_with_refinement_parity(rd, d, J, eps):
    f = front_field_rowmajor(d, J, m=2, seed=J + 1)
    say("mra refine parity d", d, "J", J, "eps", eps)
    ft = torch.tensor(f, dtype=torch.float64, device="cuda")
    keys, vals, counts = rd.mra_leaves(ft, d, J, eps, refine=True)
    ko, vo, co = M.leaves(M.row_major_to_morton(f, d, J), d, J, eps, refine=True)
    assert np.array_equal(keys.cpu().numpy().view(np.uint64), ko)
    assert np.array_equal(np.array(counts), co)
    assert np.array_equal(vals.cpu().numpy(), vo)


def leaf_centres(keys, d):
    lev, idx = M.key_level(keys), M.key_index(keys, d)
    out = np.zeros((d, keys.size))
    for j in np.unique(lev):
        sel = lev == j
        co = M.deinterleave(idx[sel], d, int(j))
        for a in range(d):
            out[a, sel] = (co[a] + 0.5) / (1 << int(j))
    return out


@pytest.mark.parametrize("d,J,eps", [(2, 8, 1e-3), (3, 5, 1e-3)])
@pytest.mark.parametrize("refine", [False, True])
@pytest.mark.parametrize("change", ["bump", "flatten"])
def test_adapt_parity(rd, d, J, eps, refine, change):
    """Adaptation after the values change: a leaf set from the oracle, its
    values changed on the CPU (a bump away from the fronts: new significant
    details; or the fronts flattened in half of the domain: details vanish
    and the tree coarsens there), then the GPU and the oracle adapt it:
    identical keys, values and per-level counts."""
    f = front_field_rowmajor(d, J, m=2, seed=J)
    ko, vo, _ = M.leaves(M.row_major_to_morton(f, d, J), d, J, eps)
    x = leaf_centres(ko, d)
    if change == "bump":
        bump = 0.3 * np.exp(-np.sum((x - 0.2) ** 2, axis=0) / 0.005)
        v2 = vo + bump[None, :] * np.array([[1.0], [0.5]])
    else:
        v2 = np.where(x[0][None, :] > 0.5, np.array([[0.7], [0.2]]), vo)
    ka, va, ca = M.adapt(ko, v2, d, J, eps, refine=refine)
    say("adapt d", d, "J", J, "refine", refine, "leaves", ko.size, "->", ka.size)
    kt = torch.tensor(ko.view(np.int64), device="cuda")
    vt = torch.tensor(np.ascontiguousarray(v2), dtype=torch.float64, device="cuda")
    kg, vg, cg = rd.mra_adapt(kt, vt, d, J, eps, refine=refine)
    assert np.array_equal(kg.cpu().numpy().view(np.uint64), ka)
    assert np.array_equal(np.array(cg), ca)
    assert np.array_equal(vg.cpu().numpy(), va)
