"""Pins of the MRA oracle (CPU).

- Morton keys: round trip, and the order of keys equals the Z-curve order
  built recursively (quadrant by quadrant) in the test.
- Projection: each node equals the brute-force average of the fine cells it
  covers.
- Prediction: third order, i.e. exact on cell averages of quadratic
  polynomials (interior nodes; averages computed in closed form), not exact
  for cubics; conservative (the 2^d predicted children average to the parent).
- Leaf sets: leaves tile the domain without overlap; the tree is graded; a
  leaf's discarded children all have details below the level threshold.
- Reconstruction: lossless at eps = 0, error shrinking with eps, and the
  projection of the reconstruction returns every leaf value.
"""
import os

import numpy as np
import pytest

from oracle import mra as M

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def zcurve(d, j):
    """Cells of level j in Z order, by recursion over quadrants (x then y[, z]
    bit order: the x half is the most significant choice)."""
    if j == 0:
        return [tuple([0] * d)]
    out = []
    for child in range(1 << d):
        bits = [(child >> (d - 1 - a)) & 1 for a in range(d)]
        for c in zcurve(d, j - 1):
            out.append(tuple(bits[a] << (j - 1) | c[a] for a in range(d)))
    return out


@pytest.mark.parametrize("d,j", [(2, 1), (2, 3), (3, 2)])
def test_morton_order_and_round_trip(d, j):
    cells = zcurve(d, j)
    coords = tuple(np.array([c[a] for c in cells]) for a in range(d))
    idx = M.interleave(coords, j)
    assert np.array_equal(idx, np.arange(len(cells)))
    back = M.deinterleave(idx, d, j)
    for a in range(d):
        assert np.array_equal(back[a], coords[a])
    keys = M.make_key(idx, j, d)
    assert np.all(np.diff(keys.astype(np.float64)) > 0)
    assert np.array_equal(M.key_index(keys, d), idx) and np.all(M.key_level(keys) == j)


def cell_avg_poly(coeff, d, j, deg):
    """Exact averages over level-j cells of sum_c coeff[c] prod_a x_a^e_a."""
    N = 1 << j
    h = 1.0 / N
    idx = np.arange(N ** d)
    co = M.deinterleave(idx, d, j)
    out = np.zeros(N ** d)
    for e, cf in coeff.items():
        term = np.full(N ** d, cf)
        for a in range(d):
            lo, hi = co[a] * h, (co[a] + 1) * h
            term *= (hi ** (e[a] + 1) - lo ** (e[a] + 1)) / ((e[a] + 1) * h)
        out += term
    return out


@pytest.mark.parametrize("d", [2, 3])
def test_prediction_exact_for_quadratics(d):
    rng = np.random.default_rng(d)
    exps = [e for e in np.ndindex(*([3] * d)) if sum(e) <= 2]
    coeff = {e: rng.normal() for e in exps}
    jc = 3
    Uc = cell_avg_poly(coeff, d, jc, 2)[None, :]
    Uf = cell_avg_poly(coeff, d, jc + 1, 2)
    k = np.arange(1 << (d * (jc + 1)))
    pred = M.predict(Uc, d, jc, k)[0]
    co = M.deinterleave(k >> d, d, jc)
    interior = np.ones(k.size, dtype=bool)
    for a in range(d):
        interior &= (co[a] >= 1) & (co[a] <= (1 << jc) - 2)
    assert np.allclose(pred[interior], Uf[interior], rtol=0, atol=1e-12)
    # a cubic term breaks it
    cub = dict(coeff)
    cub[tuple([3] + [0] * (d - 1))] = 1.0
    Uc3 = cell_avg_poly(cub, d, jc, 3)[None, :]
    Uf3 = cell_avg_poly(cub, d, jc + 1, 3)
    assert np.max(np.abs(M.predict(Uc3, d, jc, k)[0][interior] - Uf3[interior])) > 1e-6
    # conservative: children of every node average to it
    ch = pred.reshape(-1, 1 << d).mean(axis=1)
    assert np.allclose(ch, Uc[0], atol=1e-13)


@pytest.mark.parametrize("d,J", [(2, 5), (3, 3)])
def test_projection_is_the_average_of_covered_cells(d, J):
    rng = np.random.default_rng(7)
    U = rng.normal(size=(2, 1 << (d * J)))
    lv = M.project(U, d, J)
    for j in range(J + 1):
        span = 1 << (d * (J - j))
        brute = U.reshape(2, -1, span).mean(axis=2)
        assert np.allclose(lv[j], brute, atol=1e-13)


def front_field(d, J, width=0.03):
    N = 1 << J
    x = (np.arange(N) + 0.5) / N
    grids = np.meshgrid(*([x] * d), indexing="ij")          # (z, y, x) or (y, x)
    r = np.sqrt(sum((g - 0.45) ** 2 for g in grids))
    u = np.tanh((r - 0.3) / width)
    f = np.vstack([u.ravel(), (0.5 * u * u).ravel()])
    return M.row_major_to_morton(f, d, J)


@pytest.mark.parametrize("d,J,eps", [(2, 6, 1e-3), (2, 7, 1e-2), (3, 4, 1e-3)])
def test_leaf_set_properties(d, J, eps):
    U = front_field(d, J)
    keys, vals, counts = M.leaves(U, d, J, eps)
    lev = M.key_level(keys)
    idx = M.key_index(keys, d)
    assert counts.sum() == keys.size and 0 < keys.size < U.shape[1]
    # tiling: fine-index ranges [idx << d(J-j), (idx+1) << d(J-j)) are contiguous
    start = idx << (d * (J - lev))
    end = (idx + 1) << (d * (J - lev))
    assert start[0] == 0 and end[-1] == (1 << (d * J)) and np.array_equal(start[1:], end[:-1])
    # grading: every refined node (ancestor of a leaf) has its 3^d neighbours in the tree
    levels = M.project(U, d, J)
    dets = M.details(levels, d, J)
    R = M.refine_flags(levels, dets, d, J, eps, np.ones(2))
    for j in range(1, J):
        ks = np.nonzero(R[j])[0]
        co = M.deinterleave(ks, d, j)
        for off in np.ndindex(*([3] * d)):
            nb = [co[a] + off[a] - 1 for a in range(d)]
            ok = np.ones(ks.size, dtype=bool)
            for a in range(d):
                ok &= (nb[a] >= 0) & (nb[a] < (1 << j))
            assert np.all(R[j - 1][M.interleave(tuple(c[ok] for c in nb), j) >> d])
    # a leaf below the finest level has no significant child
    for j in range(J):
        sel = idx[lev == j]
        if sel.size == 0:
            continue
        ch = (sel[:, None] << d) + np.arange(1 << d)[None, :]
        nrm = M.detail_norm2(dets[j + 1][:, ch.ravel()], np.ones(2))
        assert np.all(nrm < eps * eps * 2.0 ** (d * (j + 1 - J)))
    # leaf values are the projected averages
    for j in np.unique(lev):
        sel = lev == j
        assert np.array_equal(vals[:, sel], levels[j][:, idx[sel]])


@pytest.mark.parametrize("d,J", [(2, 6), (3, 4)])
def test_reconstruction(d, J):
    U = front_field(d, J)
    k0, v0, _ = M.leaves(U, d, J, 0.0)
    assert k0.size == U.shape[1]
    assert np.max(np.abs(M.reconstruct(k0, v0, d, J) - U)) <= 1e-13
    errs = []
    for eps in [1e-1, 1e-2, 1e-3, 1e-4]:
        keys, vals, _ = M.leaves(U, d, J, eps)
        R = M.reconstruct(keys, vals, d, J)
        errs.append(np.max(np.abs(R - U)))
        # projection of the reconstruction returns the leaf values
        lv = M.project(R, d, J)
        lev, idx = M.key_level(keys), M.key_index(keys, d)
        for j in np.unique(lev):
            sel = lev == j
            assert np.allclose(lv[j][:, idx[sel]], vals[:, sel], rtol=0, atol=1e-12)
    assert all(a >= b for a, b in zip(errs, errs[1:]))
    assert errs[-1] <= 20 * 1e-4


def tree_nodes(keys, d):
    """(level, index) of every node of the tree a leaf set spans."""
    nodes = set()
    for lv, k in zip(M.key_level(keys), M.key_index(keys, d)):
        lv, k = int(lv), int(k)
        while True:
            nodes.add((lv, k))
            if lv == 0:
                break
            lv, k = lv - 1, k >> d
    return nodes


@pytest.mark.parametrize("d,J,eps", [(2, 6, 1e-3), (3, 4, 1e-3)])
def test_adapt_without_refinement_is_idempotent(d, J, eps):
    """A leaf set built from a field is the fixed point of adaptation without
    refinement: the tree values are the same averages, the nodes outside the
    tree have zero details, so flags, grading and leaves are unchanged."""
    U = front_field(d, J)
    k0, v0, c0 = M.leaves(U, d, J, eps)
    k1, v1, c1 = M.adapt(k0, v0, d, J, eps, refine=False)
    assert np.array_equal(k0, k1) and np.array_equal(v0, v1) and np.array_equal(c0, c1)


@pytest.mark.parametrize("d,J,eps", [(2, 6, 1e-3), (2, 7, 1e-2), (3, 4, 1e-3)])
def test_adapt_with_refinement(d, J, eps):
    """Refinement: every node below the finest level whose detail is
    significant has children; the adapted tree contains the old one; new
    leaves carry the values predicted from their parents' level; the result
    tiles the domain and is graded; the fine field it reconstructs is the old
    one up to rounding."""
    U = front_field(d, J)
    scale = np.ones(U.shape[0])
    k0, v0, _ = M.leaves(U, d, J, eps)
    k1, v1, _ = M.adapt(k0, v0, d, J, eps, refine=True)
    old, new = tree_nodes(k0, d), tree_nodes(k1, d)
    assert old <= new and len(new) > len(old)
    lv1, ix1 = M.key_level(k1), M.key_index(k1, d)
    start = ix1 << (d * (J - lv1))
    end = (ix1 + 1) << (d * (J - lv1))
    assert start[0] == 0 and end[-1] == (1 << (d * J)) and np.array_equal(start[1:], end[:-1])
    levels = M.tree_levels(k0, v0, d, J)
    dets = M.details(levels, d, J)
    leafset = set(zip(lv1.tolist(), ix1.tolist()))
    for j in range(1, J):
        sig = np.nonzero(M.detail_norm2(dets[j], scale) >= eps * eps * 2.0 ** (d * (j - J)))[0]
        assert not any((j, int(k)) in leafset for k in sig)       # significant nodes are refined
    for j in range(1, J + 1):                                     # new leaves: predicted values
        sel = np.nonzero(lv1 == j)[0]
        fresh = [i for i in sel if (j, int(ix1[i])) not in old]
        if fresh:
            pred = M.predict(levels[j - 1], d, j - 1, ix1[fresh])
            assert np.array_equal(v1[:, fresh], pred)
    R = M.refine_flags(levels, dets, d, J, eps, scale, refine=True)
    for j in range(1, J):                                         # graded
        ks = np.nonzero(R[j])[0]
        co = M.deinterleave(ks, d, j)
        for off in np.ndindex(*([3] * d)):
            nb = [co[a] + off[a] - 1 for a in range(d)]
            ok = np.ones(ks.size, dtype=bool)
            for a in range(d):
                ok &= (nb[a] >= 0) & (nb[a] < (1 << j))
            assert np.all(R[j - 1][M.interleave(tuple(c[ok] for c in nb), j) >> d])
    assert np.allclose(M.reconstruct(k1, v1, d, J), M.reconstruct(k0, v0, d, J), rtol=0, atol=1e-13)


@pytest.mark.parametrize("refine", [False, True])
def test_adapt_coarsens_a_flat_leaf_set(refine):
    """All leaf values equal: every detail vanishes and the tree collapses to
    the root, which holds that value."""
    d, J = 2, 6
    k0, v0, _ = M.leaves(front_field(d, J), d, J, 1e-3)
    flat = np.full_like(v0, 0.25)
    k1, v1, c1 = M.adapt(k0, flat, d, J, 1e-3, refine=refine)
    assert k1.size == 1 and M.key_level(k1)[0] == 0 and np.all(v1 == 0.25) and c1[0] == 1


def test_leaves_with_refinement_contain_the_plain_tree():
    d, J, eps = 2, 7, 3e-3
    U = front_field(d, J)
    kp, _, _ = M.leaves(U, d, J, eps)
    kr, vr, _ = M.leaves(U, d, J, eps, refine=True)
    assert tree_nodes(kp, d) < tree_nodes(kr, d)
    lev, idx = M.key_level(kr), M.key_index(kr, d)
    levels = M.project(U, d, J)
    for j in np.unique(lev):
        sel = lev == j
        assert np.array_equal(vr[:, sel], levels[j][:, idx[sel]])


def test_prediction_matches_the_paper_1d_operator():
    """tests/golden/mr_prediction_1d.txt: the paper's 1D prediction (§2.2)
    worked by hand.  A 2D coarse level that varies only along x reduces the
    tensor-product prediction to the 1D operator: the children at x = 2k and
    2k + 1 of an interior node k carry exactly the fixture's values (a wrong
    sign or a swapped child fails)."""
    rows = np.loadtxt(os.path.join(GOLDEN, "mr_prediction_1d.txt"))
    d, jc = 2, 3
    N = 1 << jc
    for um, u0, up, e0, e1 in rows:
        xs = np.full(N, 7.0)
        xs[2], xs[3], xs[4] = um, u0, up          # node k = 3 with its two neighbours
        co = M.deinterleave(np.arange(N * N), d, jc)
        Uc = xs[co[0]][None, :]                   # constant along y
        ky = 5                                    # interior row
        for cx, want in ((0, e0), (1, e1)):
            for cy in (0, 1):
                child = M.interleave((np.array([2 * 3 + cx]), np.array([2 * ky + cy])), jc + 1)
                assert M.predict(Uc, d, jc, child)[0][0] == want


def test_thresholds_match_the_paper():
    """tests/golden/mr_thresholds.txt: eps_j = 2^((d/2)(j-J)) eps (§2.2), worked
    by hand.  A field equal to v on the cells below one level-j node and 0
    elsewhere has, at level j, the detail (1 - 2^-d) v at that node (an
    interior one: its parent averages it with 2^d - 1 zero siblings, the zero
    neighbours add nothing to the prediction), smaller details at its siblings
    (2^-d v) and neighbours (at most d 2^-d v / 8), coarser details below
    their own thresholds, and no finer details.  So the node and its siblings
    are leaves exactly when (1 - 2^-d) v >= eps_j: just above, level j holds
    2^d leaves; just below, none."""
    rows = np.loadtxt(os.path.join(GOLDEN, "mr_thresholds.txt"))
    for d, J, j, eps, eps_j in rows:
        d, J, j = int(d), int(J), int(j)
        half = 1 << (j - 1)                             # an interior level-j node
        node = int(M.interleave(tuple(np.array([half]) for _ in range(d)), j)[0])
        span = 1 << (d * (J - j))
        vcrit = eps_j / (1.0 - 2.0 ** -d)
        for f, want in ((1 + 1e-9, 1 << d), (1 - 1e-9, 0)):
            U = np.zeros((1, 1 << (d * J)))
            U[0, node * span:(node + 1) * span] = vcrit * f
            _, _, counts = M.leaves(U, d, J, eps)
            assert counts[j] == want, (d, J, j, f, counts)


def test_prediction_at_the_domain_edges():
    """tests/golden/mr_prediction_edges_1d.txt: at the two ends of a row the
    missing coarse neighbour is the edge node itself (even reflection across
    the boundary face), worked by hand; checked on a 2D level that varies
    only along x, at both children of the first and of the last node."""
    rows = np.loadtxt(os.path.join(GOLDEN, "mr_prediction_edges_1d.txt"))
    d, jc = 2, 3
    N = 1 << jc
    co = M.deinterleave(np.arange(N * N), d, jc)
    for side, ue, ui, c0, c1 in rows:
        xs = np.full(N, 5.0)
        k = 0 if side == 0 else N - 1
        xs[k] = ue
        xs[1 if side == 0 else N - 2] = ui
        Uc = xs[co[0]][None, :]
        for cx, want in ((0, c0), (1, c1)):
            child = M.interleave((np.array([2 * k + cx]), np.array([7])), jc + 1)
            assert M.predict(Uc, d, jc, child)[0][0] == want, (side, cx)


def test_thresholds_average_over_species():
    """The detail norm is the mean over species of (d_i / s_i)^2 (R28): with
    a second, identically zero species the leaf transition of the single-node
    field of the threshold test moves to (1 - 2^-d) v = sqrt(2) eps_j."""
    d, J, j, eps = 2, 6, 4, 1e-3
    eps_j = eps * 2.0 ** ((d / 2) * (j - J))
    half = 1 << (j - 1)
    node = int(M.interleave(tuple(np.array([half]) for _ in range(d)), j)[0])
    span = 1 << (d * (J - j))
    vcrit = np.sqrt(2.0) * eps_j / (1.0 - 2.0 ** -d)
    for f, want in ((1 + 1e-9, 1 << d), (1 - 1e-9, 0)):
        U = np.zeros((2, 1 << (d * J)))
        U[0, node * span:(node + 1) * span] = vcrit * f
        _, _, counts = M.leaves(U, d, J, eps)
        assert counts[j] == want, (f, counts)


@pytest.mark.parametrize("d,J", [(2, 6), (3, 4)])
def test_grading_around_an_isolated_cell(d, J):
    """One nonzero fine cell: the tree refines down to it, and every node
    with children has the parents of all its 3^d neighbours refined too
    (R30), on every side of the feature."""
    N = 1 << J
    U = np.zeros((1, 1 << (d * J)))
    c = tuple(np.array([N // 2 - 1 + a]) for a in range(d))
    U[0, M.interleave(c, J)[0]] = 1.0
    levels = M.project(U, d, J)
    dets = M.details(levels, d, J)
    R = M.refine_flags(levels, dets, d, J, 1e-3, np.ones(1))
    assert R[J - 1].any()
    for j in range(1, J):
        ks = np.nonzero(R[j])[0]
        co = M.deinterleave(ks, d, j)
        for off in np.ndindex(*([3] * d)):
            nb = [co[a] + off[a] - 1 for a in range(d)]
            ok = np.ones(ks.size, dtype=bool)
            for a in range(d):
                ok &= (nb[a] >= 0) & (nb[a] < (1 << j))
            assert np.all(R[j - 1][M.interleave(tuple(cc[ok] for cc in nb), j) >> d]), (j, off)
