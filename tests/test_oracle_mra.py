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
import numpy as np
import pytest

from oracle import mra as M


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
