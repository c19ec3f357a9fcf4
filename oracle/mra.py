"""Oracle of the multiresolution (MRA) leaf-set machinery (numpy, plain loops
over levels, FP64).

TEST INFRASTRUCTURE ONLY; shares no code with the GPU library.

What it computes (Descombes et al., §2.2, after Cohen et al. 2003), on the
dyadic tree of [0,1]^d (d = 2, 3) with finest level J (2^J cells per
direction):
- projection: the value of a node is the average of its 2^d children;
- prediction: third-order centred interpolation (l = 1), the tensor product of
  the 1D operator u_{2k} = u_k + (u_{k-1} - u_{k+1})/8,
  u_{2k+1} = u_k + (u_{k+1} - u_{k-1})/8 (§2.2), applied one direction at a time
  (x, then y, then z); outside the domain the coarse values are continued by
  even reflection (u_{-1} = u_0, u_N = u_{N-1}: zero-gradient, as the
  homogeneous Neumann boundaries);
- details d_{j,k} = u_{j,k} - prediction (eq. for the detail, §2.2);
- thresholds eps_j = 2^{(d/2)(j-J)} eps (§2.2) in the L2 norm over species,
  each species scaled by s_i: a node's children are kept when
  (1/m) sum_i (d_i / s_i)^2 >= eps_j^2 for some child (compression); with
  refinement on, a node whose own detail is significant gets children too
  (§2.2: nodes whose details exceed eps_j are refined; §3.1, refinement);
- grading (§2.2, graded tree): whenever a node has children, the 3^d
  neighbours of that node must exist (their parents get children too),
  enforced from the finest level to the root;
- leaves: nodes of the tree without children; keys (paper §3.1): the Morton
  abscissa (bits of x_1, x_2[, x_3] interleaved, most significant first)
  left-aligned in the top 48 bits, the level in the next 4 bits, 12 free bits;
- reconstruction: tree values by projection of the leaves, then every node
  outside the tree predicted level by level from the coarser level;
- adaptation of a leaf set to its values (§3.1, refinement and coarsening):
  the levels of the reconstruction (tree values, predicted values elsewhere),
  their details, the flags and grading above, and the leaf set of the result:
  children created by refinement carry predicted values, nodes whose
  children are no longer significant become leaves with their projected
  values.

Storage convention (both here and in the tests): every level in Morton order,
index k = interleave(x, y[, z]) with x the most significant bit of each group,
so the children of node p are d-bit groups appended to p.
"""
from __future__ import annotations

import numpy as np

KEY_ABSCISSA_BITS = 48
KEY_LEVEL_SHIFT = 12


def interleave(coords, bits):
    """Morton index of integer coordinates (tuple of arrays x, y[, z]) with
    `bits` bits each: bit b of coordinate a goes to position d*b + (d-1-a)."""
    d = len(coords)
    out = np.zeros(np.shape(coords[0]), dtype=np.int64)
    for b in range(bits):
        for a, c in enumerate(coords):
            out |= ((np.asarray(c, dtype=np.int64) >> b) & 1) << (d * b + (d - 1 - a))
    return out


def deinterleave(idx, d, bits):
    idx = np.asarray(idx, dtype=np.int64)
    coords = []
    for a in range(d):
        c = np.zeros(idx.shape, dtype=np.int64)
        for b in range(bits):
            c |= ((idx >> (d * b + (d - 1 - a))) & 1) << b
        coords.append(c)
    return tuple(coords)


def row_major_to_morton(field, d, J):
    """field [m, N^d] with x fastest -> [m, N^d] in Morton order at level J."""
    N = 1 << J
    n = N ** d
    lin = np.arange(n)
    coords = [(lin // (N ** a)) % N for a in range(d)]   # x, y[, z]
    mort = interleave(tuple(coords), J)
    out = np.empty_like(field)
    out[:, mort] = field
    return out


def morton_to_row_major(mfield, d, J):
    N = 1 << J
    n = N ** d
    lin = np.arange(n)
    coords = [(lin // (N ** a)) % N for a in range(d)]
    mort = interleave(tuple(coords), J)
    return mfield[:, mort]


def project(U_fine, d, J):
    """Levels 0..J (each [m, 2^(d j)], Morton order) by exact averages."""
    levels = [None] * (J + 1)
    levels[J] = U_fine
    nc = 1 << d
    for j in range(J, 0, -1):
        u = levels[j]
        m, n = u.shape
        ch = u.reshape(m, n // nc, nc)
        s = ch[:, :, 0]
        for c in range(1, nc):
            s = s + ch[:, :, c]
        levels[j - 1] = s * (1.0 / nc)
    return levels


def _neighbour_values(Uc, d, jc, coords, off):
    """Values of the level-jc nodes at coords + off, reflected at the edges."""
    N = 1 << jc
    nb = []
    for a in range(d):
        c = coords[a] + off[a]
        c = np.where(c < 0, 0, np.where(c >= N, N - 1, c))
        nb.append(c)
    return Uc[:, interleave(tuple(nb), jc)]


def predict(Uc, d, jc, child_idx):
    """Prediction of the level-(jc+1) nodes child_idx from level jc values
    Uc, one direction at a time (x, then y, then z)."""
    child_idx = np.asarray(child_idx, dtype=np.int64)
    parent = child_idx >> d
    pcoords = deinterleave(parent, d, jc)
    sub = [((child_idx >> (d - 1 - a)) & 1) for a in range(d)]   # child position per axis
    sgn = [np.where(s == 0, 0.125, -0.125) for s in sub]
    # values on the 3^d stencil: table[(ox, oy[, oz])]
    offs = [-1, 0, 1]
    table = {}
    if d == 2:
        for oy in offs:
            for ox in offs:
                table[(ox, oy)] = _neighbour_values(Uc, d, jc, pcoords, (ox, oy))
        rows = {}
        for oy in offs:
            rows[oy] = table[(0, oy)] + sgn[0] * (table[(-1, oy)] - table[(1, oy)])
        return rows[0] + sgn[1] * (rows[-1] - rows[1])
    for oz in offs:
        for oy in offs:
            for ox in offs:
                table[(ox, oy, oz)] = _neighbour_values(Uc, d, jc, pcoords, (ox, oy, oz))
    planes = {}
    for oz in offs:
        rows = {}
        for oy in offs:
            rows[oy] = table[(0, oy, oz)] + sgn[0] * (table[(-1, oy, oz)] - table[(1, oy, oz)])
        planes[oz] = rows[0] + sgn[1] * (rows[-1] - rows[1])
    return planes[0] + sgn[2] * (planes[-1] - planes[1])


def details(levels, d, J):
    """d_j for j = 1..J (index 0 unused), [m, 2^(d j)]."""
    out = [None] * (J + 1)
    for j in range(1, J + 1):
        k = np.arange(levels[j].shape[1])
        out[j] = levels[j] - predict(levels[j - 1], d, j - 1, k)
    return out


def detail_norm2(dj, scale):
    """(1/m) sum_i (d_i / s_i)^2 per node, species in order."""
    m = dj.shape[0]
    acc = (dj[0] / scale[0]) * (dj[0] / scale[0])
    for i in range(1, m):
        q = dj[i] / scale[i]
        acc = acc + q * q
    return acc * (1.0 / m)


def refine_flags(levels, dets, d, J, eps, scale, refine=False):
    """R_j[k] (j = 0..J-1): node (j, k) has children in the graded tree.
    refine: a node of level < J with a significant detail has children."""
    nc = 1 << d
    R = [np.zeros(levels[j].shape[1], dtype=bool) for j in range(J)]
    for j in range(1, J + 1):
        eps_j2 = (eps * eps) * np.ldexp(1.0, d * (j - J))   # eps_j^2 = 2^(d (j-J)) eps^2
        sig = detail_norm2(dets[j], scale) >= eps_j2
        R[j - 1] |= sig.reshape(-1, nc).any(axis=1)
        if refine and j < J:
            R[j] |= sig
    # grading, finest to coarsest
    for j in range(J - 1, 0, -1):
        ks = np.nonzero(R[j])[0]
        if ks.size == 0:
            continue
        coords = deinterleave(ks, d, j)
        N = 1 << j
        for off in np.ndindex(*([3] * d)):
            nb = [coords[a] + off[a] - 1 for a in range(d)]
            ok = np.ones(ks.size, dtype=bool)
            for a in range(d):
                ok &= (nb[a] >= 0) & (nb[a] < N)
            nidx = interleave(tuple(c[ok] for c in nb), j)
            R[j - 1][nidx >> d] = True
    return R


def leaves(U_fine_morton, d, J, eps, scale=None, refine=False):
    """Leaf set of the graded tree: (keys uint64 in Morton order, values
    [m, n_leaves], per-level leaf counts [J+1])."""
    m = U_fine_morton.shape[0]
    scale = np.ones(m) if scale is None else np.asarray(scale, dtype=np.float64)
    levels = project(U_fine_morton, d, J)
    dets = details(levels, d, J)
    R = refine_flags(levels, dets, d, J, eps, scale, refine) if J >= 1 else []
    return leaf_set(levels, R, d, J)


def leaf_set(levels, R, d, J):
    """Keys (Morton order), values and per-level counts of the leaves of the
    tree given by the flags R over the level arrays."""
    keys, vals, lev = [], [], []
    counts = np.zeros(J + 1, dtype=np.int64)
    for j in range(J + 1):
        n = 1 << (d * j)
        exists = np.ones(n, dtype=bool) if j == 0 else R[j - 1][np.arange(n) >> d]
        refined = R[j] if j < J else np.zeros(n, dtype=bool)
        leaf = np.nonzero(exists & ~refined)[0]
        counts[j] = leaf.size
        keys.append(make_key(leaf, j, d))
        vals.append(levels[j][:, leaf])
        lev.append(np.full(leaf.size, j))
    keys = np.concatenate(keys)
    vals = np.concatenate(vals, axis=1)
    order = np.argsort(keys, kind="stable")
    return keys[order], vals[:, order], counts


def make_key(idx, j, d):
    """64-bit node key: level-j Morton index left-aligned in bits 63..16, the
    level in bits 15..12 (the root's abscissa is 0)."""
    idx = np.asarray(idx, dtype=np.uint64)
    lev = np.uint64(j << KEY_LEVEL_SHIFT)
    if j == 0:
        return np.zeros(idx.shape, dtype=np.uint64) | lev
    return (idx << np.uint64(64 - d * j)) | lev


def key_level(keys):
    return ((np.asarray(keys, dtype=np.uint64) >> np.uint64(KEY_LEVEL_SHIFT)) & np.uint64(15)).astype(np.int64)


def key_index(keys, d):
    keys = np.asarray(keys, dtype=np.uint64)
    j = key_level(keys)
    out = np.zeros(keys.shape, dtype=np.int64)
    for lv in np.unique(j):
        if lv == 0:
            continue
        sel = j == lv
        out[sel] = (keys[sel] >> np.uint64(64 - d * int(lv))).astype(np.int64)
    return out


def reconstruct(keys, vals, d, J):
    """Fine-level field (Morton order) from a leaf set: tree values by
    projection of the leaves, nodes outside the tree predicted."""
    return tree_levels(keys, vals, d, J)[J]


def tree_levels(keys, vals, d, J):
    """Every level of the reconstruction of a leaf set: tree nodes valued by
    projection of the leaves, the others predicted from the level above."""
    m = vals.shape[0]
    lev = key_level(keys)
    idx = key_index(keys, d)
    # tree membership and values, bottom-up
    tree_val = [np.zeros((m, 1 << (d * j))) for j in range(J + 1)]
    in_tree = [np.zeros(1 << (d * j), dtype=bool) for j in range(J + 1)]
    for j in range(J + 1):
        sel = lev == j
        tree_val[j][:, idx[sel]] = vals[:, sel]
        in_tree[j][idx[sel]] = True
    nc = 1 << d
    for j in range(J, 0, -1):
        # parents of tree nodes are tree nodes, valued by the average of children
        par = np.unique(np.nonzero(in_tree[j])[0] >> d)
        if par.size == 0:
            continue
        ch = par[:, None] * nc + np.arange(nc)[None, :]
        s = tree_val[j][:, ch[:, 0]]
        for c in range(1, nc):
            s = s + tree_val[j][:, ch[:, c]]
        tree_val[j - 1][:, par] = s * (1.0 / nc)
        in_tree[j - 1][par] = True
    V = [tree_val[0].copy()]
    for j in range(1, J + 1):
        k = np.arange(1 << (d * j))
        pred = predict(V[j - 1], d, j - 1, k)
        V.append(np.where(in_tree[j][None, :], tree_val[j], pred))
    return V


def adapt(keys, vals, d, J, eps, scale=None, refine=True):
    """Leaf set adapted to the values of a leaf set: details on the levels of
    its reconstruction (zero at predicted nodes), flags with or without
    refinement, grading, leaves."""
    m = vals.shape[0]
    scale = np.ones(m) if scale is None else np.asarray(scale, dtype=np.float64)
    levels = tree_levels(keys, vals, d, J)
    dets = details(levels, d, J)
    R = refine_flags(levels, dets, d, J, eps, scale, refine)
    return leaf_set(levels, R, d, J)
