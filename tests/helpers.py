"""Test-side matrix views of an exported hierarchy (lexicographic numbering), built with numpy/scipy."""
import os

import numpy as np
import scipy.sparse as sp

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def neighbour_table():
    rows = []
    with open(os.path.join(GOLDEN, "neighbours_sec4_4.txt")) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append([int(v) for v in line.split()])
    rows.sort()
    return [(dx, dy) for _, dx, dy in rows]


def prolongation(agg, n_coarse):
    """P_ij = 1 iff unknown i lies in aggregate j (eq. 2)."""
    n = len(agg)
    return sp.csr_matrix((np.ones(n), (np.arange(n), agg)), shape=(n, n_coarse))


def level_matrix(ex):
    """Sparse matrix of an exported quadtree level (9 slots + overflow), lexicographic numbering."""
    n = ex["n"]
    aj, ax = ex["aj"], ex["ax"]
    ns = aj.shape[1]
    m = aj >= 0
    rows = np.repeat(np.arange(n), ns).reshape(n, ns)[m]
    A = sp.csr_matrix((ax[m], (rows, aj[m])), shape=(n, n))
    if ex["ovf_ptr"][-1]:
        orow = np.repeat(np.arange(n), np.diff(ex["ovf_ptr"]))
        A = A + sp.csr_matrix((ex["ovf_val"], (orow, ex["ovf_col"])), shape=(n, n))
    return A.tocsr()


def level_matrix_structure(ex):
    """Boolean structure (slots present + overflow) of an exported level."""
    n = ex["n"]
    aj = ex["aj"]
    ns = aj.shape[1]
    m = aj >= 0
    rows = np.repeat(np.arange(n), ns).reshape(n, ns)[m]
    S = sp.csr_matrix((np.ones(m.sum()), (rows, aj[m])), shape=(n, n))
    if ex["ovf_ptr"][-1]:
        orow = np.repeat(np.arange(n), np.diff(ex["ovf_ptr"]))
        S = S + sp.csr_matrix((np.ones(len(orow)), (orow, ex["ovf_col"])), shape=(n, n))
    return S.tocsr()


def empty_rows(ex):
    """Rows whose stored row is the identity placeholder of an empty aggregate."""
    return ex.get("empty")


def lex_color(I, side):
    return (I % side) % 2 + 2 * ((I // side) % 2)


def sweep_splitting(A, color, cell, order_key):
    """Matrix form of one colored sweep: returns M_f with x_new = x + M_f^{-1}(f - A x) for the forward sweep (colors
    ascending, unknowns ascending inside a cell) when the color phase uses the residual at phase start. In the
    (color, cell, index) ordering M_f is the lower triangle of A with couplings between distinct cells of the same
    color removed (those see the phase-start iterate, i.e. they act like Jacobi)."""
    A = sp.csr_matrix(A)
    n = A.shape[0]
    perm = np.lexsort((order_key, cell, color))
    pos = np.empty(n, dtype=np.int64)
    pos[perm] = np.arange(n)
    C = A.tocoo()
    i, j, v = C.row, C.col, C.data
    keep = (pos[j] <= pos[i]) & ~((color[i] == color[j]) & (cell[i] != cell[j]))
    return sp.csr_matrix((v[keep], (i[keep], j[keep])), shape=(n, n))


def csr_of(prob):
    return sp.csr_matrix((prob.val, prob.col, prob.row_ptr), shape=(prob.n, prob.n))


def scattered_points_3d(n, seed):
    return np.random.default_rng(seed).uniform(0.0, 1.0, (n, 3))


def longrange_problem_3d(n=3000, extra=200, seed=12):
    """Scattered points in the unit cube, 3D Delaunay graph Laplacian with random positive weights plus `extra`
    long-range couplings and a positive shift: SPD, overflowing the 27-point pattern on every octree level."""
    from paper_1209_5421_amd import meshgen as mg
    from scipy.spatial import Delaunay
    rng = np.random.default_rng(seed)
    pts = scattered_points_3d(n, seed)
    tet = Delaunay(pts).simplices
    e = np.concatenate([tet[:, [a, b]] for a in range(4) for b in range(a + 1, 4)])
    e = np.unique(np.sort(e, 1), axis=0)
    i = rng.integers(0, n, extra)
    j = rng.integers(0, n, extra)
    e = np.concatenate([e, np.stack([i[i != j], j[i != j]], 1)])
    w = rng.uniform(0.5, 2.0, len(e))
    W = sp.csr_matrix((np.concatenate([-w, -w]), (np.concatenate([e[:, 0], e[:, 1]]),
                                                   np.concatenate([e[:, 1], e[:, 0]]))), shape=(n, n))
    d = -np.asarray(W.sum(1)).ravel() + rng.uniform(0.01, 0.1, n)
    A = (W + sp.diags(d)).tocsr()
    A.sum_duplicates()
    A.sort_indices()
    b = rng.uniform(-1, 1, n)
    return mg.Problem(f"longrange3d{n}", pts, A.indptr.astype(np.int64), A.indices.astype(np.int32),
                      A.data.astype(np.float64), b, None, dict(kind="longrange3d"))


def scattered_points(n, seed, box=(0.0, 1.0, 0.0, 1.0)):
    rng = np.random.default_rng(seed)
    x = rng.uniform(box[0], box[1], n)
    y = rng.uniform(box[2], box[3], n)
    return np.stack([x, y], 1)


def graph_laplacian_problem(coords, seed=0):
    """SPD test matrix on arbitrary points: Delaunay graph Laplacian with random positive edge weights plus a
    positive diagonal shift (keeps the system SPD for any point set)."""
    from scipy.spatial import Delaunay
    rng = np.random.default_rng(seed)
    n = len(coords)
    tri = Delaunay(coords).simplices
    e = np.concatenate([tri[:, [0, 1]], tri[:, [1, 2]], tri[:, [2, 0]]])
    e = np.unique(np.sort(e, 1), axis=0)
    w = rng.uniform(0.5, 2.0, len(e))
    W = sp.csr_matrix((np.concatenate([-w, -w]), (np.concatenate([e[:, 0], e[:, 1]]),
                                                   np.concatenate([e[:, 1], e[:, 0]]))), shape=(n, n))
    d = -np.asarray(W.sum(1)).ravel() + rng.uniform(0.01, 0.1, n)
    A = (W + sp.diags(d)).tocsr()
    A.sort_indices()
    return A


def longrange_problem(n=6000, extra=300, seed=11):
    """Scattered points, Delaunay graph Laplacian plus `extra` random long-range couplings and a positive shift:
    SPD, and its couplings overflow the 9-point pattern on every quadtree level. No box is given (bounding box)."""
    import scipy.sparse as sp
    from paper_1209_5421_amd import meshgen as mg
    rng = np.random.default_rng(seed)
    pts = scattered_points(n, seed)
    A = graph_laplacian_problem(pts, seed)
    i = rng.integers(0, n, extra)
    j = rng.integers(0, n, extra)
    keep = i != j
    i, j = i[keep], j[keep]
    w = rng.uniform(0.1, 1.0, len(i))
    W = sp.csr_matrix((np.concatenate([-w, -w]), (np.concatenate([i, j]), np.concatenate([j, i]))), shape=(n, n))
    D = sp.diags(np.asarray(-W.sum(1)).ravel())
    A = (A + W + D).tocsr()
    A.sum_duplicates()
    A.sort_indices()
    b = rng.uniform(-1, 1, n)
    return mg.Problem(f"longrange{n}", pts, A.indptr.astype(np.int64), A.indices.astype(np.int32),
                      A.data.astype(np.float64), b, None, dict(kind="longrange"))


def wheel_mesh(spokes=40, rings=3, seed=4):
    """A disk of `rings` rings of `spokes` points around a centre, each ring joined to the next by 2 * spokes
    triangles and the centre to the first ring by a fan: the centre lies in `spokes` triangles, so its diagonal entry
    sums `spokes` element entries. The outer ring is the Dirichlet boundary. Returns (points, tris, dirichlet)."""
    rng = np.random.default_rng(seed)
    pts = [(0.5, 0.5)]
    for r in range(1, rings + 1):
        rad = 0.45 * r / rings
        for k in range(spokes):
            a = 2 * np.pi * (k + 0.2 * rng.uniform(-1, 1) * (r < rings)) / spokes + 0.1 * r
            pts.append((0.5 + rad * np.cos(a), 0.5 + rad * np.sin(a)))
    pts = np.array(pts)
    ring = lambda r, k: 1 + (r - 1) * spokes + (k % spokes)
    tris = [(0, ring(1, k), ring(1, k + 1)) for k in range(spokes)]
    for r in range(1, rings):
        for k in range(spokes):
            tris.append((ring(r, k), ring(r + 1, k), ring(r + 1, k + 1)))
            tris.append((ring(r, k), ring(r + 1, k + 1), ring(r, k + 1)))
    tris = np.array(tris, dtype=np.int64)
    tris[1::2] = tris[1::2][:, [0, 2, 1]]  # mixed orientation: half the triangles clockwise
    dirichlet = np.zeros(len(pts), dtype=bool)
    dirichlet[1 + (rings - 1) * spokes:] = True
    return pts, tris, dirichlet


def assembly_in_stated_order(pts, tris, kappa, dirichlet):
    """Stored entries of the P1 stiffness matrix in the evaluation order the device assembly states: element
    entries in the order (a, b, triangle) per stored (row, column); the first entry plus the others' sum, sequential
    from 0 below eight terms, else eight interleaved partial sums combined pairwise, then the remainder."""
    tris = np.asarray(tris, dtype=np.int64).copy()
    a0, b0, c0 = pts[tris[:, 0]], pts[tris[:, 1]], pts[tris[:, 2]]
    s = (b0[:, 0] - a0[:, 0]) * (c0[:, 1] - a0[:, 1]) - (b0[:, 1] - a0[:, 1]) * (c0[:, 0] - a0[:, 0])
    tris[s < 0] = tris[s < 0][:, [0, 2, 1]]
    P = [pts[tris[:, k]] for k in range(3)]
    E = [P[2] - P[1], P[0] - P[2], P[1] - P[0]]
    kap = np.ones(len(tris)) if kappa is None else kappa
    dof = np.full(len(pts), -1)
    dof[~dirichlet] = np.arange(int((~dirichlet).sum()))
    terms = {}
    for a in range(3):
        for b in range(3):
            v = kap * (E[a][:, 0] * E[b][:, 0] + E[a][:, 1] * E[b][:, 1]) / (2.0 * np.abs(s))
            for t in range(len(tris)):
                r, c = dof[tris[t, a]], dof[tris[t, b]]
                if r >= 0 and c >= 0:
                    terms.setdefault((r, c), []).append(v[t])

    def rest_sum(x):
        if len(x) < 8:
            acc = 0.0
            for v in x:
                acc = acc + v
            return acc
        p = list(x[:8])
        i = 8
        while i + 8 <= len(x):
            for j in range(8):
                p[j] = p[j] + x[i + j]
            i += 8
        acc = ((p[0] + p[1]) + (p[2] + p[3])) + ((p[4] + p[5]) + (p[6] + p[7]))
        for v in x[i:]:
            acc = acc + v
        return acc

    keys = sorted(terms)
    vals = np.array([terms[k][0] + rest_sum(terms[k][1:]) if len(terms[k]) > 1 else terms[k][0] for k in keys])
    n = int((~dirichlet).sum())
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(row_ptr, np.array([k[0] for k in keys]) + 1, 1)
    return np.cumsum(row_ptr), np.array([k[1] for k in keys], dtype=np.int32), vals


def cluster_problem(side=100, cluster=13000, seed=21):
    """Poisson on a Delaunay mesh of a jittered side x side lattice of the unit square plus `cluster` uniform random
    points inside one level-L cell (L = 7 for the sizes here: cell (51, 51), [51/128, 52/128)^2), so that one cell
    holds more unknowns than the big-cell substitution stages in LDS. Dirichlet on the square's boundary."""
    from paper_1209_5421_amd import meshgen as mg
    lat = mg.jittered_points(side, seed)
    rng = np.random.default_rng(seed)
    lo, hi = 51 / 128 + 1e-4, 52 / 128 - 1e-4
    pts = np.vstack([lat, lo + (hi - lo) * rng.random((cluster, 2))])
    tris = mg.delaunay(pts)
    return mg._problem(f"cluster{side}_{cluster}", pts, tris, kind="cluster", side=side, cluster=cluster, seed=seed)
