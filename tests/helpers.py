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
    m = aj >= 0
    rows = np.repeat(np.arange(n), 9).reshape(n, 9)[m]
    A = sp.csr_matrix((ax[m], (rows, aj[m])), shape=(n, n))
    if ex["ovf_ptr"][-1]:
        orow = np.repeat(np.arange(n), np.diff(ex["ovf_ptr"]))
        A = A + sp.csr_matrix((ex["ovf_val"], (orow, ex["ovf_col"])), shape=(n, n))
    return A.tocsr()


def level_matrix_structure(ex):
    """Boolean structure (slots present + overflow) of an exported level."""
    n = ex["n"]
    aj = ex["aj"]
    m = aj >= 0
    rows = np.repeat(np.arange(n), 9).reshape(n, 9)[m]
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
