"""Pins of the CPU oracle against what the paper and the mathematics fix (no GPU needed).

Each test ties one oracle function to something other than itself: values the paper states, closed forms, exact
rational geometry, library routines (scipy's sparse products, triangular solves, CG, direct solves) and invariants.
"""
from fractions import Fraction

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla
from hypothesis import given, settings
from hypothesis import strategies as st

from paper_1209_5421_amd import meshgen as mg
from tests import helpers as H


# ---------------------------------------------------------------------------------------------------------------
# depth rule (Section 3.1): 4^L < N, coarsest = first k with 4^k <= 64
# ---------------------------------------------------------------------------------------------------------------

@pytest.mark.parametrize("n,levels,L,kc", [
    (1, 1, -1, -1), (64, 1, -1, -1),            # N <= 64: one level, dense solve
    (65, 2, 3, 3), (256, 2, 3, 3),              # 4^3 = 64 < N <= 256 -> L = 3 (256 = 4^4 is not < 256)
    (257, 3, 4, 3), (1024, 3, 4, 3), (1025, 4, 5, 3),
    (3969, 4, 5, 3),                            # 65x65 uniform grid: level-L grid 32x32 (2x2 aggregates)
    (4096, 4, 5, 3), (4097, 5, 6, 3),
    (1_044_484, 8, 9, 3), (4_194_304, 9, 10, 3), (4_194_305, 10, 11, 3),
])
def test_depth_rule(orc, n, levels, L, kc):
    assert orc.depth(n) == (levels, L, kc)


def test_depth_rule_coarse_max(orc):
    assert orc.depth(1000, coarse_max=256) == (2, 4, 4)
    assert orc.depth(5000, coarse_max=16) == (6, 6, 2)  # levels 6,5,4,3,2 + fine


# ---------------------------------------------------------------------------------------------------------------
# level-L aggregation (eq. 9)
# ---------------------------------------------------------------------------------------------------------------

def test_uniform_grid_aggregation_is_geometric_coarsening(orc):
    """Section 5.2 states that on the uniform grid the aggregation coincides with geometric coarsening: with box
    [0,1]^2 and x = j/64 the level-5 cell is j >> 1 per axis (cell 0 holds j = 1 only)."""
    p = mg.uniform_problem(64)
    o = orc.setup_problem(p)
    ex = o.export_level(0)
    j = np.rint(p.coords * 64).astype(int)
    expect = (j[:, 1] >> 1) * 32 + (j[:, 0] >> 1)
    np.testing.assert_array_equal(ex["agg"], expect)
    sizes = np.bincount(ex["agg"], minlength=1024)
    assert (sizes > 0).all() and set(np.unique(sizes)) == {1, 2, 4}
    assert sizes[0] == 1 and sizes[33] == 4


def _exact_cell(v, a, b, s):
    if b == a:
        return 0, False
    t = (Fraction(v) - Fraction(a)) / (Fraction(b) - Fraction(a)) * s
    c = min(int(t), s - 1)  # floor for t >= 0
    near = abs(t - round(t)) < Fraction(1, 2 ** 40) * max(1, s)
    return c, near


@settings(max_examples=60, deadline=None)
@given(st.integers(min_value=0, max_value=10 ** 6), st.integers(min_value=1, max_value=12),
       st.floats(-1e3, 1e3), st.floats(1e-6, 1e3), st.floats(-1e3, 1e3), st.floats(1e-6, 1e3))
def test_cell_index_exact_containment(orc, seed, L, a1, w1, a2, w2):
    """Every point lands in the cell whose exact rational interval [a + c w, a + (c+1) w) contains it (the last cell
    closed); the FP formula may differ by one cell only for points within rounding distance of a cell edge."""
    rng = np.random.default_rng(seed)
    box = (a1, a1 + w1, a2, a2 + w2)
    pts = np.stack([rng.uniform(box[0], box[1], 200), rng.uniform(box[2], box[3], 200)], 1)
    pts[:4] = [[box[0], box[2]], [box[1], box[3]], [box[0], box[3]], [box[1], box[2]]]
    cell = orc.cell_index(pts, box, L)
    s = 2 ** L
    for (x, y), c in zip(pts, cell):
        ex, nx = _exact_cell(x, box[0], box[1], s)
        ey, ny = _exact_cell(y, box[2], box[3], s)
        cx, cy = int(c) % s, int(c) // s
        assert cx == ex or (nx and abs(cx - ex) == 1)
        assert cy == ey or (ny and abs(cy - ey) == 1)


def test_cell_index_degenerate_box(orc):
    pts = np.array([[0.5, 0.1], [0.5, 0.7], [0.5, 0.9]])
    cell = orc.cell_index(pts, (0.5, 0.5, 0.0, 1.0), 3)
    np.testing.assert_array_equal(cell % 8, 0)
    np.testing.assert_array_equal(cell // 8, [0, 5, 7])


# ---------------------------------------------------------------------------------------------------------------
# coarse aggregation (eq. 10) and pattern (Section 4.4)
# ---------------------------------------------------------------------------------------------------------------

def test_coarse_aggregation_listing_and_containment(orc):
    p = mg.jittered_problem(40)
    o = orc.setup_problem(p)
    for level in range(1, o.num_levels - 1):
        ex = o.export_level(level)
        k = ex["k"]
        side = 2 ** k
        idx = np.arange(4 ** k)
        # the coarse-level listing of Section 4.2, with its power taken as the child grid's side
        listing = ((idx // side) // 2) * (side // 2) + (idx % side) // 2
        np.testing.assert_array_equal(ex["agg"], listing)
        # geometric containment in exact arithmetic: the child rectangle lies inside the parent rectangle
        for i in idx[:: max(1, len(idx) // 50)]:
            t1, t2 = i % side, i // side
            P = ex["agg"][i]
            T1, T2 = P % (side // 2), P // (side // 2)
            assert Fraction(T1, side // 2) <= Fraction(t1, side) and Fraction(t1 + 1, side) <= Fraction(T1 + 1, side // 2)
            assert Fraction(T2, side // 2) <= Fraction(t2, side) and Fraction(t2 + 1, side) <= Fraction(T2 + 1, side // 2)


def test_pattern_matches_paper_neighbour_table(orc):
    table = H.neighbour_table()
    p = mg.jittered_problem(40)
    o = orc.setup_problem(p)
    for level in range(1, o.num_levels):
        ex = o.export_level(level)
        side = 2 ** ex["k"]
        for i in range(ex["n"]):
            t1, t2 = i % side, i // side
            for slot, (dx, dy) in enumerate(table):
                u1, u2 = t1 + dx, t2 + dy
                inside = 0 <= u1 < side and 0 <= u2 < side
                assert ex["aj"][i, slot] == (u2 * side + u1 if inside else -1)
                if not inside:
                    assert ex["ax"][i, slot] == 0.0


def test_colors_are_quadtree_parity(orc):
    p = mg.jittered_problem(40)
    o = orc.setup_problem(p)
    ex0 = o.export_level(0)
    ex1 = o.export_level(1)
    side = 2 ** ex1["k"]
    I = np.arange(ex1["n"])
    np.testing.assert_array_equal(ex1["color"], H.lex_color(I, side))
    np.testing.assert_array_equal(ex0["color"], ex1["color"][ex0["agg"]])


# ---------------------------------------------------------------------------------------------------------------
# Galerkin operators (eq. 3-4, eq. 11)
# ---------------------------------------------------------------------------------------------------------------

def _hierarchy_views(o, prob):
    """Per quadtree level: (exported level, scipy P^t A P of the previous level, |.| version, empty mask)."""
    A = H.csr_of(prob)
    absA = abs(A)
    out = []
    ex0 = o.export_level(0)
    agg = ex0["agg"]
    Aprev, absprev = A, absA
    alive = np.ones(A.shape[0])  # 1 where a row holds fine unknowns
    for level in range(1, o.num_levels):
        ex = o.export_level(level)
        P = H.prolongation(agg, ex["n"])
        G = (P.T @ Aprev @ P).tocsr()
        Gabs = (P.T @ absprev @ P).tocsr()
        # a cell is empty when none of its children holds a fine unknown (all children empty counts too)
        alive = (P.T @ alive > 0).astype(np.float64)
        nonempty = alive > 0
        out.append((ex, G, Gabs, ~nonempty, P))
        # the next level is summed from this level's true operator (empty rows zero)
        Aprev, absprev = G, Gabs
        agg = ex["agg"]
    return out


def _gamma(m):
    u = 2.0 ** -53
    return m * u / (1 - m * u)


@pytest.mark.parametrize("maker", [
    lambda: mg.uniform_problem(64),
    lambda: mg.jittered_problem(48),
    lambda: mg.jittered_problem(40, kappa_tiles=16),
    lambda: mg.graded_problem(6000),
    lambda: H.longrange_problem(3000, 150),
    lambda: mg.disk_problem(48),
])
def test_galerkin_matches_scipy_triple_product(orc, maker):
    prob = maker()
    o = orc.setup_problem(prob)
    for ex, G, Gabs, empty, P in _hierarchy_views(o, prob):
        A = H.level_matrix(ex)
        ref = G.toarray()
        ref[empty, empty] = 1.0  # identity rows of empty aggregates
        bound = 4 * _gamma(int(prob.nnz)) * Gabs.toarray() + 1e-300
        assert (np.abs(A.toarray() - ref) <= bound).all()


def test_galerkin_exact_on_uniform_grid(orc):
    """Config-1 entries are small integers at every level (exact in FP64); interior rows are 2^m times the 5-point
    stencil: 8/-2 at level 5, 16/-4 at level 4, 32/-8 at level 3."""
    prob = mg.uniform_problem(64)
    o = orc.setup_problem(prob)
    for ex, G, Gabs, empty, P in _hierarchy_views(o, prob):
        assert not empty.any()
        np.testing.assert_array_equal(H.level_matrix(ex).toarray(), G.toarray())
        k, side = ex["k"], 2 ** ex["k"]
        c = 8 * 2 ** (5 - k)
        for i in range(ex["n"]):
            t1, t2 = i % side, i // side
            if 1 <= t1 <= side - 2 and 1 <= t2 <= side - 2:
                np.testing.assert_array_equal(ex["ax"][i], [c, -c / 4, 0, -c / 4, 0, -c / 4, 0, -c / 4, 0])


@pytest.mark.parametrize("maker", [lambda: mg.graded_problem(6000), lambda: H.longrange_problem(3000, 150)])
def test_overflow_structure_brute_force(orc, maker):
    """Overflow entries are exactly the aggregate pairs more than one cell apart that some stored fine entry
    couples (zero values included), found by brute force over the fine pattern."""
    prob = maker()
    o = orc.setup_problem(prob)
    ex0 = o.export_level(0)
    A = H.csr_of(prob).tocoo()
    pairs = set(zip(ex0["agg"][A.row].tolist(), ex0["agg"][A.col].tolist()))
    total = 0
    for level in range(1, o.num_levels):
        ex = o.export_level(level)
        side = 2 ** ex["k"]
        far = {(I, J) for (I, J) in pairs
               if max(abs(I % side - J % side), abs(I // side - J // side)) > 1}
        got = set()
        for I in range(ex["n"]):
            cols = ex["ovf_col"][ex["ovf_ptr"][I]:ex["ovf_ptr"][I + 1]]
            assert (np.diff(cols) > 0).all()
            got |= {(I, int(J)) for J in cols}
        assert got == far
        total += len(got)
        S = H.level_matrix_structure(ex)
        assert abs(S - S.T).max() == 0
        nxt = ex["agg"]
        pairs = {(int(nxt[I]), int(nxt[J])) for (I, J) in pairs} if level < o.num_levels - 1 else set()
    assert total > 0


@pytest.mark.parametrize("maker", [lambda: mg.jittered_problem(40), lambda: mg.graded_problem(6000),
                                   lambda: H.longrange_problem(3000, 150)])
def test_galerkin_invariants(orc, maker):
    prob = maker()
    o = orc.setup_problem(prob)
    rng = np.random.default_rng(5)
    for ex, G, Gabs, empty, P in _hierarchy_views(o, prob):
        A = H.level_matrix(ex).toarray()
        tol = 8 * _gamma(int(prob.nnz)) * Gabs.toarray()
        # symmetry
        assert (np.abs(A - A.T) <= tol + tol.T + 1e-300).all()
        # row sums aggregate: A_c 1 = P^t (A_prev 1) on non-empty rows
        Atrue = A.copy()
        Atrue[empty, empty] = 0.0
        rs = Atrue.sum(1)
        rs_ref = np.asarray(G.sum(1)).ravel()
        assert np.allclose(rs, rs_ref, rtol=0, atol=1e-9 * np.abs(Gabs).sum(1).max())
        # energy: v^t A_c v = (P v)^t A_prev (P v)
        v = rng.standard_normal(ex["n"])
        v[empty] = 0
        assert np.isclose(v @ Atrue @ v, v @ (G @ v), rtol=1e-11)
        # SPD
        assert np.linalg.eigvalsh(A).min() > 0


# ---------------------------------------------------------------------------------------------------------------
# smoother (Section 4.5)
# ---------------------------------------------------------------------------------------------------------------

def _block_splitting(A, color, cell, forward, block_max=32):
    """Matrix form of one sweep of the exact-block smoother: x_new = x + M^{-1}(f - A x), where M keeps, for the
    forward sweep, the couplings to earlier colors and the whole diagonal block of every cell of at most block_max
    unknowns (the cells of one color see each other's phase-start values, so couplings between distinct cells of
    one color are dropped); larger cells keep the lower (forward) / upper (backward) triangle of their block.
    Backward: later colors."""
    A = sp.csr_matrix(A)
    C = A.tocoo()
    i, j, v = C.row, C.col, C.data
    size = np.bincount(cell)[cell]
    same = cell[i] == cell[j]
    earlier = (color[j] < color[i]) if forward else (color[j] > color[i])
    tri = (j <= i) if forward else (j >= i)
    keep = (earlier & ~same) | (same & ((size[i] <= block_max) | tri))
    return sp.csr_matrix((v[keep], (i[keep], j[keep])), shape=A.shape)


@pytest.mark.parametrize("maker", [lambda: mg.jittered_problem(40), lambda: mg.graded_problem(6000),
                                   lambda: mg.jittered_problem(30, kappa_tiles=16), lambda: mg.disk_problem(48)])
def test_block_smoother_is_block_splitting(orc, maker):
    """The exact-block reading of the fine smoother (the cells' diagonal blocks solved exactly): one sweep equals
    the block splitting above, forward and backward, from zero and from a nonzero start."""
    prob = maker()
    o = orc.setup_problem(prob)
    o.set_block_smoother(True)
    A = H.csr_of(prob)
    ex0 = o.export_level(0)
    cell, color = ex0["agg"].astype(np.int64), ex0["color"].astype(np.int64)
    rng = np.random.default_rng(5)
    f = rng.standard_normal(prob.n)
    x0 = rng.standard_normal(prob.n)
    for forward in (True, False):
        M = _block_splitting(A, color, cell, forward).tocsc()
        np.testing.assert_allclose(o.smooth(0, f, np.zeros(prob.n), forward), spla.spsolve(M, f),
                                   rtol=1e-9, atol=1e-11)
        np.testing.assert_allclose(o.smooth(0, f, x0, forward), x0 + spla.spsolve(M, f - A @ x0),
                                   rtol=1e-9, atol=1e-10)


def test_block_smoother_single_cell_is_exact(orc):
    """When every unknown lies in one level-L cell (a cluster in a large box), one forward sweep from zero is the
    exact solve of A x = f (only that cell's color has unknowns); the substitution reading is not."""
    pts = 0.05 + 0.05 * H.scattered_points(30, 8)
    A = H.graph_laplacian_problem(pts, 8)
    o = orc.Oracle(pts, A.indptr.astype(np.int64), A.indices.astype(np.int32), A.data, box=(0, 1, 0, 1),
                   coarse_max=4)
    assert o.num_levels > 1 and len(np.unique(o.export_level(0)["agg"])) == 1
    f = np.random.default_rng(2).standard_normal(30)
    xs = np.linalg.solve(A.toarray(), f)
    assert np.linalg.norm(o.smooth(0, f, np.zeros(30), True) - xs) > 1e-6 * np.linalg.norm(xs)
    o.set_block_smoother(True)
    np.testing.assert_allclose(o.smooth(0, f, np.zeros(30), True), xs, rtol=1e-12, atol=1e-14)
    o.set_block_smoother(False)
    assert np.linalg.norm(o.smooth(0, f, np.zeros(30), True) - xs) > 1e-6 * np.linalg.norm(xs)


def test_block_smoother_preconditioner_symmetric(orc):
    """R_k and R_k^t stay adjoint with exact blocks, so the two-level B^ (fine smoothing around the exact coarsest
    solve, a linear map) stays symmetric: (B u, v) = (u, B v)."""
    prob = mg.jittered_problem(16, kappa_tiles=4)
    o = orc.setup_problem(prob)
    assert o.num_levels == 2
    o.set_block_smoother(True)
    rng = np.random.default_rng(9)
    u, v = rng.standard_normal(prob.n), rng.standard_normal(prob.n)
    bu, bv = o.apply_precond(u), o.apply_precond(v)
    assert abs(bu @ v - u @ bv) <= 1e-11 * abs(bu @ v)
    assert u @ bu > 0 and v @ bv > 0


@pytest.mark.parametrize("maker", [lambda: mg.jittered_problem(40), lambda: mg.graded_problem(6000),
                                   lambda: mg.jittered_problem(30, kappa_tiles=16)])
def test_fine_sweep_is_triangular_solve(orc, maker):
    prob = maker()
    o = orc.setup_problem(prob)
    A = H.csr_of(prob)
    ex0 = o.export_level(0)
    cell, color = ex0["agg"], ex0["color"].astype(np.int64)
    idx = np.arange(prob.n)
    Mf = H.sweep_splitting(A, color, cell, idx)
    same_color_coupled = ((color[A.tocoo().row] == color[A.tocoo().col]) &
                          (cell[A.tocoo().row] != cell[A.tocoo().col])).any()
    rng = np.random.default_rng(1)
    f = rng.standard_normal(prob.n)
    x0 = rng.standard_normal(prob.n)
    if not same_color_coupled:
        # a valid coloring: the sweep is plain Gauss-Seidel in (color, cell, index) order = lower triangular solve
        perm = np.lexsort((idx, cell, color))
        Ap = A[perm][:, perm]
        xp = spla.spsolve_triangular(sp.tril(Ap).tocsr(), f[perm], lower=True)
        x_ref = np.empty_like(xp); x_ref[perm] = xp
    else:
        x_ref = spla.spsolve(Mf.tocsc(), f)
    np.testing.assert_allclose(o.smooth(0, f, np.zeros(prob.n), True), x_ref, rtol=1e-10, atol=1e-12)
    # from a nonzero start: x + M_f^{-1}(f - A x); backward sweep: x + M_f^{-t}(f - A x)
    fwd = x0 + spla.spsolve(Mf.tocsc(), f - A @ x0)
    bwd = x0 + spla.spsolve(Mf.T.tocsc(), f - A @ x0)
    np.testing.assert_allclose(o.smooth(0, f, x0, True), fwd, rtol=1e-9, atol=1e-10)
    np.testing.assert_allclose(o.smooth(0, f, x0, False), bwd, rtol=1e-9, atol=1e-10)


@pytest.mark.parametrize("maker", [lambda: mg.graded_problem(6000), lambda: H.longrange_problem(3000, 150)])
def test_coarse_sweep_is_four_color_gauss_seidel(orc, maker):
    prob = maker()
    o = orc.setup_problem(prob)
    rng = np.random.default_rng(2)
    for level in range(1, o.num_levels - 1):
        ex = o.export_level(level)
        A = H.level_matrix(ex)
        I = np.arange(ex["n"])
        Mf = H.sweep_splitting(A, ex["color"].astype(np.int64), I, I)
        f = rng.standard_normal(ex["n"])
        x0 = rng.standard_normal(ex["n"])
        np.testing.assert_allclose(o.smooth(level, f, x0, True), x0 + spla.spsolve(Mf.tocsc(), f - A @ x0),
                                   rtol=1e-9, atol=1e-9)
        np.testing.assert_allclose(o.smooth(level, f, x0, False), x0 + spla.spsolve(Mf.T.tocsc(), f - A @ x0),
                                   rtol=1e-9, atol=1e-9)


# ---------------------------------------------------------------------------------------------------------------
# Algorithm 2.1 special cases
# ---------------------------------------------------------------------------------------------------------------

def _textbook_cg(A, b, k):
    x = np.zeros_like(b); r = b.copy(); p = r.copy(); rr = r @ r
    for _ in range(k):
        q = A @ p; a = rr / (p @ q); x = x + a * p; r = r - a * q
        rr2 = r @ r; p = r + (rr2 / rr) * p; rr = rr2
    return x


@pytest.mark.parametrize("steps", [1, 2, 3, 6])
def test_nlpcg_identity_is_cg(orc, steps):
    prob = mg.jittered_problem(20)
    A = H.csr_of(prob)
    u = orc.nlpcg_test(prob.row_ptr, prob.col, prob.val, prob.b, steps, 0)
    x_cg = spla.cg(A, prob.b, x0=np.zeros(prob.n), rtol=0.0, atol=0.0, maxiter=steps)[0]
    np.testing.assert_allclose(u, x_cg, rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(u, _textbook_cg(A, prob.b, steps), rtol=1e-9, atol=1e-12)


def test_nlpcg_exact_preconditioner_one_step(orc):
    prob = mg.jittered_problem(14)
    A = H.csr_of(prob).toarray()
    u = orc.nlpcg_test(prob.row_ptr, prob.col, prob.val, prob.b, 2, 1)
    np.testing.assert_allclose(u, np.linalg.solve(A, prob.b), rtol=1e-12, atol=1e-14)


# ---------------------------------------------------------------------------------------------------------------
# restriction and prolongation on every level (Section 4.3)
# ---------------------------------------------------------------------------------------------------------------

@pytest.mark.parametrize("maker", [lambda: mg.jittered_problem(70), lambda: mg.graded_problem(6000),
                                   lambda: H.longrange_problem(3000, 150), lambda: mg.disk_problem(48)])
def test_transfers_equal_aggregation_matrix_on_every_level(orc, maker):
    """fc = P^t r and u + P e at every level l (fine -> L and every k -> k-1), with P_{i,agg(i)} = 1 built from the
    exported aggregates (pinned above by exact containment), element by element."""
    prob = maker()
    o = orc.setup_problem(prob)
    assert o.num_levels >= 4
    rng = np.random.default_rng(7)
    for level in range(o.num_levels - 1):
        n = prob.n if level == 0 else o.level_info(level)["n"]
        nc = o.level_info(level + 1)["n"]
        P = H.prolongation(o.export_level(level)["agg"], nc)
        # integers in FP64: every sum is exact, so the comparison is exact whatever the summation order
        r = rng.integers(-1000, 1000, n).astype(np.float64)
        e = rng.integers(-1000, 1000, nc).astype(np.float64)
        u = rng.integers(-1000, 1000, n).astype(np.float64)
        np.testing.assert_array_equal(o.restrict(level, r), P.T @ r, err_msg=f"restriction at level {level}")
        np.testing.assert_array_equal(o.prolong_add(level, e, u), u + P @ e, err_msg=f"prolongation at level {level}")


# ---------------------------------------------------------------------------------------------------------------
# Algorithm 2.2: closed forms
# ---------------------------------------------------------------------------------------------------------------

def _two_level_matrix(o, prob, A_dense, coarse_level_ex, agg, exact_coarse):
    n = prob.n
    ex0 = o.export_level(0)
    Mf = H.sweep_splitting(sp.csr_matrix(A_dense), ex0["color"].astype(np.int64), ex0["agg"], np.arange(n)).toarray()
    P = H.prolongation(agg, coarse_level_ex["n"]).toarray()
    Ac = exact_coarse
    Mfi = np.linalg.inv(Mf)
    Mbi = np.linalg.inv(Mf.T)
    I = np.eye(n)
    # u1 = Mf^{-1} f; u2 = u1 + P Ac^{-1} P^t (f - A u1); B f = u2 + Mb^{-1}(f - A u2)
    U1 = Mfi
    U2 = U1 + P @ np.linalg.solve(Ac, P.T @ (I - A_dense @ U1))
    return U2 + Mbi @ (I - A_dense @ U2)


def test_two_level_kcycle_closed_form_and_symmetry(orc):
    prob = mg.jittered_problem(16)  # 196 unknowns: fine level + level 3 (coarsest, exact)
    o = orc.setup_problem(prob)
    assert o.num_levels == 2
    A = H.csr_of(prob).toarray()
    ex1 = o.export_level(1)
    Ac = H.level_matrix(ex1).toarray()
    B = _two_level_matrix(o, prob, A, ex1, o.export_level(0)["agg"], Ac)
    Bo = np.stack([o.apply_precond(e) for e in np.eye(prob.n)], 1)
    np.testing.assert_allclose(Bo, B, rtol=0, atol=1e-12 * np.abs(B).max())
    assert np.abs(Bo - Bo.T).max() <= 1e-12 * np.abs(Bo).max()


def test_kcycle_with_converged_inner_solve_equals_two_level(orc):
    """With many inner steps, B~_{L} converges to A_L^{-1}, so the 3-level cycle equals the 2-level operator with an
    exact level-L solve: this pins the recursion wiring below the first coarse level."""
    prob = mg.jittered_problem(26)  # 576 unknowns: fine, level 4, level 3
    o = orc.setup_problem(prob, inner_iters=60)
    assert o.num_levels == 3
    A = H.csr_of(prob).toarray()
    ex1 = o.export_level(1)
    AL = H.level_matrix(ex1).toarray()
    B = _two_level_matrix(o, prob, A, ex1, o.export_level(0)["agg"], AL)
    rng = np.random.default_rng(3)
    for _ in range(3):
        f = rng.standard_normal(prob.n)
        np.testing.assert_allclose(o.apply_precond(f), B @ f, rtol=0, atol=1e-9 * np.abs(B @ f).max())


# ---------------------------------------------------------------------------------------------------------------
# outer solve
# ---------------------------------------------------------------------------------------------------------------

def test_single_level_direct(orc):
    prob = mg.jittered_problem(9)  # 49 unknowns <= 64: dense Cholesky only
    o = orc.setup_problem(prob)
    assert o.num_levels == 1
    x, info = o.solve(prob.b, tol=1e-12)
    assert info["status"] == 0 and info["iters"] <= 2
    np.testing.assert_allclose(x, np.linalg.solve(H.csr_of(prob).toarray(), prob.b), rtol=1e-12)


@pytest.mark.parametrize("maker", [lambda: mg.uniform_problem(64), lambda: mg.jittered_problem(64),
                                   lambda: mg.jittered_problem(60, kappa_tiles=16), lambda: mg.graded_problem(20000),
                                   lambda: mg.disk_problem(72)])
def test_solve_matches_direct_solver(orc, maker):
    prob = maker()
    o = orc.setup_problem(prob)
    A = H.csr_of(prob)
    x, info = o.solve(prob.b, tol=1e-8)
    assert info["status"] == 0 and info["relres"] <= 1e-8
    xs = spla.spsolve(A.tocsc(), prob.b)
    np.testing.assert_allclose(np.linalg.norm(A @ x - prob.b) / np.linalg.norm(prob.b), info["relres"], rtol=1e-6)
    # ||x - x*|| / ||x*|| <= cond(A) * relres; cond from extreme eigenvalues
    lmax = spla.eigsh(A, k=1, which="LA", return_eigenvectors=False)[0]
    lmin = spla.eigsh(A, k=1, sigma=0, which="LM", return_eigenvectors=False)[0]
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) <= (lmax / lmin) * info["relres"]


def test_iterations_roughly_mesh_independent(orc):
    """The K-cycle aims at uniform convergence (Section 2): counts stay flat as the mesh is refined."""
    its = []
    for side in (34, 66, 130, 258):
        prob = mg.jittered_problem(side)
        its.append(orc.setup_problem(prob).solve(prob.b, tol=1e-8)[1]["iters"])
    assert max(its) - min(its) <= 5, its


def test_zero_rhs_and_verbatim_mode(orc):
    prob = mg.jittered_problem(30)
    o = orc.setup_problem(prob)
    x, info = o.solve(np.zeros(prob.n))
    assert info["iters"] == 0 and not x.any()
    x1, i1 = o.solve(prob.b, mmax=1)
    xa, ia = o.solve(prob.b, mmax=-1)
    assert i1["status"] == ia["status"] == 0
    np.testing.assert_allclose(x1, xa, rtol=1e-6, atol=1e-9)


def test_restart_from_true_residual(orc):
    """A forced restart after k iterations: the iteration must continue from the true residual b - A x_k with its
    direction history cleared, i.e. equal x_k plus a fresh solve of A d = b - A x_k stopped at the same absolute
    residual; both end at the true-residual tolerance."""
    prob = mg.jittered_problem(66)
    o = orc.setup_problem(prob)
    A = H.csr_of(prob)
    b, tol, k = prob.b, 1e-8, 4
    x_k, i_k = o.solve(b, tol=tol, max_iters=k)
    assert i_k["status"] == orc.NOCONV and i_k["iters"] == k
    t = b - A @ x_k
    d, i_d = o.solve(t, tol=tol * np.linalg.norm(b) / np.linalg.norm(t))
    x_r, i_r = o.solve_forced_restart(b, k, tol=tol)
    assert i_r["status"] == 0 and i_r["relres"] <= tol
    assert abs(i_r["iters"] - (k + i_d["iters"])) <= 1, (i_r, i_d)
    assert np.linalg.norm(x_r - (x_k + d)) <= 1e-10 * np.linalg.norm(x_r)
    x_n, i_n = o.solve(b, tol=tol)
    assert np.linalg.norm(x_r - x_n) <= 1e-6 * np.linalg.norm(x_n)


def test_disk_empty_cells(orc):
    """On the disk inside the unit square, the level-L cells without a point are the ones outside the circle or
    nearly so: their share approaches 1 - pi/4 (0.215) as L grows; every quadtree level keeps exactly 4^k rows, and
    each empty row is the identity row (eq. 10 on a non-rectangular domain)."""
    prob = mg.disk_problem(130)
    o = orc.setup_problem(prob)
    agg = o.export_level(0)["agg"]
    ex1 = o.export_level(1)
    assert ex1["n"] == 4 ** ex1["k"]
    share = (np.bincount(agg, minlength=ex1["n"]) == 0).mean()
    assert 0.17 < share < 0.215, share
    for ex, G, Gabs, empty, P in _hierarchy_views(o, prob):
        assert ex["n"] == 4 ** ex["k"]
        assert empty.any()
        A = H.level_matrix(ex).toarray()
        np.testing.assert_array_equal(A[np.ix_(empty, np.arange(ex["n"]))], np.eye(ex["n"])[empty])


def test_empty_cells_equal_compacted_operator(orc):
    """A point set with a hole leaves aggregates empty; their identity rows decouple, so the solve equals the direct
    solution and the non-empty block equals P^t A P on the non-empty aggregates."""
    rng = np.random.default_rng(4)
    pts = H.scattered_points(3000, 4)
    pts = pts[np.hypot(pts[:, 0] - 0.5, pts[:, 1] - 0.5) > 0.3]
    A = H.graph_laplacian_problem(pts, 4)
    o = orc.Oracle(pts, A.indptr, A.indices, A.data, box=(0, 1, 0, 1))
    ex0 = o.export_level(0)
    ex1 = o.export_level(1)
    P = H.prolongation(ex0["agg"], ex1["n"])
    ne = np.asarray(P.sum(0)).ravel() > 0
    assert (~ne).sum() > 10
    G = (P.T @ A @ P).toarray()
    Al = H.level_matrix(ex1).toarray()
    np.testing.assert_allclose(Al[np.ix_(ne, ne)], G[np.ix_(ne, ne)], rtol=1e-12, atol=1e-12)
    assert (Al[np.ix_(~ne, ~ne)] == np.eye((~ne).sum())).all()
    b = rng.standard_normal(len(pts))
    x, info = o.solve(b, tol=1e-10)
    assert info["status"] == 0
    np.testing.assert_allclose(x, spla.spsolve(A.tocsc(), b), rtol=1e-7, atol=1e-9)


# ---------------------------------------------------------------------------------------------------------------
# error behaviour
# ---------------------------------------------------------------------------------------------------------------

def test_invalid_inputs(orc):
    prob = mg.jittered_problem(12)
    args = [prob.coords, prob.row_ptr, prob.col, prob.val]
    bad_rp = prob.row_ptr.copy(); bad_rp[5] = bad_rp[4] - 1
    bad_col = prob.col.copy(); bad_col[3] = prob.n
    nan_xy = prob.coords.copy(); nan_xy[2, 1] = np.nan
    for a in ([prob.coords, bad_rp, prob.col, prob.val], [prob.coords, prob.row_ptr, bad_col, prob.val],
              [nan_xy, prob.row_ptr, prob.col, prob.val]):
        with pytest.raises(orc.OracleError) as e:
            orc.Oracle(*a)
        assert e.value.code == orc.INVALID
    with pytest.raises(orc.OracleError) as e:
        orc.Oracle(*args, box=(0.2, 1.0, 0.0, 1.0))
    assert e.value.code == orc.INVALID
    neg = prob.val.copy()
    rows = np.repeat(np.arange(prob.n), np.diff(prob.row_ptr))
    neg[(rows == 7) & (prob.col == 7)] = -1.0
    with pytest.raises(orc.OracleError) as e:
        orc.Oracle(prob.coords, prob.row_ptr, prob.col, neg)
    assert e.value.code == orc.NOT_SPD
