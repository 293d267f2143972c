"""Seeded synthetic problem generators: 2D P1 finite-element systems on the unit square.

This module holds the workloads only (meshes, stiffness matrices, right-hand sides). It contains none of the
multigrid method's arithmetic, so both the HIP path and the CPU oracle take their inputs from here.

The paper measures the P1 discretisation of the 2D Poisson problem with homogeneous Dirichlet data (Example 1,
Section 5.2) on uniform, quasi-uniform and shape-regular triangulations of the unit square (Tables 2-4). Its meshes
are not published, so these generators build stand-ins of the same kind:

* ``uniform``: (m+1)x(m+1) vertices, each square cut by its (i,j)-(i+1,j+1) diagonal (Table 2's grid).
* ``jittered``: a lattice whose interior points move by U[-0.3h, 0.3h] per coordinate, Delaunay-triangulated
  (quasi-uniform, Table 3's kind).
* ``graded``: quadtree-leaf sampling with local spacing c*(r+0.01)^0.75 towards the corner (0,0), Delaunay-
  triangulated (shape-regular with strong grading, Table 4's kind).
* ``kappa``: a 16x16 checkerboard of diffusion coefficients 10^U[-3,3] for -div(kappa grad u) = f.
* ``cube``: the 3D variant (Example 2's unit cube, Tables 6-7): one implicit Euler step of the heat equation,
  (M / dt + K) T = f, on a jittered (m+1)^3 lattice cut into six tetrahedra per cube (Kuhn), linear elements with a
  lumped mass, the inlet face x = 0 held fixed (eliminated), no-flux elsewhere.

Seeds follow ``numpy.random.default_rng``: mesh 0, right-hand side 1, kappa 2, request stream 3.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

SEED_MESH, SEED_RHS, SEED_KAPPA, SEED_STREAM = 0, 1, 2, 3
UNIT_BOX = (0.0, 1.0, 0.0, 1.0)
UNIT_CUBE = (0.0, 1.0, 0.0, 1.0, 0.0, 1.0)


@dataclasses.dataclass
class Problem:
    """An SPD system A x = b with the coordinates of its unknowns.

    ``coords`` is (n, 2) float64 (x, y interleaved), or (n, 3) for the 3D workload; ``row_ptr`` int64 (n+1),
    ``col`` int32, ``val`` float64 form a 0-based CSR matrix with columns ascending inside each row (explicit zeros
    of the stencil kept); ``box`` is the domain's bounding box (a1, b1, a2, b2[, a3, b3]).
    """
    name: str
    coords: np.ndarray
    row_ptr: np.ndarray
    col: np.ndarray
    val: np.ndarray
    b: np.ndarray
    box: tuple
    meta: dict

    @property
    def n(self) -> int:
        return int(self.coords.shape[0])

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def scipy(self):
        import scipy.sparse as sp
        return sp.csr_matrix((self.val, self.col, self.row_ptr), shape=(self.n, self.n))


# ----------------------------------------------------------------------------------------------------------------
# meshes
# ----------------------------------------------------------------------------------------------------------------

def _on_unit_boundary(p: np.ndarray) -> np.ndarray:
    return (p[:, 0] == 0.0) | (p[:, 0] == 1.0) | (p[:, 1] == 0.0) | (p[:, 1] == 1.0)


def uniform_mesh(m: int):
    """(m+1)^2 vertices at (i/m, j/m); each square split by its (i,j)-(i+1,j+1) diagonal."""
    g = np.arange(m + 1, dtype=np.float64) / m
    X, Y = np.meshgrid(g, g)  # row j = y index
    pts = np.stack([X.ravel(), Y.ravel()], 1)
    i, j = np.meshgrid(np.arange(m), np.arange(m))
    v00 = (j * (m + 1) + i).ravel()
    v10, v11, v01 = v00 + 1, v00 + m + 2, v00 + m + 1
    tris = np.concatenate([np.stack([v00, v10, v11], 1), np.stack([v00, v11, v01], 1)])
    return pts, tris


def jittered_points(side: int, seed: int = SEED_MESH, jitter: float = 0.3):
    """side x side lattice on [0,1]^2 (h = 1/(side-1)); interior points moved by U[-jitter h, jitter h]."""
    rng = np.random.default_rng(seed)
    h = 1.0 / (side - 1)
    g = np.arange(side, dtype=np.float64) / (side - 1)
    jit = rng.uniform(-jitter * h, jitter * h, size=(side * side, 2))
    P = np.empty((side, side, 2))
    P[..., 0] = g[None, :]
    P[..., 1] = g[:, None]
    # lattice points on the boundary (first / last row or column) stay put
    P[1:-1, 1:-1] += jit.reshape(side, side, 2)[1:-1, 1:-1]
    return P.reshape(-1, 2)


def disk_points(side: int, seed: int = SEED_MESH, jitter: float = 0.3):
    """Points of the disk of radius 1/2 centred at (1/2, 1/2): a side x side lattice of spacing h = 1/(side-1),
    jittered by U[-jitter h, jitter h] and kept where it lies more than h/2 inside the circle, plus round(pi / h)
    points evenly spaced on the circle. Returns (points, boundary mask). The disk covers pi/4 of its bounding box,
    so about a fifth of the quadtree cells over it are empty."""
    rng = np.random.default_rng(seed)
    h = 1.0 / (side - 1)
    g = np.arange(side, dtype=np.float64) / (side - 1)
    X, Y = np.meshgrid(g, g)
    P = np.stack([X.ravel(), Y.ravel()], 1) + rng.uniform(-jitter * h, jitter * h, size=(side * side, 2))
    inner = P[np.hypot(P[:, 0] - 0.5, P[:, 1] - 0.5) < 0.5 - 0.5 * h]
    nb = max(8, int(round(math.pi / h)))
    th = 2.0 * math.pi * np.arange(nb) / nb
    bd = np.stack([0.5 + 0.5 * np.cos(th), 0.5 + 0.5 * np.sin(th)], 1)
    pts = np.concatenate([inner, bd])
    mask = np.zeros(len(pts), dtype=bool)
    mask[len(inner):] = True
    return pts, mask


def _morton_order(pts: np.ndarray) -> np.ndarray:
    """Permutation sorting 2D points in [0,1]^2 along the Z-order curve of a 2^16 x 2^16 grid."""
    q = np.clip((pts * 65536.0).astype(np.int64), 0, 65535).astype(np.uint64)

    def spread(v):
        for shift, mask in ((8, 0x00FF00FF), (4, 0x0F0F0F0F), (2, 0x33333333), (1, 0x55555555)):
            v = (v | (v << np.uint64(shift))) & np.uint64(mask)
        return v

    return np.argsort(spread(q[:, 0]) | (spread(q[:, 1]) << np.uint64(1)), kind="stable")


def delaunay(pts: np.ndarray, local_order: bool = False) -> np.ndarray:
    """Delaunay triangles (Qhull) as an index array into ``pts``. ``local_order`` hands Qhull the points in Z-order
    (same triangles for points in general position, faster for millions of points; the triangles come out in
    another order)."""
    from scipy.spatial import Delaunay
    if not local_order:
        return np.ascontiguousarray(Delaunay(pts).simplices.astype(np.int64))
    perm = _morton_order(pts)
    return np.ascontiguousarray(perm[Delaunay(pts[perm]).simplices].astype(np.int64))


def _lattice_corners(side: int, pts: np.ndarray):
    """Corner views (a, b, c, d) = (i,j), (i+1,j), (i+1,j+1), (i,j+1) of every lattice square, each (m, m, 2) with
    m = side - 1, indexed [j, i] (vertex (i, j) is point j * side + i)."""
    P = pts.reshape(side, side, 2)
    return P[:-1, :-1], P[:-1, 1:], P[1:, 1:], P[1:, :-1]


def lattice_diagonals(side: int, pts: np.ndarray) -> np.ndarray:
    """Per lattice square ([j, i], (m, m) bool): True if its Delaunay diagonal is a-c, False for b-d. The a-c
    diagonal is taken unless d lies strictly inside the circumcircle of (a, b, c)."""
    A, B, C, D = _lattice_corners(side, pts)
    ad, bd, cd = A - D, B - D, C - D
    det = ((ad[..., 0] ** 2 + ad[..., 1] ** 2) * (bd[..., 0] * cd[..., 1] - cd[..., 0] * bd[..., 1])
           - (bd[..., 0] ** 2 + bd[..., 1] ** 2) * (ad[..., 0] * cd[..., 1] - cd[..., 0] * ad[..., 1])
           + (cd[..., 0] ** 2 + cd[..., 1] ** 2) * (ad[..., 0] * bd[..., 1] - bd[..., 0] * ad[..., 1]))
    return det <= 0.0


def local_delaunay_lattice(side: int, pts: np.ndarray) -> np.ndarray:
    """Triangles of the square-by-square triangulation (``lattice_diagonals``) as an index array: the Delaunay
    triangulation whenever all Delaunay edges stay inside lattice squares."""
    m = side - 1
    use_ac = lattice_diagonals(side, pts).ravel()
    i, j = np.meshgrid(np.arange(m), np.arange(m))
    a = (j * side + i).ravel()
    b, c, d = a + 1, a + side + 1, a + side
    t1 = np.where(use_ac[:, None], np.stack([a, b, c], 1), np.stack([a, b, d], 1))
    t2 = np.where(use_ac[:, None], np.stack([a, c, d], 1), np.stack([b, c, d], 1))
    tris = np.concatenate([t1, t2])
    if np.any(_signed_area2(pts, tris) <= 0):
        raise RuntimeError("local lattice triangulation produced an inverted triangle")
    return tris


def graded_points(target_n: int, seed: int = SEED_MESH, c: float | None = None, max_depth: int = 20):
    """Quadtree-leaf sampling of [0,1]^2 with local spacing h(x) = c (|x| + 0.01)^0.75 (density ~ (r+0.01)^-1.5
    towards the corner (0,0)). A cell is split while its size exceeds h at its centre; each leaf receives one point
    jittered by U[-0.3, 0.3] of its size around its centre. Leaves on the square's boundary contribute their corner
    points on that boundary, so the boundary is graded too. ``c`` is tuned so that the interior count is close to
    ``target_n``."""
    def leaves_for(cc):
        x0 = np.zeros(1); y0 = np.zeros(1); sz = 1.0
        out = []
        for depth in range(max_depth + 1):
            cx, cy = x0 + 0.5 * sz, y0 + 0.5 * sz
            h = cc * (np.hypot(cx, cy) + 0.01) ** 0.75
            split = (sz > h) & (depth < max_depth)
            out.append((x0[~split], y0[~split], sz))
            if not split.any():
                break
            x0, y0 = x0[split], y0[split]
            half = 0.5 * sz
            x0 = np.concatenate([x0, x0 + half, x0, x0 + half])
            y0 = np.concatenate([y0, y0, y0 + half, y0 + half])
            sz = half
        return out

    def count(cc):
        return sum(len(l[0]) for l in leaves_for(cc))

    if c is None:
        c = math.sqrt(2.56 / target_n)
        for _ in range(4):
            n_now = count(c)
            c *= math.sqrt(n_now / target_n)
    leaves = leaves_for(c)
    rng = np.random.default_rng(seed)
    xs, ys, ss = [], [], []
    for (x0, y0, sz) in leaves:
        xs.append(x0); ys.append(y0); ss.append(np.full(len(x0), sz))
    x0 = np.concatenate(xs); y0 = np.concatenate(ys); sz = np.concatenate(ss)
    jit = rng.uniform(-0.3, 0.3, size=(len(x0), 2))
    interior = np.stack([x0 + (0.5 + jit[:, 0]) * sz, y0 + (0.5 + jit[:, 1]) * sz], 1)
    bpts = [np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0], [1.0, 1.0]])]
    for sel, mk in (((x0 == 0.0), lambda a, b, s: np.stack([np.zeros_like(b), b], 1)),
                    ((y0 == 0.0), lambda a, b, s: np.stack([a, np.zeros_like(a)], 1)),
                    ((x0 + sz == 1.0), lambda a, b, s: np.stack([np.ones_like(b), b], 1)),
                    ((y0 + sz == 1.0), lambda a, b, s: np.stack([a, np.ones_like(a)], 1))):
        a, b, s = x0[sel], y0[sel], sz[sel]
        bpts.append(mk(a, b, s))
        bpts.append(mk(a + s, b + s, s))
    bnd = np.unique(np.concatenate(bpts), axis=0)
    return np.concatenate([interior, bnd]), c


def _signed_area2(pts, tris):
    a, b, c = pts[tris[:, 0]], pts[tris[:, 1]], pts[tris[:, 2]]
    return (b[:, 0] - a[:, 0]) * (c[:, 1] - a[:, 1]) - (b[:, 1] - a[:, 1]) * (c[:, 0] - a[:, 0])


# ----------------------------------------------------------------------------------------------------------------
# P1 assembly
# ----------------------------------------------------------------------------------------------------------------

def p1_assemble(pts: np.ndarray, tris: np.ndarray, kappa_t: np.ndarray | None = None,
                dirichlet: np.ndarray | None = None):
    """Stiffness matrix of -div(kappa grad u) with linear elements, Dirichlet vertices eliminated.

    Element entries use the edge-vector form K_ab = kappa (e_a . e_b) / (4 |T|), where e_a is the edge opposite
    vertex a; on right triangles with dyadic legs this gives exact 4 / -1 / 0 stencils. Every vertex pair sharing a
    triangle is kept in the pattern, zero-valued ones included. Returns (coords, row_ptr, col, val) over the
    non-Dirichlet vertices, numbered in their original order."""
    tris = np.asarray(tris, dtype=np.int64).copy()
    s = _signed_area2(pts, tris)
    flip = s < 0
    tris[flip] = tris[flip][:, [0, 2, 1]]
    area2 = np.abs(s)
    if np.any(area2 == 0):
        raise ValueError("degenerate triangle")
    P = [pts[tris[:, k]] for k in range(3)]
    E = [P[2] - P[1], P[0] - P[2], P[1] - P[0]]
    kap = np.ones(len(tris)) if kappa_t is None else np.asarray(kappa_t, dtype=np.float64)
    denom = 2.0 * area2
    rows, cols, vals = [], [], []
    for a in range(3):
        for bb in range(3):
            rows.append(tris[:, a]); cols.append(tris[:, bb])
            vals.append(kap * (E[a][:, 0] * E[bb][:, 0] + E[a][:, 1] * E[bb][:, 1]) / denom)
    rows = np.concatenate(rows); cols = np.concatenate(cols); vals = np.concatenate(vals)
    npts = len(pts)
    if dirichlet is None:
        dirichlet = _on_unit_boundary(pts)
    keep_v = ~dirichlet
    newid = np.full(npts, -1, dtype=np.int64)
    newid[keep_v] = np.arange(int(keep_v.sum()))
    keep = keep_v[rows] & keep_v[cols]
    r = newid[rows[keep]]; cc = newid[cols[keep]]; v = vals[keep]
    n = int(keep_v.sum())
    # (row, column) pairs in ascending order, equal pairs kept in element order (a stable sort of the pair key)
    key = r * n + cc
    order = np.argsort(key, kind="stable")
    r, cc, v, key = r[order], cc[order], v[order], key[order]
    first = np.ones(len(key), dtype=bool)
    first[1:] = key[1:] != key[:-1]
    starts = np.nonzero(first)[0]
    vsum = np.add.reduceat(v, starts)
    ru, cu = r[starts], cc[starts]
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(row_ptr, ru + 1, 1)
    row_ptr = np.cumsum(row_ptr)
    return (np.ascontiguousarray(pts[keep_v]), row_ptr, cu.astype(np.int32), vsum.astype(np.float64))


# corner offsets (dx, dy) of a, b, c, d inside a lattice square
_CORNER = ((0, 0), (1, 0), (1, 1), (0, 1))


class _NumpyOps:
    """The few array operations the lattice assembly needs, for numpy arrays."""
    xp = np
    i32, i64, boolean = np.int32, np.int64, bool

    @staticmethod
    def zeros(shape, like, dtype=None):
        return np.zeros(shape, dtype=like.dtype if dtype is None else dtype)

    @staticmethod
    def asarray(a, like):
        return np.asarray(a)

    @staticmethod
    def cast(a, dtype):
        return a.astype(dtype)

    @staticmethod
    def contiguous(a):
        return np.ascontiguousarray(a)

    @staticmethod
    def grid(n, like):
        """(ix, iy) of an n x n grid, indexed [iy, ix]."""
        g = np.arange(n)
        return np.broadcast_to(g[None, :], (n, n)), np.broadcast_to(g[:, None], (n, n))


class _TorchOps:
    """The same operations for torch tensors (on any device)."""
    def __init__(self):
        import torch
        self.xp = torch
        self.i32, self.i64, self.boolean = torch.int32, torch.int64, torch.bool

    def zeros(self, shape, like, dtype=None):
        return self.xp.zeros(shape, dtype=like.dtype if dtype is None else dtype, device=like.device)

    def asarray(self, a, like):
        return self.xp.as_tensor(a, device=like.device)

    def cast(self, a, dtype):
        return a.to(dtype)

    def contiguous(self, a):
        return a.contiguous()

    def grid(self, n, like):
        g = self.xp.arange(n, device=like.device)
        return g[None, :].expand(n, n), g[:, None].expand(n, n)


def _ops_for(a):
    return _NumpyOps if isinstance(a, np.ndarray) else _TorchOps()


def lattice_p1_assemble(side: int, pts, use_ac, kappa_tiles: int = 0, kappa_seed: int = SEED_KAPPA):
    """The P1 system of ``p1_assemble`` for the square-by-square triangulation of a side x side lattice, built square
    by square: each square's two element matrices are summed into a symmetric 4x4 square matrix, and each vertex
    gathers its 9-slot stencil from the four squares around it in a fixed order. Deterministic, O(N), strided slices
    and elementwise work only, so it runs unchanged on numpy arrays or on torch tensors (e.g. on the GPU, to prepare
    inputs in place). ``kappa_tiles`` > 0 gives each element the checkerboard tile value at its centroid. Boundary
    vertices are eliminated; returns (coords, row_ptr, col, val) like ``p1_assemble``, as arrays of the input kind."""
    ops = _ops_for(pts)
    xp = ops.xp
    m = side - 1
    P = pts.reshape(side, side, 2)
    X, Y = ops.contiguous(P[..., 0]), ops.contiguous(P[..., 1])
    cx = [X[:-1, :-1], X[:-1, 1:], X[1:, 1:], X[1:, :-1]]   # corner k of square [j, i]
    cy = [Y[:-1, :-1], Y[:-1, 1:], Y[1:, 1:], Y[1:, :-1]]
    ac = use_ac
    # the two triangles of each square: T1 = (a, b, c|d), T2 = (a|b, c, d); corner 0..3 of each per square
    t1x, t1y = (cx[0], cx[1], xp.where(ac, cx[2], cx[3])), (cy[0], cy[1], xp.where(ac, cy[2], cy[3]))
    t2x, t2y = (xp.where(ac, cx[0], cx[1]), cx[2], cx[3]), (xp.where(ac, cy[0], cy[1]), cy[2], cy[3])
    tile_val = None
    if kappa_tiles:
        tile_val = ops.asarray(10.0 ** np.random.default_rng(kappa_seed).uniform(-3.0, 3.0,
                                                                                (kappa_tiles, kappa_tiles)), X)
    M = {}

    def add(key, v):
        M[key] = M[key] + v if key in M else v

    for tx, ty, corner_of in ((t1x, t1y, lambda v: (0, 1, 2 if v else 3)), (t2x, t2y, lambda v: (0 if v else 1, 2, 3))):
        ex = (tx[2] - tx[1], tx[0] - tx[2], tx[1] - tx[0])
        ey = (ty[2] - ty[1], ty[0] - ty[2], ty[1] - ty[0])
        s2 = ex[2] * (-ey[1]) - ey[2] * (-ex[1])          # (p1 - p0) x (p2 - p0), twice the signed area
        if bool((s2 <= 0).any()):
            raise RuntimeError("lattice triangle inverted or degenerate")
        scale = 1.0 / (2.0 * s2)
        if tile_val is not None:
            ti = ops.cast((tx[0] + tx[1] + tx[2]) / 3.0 * kappa_tiles, ops.i64).clip(0, kappa_tiles - 1)
            tj = ops.cast((ty[0] + ty[1] + ty[2]) / 3.0 * kappa_tiles, ops.i64).clip(0, kappa_tiles - 1)
            scale = scale * tile_val[tj, ti]
        ca, cb = corner_of(True), corner_of(False)      # corner numbers for the a-c and the b-d split
        for a in range(3):
            for b in range(a, 3):
                v = scale * (ex[a] * ex[b] + ey[a] * ey[b])
                if ca[a] == cb[a] and ca[b] == cb[b]:
                    add((ca[a], ca[b]), v)
                else:
                    zero = ops.zeros(v.shape, v)
                    add((ca[a], ca[b]), xp.where(ac, v, zero))
                    add((cb[a], cb[b]), xp.where(ac, zero, v))
    # structural presence of each square-matrix pair: the 4 sides always, a-c on a-c squares, b-d on the others
    S = ops.zeros((side, side, 9), X)
    pres = ops.zeros((side, side, 9), X, dtype=ops.boolean)
    for (k, k2) in sorted(M):
        v = M[(k, k2)]
        diag = {(0, 2): ac, (1, 3): ~ac}.get((k, k2))
        for (r, c) in ((k, k2), (k2, k)) if k != k2 else ((k, k2),):
            (x0, y0), (x1, y1) = _CORNER[r], _CORNER[c]
            slot = (y1 - y0 + 1) * 3 + (x1 - x0 + 1)
            S[y0:y0 + m, x0:x0 + m, slot] += v
            if diag is None:
                pres[y0:y0 + m, x0:x0 + m, slot] = True
            else:
                pres[y0:y0 + m, x0:x0 + m, slot] |= diag
    ni = side - 2
    dxs = ops.asarray([dx for dy in (-1, 0, 1) for dx in (-1, 0, 1)], X)
    dys = ops.asarray([dy for dy in (-1, 0, 1) for dx in (-1, 0, 1)], X)
    ix, iy = ops.grid(ni, X)
    nx, ny = ix[..., None] + dxs, iy[..., None] + dys
    keep = pres[1:-1, 1:-1] & (nx >= 0) & (nx < ni) & (ny >= 0) & (ny < ni)
    counts = keep.reshape(-1, 9).sum(1)
    row_ptr = ops.zeros(ni * ni + 1, counts, dtype=ops.i64)
    row_ptr[1:] = xp.cumsum(counts, 0)
    col = ops.cast((ny * ni + nx)[keep], ops.i32)
    val = S[1:-1, 1:-1][keep]
    coords = ops.contiguous(P[1:-1, 1:-1].reshape(-1, 2))
    return coords, row_ptr, col, val


def checkerboard_kappa(pts, tris, tiles: int = 16, seed: int = SEED_KAPPA, lo: float = -3.0, hi: float = 3.0):
    """Per-element coefficient from a tiles x tiles checkerboard with tile values 10^U[lo,hi]; an element takes the
    tile of its centroid."""
    rng = np.random.default_rng(seed)
    tile_val = 10.0 ** rng.uniform(lo, hi, size=(tiles, tiles))
    cen = (pts[tris[:, 0]] + pts[tris[:, 1]] + pts[tris[:, 2]]) / 3.0
    ti = np.minimum((cen[:, 0] * tiles).astype(np.int64), tiles - 1)
    tj = np.minimum((cen[:, 1] * tiles).astype(np.int64), tiles - 1)
    return tile_val[tj, ti]


def rhs(n: int, seed: int = SEED_RHS) -> np.ndarray:
    return np.random.default_rng(seed).uniform(-1.0, 1.0, size=n)


# ----------------------------------------------------------------------------------------------------------------
# workloads
# ----------------------------------------------------------------------------------------------------------------

def _mesh_meta(pts, tris, kappa, dirichlet):
    """The mesh behind an assembled problem, for assembling it again (on the device, with new coefficients)."""
    return dict(points=pts, tris=np.ascontiguousarray(tris, dtype=np.int32), kappa=kappa, dirichlet=dirichlet)


def _problem(name, pts, tris, kappa=None, rhs_seed=SEED_RHS, **meta):
    coords, rp, col, val = p1_assemble(pts, tris, kappa)
    return Problem(name, coords, rp, col, val, rhs(len(coords), rhs_seed), UNIT_BOX,
                   dict(meta, n_points=len(pts), n_tris=len(tris),
                        **_mesh_meta(pts, tris, kappa, _on_unit_boundary(pts))))


def uniform_problem(m: int = 64, rhs_seed: int = SEED_RHS) -> Problem:
    """Poisson on the uniform right-triangle mesh with (m+1)^2 vertices (m = 64: 3,969 interior unknowns)."""
    pts, tris = uniform_mesh(m)
    return _problem(f"uniform{m + 1}", pts, tris, rhs_seed=rhs_seed, kind="uniform", m=m)


def jittered_problem(side: int = 1024, seed: int = SEED_MESH, rhs_seed: int = SEED_RHS, kappa_tiles: int = 0,
                     fast: bool = False) -> Problem:
    """Poisson (or checkerboard diffusion if kappa_tiles > 0) on a jittered side x side lattice, Delaunay-
    triangulated by Qhull (``fast``: square-by-square empty-circumcircle diagonals)."""
    pts = jittered_points(side, seed)
    name = f"jittered{side}" + (f"_kappa{kappa_tiles}" if kappa_tiles else "") + ("_fast" if fast else "")
    meta = dict(kind="jittered", side=side, seed=seed, kappa_tiles=kappa_tiles, fast=fast)
    if fast:
        coords, rp, col, val = lattice_p1_assemble(side, pts, lattice_diagonals(side, pts), kappa_tiles)
        return Problem(name, coords, rp, col, val, rhs(len(coords), rhs_seed), UNIT_BOX,
                       dict(meta, n_points=len(pts), n_tris=2 * (side - 1) ** 2))
    tris = delaunay(pts)
    kap = checkerboard_kappa(pts, tris, kappa_tiles) if kappa_tiles else None
    return _problem(name, pts, tris, kap, rhs_seed=rhs_seed, **meta)


def disk_problem(side: int = 1024, seed: int = SEED_MESH, rhs_seed: int = SEED_RHS) -> Problem:
    """Poisson on a Delaunay mesh of the disk (Dirichlet on the circle); the quadtree box is the unit square, so
    the cells outside the disk are empty aggregates on every level."""
    pts, mask = disk_points(side, seed)
    tris = delaunay(pts)
    coords, rp, col, val = p1_assemble(pts, tris, None, dirichlet=mask)
    return Problem(f"disk{side}", coords, rp, col, val, rhs(len(coords), rhs_seed), UNIT_BOX,
                   dict(kind="disk", side=side, seed=seed, n_points=len(pts), n_tris=len(tris),
                        **_mesh_meta(pts, tris, None, mask)))


def lattice_system(side: int, seed: int = SEED_MESH, kappa_tiles: int = 0, device=None):
    """(coords, row_ptr, col, val) of the square-by-square jittered-lattice system. With ``device`` (a torch device)
    the points are drawn on the host as usual and the assembly runs there, leaving the system resident on it."""
    pts = jittered_points(side, seed)
    if device is not None:
        import torch
        pts = torch.as_tensor(pts, device=device)
    return lattice_p1_assemble(side, pts, lattice_diagonals(side, pts), kappa_tiles)


def graded_problem(target_n: int = 4_000_000, seed: int = SEED_MESH, rhs_seed: int = SEED_RHS,
                   progress=None) -> Problem:
    """Poisson on a graded Delaunay mesh refined towards (0,0). ``progress(msg)`` is told when each stage ends (a
    few million points take minutes on one core)."""
    say = progress or (lambda msg: None)
    pts, c = graded_points(target_n, seed)
    say(f"graded mesh: {len(pts)} points sampled")
    tris = delaunay(pts, local_order=True)
    say(f"graded mesh: {len(tris)} Delaunay triangles")
    return _problem(f"graded{target_n}", pts, tris, rhs_seed=rhs_seed, kind="graded", target_n=target_n, c=c,
                    seed=seed)


# ----------------------------------------------------------------------------------------------------------------
# 3D: heat-transfer step on the unit cube
# ----------------------------------------------------------------------------------------------------------------

# the six tetrahedra of a unit cube around its diagonal (0,0,0)-(1,1,1): vertex path 0 -> +e_a -> +e_b -> (1,1,1)
# for every order (a, b, c) of the axes; corners numbered x + 2 y + 4 z
_KUHN = np.array([[0, 1, 3, 7], [0, 1, 5, 7], [0, 2, 3, 7], [0, 2, 6, 7], [0, 4, 5, 7], [0, 4, 6, 7]], dtype=np.int64)


def cube_mesh(m: int, seed: int = SEED_MESH, jitter: float = 0.15):
    """(points (m+1)^3 x 3, tetrahedra (6 m^3) x 4 positively oriented, inlet mask) of a jittered lattice of the unit
    cube: interior points move by U[-jitter h, jitter h] per coordinate, boundary points stay on their faces (moved
    only along them)."""
    h = 1.0 / m
    g = np.arange(m + 1, dtype=np.float64) * h
    z, y, x = np.meshgrid(g, g, g, indexing="ij")
    pts = np.stack([x.ravel(), y.ravel(), z.ravel()], 1)
    rng = np.random.default_rng(seed)
    d = rng.uniform(-jitter * h, jitter * h, size=pts.shape)
    on_face = (pts <= 0.0) | (pts >= 1.0)
    d[on_face] = 0.0  # a boundary coordinate stays on its face
    pts = pts + d
    i = np.arange(m)
    kk, jj, ii = np.meshgrid(i, i, i, indexing="ij")
    base = (kk * (m + 1) + jj) * (m + 1) + ii
    corner = np.array([(c & 1) + ((c >> 1) & 1) * (m + 1) + (c >> 2) * (m + 1) ** 2 for c in range(8)])
    tets = (base.ravel()[:, None, None] + corner[_KUHN][None, :, :]).reshape(-1, 4)
    e = pts[tets[:, 1:]] - pts[tets[:, :1]]
    vol6 = np.einsum("ij,ij->i", e[:, 0], np.cross(e[:, 1], e[:, 2]))
    if not (np.abs(vol6) > 0.05 * h ** 3).all():
        raise ValueError("degenerate tetrahedron")
    neg = vol6 < 0
    tets[neg, 2], tets[neg, 3] = tets[neg, 3].copy(), tets[neg, 2].copy()
    return pts, tets, pts[:, 0] <= 0.0


def heat_step_assemble(pts, tets, dt, fixed):
    """CSR (columns ascending) of M / dt + K over the unknowns (vertices not ``fixed``, in vertex order): K the
    linear-element stiffness of -div(grad T), sum over tetrahedra of |T| grad(phi_a) . grad(phi_b), M the lumped
    mass |T| / 4 per vertex and tetrahedron. Returns (coords, row_ptr, col, val)."""
    import scipy.sparse as sp
    e = pts[tets[:, 1:]] - pts[tets[:, :1]]                      # (nt, 3, 3): edges from vertex 0
    vol = np.abs(np.linalg.det(e)) / 6.0
    inv = np.linalg.inv(e)                                       # columns: gradients of phi_1..3
    g = np.concatenate([-inv.sum(axis=2, keepdims=True), inv], axis=2)  # (nt, 3, 4): grad phi_a as column a
    k = vol[:, None, None] * np.einsum("tia,tib->tab", g, g)
    nv = len(pts)
    rows = np.repeat(tets, 4, axis=1).ravel()
    cols = np.tile(tets, (1, 4)).ravel()
    K = sp.csr_matrix((k.ravel(), (rows, cols)), shape=(nv, nv))
    mass = np.bincount(tets.ravel(), weights=np.repeat(vol / 4.0, 4), minlength=nv)
    A = (K + sp.diags(mass / dt)).tocsr()
    keep = np.flatnonzero(~fixed)
    A = A[keep][:, keep].tocsr()
    A.sort_indices()
    return (np.ascontiguousarray(pts[keep]), A.indptr.astype(np.int64), A.indices.astype(np.int32),
            A.data.astype(np.float64))


def cube_problem(m: int = 100, seed: int = SEED_MESH, rhs_seed: int = SEED_RHS) -> Problem:
    """One implicit Euler step (dt = h) of the heat equation on the unit cube (the 3D variant): m = 100 gives
    101^3 - 101^2 = 1,020,100 unknowns."""
    pts, tets, inlet = cube_mesh(m, seed)
    coords, rp, col, val = heat_step_assemble(pts, tets, 1.0 / m, inlet)
    return Problem(f"cube{m + 1}", coords, rp, col, val, rhs(len(coords), rhs_seed), UNIT_CUBE,
                   dict(kind="cube", m=m, seed=seed, n_points=len(pts), n_tets=len(tets)))


def serving_sides(n_req: int = 512, seed: int = SEED_STREAM, dof_lo: float = 1e4, dof_hi: float = 2e6,
                  repeat_p: float = 0.3):
    """Request stream shape: per request a lattice side (DOF log-uniform in [dof_lo, dof_hi], side ~ sqrt(DOF)+2)
    and whether it repeats an earlier mesh (probability ``repeat_p``). Returns a list of (mesh_id, side, rhs_seed)."""
    rng = np.random.default_rng(seed)
    reqs, meshes = [], []
    for q in range(n_req):
        if meshes and rng.uniform() < repeat_p:
            mid = int(rng.integers(len(meshes)))
        else:
            dof = math.exp(rng.uniform(math.log(dof_lo), math.log(dof_hi)))
            meshes.append(int(round(math.sqrt(dof))) + 2)
            mid = len(meshes) - 1
        reqs.append((mid, meshes[mid], 1000 + q))
    return reqs


def config(name: str, scale: float = 1.0) -> Problem:
    """Named workloads. ``scale`` < 1 shrinks the unknown count for tests (same generator, same seeds)."""
    if name == "c1":
        return uniform_problem(64)
    if name == "c2":
        return jittered_problem(max(8, int(round(1024 * math.sqrt(scale)))))
    if name == "c3":
        return graded_problem(int(4_000_000 * scale))
    if name == "c4":
        return jittered_problem(max(8, int(round(1416 * math.sqrt(scale)))), kappa_tiles=16)
    if name == "cube":
        return cube_problem(max(4, int(round(100 * scale ** (1.0 / 3.0)))))
    raise KeyError(name)
