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

Seeds follow ``numpy.random.default_rng``: mesh 0, right-hand side 1, kappa 2, request stream 3.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

SEED_MESH, SEED_RHS, SEED_KAPPA, SEED_STREAM = 0, 1, 2, 3
UNIT_BOX = (0.0, 1.0, 0.0, 1.0)


@dataclasses.dataclass
class Problem:
    """An SPD system A x = b with the coordinates of its unknowns.

    ``coords`` is (n, 2) float64 (x, y interleaved); ``row_ptr`` int64 (n+1), ``col`` int32, ``val`` float64 form a
    0-based CSR matrix with columns ascending inside each row (explicit zeros of the stencil kept); ``box`` is the
    domain's bounding box (a1, b1, a2, b2).
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
    X, Y = np.meshgrid(g, g)
    pts = np.stack([X.ravel(), Y.ravel()], 1)
    bnd = _on_unit_boundary(pts)
    jit = rng.uniform(-jitter * h, jitter * h, size=pts.shape)
    pts[~bnd] += jit[~bnd]
    return pts


def delaunay(pts: np.ndarray) -> np.ndarray:
    from scipy.spatial import Delaunay
    return np.ascontiguousarray(Delaunay(pts).simplices.astype(np.int64))


def local_delaunay_lattice(side: int, pts: np.ndarray) -> np.ndarray:
    """Triangulate a jittered lattice square by square, taking in each square the diagonal that passes the
    empty-circumcircle test (the Delaunay choice whenever all Delaunay edges stay inside lattice squares).
    Vectorised and fast; used for the serving request stream where Qhull on hundreds of meshes would dominate."""
    m = side - 1
    i, j = np.meshgrid(np.arange(m), np.arange(m))
    a = (j * side + i).ravel()
    b, c, d = a + 1, a + side + 1, a + side
    A, B, C, D = pts[a], pts[b], pts[c], pts[d]
    # d inside circumcircle(a,b,c) (a,b,c counter-clockwise) <=> incircle determinant > 0
    ad, bd, cd = A - D, B - D, C - D
    det = ((ad[:, 0] ** 2 + ad[:, 1] ** 2) * (bd[:, 0] * cd[:, 1] - cd[:, 0] * bd[:, 1])
           - (bd[:, 0] ** 2 + bd[:, 1] ** 2) * (ad[:, 0] * cd[:, 1] - cd[:, 0] * ad[:, 1])
           + (cd[:, 0] ** 2 + cd[:, 1] ** 2) * (ad[:, 0] * bd[:, 1] - bd[:, 0] * ad[:, 1]))
    use_ac = det <= 0.0
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
    order = np.lexsort((np.arange(len(r)), cc, r))
    r, cc, v = r[order], cc[order], v[order]
    key = r * n + cc
    first = np.ones(len(key), dtype=bool)
    first[1:] = key[1:] != key[:-1]
    starts = np.nonzero(first)[0]
    vsum = np.add.reduceat(v, starts)
    ru, cu = r[starts], cc[starts]
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(row_ptr, ru + 1, 1)
    row_ptr = np.cumsum(row_ptr)
    return (np.ascontiguousarray(pts[keep_v]), row_ptr, cu.astype(np.int32), vsum.astype(np.float64))


def lattice_p1_assemble(side: int, pts: np.ndarray, tris: np.ndarray, kappa_t: np.ndarray | None = None):
    """The same P1 system as ``p1_assemble`` for a triangulation whose edges join lattice neighbours (the
    square-by-square triangulation of a side x side lattice), in O(N): element entries are accumulated into a 9-slot
    stencil per vertex with bincount instead of sorting all entry pairs. Boundary vertices are eliminated."""
    tris = np.asarray(tris, dtype=np.int64)
    npts = len(pts)
    s = _signed_area2(pts, tris)
    if np.any(s <= 0):
        raise ValueError("lattice triangles must be counter-clockwise and non-degenerate")
    P = [pts[tris[:, k]] for k in range(3)]
    E = [P[2] - P[1], P[0] - P[2], P[1] - P[0]]
    kap = np.ones(len(tris)) if kappa_t is None else np.asarray(kappa_t, dtype=np.float64)
    scale = kap / (2.0 * s)
    tx = [tris[:, k] % side for k in range(3)]
    ty = [tris[:, k] // side for k in range(3)]
    idx, w = [], []
    for a in range(3):
        for b in range(3):
            dx, dy = tx[b] - tx[a], ty[b] - ty[a]
            if np.abs(dx).max() > 1 or np.abs(dy).max() > 1:
                raise ValueError("an edge leaves the lattice neighbourhood")
            idx.append(tris[:, a] * 9 + (dy + 1) * 3 + (dx + 1))
            w.append(scale * (E[a][:, 0] * E[b][:, 0] + E[a][:, 1] * E[b][:, 1]))
    idx = np.concatenate(idx)
    S = np.bincount(idx, weights=np.concatenate(w), minlength=npts * 9).reshape(npts, 9)
    present = (np.bincount(idx, minlength=npts * 9) > 0).reshape(npts, 9)
    vx, vy = np.arange(npts) % side, np.arange(npts) // side
    interior = ~((vx == 0) | (vy == 0) | (vx == side - 1) | (vy == side - 1))
    newid = np.full(npts, -1, dtype=np.int64)
    newid[interior] = np.arange(int(interior.sum()))
    rows = np.nonzero(interior)[0]
    off = np.array([(dy * side + dx) for dy in (-1, 0, 1) for dx in (-1, 0, 1)])
    nb = rows[:, None] + off[None, :]
    keep = present[rows] & interior[nb]
    row_ptr = np.zeros(len(rows) + 1, dtype=np.int64)
    row_ptr[1:] = np.cumsum(keep.sum(1))
    col = newid[nb[keep]].astype(np.int32)
    vals = S[rows][keep].astype(np.float64)
    return np.ascontiguousarray(pts[interior]), row_ptr, col, vals


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

def _problem(name, pts, tris, kappa=None, rhs_seed=SEED_RHS, **meta):
    coords, rp, col, val = p1_assemble(pts, tris, kappa)
    return Problem(name, coords, rp, col, val, rhs(len(coords), rhs_seed), UNIT_BOX,
                   dict(meta, n_points=len(pts), n_tris=len(tris)))


def uniform_problem(m: int = 64, rhs_seed: int = SEED_RHS) -> Problem:
    """Poisson on the uniform right-triangle mesh with (m+1)^2 vertices (m = 64: 3,969 interior unknowns)."""
    pts, tris = uniform_mesh(m)
    return _problem(f"uniform{m + 1}", pts, tris, rhs_seed=rhs_seed, kind="uniform", m=m)


def jittered_problem(side: int = 1024, seed: int = SEED_MESH, rhs_seed: int = SEED_RHS, kappa_tiles: int = 0,
                     fast: bool = False) -> Problem:
    """Poisson (or checkerboard diffusion if kappa_tiles > 0) on a jittered side x side lattice, Delaunay-
    triangulated by Qhull (``fast``: square-by-square empty-circumcircle diagonals)."""
    pts = jittered_points(side, seed)
    tris = local_delaunay_lattice(side, pts) if fast else delaunay(pts)
    kap = checkerboard_kappa(pts, tris, kappa_tiles) if kappa_tiles else None
    name = f"jittered{side}" + (f"_kappa{kappa_tiles}" if kappa_tiles else "") + ("_fast" if fast else "")
    meta = dict(kind="jittered", side=side, seed=seed, kappa_tiles=kappa_tiles, fast=fast)
    if fast:
        coords, rp, col, val = lattice_p1_assemble(side, pts, tris, kap)
        return Problem(name, coords, rp, col, val, rhs(len(coords), rhs_seed), UNIT_BOX,
                       dict(meta, n_points=len(pts), n_tris=len(tris)))
    return _problem(name, pts, tris, kap, rhs_seed=rhs_seed, **meta)


def graded_problem(target_n: int = 4_000_000, seed: int = SEED_MESH, rhs_seed: int = SEED_RHS) -> Problem:
    """Poisson on a graded Delaunay mesh refined towards (0,0)."""
    pts, c = graded_points(target_n, seed)
    tris = delaunay(pts)
    return _problem(f"graded{target_n}", pts, tris, rhs_seed=rhs_seed, kind="graded", target_n=target_n, c=c,
                    seed=seed)


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
    raise KeyError(name)
