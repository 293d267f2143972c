"""Input generators (no GPU): the square-by-square lattice assembly against the generic element-by-element one."""
import numpy as np
import pytest

from paper_1209_5421_amd import meshgen as mg
from tests import helpers as H


@pytest.mark.parametrize("side,kappa,seed", [(12, 0, 0), (40, 0, 0), (40, 16, 2), (30, 16, 1)])
def test_lattice_assembly_matches_generic_assembly(side, kappa, seed):
    """Where Qhull's Delaunay triangulation keeps to lattice squares, both give the same pattern and values to
    rounding."""
    f = mg.jittered_problem(side, seed=seed, kappa_tiles=kappa, fast=True)
    g = mg.jittered_problem(side, seed=seed, kappa_tiles=kappa, fast=False)
    np.testing.assert_array_equal(f.coords, g.coords)
    np.testing.assert_array_equal(f.row_ptr, g.row_ptr)
    np.testing.assert_array_equal(f.col, g.col)
    assert np.abs(f.val - g.val).max() <= 1e-14 * np.abs(g.val).max()


def test_lattice_triangulation_is_the_local_delaunay_choice():
    side = 100
    pts = mg.jittered_points(side, 0)
    tris = mg.local_delaunay_lattice(side, pts)
    qh = mg.delaunay(pts)

    def edges(t):
        e = np.sort(np.concatenate([t[:, [0, 1]], t[:, [1, 2]], t[:, [2, 0]]]), 1)
        return set(map(tuple, e))
    diff = edges(qh) - edges(tris)
    # jitter of 0.3h lets a Delaunay edge leave its square only rarely; every other edge agrees
    assert len(tris) == len(qh) and len(diff) <= 3
    for a, b in diff:
        assert max(abs(a % side - b % side), abs(a // side - b // side)) == 2


def test_lattice_system_properties():
    p = mg.jittered_problem(64, seed=4, fast=True)
    A = p.scipy()
    assert abs(A - A.T).max() <= 1e-15 * abs(A).max()
    assert np.all(A.diagonal() > 0)
    # Poisson rows away from the boundary sum to zero (constants are in the kernel of the Neumann operator)
    x = p.coords
    h = 1.0 / 63
    inner = np.all((x > 2.5 * h) & (x < 1 - 2.5 * h), axis=1)
    rs = np.asarray(A.sum(1)).ravel()
    assert np.abs(rs[inner]).max() <= 1e-13 * A.diagonal().max()


def test_torch_backend_is_bitwise_numpy():
    torch = pytest.importorskip("torch")
    for side, kappa in ((33, 0), (33, 16)):
        f = mg.jittered_problem(side, seed=7, kappa_tiles=kappa, fast=True)
        pts = torch.as_tensor(mg.jittered_points(side, 7))
        out = mg.lattice_p1_assemble(side, pts, mg.lattice_diagonals(side, pts), kappa)
        for a, b in zip((f.coords, f.row_ptr, f.col, f.val), out):
            assert a.dtype == b.numpy().dtype
            np.testing.assert_array_equal(a, b.numpy())


def test_disk_mesh_properties():
    """The disk mesh: unknowns strictly inside the circle, as many as lattice points fit there; an SPD P1 Laplacian whose rows
    away from the circle sum to zero; the triangulation covers the disk (total area within the inscribed polygon's)."""
    side = 80
    pts, mask = mg.disk_points(side, 0)
    r = np.hypot(pts[:, 0] - 0.5, pts[:, 1] - 0.5)
    np.testing.assert_allclose(r[mask], 0.5, rtol=1e-15)
    assert (r[~mask] < 0.5).all()
    n_in = int((~mask).sum())
    h = 1.0 / (side - 1)
    expect = np.pi * (0.5 - 0.5 * h) ** 2 / h ** 2  # lattice points within radius 1/2 - h/2
    assert abs(n_in / expect - 1) < 0.02
    tris = mg.delaunay(pts)
    area = 0.5 * np.abs(mg._signed_area2(pts, tris)).sum()
    nb = int(mask.sum())
    polygon = 0.5 * nb * 0.25 * np.sin(2 * np.pi / nb)
    assert abs(area - polygon) <= 1e-12
    p = mg.disk_problem(side)
    assert p.n == n_in
    A = p.scipy()
    assert abs(A - A.T).max() <= 1e-15 * abs(A).max()
    far = np.hypot(p.coords[:, 0] - 0.5, p.coords[:, 1] - 0.5) < 0.5 - 3 * h
    rs = np.asarray(A.sum(1)).ravel()
    assert np.abs(rs[far]).max() <= 1e-13 * A.diagonal().max()
    assert np.linalg.eigvalsh(A.toarray()).min() > 0


@pytest.mark.parametrize("mesh", ["wheel40", "wheel100", "jittered40_kappa"])
def test_p1_assembly_follows_the_stated_summation_order(mesh):
    """The host generator's assembly equals, bit for bit, the evaluation order the device assembly states (long
    sums included: the wheel's centre sums 40 or 100 element entries), so the device result can be compared with
    the generator's exactly."""
    if mesh.startswith("wheel"):
        pts, tris, dirichlet = H.wheel_mesh(spokes=int(mesh[5:]))
        kap = None
    else:
        pts = mg.jittered_points(40)
        tris = mg.delaunay(pts)
        kap = mg.checkerboard_kappa(pts, tris, 4)
        dirichlet = mg._on_unit_boundary(pts)
    _, rp, col, val = mg.p1_assemble(pts, tris, kap, dirichlet=dirichlet)
    rp2, col2, val2 = H.assembly_in_stated_order(pts, tris, kap, dirichlet)
    np.testing.assert_array_equal(rp, rp2)
    np.testing.assert_array_equal(col, col2)
    np.testing.assert_array_equal(val, val2)
