"""Parity of the octree (3D) variant of the HIP path (amg_setup3d, through the C ABI) with the CPU oracle's octree
setup and solve, element by element on seeded inputs.

Workloads: one implicit heat step on jittered lattices of the unit cube (P1 tetrahedra, Dirichlet inlet face; the
synthetic stand-in for the paper's 3D heat-transfer example), sized for two to four octree levels, and scattered
points with long-range couplings (overflow beyond the 27-point pattern on every level, no box given).
Bars as for the quadtree: aggregates, colors, 27-slot columns and overflow lists bit-exact; FP64 hierarchy values
bit-exact and the FP32 copy their rounding; level SpMV 1e-13 and sweeps 1e-11 of the maximum; preconditioner 1e-10;
FP64 solve iterations +-1 and relative error <= 1e-6 at 1e-8; mixed solve true residual <= 1e-8 and within 1e-6 of
the oracle solved to 1e-12.
"""
import numpy as np
import pytest

import oracle
from paper_1209_5421_amd import meshgen as mg
from tests import helpers as H

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

PROBLEMS = {
    "cube9": lambda: mg.cube_problem(8),          # 648 unknowns: octree levels 3, 2
    "cube17": lambda: mg.cube_problem(16),        # 4,624 unknowns: levels 4, 3, 2
    "cube33": lambda: mg.cube_problem(32),        # 34,848 unknowns: levels 5, 4, 3, 2
    "longrange3d": lambda: H.longrange_problem_3d(3000, 200),  # overflow on every level, bounding box
}

_cache = {}


def problem(name):
    if name not in _cache:
        _cache[name] = PROBLEMS[name]()
    return _cache[name]


def T(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda:0")


def gpu_hier(prob, **kw):
    from paper_1209_5421_amd import amg
    print(f"[octree] setup {prob.name} n={prob.n} nnz={prob.nnz} {kw}", flush=True)
    return amg.Hierarchy.from_problem(prob, device="cuda:0", **kw)


@pytest.mark.parametrize("name", list(PROBLEMS))
def test_octree_hierarchy_bit_exact(name):
    prob = problem(name)
    g = gpu_hier(prob)
    o = oracle.setup_problem(prob)
    assert g.num_levels == o.num_levels >= 2
    e0g, e0o = g.export_level(0), o.export_level(0)
    np.testing.assert_array_equal(e0g["agg"], e0o["agg"])
    np.testing.assert_array_equal(e0g["color"], e0o["color"])
    assert e0g["color"].max() == 7
    ovf = 0
    for level in range(1, g.num_levels):
        eg, eo = g.export_level(level, f32=True), o.export_level(level)
        assert eg["n"] == eo["n"] and eg["k"] == eo["k"] and eg["ovf_nnz"] == eo["ovf_nnz"]
        assert eg["aj"].shape[1] == 27
        for key in ("agg", "color", "aj", "ovf_ptr", "ovf_col"):
            np.testing.assert_array_equal(eg[key], eo[key], err_msg=f"level {level} {key}")
        np.testing.assert_array_equal(eg["ax"], eo["ax"], err_msg=f"level {level} ax")
        np.testing.assert_array_equal(eg["ovf_val"], eo["ovf_val"], err_msg=f"level {level} ovf_val")
        np.testing.assert_array_equal(eg["ax32"], eo["ax"].astype(np.float32), err_msg=f"level {level} fp32")
        ovf += eg["ovf_nnz"]
    if name == "longrange3d":
        assert ovf > 0
    g.close()
    o.close()


@pytest.mark.parametrize("name", list(PROBLEMS))
def test_octree_level_spmv_and_smoother(name):
    prob = problem(name)
    g = gpu_hier(prob)
    o = oracle.setup_problem(prob)
    rng = np.random.default_rng(7)
    for level in range(g.num_levels):
        n = g.level_info(level)["n"]
        x, f = rng.standard_normal(n), rng.standard_normal(n)
        y_o = o.spmv(level, x)
        y_g = g.spmv(level, T(x)).cpu().numpy()
        np.testing.assert_allclose(y_g, y_o, rtol=0, atol=1e-13 * np.abs(y_o).max(), err_msg=f"spmv {level}")
        if level == g.num_levels - 1:
            continue
        for fwd in (True, False):
            s_o = o.smooth(level, f, x, fwd)
            s_g = g.smooth(level, T(f), T(x), fwd).cpu().numpy()
            np.testing.assert_allclose(s_g, s_o, rtol=0, atol=1e-11 * np.abs(s_o).max(), err_msg=f"{level} {fwd}")
    g.close()
    o.close()


@pytest.mark.parametrize("smoother", [0, 1])
@pytest.mark.parametrize("name", list(PROBLEMS))
def test_octree_preconditioner_and_solves(name, smoother):
    prob = problem(name)
    g = gpu_hier(prob, smoother=smoother)
    o = oracle.setup_problem(prob)
    if smoother:
        o.set_block_smoother(True)
    r = np.random.default_rng(9).standard_normal(prob.n)
    z_o = o.apply_precond(r)
    z_g = g.apply_precond(T(r)).cpu().numpy()
    assert np.linalg.norm(z_g - z_o) <= 1e-10 * np.linalg.norm(z_o)
    z32 = g.apply_precond(T(r), precision=1).cpu().numpy()
    assert np.linalg.norm(z32 - z_o) <= 1e-3 * np.linalg.norm(z_o)
    x_o, io = o.solve(prob.b, tol=1e-8)
    x_12, _ = o.solve(prob.b, tol=1e-12)
    A = H.csr_of(prob)
    bn = np.linalg.norm(prob.b)
    x_g, ig = g.solve(T(prob.b), tol=1e-8)
    x_g = x_g.cpu().numpy()
    assert ig["status"] == 0 and np.linalg.norm(A @ x_g - prob.b) <= 1e-8 * bn * (1 + 1e-6)
    assert abs(ig["iters"] - io["iters"]) <= 1, (ig, io)
    assert np.linalg.norm(x_g - x_o) <= 1e-6 * np.linalg.norm(x_o)
    g.set_precision(1)
    x_m, im = g.solve(T(prob.b), tol=1e-8)
    x_m = x_m.cpu().numpy()
    err = np.linalg.norm(x_m - x_12) / np.linalg.norm(x_12)
    print(f"[octree] {name} smoother {smoother}: fp64 iters {ig['iters']} (oracle {io['iters']}); fp32-precond "
          f"iters {im['iters']} err vs fp64 oracle (1e-12) {err:.2e}", flush=True)
    assert im["status"] == 0 and np.linalg.norm(A @ x_m - prob.b) <= 1e-8 * bn * (1 + 1e-6)
    assert err <= 1e-6
    g.close()
    o.close()


def test_octree_values_update_equals_fresh_setup():
    """A values update on an octree hierarchy (new coefficients, same mesh) equals a fresh octree setup of the new
    system bit for bit, and the oracle's hierarchy of it."""
    prob = problem("cube17")
    d = np.random.default_rng(11).uniform(0.5, 2.0, prob.n)
    A = H.csr_of(prob)
    import scipy.sparse as sp
    B = (sp.diags(d) @ A @ sp.diags(d)).tocsr()
    B.sort_indices()
    new = mg.Problem("cube17_scaled", prob.coords, prob.row_ptr, prob.col, _values_on_pattern(prob, B), prob.b,
                     prob.box, {})
    g = gpu_hier(prob)
    g.update_problem(new)
    f = gpu_hier(new)
    o = oracle.setup_problem(new)
    for level in range(1, g.num_levels):
        eg, ef, eo = g.export_level(level), f.export_level(level), o.export_level(level)
        np.testing.assert_array_equal(eg["ax"], ef["ax"])
        np.testing.assert_array_equal(eg["ax"], eo["ax"])
    xg, ig = g.solve(T(new.b), tol=1e-8)
    xf, if_ = f.solve(T(new.b), tol=1e-8)
    assert ig["iters"] == if_["iters"] and torch.equal(xg, xf)
    g.close()
    f.close()
    o.close()


def _values_on_pattern(prob, B):
    """B's entries in the order of prob's CSR (same pattern)."""
    rows = np.repeat(np.arange(prob.n), np.diff(prob.row_ptr))
    return np.asarray(B[rows, prob.col]).ravel()
