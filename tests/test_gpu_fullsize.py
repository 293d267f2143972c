"""Parity at the benchmark configurations' full sizes, in the launch configuration bench.py times (engine on, the
exact-block fine smoother bench.py uses by default; the 1M-unknown system also with the substitution smoother).

- quasi-uniform 1024x1024 jittered Delaunay (1,044,484 unknowns) and the 16x16 kappa checkerboard on 1416x1416
  (1,999,396 unknowns), each with both fine smoothers: whole hierarchy bit-exact, FP64 solve vs the oracle's solve
  (iterations +-1, relative error <= 1e-6 at 1e-8), mixed solve (true residual <= 1e-8) within 1e-6 of the FP64
  oracle solved to 1e-12.
- graded Delaunay, ~4.0M unknowns, with both fine smoothers: whole hierarchy bit-exact, one preconditioner
  application vs the oracle's, FP64 solve vs the oracle's (iterations +-1, relative error <= 1e-6 at 1e-8) and the
  mixed solve within 1e-6 of the oracle's.
"""
import time

import numpy as np
import pytest

import oracle
from paper_1209_5421_amd import meshgen as mg
from tests import helpers as H

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def log(msg):
    print(f"[fullsize] {msg}", flush=True)


_cache = {}


def problem(name):
    if name not in _cache:
        t = time.time()
        _cache[name] = {"c2": lambda: mg.jittered_problem(1024),
                        "c4": lambda: mg.jittered_problem(1416, kappa_tiles=16),
                        "c3": lambda: mg.graded_problem(4_000_000, progress=log)}[name]()
        log(f"{name}: n={_cache[name].n} generated in {time.time() - t:.1f}s")
    return _cache[name]


def T(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda:0")


def hier(prob, **kw):
    from paper_1209_5421_amd import amg
    return amg.Hierarchy.from_problem(prob, device="cuda:0", **kw)


def assert_hierarchy_equal(g, o):
    assert g.num_levels == o.num_levels
    a, b = g.export_level(0), o.export_level(0)
    np.testing.assert_array_equal(a["agg"], b["agg"])
    np.testing.assert_array_equal(a["color"], b["color"])
    for level in range(1, g.num_levels):
        a, b = g.export_level(level, f32=True), o.export_level(level)
        for key in ("aj", "ax", "ovf_ptr", "ovf_col", "ovf_val"):
            np.testing.assert_array_equal(a[key], b[key], err_msg=f"level {level} {key}")
        np.testing.assert_array_equal(a["ax32"], b["ax"].astype(np.float32))


@pytest.mark.timeout(600)
@pytest.mark.parametrize("name,smoother", [("c2", 1), ("c2", 0), ("c4", 1), ("c4", 0)])
def test_fullsize_solve_parity(name, smoother):
    prob = problem(name)
    g = hier(prob, smoother=smoother)
    o = oracle.setup_problem(prob)
    if smoother:
        o.set_block_smoother(True)
    assert_hierarchy_equal(g, o)
    log(f"{name}: hierarchy bit-exact over {g.num_levels} levels")
    t = time.time()
    x_o, io = o.solve(prob.b, tol=1e-8)
    x_12, i12 = o.solve(prob.b, tol=1e-12)
    log(f"{name}: oracle solves {time.time() - t:.1f}s, {io['iters']} iterations to 1e-8, {i12['iters']} to 1e-12")
    x_g, ig = g.solve(T(prob.b), tol=1e-8)
    x_g = x_g.cpu().numpy()
    assert ig["status"] == 0 and ig["relres"] <= 1e-8
    assert abs(ig["iters"] - io["iters"]) <= 1, (ig, io)
    err = np.linalg.norm(x_g - x_o) / np.linalg.norm(x_o)
    assert err <= 1e-6
    g.set_precision(1)
    x_m, im = g.solve(T(prob.b), tol=1e-8)
    x_m = x_m.cpu().numpy()
    A = H.csr_of(prob)
    assert im["status"] == 0 and np.linalg.norm(A @ x_m - prob.b) <= 1e-8 * np.linalg.norm(prob.b) * (1 + 1e-6)
    err_m = np.linalg.norm(x_m - x_12) / np.linalg.norm(x_12)
    log(f"{name} smoother {smoother}: fp64 iters {ig['iters']} err {err:.2e}; fp32-precond iters {im['iters']} "
        f"relres {im['relres']:.2e} err vs fp64 oracle (1e-12) {err_m:.2e}")
    assert err_m <= 1e-6
    g.close()
    o.close()


@pytest.mark.timeout(900)
@pytest.mark.parametrize("smoother", [1, 0])
def test_fullsize_graded(smoother):
    prob = problem("c3")
    assert 4 ** 10 < prob.n <= 4 ** 11
    g = hier(prob, smoother=smoother)
    o = oracle.setup_problem(prob)
    if smoother:
        o.set_block_smoother(True)
    assert_hierarchy_equal(g, o)
    log(f"c3: hierarchy bit-exact over {g.num_levels} levels, level-L overflow {g.level_info(1)['ovf_nnz']}")
    r = np.random.default_rng(5).standard_normal(prob.n)
    z_o = o.apply_precond(r)
    z_g = g.apply_precond(T(r)).cpu().numpy()
    assert np.linalg.norm(z_g - z_o) <= 1e-10 * np.linalg.norm(z_o)
    t = time.time()
    x_o, io = o.solve(prob.b, tol=1e-8)
    log(f"c3 smoother {smoother}: oracle solve {time.time() - t:.1f}s, {io['iters']} iterations")
    A = H.csr_of(prob)
    g.set_precision(1)
    x_m, im = g.solve(T(prob.b), tol=1e-8)
    g.set_precision(0)
    x_d, idd = g.solve(T(prob.b), tol=1e-8)
    x_m, x_d = x_m.cpu().numpy(), x_d.cpu().numpy()
    bn = np.linalg.norm(prob.b)
    assert io["status"] == 0 and im["status"] == 0 and idd["status"] == 0
    assert np.linalg.norm(A @ x_m - prob.b) <= 1e-8 * bn * (1 + 1e-6)
    assert np.linalg.norm(A @ x_d - prob.b) <= 1e-8 * bn * (1 + 1e-6)
    err = np.linalg.norm(x_d - x_o) / np.linalg.norm(x_o)
    err_m = np.linalg.norm(x_m - x_o) / np.linalg.norm(x_o)
    log(f"c3 smoother {smoother}: fp64 iters {idd['iters']} err {err:.2e}; fp32-precond iters {im['iters']} "
        f"err vs fp64 oracle {err_m:.2e}")
    assert abs(idd["iters"] - io["iters"]) <= 1, (idd, io)
    assert err <= 1e-6 and err_m <= 1e-6
    g.close()
    o.close()


@pytest.mark.timeout(600)
def test_fullsize_time_step():
    """The benchmark's time step on the 1M-unknown mesh: device assembly of a smooth coefficient field (bit-exact
    against the host generator's assembly), a values update of the resident hierarchy (whole hierarchy bit-exact
    against the oracle's setup of the new system), then the FP64 solve against the oracle's."""
    from paper_1209_5421_amd import amg
    prob = problem("c2")
    mesh = prob.meta
    pts, tris, dirichlet = mesh["points"], mesh["tris"], mesh["dirichlet"]
    dof = np.full(len(pts), -1, dtype=np.int32)
    dof[~dirichlet] = np.arange(prob.n, dtype=np.int32)
    ti = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.int32, device="cuda:0")
    pm = amg.P1Mesh(T(pts), ti(tris), ti(dof), prob.n)
    rp, col = pm.pattern()
    np.testing.assert_array_equal(rp.cpu().numpy(), prob.row_ptr)
    np.testing.assert_array_equal(col.cpu().numpy(), prob.col)
    cen = (pts[tris[:, 0]] + pts[tris[:, 1]] + pts[tris[:, 2]]) / 3.0
    kap = 1.0 + 0.5 * np.sin(2 * np.pi * cen[:, 0]) * np.sin(2 * np.pi * cen[:, 1])
    vals = pm.assemble(T(kap))
    _, hrp, hcol, hval = mg.p1_assemble(pts, tris, kap, dirichlet=dirichlet)
    np.testing.assert_array_equal(vals.cpu().numpy(), hval)
    new = mg.Problem("c2_kappa_smooth", prob.coords, hrp, hcol, hval, prob.b, prob.box, {})
    g = hier(prob, precision=1, smoother=1)
    g.solve(T(prob.b), tol=1e-8)
    log("update")
    g.update_values(rp, col, vals)
    o = oracle.setup_problem(new)
    o.set_block_smoother(True)
    assert_hierarchy_equal(g, o)
    x_o, io = o.solve(new.b, tol=1e-8)
    g.set_precision(0)
    x_g, ig = g.solve(T(new.b), tol=1e-8)
    x_g = x_g.cpu().numpy()
    assert ig["status"] == 0 and abs(ig["iters"] - io["iters"]) <= 1, (ig, io)
    assert np.linalg.norm(x_g - x_o) <= 1e-6 * np.linalg.norm(x_o)
    log(f"time step: iters {ig['iters']} (oracle {io['iters']})")
    g.close()
    pm.close()
