"""Parity of the HIP path (through the C ABI) with the CPU oracle, element by element on seeded inputs.

Bars: integer outputs (aggregates, colors, patterns, overflow columns) bit-exact; hierarchy values bit-exact (both
sides sum the same terms in the same order with plain IEEE additions); FP32 hierarchy = round-to-nearest of the FP64
one; smoother / SpMV / preconditioner within a few ulps of accumulated rounding; solves agree to 1e-6 relative error
at 1e-8 relative residual with iteration counts equal within one.
"""
import numpy as np
import pytest

import oracle
from paper_1209_5421_amd import meshgen as mg
from tests import helpers as H

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _amg():
    from paper_1209_5421_amd import amg
    return amg


PROBLEMS = {
    "uniform65": lambda: mg.uniform_problem(64),
    "jittered130": lambda: mg.jittered_problem(130),                 # 16,384 unknowns, L = 6
    "jittered177_kappa": lambda: mg.jittered_problem(177, kappa_tiles=16),  # level-L overflow, same-color pairs
    "graded20k": lambda: mg.graded_problem(20000),                    # level-L overflow, big cells
    "longrange6k": lambda: H.longrange_problem(6000),                 # overflow on every level, no box given
    "two_level": lambda: mg.jittered_problem(16),                     # 196 unknowns: fine + coarsest
    "disk130": lambda: mg.disk_problem(130),                          # a fifth of the cells empty on every level
}

_cache = {}


def problem(name):
    if name not in _cache:
        _cache[name] = PROBLEMS[name]()
    return _cache[name]


def dev():
    return torch.device("cuda:0")


def gpu_hier(prob, **kw):
    print(f"[gpu] setup {prob.name} n={prob.n} nnz={prob.nnz} {kw}", flush=True)
    return _amg().Hierarchy.from_problem(prob, device=dev(), **kw)


def T(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev())


@pytest.mark.parametrize("name", list(PROBLEMS))
def test_hierarchy_bit_exact(name):
    prob = problem(name)
    g = gpu_hier(prob)
    o = oracle.setup_problem(prob)
    assert g.num_levels == o.num_levels
    e0g, e0o = g.export_level(0), o.export_level(0)
    np.testing.assert_array_equal(e0g["agg"], e0o["agg"])
    np.testing.assert_array_equal(e0g["color"], e0o["color"])
    for level in range(1, g.num_levels):
        eg, eo = g.export_level(level, f32=True), o.export_level(level)
        assert eg["n"] == eo["n"] and eg["k"] == eo["k"] and eg["ovf_nnz"] == eo["ovf_nnz"]
        for key in ("agg", "color", "aj", "ovf_ptr", "ovf_col"):
            np.testing.assert_array_equal(eg[key], eo[key], err_msg=f"level {level} {key}")
        np.testing.assert_array_equal(eg["ax"], eo["ax"], err_msg=f"level {level} ax")
        np.testing.assert_array_equal(eg["ovf_val"], eo["ovf_val"], err_msg=f"level {level} ovf_val")
        np.testing.assert_array_equal(eg["ax32"], eo["ax"].astype(np.float32), err_msg=f"level {level} fp32")
    g.close()


@pytest.mark.parametrize("name", ["uniform65", "jittered177_kappa", "graded20k", "longrange6k", "disk130"])
def test_level_spmv_and_smoother(name):
    prob = problem(name)
    g = gpu_hier(prob)
    o = oracle.setup_problem(prob)
    rng = np.random.default_rng(7)
    for level in range(g.num_levels):
        n = g.level_info(level)["n"]
        x = rng.standard_normal(n)
        f = rng.standard_normal(n)
        y_o = o.spmv(level, x)
        y_g = g.spmv(level, T(x)).cpu().numpy()
        scale = np.abs(y_o).max()
        np.testing.assert_allclose(y_g, y_o, rtol=0, atol=1e-13 * scale)
        y32 = g.spmv(level, T(x), precision=1).cpu().numpy()
        np.testing.assert_allclose(y32, y_o, rtol=0, atol=2e-5 * scale)
        if level == g.num_levels - 1:
            continue
        for fwd in (True, False):
            s_o = o.smooth(level, f, x, fwd)
            s_g = g.smooth(level, T(f), T(x), fwd).cpu().numpy()
            np.testing.assert_allclose(s_g, s_o, rtol=0, atol=1e-11 * np.abs(s_o).max(), err_msg=f"{level} {fwd}")
    g.close()


@pytest.mark.parametrize("name", ["jittered130", "jittered177_kappa", "graded20k", "longrange6k", "disk130"])
def test_block_smoother_parity(name):
    """The exact-block fine smoother (smoother=1): sweeps in both directions, the preconditioner and both solve
    precisions against the oracle's exact-block reading (graded20k also has cells above 32 unknowns, which keep the
    substitution on both sides)."""
    prob = problem(name)
    g = gpu_hier(prob, smoother=1)
    o = oracle.setup_problem(prob)
    o.set_block_smoother(True)
    rng = np.random.default_rng(7)
    x, f = rng.standard_normal(prob.n), rng.standard_normal(prob.n)
    for fwd in (True, False):
        s_o = o.smooth(0, f, x, fwd)
        s_g = g.smooth(0, T(f), T(x), fwd).cpu().numpy()
        np.testing.assert_allclose(s_g, s_o, rtol=0, atol=1e-11 * np.abs(s_o).max(), err_msg=f"fwd={fwd}")
        s32 = g.smooth(0, T(f), T(x), fwd, precision=1).cpu().numpy()
        np.testing.assert_allclose(s32, s_o, rtol=0, atol=1e-4 * np.abs(s_o).max(), err_msg=f"fp32 fwd={fwd}")
    r = rng.standard_normal(prob.n)
    z_o = o.apply_precond(r)
    z_g = g.apply_precond(T(r)).cpu().numpy()
    assert np.linalg.norm(z_g - z_o) <= 1e-10 * np.linalg.norm(z_o)
    x_o, io = o.solve(prob.b, tol=1e-8)
    A = H.csr_of(prob)
    for prec in (0, 1):
        g.set_precision(prec)
        x_g, ig = g.solve(T(prob.b), tol=1e-8)
        x_g = x_g.cpu().numpy()
        assert ig["status"] == 0 and ig["relres"] <= 1e-8
        assert np.linalg.norm(A @ x_g - prob.b) <= 1e-8 * np.linalg.norm(prob.b) * (1 + 1e-6)
        assert abs(ig["iters"] - io["iters"]) <= 1, (prec, ig, io)
        assert np.linalg.norm(x_g - x_o) <= 1e-6 * np.linalg.norm(x_o)
    g.close()


@pytest.mark.parametrize("name", list(PROBLEMS))
def test_preconditioner_parity(name):
    prob = problem(name)
    g = gpu_hier(prob)
    o = oracle.setup_problem(prob)
    r = np.random.default_rng(9).standard_normal(prob.n)
    z_o = o.apply_precond(r)
    z_g = g.apply_precond(T(r)).cpu().numpy()
    assert np.linalg.norm(z_g - z_o) <= 1e-10 * np.linalg.norm(z_o)
    z32 = g.apply_precond(T(r), precision=1).cpu().numpy()
    assert np.linalg.norm(z32 - z_o) <= 1e-3 * np.linalg.norm(z_o)
    g.close()


@pytest.mark.parametrize("name", list(PROBLEMS))
def test_solve_parity_fp64(name):
    prob = problem(name)
    g = gpu_hier(prob)
    o = oracle.setup_problem(prob)
    x_o, io = o.solve(prob.b, tol=1e-8)
    x_g, ig = g.solve(T(prob.b), tol=1e-8)
    x_g = x_g.cpu().numpy()
    A = H.csr_of(prob)
    assert io["status"] == 0 and ig["status"] == 0
    assert ig["relres"] <= 1e-8
    assert np.linalg.norm(A @ x_g - prob.b) <= 1e-8 * np.linalg.norm(prob.b) * (1 + 1e-6)
    assert abs(ig["iters"] - io["iters"]) <= 1, (ig, io)
    assert np.linalg.norm(x_g - x_o) <= 1e-6 * np.linalg.norm(x_o)
    g.close()


@pytest.mark.parametrize("name", ["uniform65", "jittered130", "jittered177_kappa", "graded20k", "disk130"])
def test_solve_mixed_precision(name):
    prob = problem(name)
    g = gpu_hier(prob, precision=1)
    o = oracle.setup_problem(prob)
    x_ref, _ = o.solve(prob.b, tol=1e-12)
    x_g, ig = g.solve(T(prob.b), tol=1e-8)
    x_g = x_g.cpu().numpy()
    A = H.csr_of(prob)
    assert ig["status"] == 0 and ig["relres"] <= 1e-8
    assert np.linalg.norm(A @ x_g - prob.b) <= 1e-8 * np.linalg.norm(prob.b) * (1 + 1e-6)
    err = np.linalg.norm(x_g - x_ref) / np.linalg.norm(x_ref)
    print(f"[gpu] mixed {name}: iters={ig['iters']} relres={ig['relres']:.2e} err_vs_fp64_oracle={err:.2e}")
    assert err <= 1e-6
    g.close()


@pytest.mark.parametrize("name", ["uniform65", "jittered130", "longrange6k", "disk130"])
@pytest.mark.parametrize("precision", [0, 1])
def test_engine_matches_per_step_launches(name, precision):
    """The persistent small-level workgroup and the launch-per-step path compute the same preconditioner (their
    inner products use different reduction trees, so agreement is to rounding)."""
    prob = problem(name)
    ga = gpu_hier(prob, engine=1)
    gb = gpu_hier(prob, engine=0)
    r = T(np.random.default_rng(3).standard_normal(prob.n))
    za = ga.apply_precond(r, precision=precision).cpu().numpy()
    zb = gb.apply_precond(r, precision=precision).cpu().numpy()
    tol = 1e-11 if precision == 0 else 1e-4
    assert np.linalg.norm(za - zb) <= tol * np.linalg.norm(zb)
    ga.set_precision(precision)
    gb.set_precision(precision)
    xa, ia = ga.solve(T(prob.b))
    xb, ib = gb.solve(T(prob.b))
    assert abs(ia["iters"] - ib["iters"]) <= 1
    assert torch.linalg.norm(xa - xb) <= 1e-6 * torch.linalg.norm(xb)
    ga.close()
    gb.close()


def _tile_problem():
    # 88,804 unknowns, L = 8: levels of 4,096 to 65,536 cells above the engine in both precisions, each with squares
    # of 16 x 16 super-cells inside the grid and along its edges
    if "jittered300" not in _cache:
        _cache["jittered300"] = mg.jittered_problem(300)
    return _cache["jittered300"]


@pytest.mark.parametrize("precision", [0, 1])
def test_tiled_tree_levels(precision):
    """The tree levels' tiled launches (engine on: presmoothing with the restriction, and the first post-smoothing
    sweep, on 16 x 16 super-cell squares with staged rings) against one launch per color phase (engine off) and, in
    FP64, the oracle: the same preconditioner to rounding (the engine's levels below use other reduction trees)."""
    prob = _tile_problem()
    ga = gpu_hier(prob, engine=1)
    gb = gpu_hier(prob, engine=0)
    info = ga.engine_info(precision)
    print(f"[gpu] tiles p{precision}: engine {info}", flush=True)
    assert info["top_level"] >= 2, "no tree level above the engine"
    r = T(np.random.default_rng(5).standard_normal(prob.n))
    za = ga.apply_precond(r, precision=precision).cpu().numpy()
    zb = gb.apply_precond(r, precision=precision).cpu().numpy()
    tol = 1e-11 if precision == 0 else 1e-4
    assert np.linalg.norm(za - zb) <= tol * np.linalg.norm(zb)
    if precision == 0:
        o = oracle.setup_problem(prob)
        z_o = o.apply_precond(r.cpu().numpy())
        assert np.linalg.norm(za - z_o) <= 1e-10 * np.linalg.norm(z_o)
        o.close()
    ga.set_precision(precision)
    gb.set_precision(precision)
    xa, ia = ga.solve(T(prob.b))
    xb, ib = gb.solve(T(prob.b))
    assert ia["status"] == 0 and abs(ia["iters"] - ib["iters"]) <= 1
    assert torch.linalg.norm(xa - xb) <= 1e-6 * torch.linalg.norm(xb)
    ga.close()
    gb.close()


@pytest.mark.parametrize("name", ["uniform65", "jittered130", "jittered177_kappa", "graded20k", "disk130"])
@pytest.mark.parametrize("precision", [0, 1])
def test_specialised_engine_matches_interpreter(name, precision):
    """The specialised small-level engine (compile-time levels, B~ of the 256-cell level in one wavefront) against
    the generic step interpreter (engine = 2) and the oracle: the same preconditioner to rounding (different
    reduction trees; in FP32 the interpreter applies B^ of the 256-cell level as a precomputed matrix), the solves
    within the parity bar."""
    prob = problem(name)
    ga = gpu_hier(prob, engine=1)
    gb = gpu_hier(prob, engine=2)
    ia, ib = ga.engine_info(precision), gb.engine_info(precision)
    print(f"[gpu] engine {name} p{precision}: specialised {ia} interpreter {ib}", flush=True)
    assert ia["steps"] < ib["steps"], "the specialised engine was not selected"
    r = T(np.random.default_rng(3).standard_normal(prob.n))
    za = ga.apply_precond(r, precision=precision).cpu().numpy()
    zb = gb.apply_precond(r, precision=precision).cpu().numpy()
    tol = 1e-11 if precision == 0 else 1e-4
    assert np.linalg.norm(za - zb) <= tol * np.linalg.norm(zb)
    if precision == 0:
        o = oracle.setup_problem(prob)
        z_o = o.apply_precond(r.cpu().numpy())
        assert np.linalg.norm(za - z_o) <= 1e-10 * np.linalg.norm(z_o)
        o.close()
    ga.set_precision(precision)
    gb.set_precision(precision)
    xa, ia_ = ga.solve(T(prob.b))
    xb, ib_ = gb.solve(T(prob.b))
    assert ia_["status"] == 0 and abs(ia_["iters"] - ib_["iters"]) <= 1
    assert torch.linalg.norm(xa - xb) <= 1e-6 * torch.linalg.norm(xb)
    ga.close()
    gb.close()


@pytest.mark.parametrize("name", ["uniform65", "jittered130", "graded20k", "disk130"])
@pytest.mark.parametrize("precision", [0, 1])
def test_all_directions_outer_iteration(name, precision):
    """outer_mmax = -1: Algorithm 2.1 as written, every new direction orthogonalised against all earlier ones,
    against the oracle's same form (mmax = -1): iterations +-1, relative error <= 1e-6 at 1e-8 (the FP32
    preconditioner against the oracle solved to 1e-12)."""
    prob = problem(name)
    g = gpu_hier(prob, outer_mmax=-1, precision=precision)
    o = oracle.setup_problem(prob)
    x_o, io = o.solve(prob.b, tol=1e-8, mmax=-1)
    x_g, ig = g.solve(T(prob.b), tol=1e-8)
    x_g = x_g.cpu().numpy()
    A = H.csr_of(prob)
    assert ig["status"] == 0 and np.linalg.norm(A @ x_g - prob.b) <= 1e-8 * np.linalg.norm(prob.b) * (1 + 1e-6)
    ref = x_o if precision == 0 else o.solve(prob.b, tol=1e-12, mmax=-1)[0]
    err = np.linalg.norm(x_g - ref) / np.linalg.norm(ref)
    print(f"[gpu] all directions {name} p{precision}: iters {ig['iters']} (oracle {io['iters']}) err {err:.2e}")
    if precision == 0:
        assert abs(ig["iters"] - io["iters"]) <= 1, (ig, io)
    assert err <= 1e-6
    # a second solve on the same hierarchy reuses the kept direction storage and gives the same result
    x_2, i2 = g.solve(T(prob.b), tol=1e-8)
    assert i2["iters"] == ig["iters"] and np.array_equal(x_2.cpu().numpy(), x_g)
    g.close()
    o.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_caller_allocator(precision):
    """Hierarchy memory from the caller's allocator (amg_options.alloc / dealloc: torch's caching allocator): the
    same hierarchy and solution as the library's own pool, bit for bit, and every block handed back on free."""
    from paper_1209_5421_amd import amg
    prob = problem("jittered130")
    ta = amg.TorchAllocator("cuda:0")
    ga = gpu_hier(prob, precision=precision, allocator=ta)
    gb = gpu_hier(prob, precision=precision)
    assert ta.live > 0
    for level in range(1, ga.num_levels):
        np.testing.assert_array_equal(ga.export_level(level)["ax"], gb.export_level(level)["ax"])
    xa, ia = ga.solve(T(prob.b))
    xb, ib = gb.solve(T(prob.b))
    assert ia["iters"] == ib["iters"] and torch.equal(xa, xb)
    ga.update_problem(prob)  # temporaries of a values update come from the same allocator
    xa2, _ = ga.solve(T(prob.b))
    assert torch.equal(xa2, xb)
    ga.close()
    gb.close()
    assert ta.live == 0


@pytest.mark.parametrize("sweeps,inner", [(2, 2), (1, 1), (3, 1)])
@pytest.mark.parametrize("engine", [1, 0])
@pytest.mark.parametrize("name", ["jittered130", "jittered177_kappa"])
def test_cycle_options_parity(name, engine, sweeps, inner):
    """Non-default cycle options against the oracle with the same options: several smoothing sweeps (the folds of
    the first and last relaxation then apply to one sweep only) and one inner step of Algorithm 2.1 (nothing
    folded, no deferred update); engine on (small levels in the persistent workgroup) and off (every level per
    step)."""
    prob = problem(name)
    g = gpu_hier(prob, engine=engine, sweeps=sweeps, inner_iters=inner)
    o = oracle.setup_problem(prob, sweeps=sweeps, inner_iters=inner)
    r = np.random.default_rng(11).standard_normal(prob.n)
    z_o = o.apply_precond(r)
    z_g = g.apply_precond(T(r)).cpu().numpy()
    assert np.linalg.norm(z_g - z_o) <= 1e-10 * np.linalg.norm(z_o)
    x_o, io = o.solve(prob.b, tol=1e-8)
    A = H.csr_of(prob)
    for prec in (0, 1):
        g.set_precision(prec)
        x_g, ig = g.solve(T(prob.b), tol=1e-8)
        x_g = x_g.cpu().numpy()
        assert ig["status"] == 0 and np.linalg.norm(A @ x_g - prob.b) <= 1e-8 * np.linalg.norm(prob.b) * (1 + 1e-6)
        assert abs(ig["iters"] - io["iters"]) <= 1, (prec, ig, io)
        assert np.linalg.norm(x_g - x_o) <= 1e-6 * np.linalg.norm(x_o)
    g.close()


def test_single_level_direct():
    prob = mg.jittered_problem(9)  # 49 unknowns <= 64
    g = gpu_hier(prob)
    assert g.num_levels == 1
    x, info = g.solve(T(prob.b), tol=1e-12)
    xs = np.linalg.solve(H.csr_of(prob).toarray(), prob.b)
    np.testing.assert_allclose(x.cpu().numpy(), xs, rtol=1e-11, atol=1e-13)
    assert info["iters"] <= 2
    g.close()


def test_repeated_setup_reuses_memory():
    """Freed hierarchies leave their blocks for later ones of the same size: a run of setup / solve / free cycles
    on one system holds the device memory of one hierarchy (plus the cache), not one per cycle, and every cycle
    gives the same solution."""
    prob = problem("jittered177_kappa")
    b = T(prob.b)
    xs, used = [], []
    for cycle in range(6):
        g = gpu_hier(prob, smoother=cycle % 2)
        x, info = g.solve(b, tol=1e-8)
        assert info["status"] == 0
        xs.append((cycle % 2, x.cpu().numpy()))
        g.close()
        torch.cuda.synchronize()
        free, total = torch.cuda.mem_get_info()
        used.append(total - free)
    # after the first cycle of each smoother, device use stays flat (within 1 MiB of slack)
    assert max(used[2:]) - used[1] <= 1 << 20, used
    for sm in (0, 1):
        same = [x for s_, x in xs if s_ == sm]
        for x in same[1:]:
            np.testing.assert_array_equal(x, same[0])


def test_zero_rhs_and_determinism():
    prob = problem("jittered130")
    g = gpu_hier(prob)
    x, info = g.solve(torch.zeros(prob.n, dtype=torch.float64, device=dev()))
    assert info["iters"] == 0 and not x.any()
    x1, i1 = g.solve(T(prob.b))
    x2, i2 = g.solve(T(prob.b))
    assert torch.equal(x1, x2) and i1["iters"] == i2["iters"]
    g.set_precision(1)
    y1, _ = g.solve(T(prob.b))
    y2, _ = g.solve(T(prob.b))
    assert torch.equal(y1, y2)
    g.close()


def test_error_paths():
    amg = _amg()
    prob = mg.jittered_problem(20)
    with pytest.raises(amg.AMGError) as e:
        gpu_hier(prob, box=(0.2, 1.0, 0.0, 1.0))
    assert e.value.code == amg.INVALID
    bad = mg.jittered_problem(20)
    bad.coords = bad.coords.copy()
    bad.coords[3, 0] = np.nan
    with pytest.raises(amg.AMGError) as e:
        gpu_hier(bad)
    assert e.value.code == amg.INVALID
    neg = mg.jittered_problem(20)
    rows = np.repeat(np.arange(neg.n), np.diff(neg.row_ptr))
    neg.val = neg.val.copy()
    neg.val[(rows == 5) & (neg.col == 5)] = -2.0
    with pytest.raises(amg.AMGError) as e:
        gpu_hier(neg)
    assert e.value.code == amg.NOT_SPD
    with pytest.raises(amg.AMGError) as e:
        gpu_hier(prob, smoother=2)
    assert e.value.code == amg.INVALID
    badcol = mg.jittered_problem(20)
    badcol.col = badcol.col.copy()
    badcol.col[10] = badcol.n + 5
    with pytest.raises(amg.AMGError) as e:
        gpu_hier(badcol)
    assert e.value.code == amg.INVALID
    g = gpu_hier(prob, max_iters=1)
    x, info = g.solve(T(prob.b), check=False)
    assert info["status"] == amg.NOCONV and info["iters"] == 1
    g.close()


@pytest.mark.parametrize("smoother", [0, 1])
@pytest.mark.parametrize("name", list(PROBLEMS))
def test_footprint_within_estimate(name, smoother):
    """amg_estimate_bytes (used for admission by HBM footprint) bounds what a hierarchy actually holds."""
    prob = problem(name)
    g = gpu_hier(prob, smoother=smoother)
    est = _amg().estimate_bytes(prob.n, prob.nnz, smoother=smoother)
    print(f"[gpu] {name} smoother {smoother}: {g.bytes()} bytes held, estimate {est}", flush=True)
    assert 0 < g.bytes() <= est
    g.close()


@pytest.mark.parametrize("smoother", [0, 1])
def test_footprint_within_estimate_large(smoother):
    prob = mg.jittered_problem(700, fast=True)
    g = gpu_hier(prob, smoother=smoother)
    est = _amg().estimate_bytes(prob.n, prob.nnz, smoother=smoother)
    print(f"[gpu] jittered700: {g.bytes()} bytes held ({g.bytes() / prob.n:.0f} per unknown), estimate {est}",
          flush=True)
    assert 0 < g.bytes() <= est
    g.close()


_cluster = {}


@pytest.mark.parametrize("smoother", [1, 0])
def test_big_cell_beyond_lds(smoother):
    """One level-L cell of 13,001 unknowns (a random cluster inside a jittered lattice): more than the big-cell
    substitution stages in LDS (12,288 FP32 or 6,144 FP64 values), so its in-cell substitution takes the kernel's
    global-memory path in both precisions. Hierarchy bit-exact; one preconditioner application against the oracle's
    (FP64 1e-10, FP32 1e-4); the FP64 solve to 1e-8 within one iteration of the oracle's and 1e-6 of its solution."""
    if "p" not in _cluster:
        _cluster["p"] = H.cluster_problem()
    prob = _cluster["p"]
    g = gpu_hier(prob, smoother=smoother)
    agg = g.export_level(0)["agg"]
    assert np.bincount(agg).max() > 12288, "the cluster does not exceed the LDS staging"
    o = oracle.setup_problem(prob)
    o.set_block_smoother(bool(smoother))
    for level in range(g.num_levels):
        assert _level_bytes(g.export_level(level)) == _level_bytes(o.export_level(level)), level
    r = np.random.default_rng(7).standard_normal(prob.n)
    z_o = o.apply_precond(r)
    z64 = g.apply_precond(T(r), precision=0).cpu().numpy()
    z32 = g.apply_precond(T(r), precision=1).cpu().numpy()
    e64 = np.linalg.norm(z64 - z_o) / np.linalg.norm(z_o)
    e32 = np.linalg.norm(z32 - z_o) / np.linalg.norm(z_o)
    x_o, io = o.solve(prob.b, tol=1e-8)
    x, info = g.solve(T(prob.b), tol=1e-8)
    x = x.cpu().numpy()
    ex = np.linalg.norm(x - x_o) / np.linalg.norm(x_o)
    print(f"[gpu] cluster smoother {smoother}: precond {e64:.1e} (FP32 {e32:.1e}); iters {info['iters']} "
          f"(oracle {io['iters']}), solution {ex:.1e}", flush=True)
    assert e64 <= 1e-10 and e32 <= 1e-4
    assert info["status"] == 0 and abs(info["iters"] - io["iters"]) <= 1 and ex <= 1e-6
    g.close()
    o.close()


def _level_bytes(lv):
    """Integer and value arrays of an exported level, for an exact comparison."""
    keys = [k for k in ("agg", "color", "aj", "ax", "ovf_ptr", "ovf_col", "ovf_val") if k in lv]
    return [(k, lv[k].tobytes()) for k in keys]
