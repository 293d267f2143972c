"""amg_update_values: new matrix values on the pattern given to setup.

The aggregation of Section 3 depends on the points and the pattern only, so an update re-runs the numeric part of
setup (eq. 11 on every level, the smoother's data, the coarsest factor) in place. Bars: the updated hierarchy equals
a fresh setup on the new values bit for bit (levels, FP32 copies, smoother, preconditioner, solves), its levels
equal the oracle's bit for bit, and its solves meet the usual parity bar against the oracle. The new values are
D A D + diag(sigma) for a random positive diagonal D and shift sigma (an implicit time step's M / dt + A has this
form), or a coefficient field on the same mesh.
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


def dev():
    return torch.device("cuda:0")


def T(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev())


def rescaled(prob, seed):
    """D A D + diag(sigma): same pattern, symmetric positive definite, new values on every level."""
    rng = np.random.default_rng(seed)
    d = rng.uniform(0.5, 2.0, prob.n)
    rows = np.repeat(np.arange(prob.n), np.diff(prob.row_ptr))
    on_diag = rows == prob.col
    diag = np.zeros(prob.n)
    np.add.at(diag, rows[on_diag], prob.val[on_diag])
    sigma = rng.uniform(0.0, 0.1, prob.n) * diag
    val = prob.val * (d[rows] * d[prob.col]) + np.where(on_diag, sigma[rows], 0.0)
    return mg.Problem(**{**prob.__dict__, "name": prob.name + f"_rescaled{seed}", "val": val})


PROBLEMS = {
    "uniform65": lambda: mg.uniform_problem(64),
    "jittered130": lambda: mg.jittered_problem(130),
    "graded20k": lambda: mg.graded_problem(20000),        # level-L overflow, cells above 32 unknowns
    "longrange6k": lambda: H.longrange_problem(6000),     # overflow on every level
    "two_level": lambda: mg.jittered_problem(16),
    "disk130": lambda: mg.disk_problem(130),              # empty cells on every level
}

_cache = {}


def problem(name):
    if name not in _cache:
        _cache[name] = PROBLEMS[name]()
    return _cache[name]


def gpu_hier(prob, **kw):
    print(f"[gpu] setup {prob.name} n={prob.n} nnz={prob.nnz} {kw}", flush=True)
    return _amg().Hierarchy.from_problem(prob, device=dev(), **kw)


def assert_same_hierarchy(a, b):
    assert a.num_levels == b.num_levels
    for level in range(1, a.num_levels):
        ea, eb = a.export_level(level, f32=True), b.export_level(level, f32=True)
        for key in ("agg", "color", "aj", "ax", "ax32", "ovf_ptr", "ovf_col", "ovf_val"):
            np.testing.assert_array_equal(ea[key], eb[key], err_msg=f"level {level} {key}")


@pytest.mark.parametrize("smoother", [0, 1])
@pytest.mark.parametrize("name", list(PROBLEMS))
def test_update_equals_fresh_setup(name, smoother):
    prob = problem(name)
    new = rescaled(prob, 11)
    g = gpu_hier(prob, smoother=smoother)
    x_old, _ = g.solve(T(prob.b), tol=1e-8)      # the hierarchy has been used before it is updated
    print(f"[gpu] update {name} smoother={smoother}", flush=True)
    g.update_problem(new)
    f = gpu_hier(new, smoother=smoother)
    assert_same_hierarchy(g, f)
    rng = np.random.default_rng(3)
    r, x0 = rng.standard_normal(prob.n), rng.standard_normal(prob.n)
    for prec in (0, 1):
        assert torch.equal(g.apply_precond(T(r), precision=prec), f.apply_precond(T(r), precision=prec))
        if g.num_levels > 1:
            for fwd in (True, False):
                assert torch.equal(g.smooth(0, T(r), T(x0), fwd, precision=prec),
                                   f.smooth(0, T(r), T(x0), fwd, precision=prec))
        g.set_precision(prec)
        f.set_precision(prec)
        xg, ig = g.solve(T(new.b), tol=1e-8)
        xf, if_ = f.solve(T(new.b), tol=1e-8)
        assert ig["status"] == 0 and ig["iters"] == if_["iters"]
        assert torch.equal(xg, xf), prec
    # against the oracle on the new values
    o = oracle.setup_problem(new)
    o.set_block_smoother(bool(smoother))
    for level in range(1, g.num_levels):
        eg, eo = g.export_level(level), o.export_level(level)
        np.testing.assert_array_equal(eg["ax"], eo["ax"], err_msg=f"level {level}")
        np.testing.assert_array_equal(eg["ovf_val"], eo["ovf_val"], err_msg=f"level {level}")
    x_o, io = o.solve(new.b, tol=1e-8)
    g.set_precision(0)
    x_g, ig = g.solve(T(new.b), tol=1e-8)
    x_g = x_g.cpu().numpy()
    A = H.csr_of(new)
    assert np.linalg.norm(A @ x_g - new.b) <= 1e-8 * np.linalg.norm(new.b) * (1 + 1e-6)
    assert abs(ig["iters"] - io["iters"]) <= 1, (ig, io)
    assert np.linalg.norm(x_g - x_o) <= 1e-6 * np.linalg.norm(x_o)
    assert not np.array_equal(x_g, x_old.cpu().numpy())
    g.close()
    f.close()


def test_update_coefficient_field():
    """Poisson, then a 16 x 16 checkerboard of coefficients 10^U[-3,3] on the same mesh, in mixed precision."""
    pois = mg.jittered_problem(177)
    kap = mg.jittered_problem(177, kappa_tiles=16)
    np.testing.assert_array_equal(pois.row_ptr, kap.row_ptr)
    np.testing.assert_array_equal(pois.col, kap.col)
    g = gpu_hier(pois, precision=1, smoother=1)
    g.update_problem(kap)
    f = gpu_hier(kap, precision=1, smoother=1)
    assert_same_hierarchy(g, f)
    xg, ig = g.solve(T(kap.b), tol=1e-8)
    xf, if_ = f.solve(T(kap.b), tol=1e-8)
    assert ig["status"] == 0 and ig["iters"] == if_["iters"] and torch.equal(xg, xf)
    o = oracle.setup_problem(kap)
    o.set_block_smoother(True)
    x_o, io = o.solve(kap.b, tol=1e-8)
    assert abs(ig["iters"] - io["iters"]) <= 1
    assert np.linalg.norm(xg.cpu().numpy() - x_o) <= 1e-6 * np.linalg.norm(x_o)
    g.close()
    f.close()


def test_update_single_level():
    prob = mg.jittered_problem(9)  # 49 unknowns: the coarsest solve only
    new = rescaled(prob, 5)
    g = gpu_hier(prob)
    assert g.num_levels == 1
    g.update_problem(new)
    x, info = g.solve(T(new.b), tol=1e-12)
    xs = np.linalg.solve(H.csr_of(new).toarray(), new.b)
    np.testing.assert_allclose(x.cpu().numpy(), xs, rtol=1e-11, atol=1e-13)
    g.close()


def test_update_rejections_leave_hierarchy_unchanged():
    amg = _amg()
    prob = problem("jittered130")
    g = gpu_hier(prob, smoother=1)
    x_ref, i_ref = g.solve(T(prob.b), tol=1e-8)
    # a column order that differs in one row
    swapped = mg.Problem(**{**prob.__dict__, "col": prob.col.copy()})
    r0 = prob.row_ptr[7]
    swapped.col[r0], swapped.col[r0 + 1] = prob.col[r0 + 1], prob.col[r0]
    # another mesh of the same size has another pattern
    other = mg.jittered_problem(130, seed=5)
    # a non-positive diagonal entry
    neg = mg.Problem(**{**prob.__dict__, "val": prob.val.copy()})
    rows = np.repeat(np.arange(prob.n), np.diff(prob.row_ptr))
    neg.val[(rows == 5) & (prob.col == 5)] = -1.0
    for bad, code in ((swapped, amg.INVALID), (other, amg.INVALID), (neg, amg.NOT_SPD)):
        if bad is other and other.nnz == prob.nnz and np.array_equal(other.col, prob.col):
            continue
        with pytest.raises(amg.AMGError) as e:
            g.update_problem(bad)
        assert e.value.code == code
        x, info = g.solve(T(prob.b), tol=1e-8)
        assert torch.equal(x, x_ref) and info["iters"] == i_ref["iters"]
    # wrong length: refused before any device work
    t = lambda a, dt: torch.as_tensor(a, dtype=dt, device=dev())
    with pytest.raises(amg.AMGError) as e:
        g.update_values(t(prob.row_ptr, torch.int64), t(prob.col[:-1], torch.int32), t(prob.val[:-1], torch.float64))
    assert e.value.code == amg.INVALID
    g.close()


def test_failed_update_is_refused_until_a_good_one():
    """Positive diagonals but indefinite cell blocks: the exact-block factors fail after the values began to change,
    so the hierarchy refuses solves until a valid update."""
    amg = _amg()
    prob = problem("jittered130")
    g = gpu_hier(prob, smoother=1)
    x_ref, _ = g.solve(T(prob.b), tol=1e-8)
    rows = np.repeat(np.arange(prob.n), np.diff(prob.row_ptr))
    bad = mg.Problem(**{**prob.__dict__, "val": np.where(rows == prob.col, prob.val, 10.0 * prob.val)})
    with pytest.raises(amg.AMGError) as e:
        g.update_problem(bad)
    assert e.value.code == amg.NOT_SPD
    x, info = g.solve(T(prob.b), check=False)
    assert info["status"] == amg.INVALID
    with pytest.raises(amg.AMGError) as e:
        g.apply_precond(T(prob.b))
    assert e.value.code == amg.INVALID
    g.update_problem(prob)
    x, info = g.solve(T(prob.b), tol=1e-8)
    assert info["status"] == 0 and torch.equal(x, x_ref)
    g.close()


def test_repeated_updates_hold_memory_flat():
    """Updates return their temporaries: the hierarchy's bytes and the device's use stay flat over many updates, and
    the two alternating value sets give the same solutions every time."""
    prob = problem("disk130")
    vals = [prob, rescaled(prob, 21)]
    g = gpu_hier(prob, precision=1, smoother=1)
    held = g.bytes()
    xs, used = {0: [], 1: []}, []
    for step in range(8):
        g.update_problem(vals[step % 2])
        x, info = g.solve(T(prob.b), tol=1e-8)
        assert info["status"] == 0 and g.bytes() == held
        xs[step % 2].append(x.cpu().numpy())
        torch.cuda.synchronize()
        free, total = torch.cuda.mem_get_info()
        used.append(total - free)
    assert max(used[2:]) - used[1] <= 1 << 20, used
    for k in (0, 1):
        for x in xs[k][1:]:
            np.testing.assert_array_equal(x, xs[k][0])
    g.close()
