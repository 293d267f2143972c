"""The batched serving path (amg_solve_batch): small systems as one whole-solve workgroup each in a shared launch,
large systems on their own host thread and stream, all overlapping.

Bars: a system's result is bit-identical alone and in any mix (same route, no cross-system reduction); the
whole-solve route matches the oracle like amg_solve does (iterations +-1, relative error <= 1e-6 at 1e-8); the two
routes agree to rounding.
"""
import numpy as np
import pytest

import oracle
from paper_1209_5421_amd import meshgen as mg
from tests import helpers as H

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

SIDES = [40, 66, 100, 140, 200, 258]  # 1.4k .. 65.5k unknowns (all take the whole-solve route)

_cache = {}


def prob(side, kappa=0):
    key = (side, kappa)
    if key not in _cache:
        _cache[key] = mg.jittered_problem(side, kappa_tiles=kappa, rhs_seed=100 + side, fast=True)
    return _cache[key]


def T(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda:0")


def hier(p, **kw):
    from paper_1209_5421_amd import amg
    print(f"[batch] setup n={p.n} {kw}", flush=True)
    return amg.Hierarchy.from_problem(p, device="cuda:0", **kw)


def solve_batch(hs, probs, tol=1e-8):
    from paper_1209_5421_amd import amg
    bs = [T(p.b) for p in probs]
    xs = [torch.empty_like(b) for b in bs]
    code, infos = amg.solve_batch(hs, bs, xs, [tol] * len(hs))
    torch.cuda.synchronize()
    return code, [x.cpu().numpy() for x in xs], infos


@pytest.mark.parametrize("precision", [0, 1])
def test_alone_equals_in_the_mix(precision):
    probs = [prob(s) for s in SIDES] + [prob(120, 16)]
    hs = [hier(p, precision=precision) for p in probs]
    code, xs_mix, infos_mix = solve_batch(hs, probs)
    assert code == 0
    for h, p, x_mix, i_mix in zip(hs, probs, xs_mix, infos_mix):
        code1, (x1,), (i1,) = solve_batch([h], [p])
        assert code1 == 0
        assert np.array_equal(x1, x_mix) and i1["iters"] == i_mix["iters"], p.name
        A = H.csr_of(p)
        assert np.linalg.norm(A @ x1 - p.b) <= 1e-8 * np.linalg.norm(p.b) * (1 + 1e-6)
    for h in hs:
        h.close()


def test_whole_solve_route_matches_oracle_and_amg_solve():
    for side in (66, 140, 258):
        p = prob(side)
        h = hier(p)
        code, (xb,), (ib,) = solve_batch([h], [p])
        assert code == 0 and ib["relres"] <= 1e-8
        xs, isolo = h.solve(T(p.b))
        xs = xs.cpu().numpy()
        o = oracle.setup_problem(p)
        xo, io = o.solve(p.b, tol=1e-8)
        assert abs(ib["iters"] - io["iters"]) <= 1 and abs(isolo["iters"] - io["iters"]) <= 1
        assert np.linalg.norm(xb - xo) <= 1e-6 * np.linalg.norm(xo)
        assert np.linalg.norm(xb - xs) <= 1e-6 * np.linalg.norm(xs)
        h.close()


def test_whole_solve_route_fp32_preconditioner_matches_oracle():
    """The serving default (FP32 preconditioner, FP64 outer) through the whole-solve workgroup: true residual at the
    tolerance and error <= 1e-6 against the FP64 oracle solved to 1e-12."""
    probs = [prob(s) for s in (40, 140, 258)] + [prob(120, 16)]
    hs = [hier(p, precision=1) for p in probs]
    code, xs, infos = solve_batch(hs, probs)
    assert code == 0
    for p, x, info in zip(probs, xs, infos):
        o = oracle.setup_problem(p)
        x12, _ = o.solve(p.b, tol=1e-12)
        _, i8 = o.solve(p.b, tol=1e-8)
        A = H.csr_of(p)
        err = np.linalg.norm(x - x12) / np.linalg.norm(x12)
        print(f"[batch] fp32-precond whole-solve n={p.n}: iters {info['iters']} (oracle fp64 {i8['iters']}), "
              f"relres {info['relres']:.2e}, err vs oracle {err:.2e}", flush=True)
        assert info["relres"] <= 1e-8
        assert np.linalg.norm(A @ x - p.b) <= 1e-8 * np.linalg.norm(p.b) * (1 + 1e-6)
        assert err <= 1e-6
    for h in hs:
        h.close()


def test_mix_of_small_and_large_systems():
    small = [prob(s) for s in (66, 140)]
    large = [prob(300), prob(420)]          # > 65,536 unknowns: threaded amg_solve route
    hs = [hier(p, precision=1) for p in small + large]
    code, xs, infos = solve_batch(hs, small + large)
    assert code == 0
    for h, p, x, info in zip(hs, small + large, xs, infos):
        A = H.csr_of(p)
        assert info["relres"] <= 1e-8
        assert np.linalg.norm(A @ x - p.b) <= 1e-8 * np.linalg.norm(p.b) * (1 + 1e-6)
    # a large system in the mix equals amg_solve alone bit for bit (same route, deterministic)
    xl, il = hs[-1].solve(T(large[-1].b))
    assert np.array_equal(xl.cpu().numpy(), xs[-1]) and il["iters"] == infos[-1]["iters"]
    for h in hs:
        h.close()


def test_batch_with_batching_disabled_routes_to_amg_solve():
    p = prob(100)
    h = hier(p, batch=0)
    code, (xb,), (ib,) = solve_batch([h], [p])
    xs, isolo = h.solve(T(p.b))
    assert code == 0 and np.array_equal(xb, xs.cpu().numpy()) and ib["iters"] == isolo["iters"]
    h.close()
