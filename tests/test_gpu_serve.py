"""The serving loop end to end on the GPU: requests for meshes of uneven sizes arrive over time (Poisson arrivals),
some repeat a right-hand side on a cached hierarchy, several dispatchers batch and overlap them on the device.

Bars: every request converges to 1e-8 in the true FP64 residual; each result is bit-identical to the same system
solved alone (a fresh hierarchy, a batch of one); repeats hit the cache; admission under a tight HBM budget evicts
and still serves everything.
"""
import numpy as np
import pytest

from paper_1209_5421_amd import meshgen as mg
from tests import helpers as H

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def stream_of_requests(nreq=40, seed=11, lo=1e3, hi=3e5, repeat=0.3, rate=200.0):
    from paper_1209_5421_amd.serve import Request
    rng = np.random.default_rng(seed)
    meshes, reqs, t = [], [], 0.0
    for rid in range(nreq):
        t += rng.exponential(1.0 / rate)
        if meshes and rng.random() < repeat:
            mid = int(rng.integers(len(meshes)))
        else:
            side = int(round(np.sqrt(np.exp(rng.uniform(np.log(lo), np.log(hi)))))) + 2
            meshes.append(mg.jittered_problem(side, seed=1000 + rid, rhs_seed=rid, fast=True))
            mid = len(meshes) - 1
        rhs = np.random.default_rng(5000 + rid).uniform(-1, 1, meshes[mid].n)
        reqs.append(Request(rid, mid, meshes[mid], rhs, t))
    return meshes, reqs


def alone(p, rhs):
    from paper_1209_5421_amd import amg
    h = amg.Hierarchy.from_problem(p, device="cuda:0", precision=1)
    b = torch.as_tensor(rhs, dtype=torch.float64, device="cuda:0")
    x = torch.empty_like(b)
    code, (info,) = amg.solve_batch([h], [b], [x], [1e-8])
    torch.cuda.synchronize()
    out = x.cpu().numpy()
    h.close()
    return code, out, info


@pytest.mark.timeout(300)
def test_serving_stream_results_equal_alone():
    from paper_1209_5421_amd.serve import Server, summarize
    meshes, reqs = stream_of_requests()
    print(f"[serve] {len(reqs)} requests over {len(meshes)} meshes, n in "
          f"[{min(m.n for m in meshes)}, {max(m.n for m in meshes)}]", flush=True)
    srv = Server(dispatchers=4, precision=1)
    res = srv.serve(reqs)
    m = summarize(res)
    print(f"[serve] {m} setups {srv.setups} batches {srv.batches}", flush=True)
    assert len(res) == len(reqs) and srv.setups == len(meshes)
    assert m["all_converged"]
    assert m["cache_hit_rate"] == pytest.approx(1 - len(meshes) / len(reqs))
    for r in reqs:
        got = res[r.rid]
        A = H.csr_of(r.problem)
        assert np.linalg.norm(A @ got.x - r.rhs) <= 1e-8 * np.linalg.norm(r.rhs) * (1 + 1e-6)
        code, x1, i1 = alone(r.problem, r.rhs)
        assert code == 0 and i1["iters"] == got.iters
        assert np.array_equal(x1, got.x), r.rid
    srv.close()


@pytest.mark.timeout(300)
def test_serving_under_tight_memory_budget():
    from paper_1209_5421_amd import amg
    from paper_1209_5421_amd.serve import Server, summarize
    meshes, reqs = stream_of_requests(nreq=24, seed=3, lo=1e4, hi=2e5, repeat=0.3)
    biggest = max(amg.estimate_bytes(m.n, m.nnz, precision=1) for m in meshes)
    srv = Server(dispatchers=2, precision=1, mem_budget=int(2.2 * biggest))
    res = srv.serve(reqs)
    m = summarize(res)
    print(f"[serve] tight budget: {m} setups {srv.setups} evictions {srv.evictions}", flush=True)
    assert len(res) == len(reqs) and m["all_converged"] and srv.evictions > 0
    assert srv.sched.mem_used <= srv.sched.mem_budget
    for r in reqs:
        A = H.csr_of(r.problem)
        assert np.linalg.norm(A @ res[r.rid].x - r.rhs) <= 1e-8 * np.linalg.norm(r.rhs) * (1 + 1e-6)
    srv.close()


def test_cache_limit_bounds_the_freed_block_cache():
    """amg_cache_control: freed hierarchies' blocks stay cached up to the limit, a lower limit returns the excess to
    the driver at once, and with limit 0 nothing is kept."""
    from paper_1209_5421_amd import amg
    prob = mg.jittered_problem(130, fast=True)
    try:
        amg.cache_control(0, 8 << 30)
        before = amg.cache_control(0)
        h = amg.Hierarchy.from_problem(prob, device="cuda:0")
        h.close()
        held = amg.cache_control(0)
        assert held > before
        assert amg.cache_control(0, 0) == 0
        h = amg.Hierarchy.from_problem(prob, device="cuda:0")
        h.close()
        assert amg.cache_control(0) == 0
    finally:
        amg.cache_control(0, 32 << 30)
