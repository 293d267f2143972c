"""amg_solve_batch_noalloc (static device scratch, no allocation per call) against amg_solve_batch through the C ABI:
two calls in a row, the second with fewer and smaller systems, each result bit-identical to the allocating entry
point's (the same whole-solve launches on the same inputs), in both precisions. Also: a batch larger than the static
array, and a system that would not take the whole-solve route, are rejected before any device work."""
import numpy as np
import pytest

from paper_1209_5421_amd import meshgen as mg

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def T(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda:0")


def run(hs, probs, noalloc):
    from paper_1209_5421_amd import amg
    bs = [T(p.b) for p in probs]
    xs = [torch.full_like(b, float("nan")) for b in bs]
    code, infos = amg.solve_batch(hs, bs, xs, [1e-8] * len(hs), noalloc=noalloc)
    torch.cuda.synchronize()
    return code, [x.cpu().numpy() for x in xs], infos


@pytest.mark.parametrize("precision", [0, 1])
def test_noalloc_equals_batch_on_two_calls(precision):
    from paper_1209_5421_amd import amg
    first = [mg.jittered_problem(s, rhs_seed=200 + s, fast=True) for s in (40, 100, 160, 258)]
    second = [mg.jittered_problem(s, rhs_seed=300 + s, fast=True) for s in (30, 66)]
    for probs in (first, second):
        print(f"[noalloc] precision {precision}: sizes {[p.n for p in probs]}", flush=True)
        hs = [amg.Hierarchy.from_problem(p, device="cuda:0", precision=precision) for p in probs]
        code_a, xa, ia = run(hs, probs, noalloc=False)
        code_s, xs, is_ = run(hs, probs, noalloc=True)
        assert code_a == 0 and code_s == 0
        for p, a, s, i1, i2 in zip(probs, xa, xs, ia, is_):
            assert np.array_equal(a, s), p.name
            assert i1["iters"] == i2["iters"] and i1["relres"] == i2["relres"] and i2["status"] == 0
        for h in hs:
            h.close()


def test_noalloc_rejects_what_it_cannot_run():
    from paper_1209_5421_amd import amg
    p = mg.jittered_problem(40, rhs_seed=7, fast=True)
    h_block = amg.Hierarchy.from_problem(p, device="cuda:0", smoother=1)  # never takes the whole-solve route
    b = T(p.b)
    x = torch.zeros_like(b)
    code, _ = amg.solve_batch([h_block], [b], [x], [1e-8], noalloc=True)
    assert code == amg.INVALID
    h_block.close()
    hs = [amg.Hierarchy.from_problem(p, device="cuda:0") for _ in range(257)]
    bs = [b] * 257
    xs = [torch.zeros_like(b) for _ in range(257)]
    code, _ = amg.solve_batch(hs, bs, xs, [1e-8] * 257, noalloc=True)
    assert code == amg.INVALID
    for h in hs:
        h.close()
