"""Expected values of the full-size parity tests (tests/test_gpu_fullsize.py), written by the oracle alone.

Test infrastructure: this script calls only the CPU oracle (oracle/) and the seeded input generators
(paper_1209_5421_amd/meshgen.py). For each full-size workload and each reading of the fine smoother it stores

- a digest of the generated system (coordinates, CSR, right-hand side), so that a test knows it regenerated the
  same system;
- SHA-256 digests of every exported level of the oracle's hierarchy: the aggregates and colors, and per quadtree
  level the 9-slot columns, the FP64 values, their FP32 rounding and the overflow lists;
- the oracle's FP64 solves (Algorithm 2.1 with the K-cycle of Algorithm 2.2) to 1e-8, and to a tighter reference
  tolerance (1e-12, or 1e-11 where FP64 cannot reach 1e-12) against which the mixed-precision solve is compared, as
  iteration counts, true relative residuals, solution norms and the solution at
  512 seeded sample indices;
- one application of the preconditioner to a seeded vector, at the same sample indices.

A full solve of these systems takes the single-threaded oracle minutes; the GPU tests compare against the stored
samples (the relative error over 512 seeded entries and the norms) instead of re-running it.

Usage: python tests/golden/make_fullsize.py c2 c4 c3   (one process per workload can run side by side)
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1209_5421_amd import meshgen as mg  # noqa: E402

OUT = os.path.dirname(os.path.abspath(__file__))
N_SAMPLES = 512
SAMPLE_SEED = 17
PRECOND_SEED = 5

# workload: (description, generator, tolerance of the reference solve the mixed-precision form is compared with, or
# None). On the checkerboard (coefficients spanning six decades) the FP64 true residual stalls near 5e-12, so its
# reference is solved to 1e-11, the smallest attainable power of ten.
WORKLOADS = {
    "c2": ("quasi-uniform jittered Delaunay 1024x1024", lambda: mg.jittered_problem(1024), 1e-12),
    "c4": ("jittered Delaunay 1416x1416, 16x16 kappa checkerboard", lambda: mg.jittered_problem(1416, kappa_tiles=16),
           1e-11),
    "c3": ("graded Delaunay, 4.0M points", lambda: mg.graded_problem(4_000_000), None),
}


def digest(*arrays):
    h = hashlib.sha256()
    for a in arrays:
        a = np.ascontiguousarray(a)
        h.update(str(a.dtype).encode())
        h.update(str(a.shape).encode())
        h.update(a.tobytes())
    return h.hexdigest()


def problem_digest(prob):
    return digest(prob.coords, prob.row_ptr, prob.col, prob.val, prob.b)


def level_digests(lv):
    """Digests of one exported level (the same function is applied to the GPU's export)."""
    if "aj" not in lv:
        return {"agg": digest(lv["agg"]), "color": digest(lv["color"])}
    return {"agg": digest(lv["agg"]), "color": digest(lv["color"]), "aj": digest(lv["aj"]),
            "ax": digest(lv["ax"]), "ax32": digest(lv["ax"].astype(np.float32)),
            "ovf": digest(lv["ovf_ptr"], lv["ovf_col"], lv["ovf_val"])}


def sample_indices(n):
    return np.sort(np.random.default_rng(SAMPLE_SEED).choice(n, size=min(N_SAMPLES, n), replace=False))


def log(msg):
    print(f"[make_fullsize] {msg}", flush=True)


def make(name):
    desc, gen, ref_tol = WORKLOADS[name]
    t = time.time()
    prob = gen()
    log(f"{name}: n={prob.n} nnz={prob.nnz} generated in {time.time() - t:.1f}s")
    idx = sample_indices(prob.n)
    rec = {"workload": desc, "n": prob.n, "nnz": prob.nnz, "problem_digest": problem_digest(prob),
           "sample_seed": SAMPLE_SEED, "samples": idx.tolist(), "precond_seed": PRECOND_SEED, "smoothers": {}}
    o = oracle.setup_problem(prob)
    for smoother in (1, 0):
        o.set_block_smoother(bool(smoother))
        levels = [level_digests(o.export_level(l)) for l in range(o.num_levels)]
        r = np.random.default_rng(PRECOND_SEED).standard_normal(prob.n)
        z = o.apply_precond(r)
        t = time.time()
        x8, i8 = o.solve(prob.b, tol=1e-8)
        log(f"{name} smoother {smoother}: 1e-8 in {i8['iters']} iterations, {time.time() - t:.1f}s")
        s = {"levels": levels, "num_levels": o.num_levels,
             "precond": {"z_samples": z[idx].tolist(), "z_norm": float(np.linalg.norm(z))},
             "tol_1e-8": {"iters": i8["iters"], "relres": i8["relres"], "x_norm": float(np.linalg.norm(x8)),
                          "x_samples": x8[idx].tolist()}}
        if ref_tol:
            t = time.time()
            xr, ir = o.solve(prob.b, tol=ref_tol)
            assert ir["status"] == 0, ir
            log(f"{name} smoother {smoother}: {ref_tol:g} in {ir['iters']} iterations, {time.time() - t:.1f}s")
            s["reference"] = {"tol": ref_tol, "iters": ir["iters"], "relres": ir["relres"],
                              "x_norm": float(np.linalg.norm(xr)), "x_samples": xr[idx].tolist()}
        rec["smoothers"][str(smoother)] = s
    o.close()
    path = os.path.join(OUT, f"fullsize_{name}.json")
    with open(path, "w") as f:
        json.dump(rec, f)
    log(f"wrote {path}")


if __name__ == "__main__":
    oracle.build(force=False)
    for name in sys.argv[1:] or list(WORKLOADS):
        make(name)
