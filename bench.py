"""Benchmark: auxiliary-grid AMG on one MI355X.

A step is one pass of the whole hot path over the workload: amg_setup (box, cell keys, counting sort, sliced ELL,
Galerkin hierarchy, coarsest factor) followed by one amg_solve to a 1e-8 relative residual with the FP32
preconditioner / FP64 outer iteration, the fine smoother solving each cell's diagonal block exactly (the 4-color
block Gauss-Seidel of Section 4.5 with the aggregates as blocks; --smoother 0 takes the substitution reading). The
default workload is the quasi-uniform 2D P1 Poisson system: a 1024 x 1024
lattice jittered by U[-0.3h, 0.3h], Delaunay-triangulated, Dirichlet boundary eliminated (1,044,484 unknowns),
right-hand side U[-1, 1]. Inputs are resident in HBM before the timed region starts.

Printed: one JSON line. value = unknowns x steps / wall time of the K timed steps (DOF/s of setup + solve). Extra
fields give the first (cold) step's setup and solve times; solve-only rates on a resident hierarchy for both forms
(solves/s, DOF/s, p50/p99 latency); a time step with new coefficients on the resident hierarchy (device P1
assembly, values update, solve); the roofline of the dominant kernel (the persistent small-level workgroup:
algorithmic flops per launch over its duration, and its share of the solve); the same for the HBM-bound fine
residual with its counter-measured traffic (roofline_hbm), both from HIP-event timing of their launches inside the
timed steps (alternate steps time one or the other); and the oracle timed on the host (cpu_baseline).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "DOF/s + solves/s to 1e-8 rel residual (FP32-precond vs FP64); p50/p99 latency"
HBM_PEAK_GBS = 8000.0
WORKLOADS = {
    "c1": ("uniform 65x65 vertices P1 Poisson (3,969 DOF)", lambda mg: mg.uniform_problem(64)),
    "c2": ("quasi-uniform jittered Delaunay 1024x1024 P1 Poisson (1,044,484 DOF)", lambda mg: mg.jittered_problem(1024)),
    "c3": ("graded Delaunay ~4.0M points, density (r+0.01)^-1.5, P1 Poisson",
           lambda mg: mg.graded_problem(4_000_000, progress=log)),
    "c4": ("jittered Delaunay 1416x1416, kappa 10^U[-3,3] 16x16 checkerboard (1,999,396 DOF)",
           lambda mg: mg.jittered_problem(1416, kappa_tiles=16)),
    "disk": ("Delaunay mesh of the disk r = 1/2 inside the unit square, jittered 1156x1156 lattice points plus 3,629 "
             "on the circle, P1 Poisson (about 1.05M DOF; a fifth of the quadtree cells empty)",
             lambda mg: mg.disk_problem(1156)),
    "c5": ("serving stream: 512 Poisson-arrival requests, jittered-lattice P1 Poisson systems with DOF log-uniform in "
           "[1e4, 2e6], 30% repeat right-hand sides on a cached hierarchy", None),
    "cube": ("octree variant: one implicit heat step (dt = h) on a jittered 101^3 lattice of the unit cube, P1 "
             "tetrahedra, Dirichlet inlet face (1,020,100 DOF)", lambda mg: mg.cube_problem(100)),
}
ROOFLINE_KERNELS = {"engine32": "k_engine_fast<float>", "spmv64": "k_outer_spmv_dot",
                    "resid_fine32": "k_fine_resid_full<float>", "gs_fine32": "k_fine_gs<float> (fused color phase)"}
# counter rows of a family: the fused phase's exact-block variants only (the smoother the benchmark runs and times)
COUNTER_TAGS = {"gs_fine32": "k_fine_gs<float, 1,"}
GOLDEN = os.path.join(ROOT, "tests", "golden")
FP32_VECTOR_PEAK_TFLOPS = 157.3  # MI355X dense FP32 vector, 256 CUs at 2.4 GHz
N_CU = 256
# c5 arrival rate: 0.7 x the saturated FP32-preconditioned served throughput measured by --calibrate (frozen)
C5_RATE = 112.2
MALL_BYTES = 256 << 20           # Infinity Cache: operands smaller than this may be served from it
ROW_VISIT_BYTES = 250.0          # algorithmic bytes per visit of a tree-level row (9 FP32 values, its vectors)


def coarse_row_visits(levels, top):
    """Tree-level rows one launch of the small-level workgroup passes over: B~ at level `top` runs B^ there twice,
    and each B^ one B~ below, so level top + j is visited 2^(j+1) times (the coarsest, a dense solve, not counted)."""
    return sum(2 ** (l - top + 1) * levels[l]["n"] for l in range(top, len(levels) - 1))


def solve_bytes_per_iteration(n, nnz, n_level_L):
    """Algorithmic bytes of one outer iteration of the FP32-preconditioned solve: the outer FP64 SpMV (12 B per
    entry + 24 B per row), the outer vector work of FCG(1) (about 108 B per row), the fine preconditioner's three
    FP32 passes over the matrix (8 B per entry + 12 B per row each), and the tree levels (about 1000 B per level-L
    row: 4 N_L row visits of about 250 B)."""
    return (12.0 * nnz + 24.0 * n) + 108.0 * n + 3 * (8.0 * nnz + 12.0 * n) + 1000.0 * n_level_L


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def err_vs_oracle_reference(workload, smoother, n, x):
    """Relative error of a solution of the workload's own right-hand side against the oracle's FP64 solve stored in
    tests/golden/fullsize_<workload>.json (written by the oracle alone): over its 512 seeded sample entries, and of
    the norm. The reference is the tightest stored solve (1e-12 on the quasi-uniform mesh, 1e-11 on the
    checkerboard, else 1e-8)."""
    path = os.path.join(GOLDEN, f"fullsize_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        g = json.load(f)
    if g["n"] != n:
        return None
    ref = g["smoothers"][str(smoother)]
    r = ref.get("reference") or dict(ref["tol_1e-8"], tol=1e-8)
    idx = np.asarray(g["samples"])
    xs = np.asarray(r["x_samples"])
    return {"oracle_tol": r["tol"], "oracle_iters": r["iters"], "samples": len(idx),
            "rel_err_samples": float(np.linalg.norm(x[idx] - xs) / np.linalg.norm(xs)),
            "rel_err_norm": float(abs(np.linalg.norm(x) - r["x_norm"]) / r["x_norm"])}


def kernel_source_hash(kernel="resid_fine32"):
    """Hash of the sources a kernel family depends on: for the small-level engine qa_engine.hip, else the fine-level
    section of qa_solve.hip and the sliced-ELL layout built in qa_setup.hip; the shared header for both. A counter
    record taken on other sources is not used."""
    csrc = os.path.join(ROOT, "paper_1209_5421_amd", "csrc")
    h = hashlib.sha256()
    if kernel.startswith("engine"):
        names = ("qa_engine.hip", "qa_internal.hpp")
    else:
        with open(os.path.join(csrc, "qa_solve.hip")) as f:
            text = f.read()
        start = text.index("\n// fine level kernels\n")
        end = text.index("\n// -----", start + 1)
        h.update(text[start:end].encode())
        names = ("qa_setup.hip", "qa_internal.hpp")
    for name in names:
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_from_profiles(kernel, workload):
    """HBM bytes per launch from committed rocprofv3 counter runs, if taken on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("source_hash") != kernel_source_hash(kernel):
        return None
    return rec.get("bytes_per_launch")


COPY_ELEMS = 1 << 28           # calibration copy: 1 GiB of float32 read, 1 GiB written
COPY_KERNEL_TAG = "neg_kernel"


def copy_calibration():
    """A plain streaming kernel of known size for scaling the FETCH_SIZE / WRITE_SIZE counters: y = -x over 1 GiB."""
    import torch
    x = torch.ones(COPY_ELEMS, dtype=torch.float32, device="cuda:0")
    y = torch.empty_like(x)
    for _ in range(3):
        torch.neg(x, out=y)
    torch.cuda.synchronize()
    del x, y


def _counter_rows(d):
    import csv
    import glob
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise SystemExit(f"no counter_collection.csv under {d}")
    rows = []
    for fn in files:
        with open(fn) as f:
            rows += list(csv.DictReader(f))
    return rows


def _per_dispatch(rows, counter, tag):
    vals = {}
    for r in rows:
        if r.get("Counter_Name") == counter and tag in r.get("Kernel_Name", ""):
            key = r.get("Dispatch_Id") or r.get("Correlation_Id")
            vals[key] = vals.get(key, 0.0) + float(r["Counter_Value"])
    if not vals:
        raise SystemExit(f"no {counter} rows for kernels matching {tag!r}")
    return float(np.mean(list(vals.values()))), len(vals)


def traffic_record(fetch_dir, write_dir, kernel, workload, commands):
    """Combine a FETCH_SIZE run and a WRITE_SIZE run (KiB per dispatch) into HBM bytes per launch of `kernel`,
    each counter scaled by what it reads for the calibration copy (expected / measured)."""
    tag = COUNTER_TAGS.get(kernel) or ROOFLINE_KERNELS[kernel].split(" ")[0].rstrip(">")
    fr, wr = _counter_rows(fetch_dir), _counter_rows(write_dir)
    f_k, nf = _per_dispatch(fr, "FETCH_SIZE", tag)
    w_k, nw = _per_dispatch(wr, "WRITE_SIZE", tag)
    f_c, _ = _per_dispatch(fr, "FETCH_SIZE", COPY_KERNEL_TAG)
    w_c, _ = _per_dispatch(wr, "WRITE_SIZE", COPY_KERNEL_TAG)
    expect_kib = COPY_ELEMS * 4 / 1024.0
    sf, sw = expect_kib / f_c, expect_kib / w_c
    return {"kernel": kernel, "kernel_name": ROOFLINE_KERNELS[kernel], "workload": workload,
            "source_hash": kernel_source_hash(kernel),
            "fetch_kib_per_launch": f_k, "write_kib_per_launch": w_k, "dispatches": [nf, nw],
            "copy_calibration": {"bytes_read": COPY_ELEMS * 4, "bytes_written": COPY_ELEMS * 4,
                                 "fetch_kib": f_c, "write_kib": w_c, "fetch_scale": sf, "write_scale": sw},
            "bytes_per_launch": (f_k * sf + w_k * sw) * 1024.0, "commands": commands}


def cpu_baseline(prob, tol, smoother):
    import oracle
    cores = len(os.sched_getaffinity(0))
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    t0 = time.perf_counter()
    o = oracle.setup_problem(prob)
    if smoother:
        o.set_block_smoother(True)  # the same reading of the fine smoother as the GPU run (its factors: setup)
    t1 = time.perf_counter()
    x, info = o.solve(prob.b, tol=tol)
    t2 = time.perf_counter()
    o.close()
    total = t2 - t0
    return {"value": prob.n / total, "unit": "DOF/s", "cores": 1, "kind": "oracle",
            "sample": f"one full oracle setup + FP64 solve of the same {prob.n}-unknown system to {tol:g}, same "
                      f"fine smoother "
                      f"(setup {t1 - t0:.2f} s, solve {t2 - t1:.2f} s, {info['iters']} iterations); "
                      f"single-threaded, 1 of {cores} host cores ({model})",
            "setup_s": t1 - t0, "solve_s": t2 - t1, "iters": info["iters"]}, x


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c2", choices=sorted(WORKLOADS))
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--smoother", type=int, default=1, choices=[0, 1],
                    help="fine block Gauss-Seidel of Section 4.5: 1 (default) the exact solve of each cell's diagonal "
                         "block (cells of at most 32 unknowns), 0 one substitution over each cell's unknowns")
    ap.add_argument("--repeats", type=int, default=20, help="resident-hierarchy solves per form for latency")
    ap.add_argument("--roofline-kernel", default="engine32", choices=sorted(ROOFLINE_KERNELS),
                    help="kernel of the roofline entry: the dominant one by time (the persistent small-level "
                         "workgroup of the FP32 preconditioner)")
    ap.add_argument("--hbm-kernel", default="resid_fine32", choices=["resid_fine32", "spmv64", "gs_fine32"],
                    help="HBM-bound kernel reported beside it (roofline_hbm), with counter-measured traffic")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--big-leg", default="c3", choices=["c3", "c4", "none"],
                    help="after the timed steps: a system beyond the Infinity Cache solved for 8 right-hand sides, "
                         "with per-kernel HBM fractions")
    ap.add_argument("--requests", type=int, default=512, help="c5: requests in the stream")
    ap.add_argument("--rate", type=float, default=C5_RATE,
                    help="c5: Poisson arrival rate (requests/s); the default is frozen at 0.7 x the saturated "
                         "throughput of the FP32-preconditioned served form (--calibrate measures it)")
    ap.add_argument("--calibrate", action="store_true",
                    help="c5: serve the stream with every request arriving at once and report the saturated "
                         "solves/s and the rate 0.7 x that")
    ap.add_argument("--oracle-sample", type=int, default=32, help="c5: requests in the oracle latency sample")
    ap.add_argument("--dispatchers", type=int, default=4, help="c5: concurrent batch dispatchers")
    ap.add_argument("--mem-gb", type=float, default=200.0, help="c5: HBM budget for resident hierarchies")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run the 1 GiB streaming kernel that scales the HBM counters")
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="write profiles/traffic_<kernel>_<workload>.json from two rocprofv3 --pmc runs and exit")
    ap.add_argument("--traffic-commands", nargs="*", default=[], help="commands that produced the counter runs")
    ap.add_argument("--traffic-kernel", default=None, choices=sorted(ROOFLINE_KERNELS),
                    help="--traffic-from: the kernel family the counters are for (default: --hbm-kernel)")
    args = ap.parse_args()
    if args.traffic_from:
        tk = args.traffic_kernel or args.hbm_kernel
        rec = traffic_record(*args.traffic_from, tk, args.workload, args.traffic_commands)
        out = os.path.join(ROOT, "profiles", f"traffic_{tk}_{args.workload}.json")
        with open(out, "w") as f:
            json.dump(rec, f, indent=1)
        print(json.dumps(rec))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the solver runs on one GPU: sharding across GPUs is not implemented; "
                                   "run with --gpus 1"}))
        sys.exit(2)

    from paper_1209_5421_amd import amg, meshgen
    import torch

    if args.workload == "c5":
        return serve_bench(args)
    desc, make = WORKLOADS[args.workload]
    log(f"workload {args.workload}: generating the mesh and its system on the host ...")
    t = time.time()
    prob = make(meshgen)
    log(f"workload {args.workload}: n={prob.n} nnz={prob.nnz} generated in {time.time() - t:.1f}s")
    dev = torch.device("cuda:0")
    amg.load()
    tt = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=dev)
    coords, rp, ci, va = tt(prob.coords, torch.float64), tt(prob.row_ptr, torch.int64), tt(prob.col, torch.int32), \
        tt(prob.val, torch.float64)
    b = tt(prob.b, torch.float64)
    x = torch.empty_like(b)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()

    wall = {"setup_call": [], "timing_enable": [], "solve_call": [], "timing_read": [], "free": []}

    def step(timing_kernel=None):
        c0 = time.perf_counter()
        h = amg.Hierarchy(coords, rp, ci, va, box=prob.box, precision=1, stream=stream, smoother=args.smoother)
        c1 = time.perf_counter()
        if timing_kernel:
            h.timing_enable(timing_kernel)
        c2 = time.perf_counter()
        _, info = h.solve(b, tol=args.tol, x=x)
        c3 = time.perf_counter()
        tm = h.timing_read() if timing_kernel else None
        c4 = time.perf_counter()
        h.close()
        c5 = time.perf_counter()
        for key, dt in zip(wall, (c1 - c0, c2 - c1, c3 - c2, c4 - c3, c5 - c4)):
            wall[key].append(dt * 1e3)
        return info, tm

    cold = None
    for w in range(args.warmup):
        info, _ = step()
        log(f"warmup {w}: setup {info['setup_ms']:.2f} ms solve {info['solve_ms']:.2f} ms iters {info['iters']}")
        if w == 0:  # the process's first setup and solve: module load, memory pool and block cache still empty
            cold = {"setup_ms": info["setup_ms"], "solve_ms": info["solve_ms"],
                    "step_wall_ms": sum(v[-1] for v in wall.values())}

    # the timed steps alternate between timing the launches of the roofline kernel and of the HBM kernel
    timed = {args.roofline_kernel: [0, 0.0, 0.0, 0], args.hbm_kernel: [0, 0.0, 0.0, 0]}
    infos = []
    for v in wall.values():
        v.clear()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        kind = args.roofline_kernel if k % 2 == 0 else args.hbm_kernel
        info, tm = step(kind)
        infos.append(info)
        acc = timed[kind]
        acc[0] += tm["launches"]
        acc[1] += tm["total_ms"]
        acc[2] = tm["bytes_per_launch"]
        acc[3] += 1
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    for k, info in enumerate(infos):
        log(f"step {k}: setup {info['setup_ms']:.2f} ms solve {info['solve_ms']:.2f} ms iters {info['iters']} "
            f"relres {info['relres']:.2e}")

    # resident-hierarchy solves: both forms
    forms = {}
    h = amg.Hierarchy(coords, rp, ci, va, box=prob.box, precision=0, stream=stream, smoother=args.smoother)
    engine = {name: h.engine_info(prec) for name, prec in (("fp64", 0), ("fp32_precond", 1))}
    levels = [h.level_info(l) for l in range(h.num_levels)]
    log(f"levels {[(lv['k'], lv['n']) for lv in levels]} engine {engine}")
    for name, prec in (("fp64", 0), ("fp32_precond", 1)):
        h.set_precision(prec)
        h.solve(b, tol=args.tol, x=x)
        lat = []
        for _ in range(args.repeats):
            torch.cuda.synchronize()
            s0 = time.perf_counter()
            _, info = h.solve(b, tol=args.tol, x=x)
            torch.cuda.synchronize()
            lat.append((time.perf_counter() - s0) * 1e3)
        lat = np.array(lat)
        forms[name] = {"iters": info["iters"], "relres": info["relres"], "p50_ms": float(np.percentile(lat, 50)),
                       "p99_ms": float(np.percentile(lat, 99)), "solves_per_s": float(1e3 / np.median(lat)),
                       "dof_per_s": float(prob.n * 1e3 / np.median(lat))}
        log(f"resident {name}: {forms[name]}")
    x_gpu = x.cpu().numpy()
    err_ref = err_vs_oracle_reference(args.workload, args.smoother, prob.n, x_gpu)
    log(f"fp32-precond solution against the stored oracle reference: {err_ref}")
    # the other reading of the fine smoother on the same resident system (both forms)
    other = 1 - args.smoother
    ho = amg.Hierarchy(coords, rp, ci, va, box=prob.box, precision=0, stream=stream, smoother=other)
    forms_other = {}
    for name, prec in (("fp64", 0), ("fp32_precond", 1)):
        ho.set_precision(prec)
        ho.solve(b, tol=args.tol, x=x)
        lat = []
        for _ in range(args.repeats):
            torch.cuda.synchronize()
            s0 = time.perf_counter()
            _, info = ho.solve(b, tol=args.tol, x=x)
            torch.cuda.synchronize()
            lat.append((time.perf_counter() - s0) * 1e3)
        forms_other[name] = {"iters": info["iters"], "relres": info["relres"],
                             "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                             "solves_per_s": float(1e3 / np.median(lat)),
                             "dof_per_s": float(prob.n * 1e3 / np.median(lat))}
    forms_other = {"smoother": ["cell substitution", "exact cell blocks"][other], **forms_other}
    log(f"resident, other smoother: {forms_other}")
    ho.close()
    # time stepping with changing coefficients on the same mesh: per step the device assembly of the new
    # coefficients (amg_p1_assemble), a values update of the resident hierarchy (amg_update_values) and a solve, in
    # the mixed form; kappa alternates between 1 + sin(2 pi x) sin(2 pi y) / 2 at the triangles' centroids and the
    # workload's own coefficients. The device assembly of the workload's coefficients is checked against its matrix.
    update = None
    if prob.coords.shape[1] == 2:  # device P1 assembly is for triangle meshes
        mesh = prob.meta
        dof = np.full(len(mesh["points"]), -1, dtype=np.int32)
        dof[~mesh["dirichlet"]] = np.arange(prob.n, dtype=np.int32)
        c0 = time.perf_counter()
        pm = amg.P1Mesh(tt(mesh["points"], torch.float64), tt(mesh["tris"], torch.int32), tt(dof, torch.int32), prob.n,
                        stream=stream)
        pattern_ms = (time.perf_counter() - c0) * 1e3
        prp, pcol = pm.pattern()
        kap0 = None if mesh["kappa"] is None else tt(mesh["kappa"], torch.float64)
        same = bool(torch.equal(prp, rp) and torch.equal(pcol, ci) and torch.equal(pm.assemble(kap0), va))
        del prp, pcol
        pts_, tri_ = mesh["points"], mesh["tris"]
        cen = (pts_[tri_[:, 0]] + pts_[tri_[:, 1]] + pts_[tri_[:, 2]]) / 3.0
        kap1 = tt(1.0 + 0.5 * np.sin(2 * np.pi * cen[:, 0]) * np.sin(2 * np.pi * cen[:, 1]), torch.float64)
        vals = torch.empty_like(va)
        h.set_precision(1)
        asm, upd, step_ms, upd_iters = [], [], [], []
        for k in range(args.repeats):
            torch.cuda.synchronize()
            s0 = time.perf_counter()
            pm.assemble(kap1 if k % 2 == 0 else kap0, out=vals)
            s1 = time.perf_counter()
            h.update_values(rp, ci, vals)
            s2 = time.perf_counter()
            _, info = h.solve(b, tol=args.tol, x=x)
            torch.cuda.synchronize()
            asm.append((s1 - s0) * 1e3)
            upd.append((s2 - s1) * 1e3)
            step_ms.append((time.perf_counter() - s0) * 1e3)
            upd_iters.append(info["iters"])
        pm.close()
        update = {"coefficients": "alternately 1 + sin(2 pi x) sin(2 pi y) / 2 at the centroids and the workload's own",
                  "device_assembly_equals_matrix": same, "pattern_ms": pattern_ms,
                  "assemble_ms_p50": float(np.median(asm)), "update_ms_p50": float(np.median(upd)),
                  "update_ms_p99": float(np.percentile(upd, 99)), "step_ms_p50": float(np.median(step_ms)),
                  "iters": sorted(set(upd_iters))}
        log(f"values update: {update}")
    h.close()

    solve_ms = float(np.median([i["solve_ms"] for i in infos]))

    def entry(kind):
        launches, kern_ms, per_launch, nsteps = timed[kind]
        avg_ms = kern_ms / max(launches, 1)
        if kind.startswith("engine"):
            # one workgroup runs the cycle below ~4,096 cells as a chain of dependent steps (barrier after each);
            # its algorithmic bytes are the tree-level row visits of one launch at 250 B each
            eng = engine["fp32_precond" if kind == "engine32" else "fp64"]
            top = eng["top_level"]
            rows = coarse_row_visits(levels, top) if top >= 0 else 0
            nbytes = rows * ROW_VISIT_BYTES
            gbs = nbytes / (avg_ms * 1e-3) / 1e9 if launches else None
            name = ROOFLINE_KERNELS[kind]
            if top >= 0:  # the specialised engine's instance: <precision, top level k, last LDS level k>
                name = f"{name[:-1]}, {levels[top]['k']}, {levels[eng['lds_level']]['k']}>"
            return {"bound": "hbm", "kernel": name, "achieved": gbs, "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": (gbs / HBM_PEAK_GBS) if gbs else None,
                    "traffic": traffic_from_profiles(kind, args.workload),
                    "launches": launches, "avg_us": avg_ms * 1e3, "algorithmic_bytes_per_launch": nbytes,
                    "row_visits_per_launch": rows, "bytes_per_row_visit": ROW_VISIT_BYTES,
                    "share_of_solve": (kern_ms / max(nsteps, 1)) / solve_ms if nsteps else None,
                    "operands_fit_infinity_cache": True,
                    "limit": "latency of one workgroup's chain of dependent steps (operands in LDS and L2)"}
        gbs = per_launch / (avg_ms * 1e-3) / 1e9 if launches else None
        return {"bound": "hbm", "kernel": ROOFLINE_KERNELS[kind], "achieved": gbs, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": (gbs / HBM_PEAK_GBS) if gbs else None,
                "traffic": traffic_from_profiles(kind, args.workload),
                "launches": launches, "avg_us": avg_ms * 1e3, "algorithmic_bytes_per_launch": per_launch,
                "operands_fit_infinity_cache": bool(per_launch < MALL_BYTES)}

    roofline = entry(args.roofline_kernel)
    roofline_hbm = entry(args.hbm_kernel) if args.hbm_kernel != args.roofline_kernel else None
    it_med = float(np.median([i["iters"] for i in infos]))
    bpi = solve_bytes_per_iteration(prob.n, prob.nnz, levels[1]["n"] if len(levels) > 1 else 0)
    solve_roofline = {"bytes_per_iteration": bpi, "bytes_per_dof_per_iteration": bpi / prob.n,
                      "iterations": it_med, "solve_ms": solve_ms,
                      "achieved_gbs": bpi * it_med / (solve_ms * 1e-3) / 1e9,
                      "frac": bpi * it_med / (solve_ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
    log(f"solve-level roofline: {solve_roofline}")
    big = None
    if args.big_leg != "none":
        big = big_leg(args, amg, meshgen, torch, stream)

    if args.copy_calibration:
        copy_calibration()

    cpu = None
    err_vs_oracle = None
    if not args.no_cpu_baseline:
        log("oracle (CPU baseline) ...")
        cpu, x_orc = cpu_baseline(prob, args.tol, args.smoother)
        err_vs_oracle = float(np.linalg.norm(x_gpu - x_orc) / np.linalg.norm(x_orc))
        log(f"oracle: {cpu['sample']}; fp32-precond solution vs oracle rel err {err_vs_oracle:.2e}")

    out = {
        "metric": METRIC, "value": prob.n * 1e3 / ms_per_step, "unit": "DOF/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32/f64", "data": "synthetic",
        "config": {"workload": f"{args.workload}: {desc}", "n": prob.n, "nnz": prob.nnz, "tol": args.tol,
                   "step": "amg_setup + amg_solve (FP32 preconditioner, FP64 outer)",
                   "smoother": ["cell substitution", "exact cell blocks"][args.smoother],
                   "setup_ms_median": float(np.median([i["setup_ms"] for i in infos])),
                   "solve_ms_median": solve_ms,
                   "iters": infos[-1]["iters"], "relres": infos[-1]["relres"]},
        "step_wall_ms": {k: float(np.median(v)) for k, v in wall.items()},
        "cold": cold,
        "solve_resident": forms,
        "update_resident": update,
        "engine": engine,
        "err_vs_oracle": err_vs_oracle,
        "err_vs_oracle_reference": err_ref,
        "solve_resident_other_smoother": forms_other,
        "roofline": roofline,
        "roofline_hbm": roofline_hbm,
        "solve_roofline": solve_roofline,
        "beyond_cache": big,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def big_leg(args, amg, meshgen, torch, stream):
    """A system whose operands exceed the 256 MB Infinity Cache, on one resident hierarchy (FP32 preconditioner):
    the graded 4.0M-unknown mesh (default) solved for 8 right-hand sides in sequence (each solve, p50/p99, aggregate
    solves/s), then one solve per HBM-bound kernel family with its launches timed by HIP events, giving each family's
    HBM fraction from its algorithmic bytes and the solve-level fraction."""
    name = args.big_leg
    desc, make = WORKLOADS[name]
    log(f"{name} leg: generating the mesh and its system on the host ...")
    t = time.time()
    prob = make(meshgen)
    log(f"{name} leg: n={prob.n} nnz={prob.nnz} generated in {time.time() - t:.1f}s")
    dev = torch.device("cuda:0")
    tt = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=dev)
    coords, rp, ci, va = tt(prob.coords, torch.float64), tt(prob.row_ptr, torch.int64), tt(prob.col, torch.int32), \
        tt(prob.val, torch.float64)
    h = amg.Hierarchy(coords, rp, ci, va, box=prob.box, precision=1, stream=stream, smoother=args.smoother)
    levels = [h.level_info(l) for l in range(h.num_levels)]
    x = torch.empty(prob.n, dtype=torch.float64, device=dev)
    rhs = [tt(meshgen.rhs(prob.n, 1000 + j), torch.float64) for j in range(8)]
    h.solve(rhs[0], tol=args.tol, x=x)  # warm
    lat, its = [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for bj in rhs:
        s0 = time.perf_counter()
        _, info = h.solve(bj, tol=args.tol, x=x)
        lat.append((time.perf_counter() - s0) * 1e3)
        its.append(info["iters"])
        assert info["status"] == 0 and info["relres"] <= args.tol
    wall = time.perf_counter() - t0
    lat = np.array(lat)
    seq = {"solve_ms": [float(v) for v in lat], "iters": its, "p50_ms": float(np.percentile(lat, 50)),
           "p99_ms": float(np.percentile(lat, 99)), "solves_per_s": len(rhs) / wall,
           "dof_per_s": prob.n * len(rhs) / wall}
    log(f"{name} 8 sequential right-hand sides: {seq}")
    b0 = tt(prob.b, torch.float64)
    _, info0 = h.solve(b0, tol=args.tol, x=x)
    err_ref = err_vs_oracle_reference(name, args.smoother, prob.n, x.cpu().numpy())
    log(f"{name} own right-hand side: iters {info0['iters']}, against the stored oracle reference {err_ref}")
    kernels = {}
    for kind in ("spmv64", "resid_fine32", "gs_fine32"):
        h.timing_enable(kind)
        h.solve(rhs[0], tol=args.tol, x=x)
        tm = h.timing_read()
        h.timing_enable(None)
        avg_ms = tm["total_ms"] / max(tm["launches"], 1)
        gbs = tm["bytes_per_launch"] / (avg_ms * 1e-3) / 1e9
        kernels[kind] = {"kernel": ROOFLINE_KERNELS[kind], "launches": tm["launches"], "avg_us": avg_ms * 1e3,
                         "algorithmic_bytes_per_launch": tm["bytes_per_launch"], "achieved": gbs,
                         "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
                         "traffic": traffic_from_profiles(kind, name)}
        log(f"{name} {kind}: {kernels[kind]}")
    bpi = solve_bytes_per_iteration(prob.n, prob.nnz, levels[1]["n"] if len(levels) > 1 else 0)
    it_med = float(np.median(its))
    med_ms = float(np.median(lat))
    h.close()
    return {"workload": f"{name}: {desc}", "n": prob.n, "nnz": prob.nnz, "precision": "fp32_precond",
            "smoother": ["cell substitution", "exact cell blocks"][args.smoother],
            "levels": [(lv["k"], lv["n"]) for lv in levels], "sequential_rhs": seq,
            "own_rhs": {"iters": info0["iters"], "err_vs_oracle_reference": err_ref}, "kernels": kernels,
            "solve_roofline": {"bytes_per_iteration": bpi, "iterations": it_med, "solve_ms": med_ms,
                               "achieved_gbs": bpi * it_med / (med_ms * 1e-3) / 1e9,
                               "frac": bpi * it_med / (med_ms * 1e-3) / 1e9 / HBM_PEAK_GBS}}


def _oracle_request(item):
    """One request on the CPU oracle: lattice mesh generated on the host, setup and FP64 solve (test infrastructure:
    the baseline of the served form)."""
    import oracle
    from paper_1209_5421_amd import meshgen as mg
    mid, side, rs, tol = item
    c, rp, ci, va = mg.lattice_system(side, seed=100 + mid)
    b = mg.rhs(len(c), rs)
    t0 = time.perf_counter()
    o = oracle.Oracle(c, rp, ci, va, box=mg.UNIT_BOX)
    _, info = o.solve(b, tol=tol)
    o.close()
    return len(c), time.perf_counter() - t0, info["status"]


def oracle_serving_baseline(stream, sample, tol):
    """The oracle on the host: throughput of a pool of one worker per host core over the whole request list (each
    request set up and solved from scratch, no cache), and the latency of one request at a time on a sample of the
    first `sample` requests."""
    import multiprocessing as mp
    import oracle
    oracle.build(force=False)
    cores = len(os.sched_getaffinity(0))
    items = [(mid, side, rs, tol) for mid, side, rs in stream]
    log(f"c5 oracle: latency sample of {sample} requests ...")
    lat = [_oracle_request(it)[1] for it in items[:sample]]
    log(f"c5 oracle: pool of {cores} processes over {len(items)} requests ...")
    t0 = time.perf_counter()
    with mp.get_context("spawn").Pool(cores) as pool:
        res = pool.map(_oracle_request, items, chunksize=1)
    wall = time.perf_counter() - t0
    ok = all(r[2] == 0 for r in res)
    lat_ms = np.array(lat) * 1e3
    return {"value": len(items) / wall, "unit": "solves/s", "cores": cores, "kind": "oracle",
            "sample": f"the whole {len(items)}-request stream solved by the oracle in a pool of {cores} processes "
                      f"(setup + FP64 solve per request, meshes generated outside the timing); latency p50/p99 from "
                      f"the first {sample} requests one at a time",
            "dof_per_s": sum(r[0] for r in res) / wall, "wall_s": wall, "all_converged": ok,
            "latency_p50_ms": float(np.percentile(lat_ms, 50)), "latency_p99_ms": float(np.percentile(lat_ms, 99))}


def serve_bench(args):
    """The served form: a request stream through the continuous-batching loop, three ways over the same stream
    (FP32-preconditioned and FP64 served with batching and overlap, and the plain FP64 solver taking one request at a
    time in arrival order). Meshes and right-hand sides are made resident in HBM before the stream starts; each pass
    starts with an empty hierarchy cache, so a new mesh pays its setup inside its request's latency."""
    import types
    import torch
    from paper_1209_5421_amd import amg, meshgen as mg
    from paper_1209_5421_amd.serve import Request, Server, summarize

    dev = torch.device("cuda:0")
    amg.load()
    stream = mg.serving_sides(args.requests)
    t = time.time()
    meshes = {}
    for mid, side, _ in stream:
        if mid not in meshes:
            c, rp, ci, va = mg.lattice_system(side, seed=100 + mid, device=dev)
            meshes[mid] = types.SimpleNamespace(coords=c, row_ptr=rp, col=ci, val=va, n=int(c.shape[0]),
                                                nnz=int(va.shape[0]), box=mg.UNIT_BOX)
    rng = np.random.default_rng(mg.SEED_STREAM + 1)
    gaps = rng.exponential(1.0 / args.rate, size=len(stream))
    arrivals = np.cumsum(gaps) - gaps[0]
    reqs = [Request(q, mid, meshes[mid], torch.as_tensor(mg.rhs(meshes[mid].n, rs), device=dev), float(arrivals[q]))
            for q, (mid, _, rs) in enumerate(stream)]
    torch.cuda.synchronize()
    dof = {r.rid: r.problem.n for r in reqs}
    log(f"c5: {len(reqs)} requests over {len(meshes)} meshes ({sum(m.n for m in meshes.values()) / 1e6:.1f}M unique "
        f"DOF, {sum(dof.values()) / 1e6:.1f}M requested DOF), arrivals over {arrivals[-1]:.1f}s at {args.rate}/s; "
        f"inputs resident in {time.time() - t:.1f}s")

    # warm-up: a short stream on separate small meshes (kernels loaded, pools primed)
    warm = []
    for q in range(8):
        c, rp, ci, va = mg.lattice_system(60 + 40 * q, seed=50 + q, device=dev)
        p = types.SimpleNamespace(coords=c, row_ptr=rp, col=ci, val=va, n=int(c.shape[0]), nnz=int(va.shape[0]),
                                  box=mg.UNIT_BOX)
        warm.append(Request(q, ("warm", q), p, torch.as_tensor(mg.rhs(p.n, q), device=dev), 0.002 * q))
    for prec in (1, 0):
        srv = Server(precision=prec, dispatchers=args.dispatchers, mem_budget=int(args.mem_gb * 2**30))
        srv.serve(warm)
        srv.close()

    if args.calibrate:
        # saturation: the whole stream queued at t = 0, the FP32-preconditioned served form
        sat_reqs = [Request(r.rid, r.mesh_id, r.problem, r.rhs, 0.0) for r in reqs]
        srv = Server(mem_budget=int(args.mem_gb * 2**30), precision=1, dispatchers=args.dispatchers)
        m = summarize(srv.serve(sat_reqs), dof=dof)
        srv.close()
        out = {"saturated_fp32_precond": m, "rate_0p7": 0.7 * m["solves_per_s"]}
        log(f"c5 calibration: {out}")
        print(json.dumps(out), flush=True)
        return

    passes = {"fp32_precond": dict(precision=1, dispatchers=args.dispatchers),
              "fp64": dict(precision=0, dispatchers=args.dispatchers),
              "plain_fp64_fifo": dict(precision=0, dispatchers=1, max_batch=1, batch=0)}
    served = {}
    for name, kw in passes.items():
        srv = Server(mem_budget=int(args.mem_gb * 2**30), **kw)
        res = srv.serve(reqs)
        m = summarize(res, dof=dof)
        m.update(setups=srv.setups, evictions=srv.evictions, config=kw)
        served[name] = m
        log(f"c5 {name}: {m}")
        srv.close()
        torch.cuda.synchronize()

    main_pass = served["fp32_precond"]
    cpu = None if args.no_cpu_baseline else oracle_serving_baseline(stream, args.oracle_sample, args.tol)
    out = {
        "metric": METRIC, "value": main_pass["dof_per_s"], "unit": "DOF/s", "n_gpus": 1, "steps": 1, "warmup": 1,
        "ms_per_step": main_pass["makespan_s"] * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32/f64", "data": "synthetic",
        "config": {"workload": f"c5: {WORKLOADS['c5'][0]}", "requests": len(reqs), "unique_meshes": len(meshes),
                   "rate_per_s": args.rate, "tol": 1e-8, "dispatchers": args.dispatchers,
                   "step": "the whole stream served once (FP32 preconditioner, FP64 outer)"},
        "serving": served,
        "roofline": None,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
