"""Benchmark of the SIPG Helmholtz operator on one MI355X.

Workload: 3-D 32^3 perturbed hex mesh on [0,1]^3, per-element order
U{3..6} (seeded), lambda = 10, Legendre modes, GLL p+2 points per direction.

A step is one FP64 operator application y = A x (both kernel stages) on
seeded N(0,1) coefficients already resident in HBM.  value = N_dof / time
(GDOF/s).  The same line reports the FP32 application, the per-stage kernel
times, the HBM roofline of the dominant kernel launch (the algorithmic bytes
of its elements / its duration from HIP events around each launch) and of
the whole application, the Jacobi-PCG time to a 1e-10 relative residual in FP64 and as FP32
inner solves inside FP64 iterative refinement (manufactured solution
sin(pi x) sin(pi y) sin(pi z)), and the CPU oracle timed on a bounded sample
of the same workload.  `geometry_map` repeats the application and the solves
with deformed elements' geometric factors derived at every point from their
trilinear maps instead of read from HBM (a variant of the method, reported
beside the metric); `p2p` times the application with the point-to-point
interpolation flux instead of the shared trace (the paper's alternative);
`modal` times it in the modified C0 modal basis of Table 1, and `gauss` with
p+2 Gauss (Gauss-Legendre) volume points instead of GLL (the faces keep the
shared trace's GLL points), with its FP64 PCG solve.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cg] [--no-cpu] [--no-map] [--no-p2p] [--no-modal]
                    [--no-gauss]
"""

from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "SIPG matvec GDOF/s (FP64 vs FP32+refine) + CG time to 1e-10 residual, 1 GPU"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
WORKLOAD = 3


def algorithmic_bytes(st, dim, word):
    """Bytes one application must move: x in, y out, per-point volume
    factors (G w, d(d+1)/2 values, and w|J|), per trace point the factors
    (a, and C for each side: 2d+1 interior, d+1 boundary), lambda per element
    and 32 bytes of connectivity per face."""
    nvol = st["n_volume_points"]
    nint = st["n_interior_trace_points"]
    nbnd = st["n_boundary_trace_points"]
    nfaces = st["n_interior_faces"] + st["n_boundary_faces"]
    words = (2 * st["n_dofs"] + nvol * (dim * (dim + 1) // 2 + 1) + nint * (2 * dim + 1)
             + nbnd * (dim + 1) + st["n_elems"])
    return word * words + 32 * nfaces


def algorithmic_flops(mesh, st):
    """Sum-factorised flop count of one application (FMA = 2): BwdTrans and
    IProduct, collocation derivatives and their transposes, pointwise terms,
    interpolation to and from the trace for the lower-order side of each
    non-conforming face, and the per-trace-point flux."""
    import numpy as np
    d = mesh.dim
    p = mesh.order.astype(np.int64)
    n, np_ = p + 2, p + 1
    if d == 3:
        bt = 2 * (n * np_ ** 3 + n * n * np_ ** 2 + n ** 3 * np_)
        der = 2 * d * n ** (d + 1)
        pw = 20 * n ** 3
    else:
        bt = 2 * (n * np_ ** 2 + n * n * np_)
        der = 2 * d * n ** (d + 1)
        pw = 10 * n ** 2
    # trace kernel repeats BwdTrans and derivatives
    vol = int((2 * bt + 2 * der + pw).sum() + (bt + der).sum())
    trace = (st["n_interior_trace_points"] * 2 + st["n_boundary_trace_points"]) * (4 * (1 + d) + 12)
    return vol + trace


# The sources the FP64 application kernels are compiled from (the trace
# stage, the per-order applies and their multi-element tiles, with the
# argument and descriptor layouts they read): a stored traffic figure is used
# only while this hash matches, i.e. until one of those kernels changes.
KERNEL_SOURCES = ("context.hpp", "launch.hpp", "gfold3d.hpp", "gfold_tile.hpp", "k_tile.hpp", "tile_shapes.hpp",
                  "k_gfold3d_f64.hip", "k_tile_f64.hip")


def source_hash():
    h = hashlib.sha256()
    cdir = os.path.join(ROOT, "paper_2504_03573_amd", "csrc")
    for f in KERNEL_SOURCES:
        with open(os.path.join(cdir, f), "rb") as fh:
            h.update(f.encode())
            h.update(fh.read())
    return h.hexdigest()[:16]


def kernel_name(variant, order, stage=2, geo_map=False, tuning=None):
    """Kernel symbol (as rocprofv3 prints it, FP64) of one launch; tuning (the
    handle's tile shapes) names the multi-element tile kernel of an order
    group tuned to one."""
    if variant == "gather_fold":
        if stage == 1:
            return ("sipdg::g3::k3t_all<double, 0, false, false>" if order == 0
                    else "sipdg::g3::k3t<double, %d, 0, false>" % order)
        if tuning and 1 <= order <= 5 and (tuning["tile"][order], tuning["budget"][order]) != (1, 2):
            e, bud = tuning["tile"][order], tuning["budget"][order]
            nw = (e * (order + 2) ** 2 + 63) // 64
            return "sipdg::g3::k3gm<double, %d, %d, %d, %d, %d>" % (order, e, nw, 2 if geo_map else 0, bud)
        return "sipdg::g3::k3g<double, %d, 1, %d>" % (order, 2 if geo_map else 0)
    if variant == "gather_fold_persistent" and order == 0:
        return "sipdg::g3::k3g_persistent<double, %d>" % (0 if stage == 1 else 1)
    if variant == "gather_fold_fused":
        return "sipdg::g3::k3g<double, %d, 2, 0>" % order
    if variant == "two_stage":
        return ("sipdg::f3::k3_trace<double, %d>" % order if stage == 1
                else "sipdg::f3::k3_apply<double, %d, false>" % order)
    if variant == "fused":
        return "sipdg::f3::k3_apply<double, %d, true>" % order
    return "sipdg::k_%s<double, 3, %d>" % ("trace" if stage == 1 else "apply", order)


def p2p_kernel_name(variant, order, stage):
    """Kernel symbol of a launch of the point-to-point application."""
    if variant == "gather":
        return "sipdg::k_p2p_%s<double, %d>" % ("trace" if stage == 1 else "apply", order)
    if stage == 1:
        return "sipdg::g3::k3t_all<double, 0, true, false>" if order == 0 else "sipdg::g3::k3t<double, %d, 0, true>" % order
    return "sipdg::g3::k3g<double, %d, 1, 0>" % order


# CG vector traffic per iteration, in vector lengths: the dot p.q reads p and
# q; the fused update reads x, r, p, q and the inverse diagonal and writes x,
# r and z (with the two dot products r.z and r.r on the way); the direction
# update reads z and p and writes p.  The operator application's own bytes
# (p in, q out, factors) are its algorithmic bytes.
CG_VECTOR_WORDS = 2 + 8 + 3


def solve_record(info, ndof, apply_bytes, word):
    """Time to tolerance and the throughput of one solve: DOF-iterations per
    second (N_dof x iterations / time) and the HBM roofline fraction of an
    average iteration (one application's algorithmic bytes plus the CG
    vector traffic, over time per iteration).  For FP32 inside FP64
    refinement the iterations are the inner FP32 ones, and time includes the
    FP64 residual evaluations between them."""
    t = info["time_ms"] * 1e-3
    it = max(1, info["iters"])
    per_iter = apply_bytes + CG_VECTOR_WORDS * word * ndof
    return {"time_s": t, "iters": info["iters"], "outer_iters": info["outer_iters"],
            "rel_resid": info["rel_resid"], "converged": info["converged"],
            "ms_per_iter": info["time_ms"] / it,
            "gdofs": ndof * it / t / 1e9 if t > 0 else None,
            "bytes_per_iter": per_iter,
            "roofline_frac": per_iter / (t / it) / 1e9 / HBM_PEAK_GBS if t > 0 else None}


def time_events(fn, n, stream):
    import torch
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(n):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / n


def cpu_baseline(mesh, x, budget_s=12.0):
    """The oracle on a bounded random sample of elements (rows of y = A x)."""
    import numpy as np
    import oracle
    oracle.build(force=False)
    om = oracle.prepare(mesh)
    rng = np.random.default_rng(123)
    perm = rng.permutation(mesh.n_elems)
    dofs = (mesh.order.astype(np.int64) + 1) ** mesh.dim
    k = min(mesh.n_elems, 512)
    t0 = time.perf_counter()
    om.apply(x, elems=perm[:k])
    dt = time.perf_counter() - t0
    k2 = int(min(mesh.n_elems, max(k, k * budget_s / max(dt, 1e-3))))
    sel = np.sort(perm[:k2])
    t0 = time.perf_counter()
    om.apply(x, elems=sel)
    dt = time.perf_counter() - t0
    nd = int(dofs[sel].sum())
    threads = oracle.num_threads()
    # the same oracle on one thread, a smaller sample of the same rows
    k1 = max(16, min(k2, int(k2 * 0.25 / threads) + 1))
    sel1 = np.sort(perm[:k1])
    oracle.set_num_threads(1)
    try:
        t0 = time.perf_counter()
        om.apply(x, elems=sel1)
        dt1 = time.perf_counter() - t0
    finally:
        oracle.set_num_threads(threads)
    nd1 = int(dofs[sel1].sum())
    return {
        "value": nd / dt / 1e9, "unit": "GDOF/s", "cores": threads, "kind": "oracle",
        "sample": f"rows of {k2} of {mesh.n_elems} elements ({nd} of {int(dofs.sum())} DOFs), "
                  f"{dt:.1f} s, plain FP64 oracle, OpenMP over elements",
        "seconds": dt,
        "one_thread": {"value": nd1 / dt1 / 1e9, "unit": "GDOF/s", "seconds": dt1,
                       "sample": f"rows of {k1} elements ({nd1} DOFs)"},
        "host_cpu": _cpu_model(),
    }


def _sines_source(dim, lam):
    import torch

    def src(X):
        v = torch.ones(X.shape[0], dtype=torch.float64, device=X.device)
        for a in range(dim):
            v = v * torch.sin(math.pi * X[:, a])
        return (lam + dim * math.pi ** 2) * v
    return src


def _zero(X):
    import torch
    return torch.zeros(X.shape[0], dtype=torch.float64, device=X.device)


def bench_2d(args, stream):
    """The two 2-D workloads: FP64 and FP32 application times (back to back)
    and the FP64 PCG solve of the manufactured sin(pi x) sin(pi y) problem."""
    import torch

    import synth
    from paper_2504_03573_amd import SipdgOperator, inspect_mesh
    res = {}
    for k in (1, 2):
        m = synth.workload(k)
        st = inspect_mesh(m)
        op = SipdgOperator(m)
        tuned = op.autotune(200)   # applications of ~10 us: many repetitions against timer noise
        x = torch.tensor(synth.random_coefficients(m, 4000 + k), device="cuda")
        y = torch.empty_like(x)
        x32, y32 = x.float(), torch.empty_like(x, dtype=torch.float32)
        for _ in range(args.warmup):
            op.apply(x, out=y)
            op.apply(x32, out=y32)
        reps = max(args.steps, 100)
        ms = time_events(lambda: op.apply(x, out=y), reps, stream)
        ms32 = time_events(lambda: op.apply(x32, out=y32), reps, stream)
        b = op.rhs(_sines_source(2, 1.0), _zero)
        op.cg_solve(b, tol=1e-10, maxit=50, raise_on_fail=False)
        torch.cuda.synchronize()
        _, info = op.cg_solve(b, tol=1e-10, maxit=getattr(args, "cg_iters", 100000), raise_on_fail=False)
        res["workload_%d" % k] = {
            "workload": synth.WORKLOADS[k], "n_dofs": op.n_dofs,
            "apply_us": ms * 1e3, "gdofs": op.n_dofs / (ms * 1e-3) / 1e9,
            "apply_fp32_us": ms32 * 1e3, "gdofs_fp32": op.n_dofs / (ms32 * 1e-3) / 1e9,
            "launches_per_apply": len(op.apply_timed(x, y, reps=5, stream=stream)),
            "variant": op.variant, "autotune_ms": tuned,
            "cg_f64": solve_record(info, op.n_dofs, algorithmic_bytes(st, 2, 8), 8),
        }
        op.close()
    return res


def _lam_points(m):
    """lambda of the element owning each volume quadrature point (points
    element after element, (p+2)^d per element)."""
    import numpy as np
    npts = (m.order.astype(np.int64) + 2) ** m.dim
    return np.repeat(np.broadcast_to(np.asarray(m.lam, dtype=np.float64), (m.n_elems,)), npts)


def bench_batched(args, stream):
    """The 64-problem batch (problem i: n_i^3 perturbed hexes, order p_i,
    lambda_i; one handle, every order group of all problems in one launch):
    FP64 and FP32 application after autotuning, and Jacobi-PCG to 1e-10 of
    every problem (FP64, FP32 inside FP64 refinement) on the manufactured
    sin(pi x) sin(pi y) sin(pi z) problems."""
    import torch

    import synth
    from paper_2504_03573_amd import SipdgOperator, inspect_mesh
    meshes = synth.workload(4)
    op = SipdgOperator.batch(meshes)
    tuned = op.autotune(10)
    x = torch.randn(op.n_dofs, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    x32, y32 = x.float(), torch.empty(op.n_dofs, dtype=torch.float32, device="cuda")
    for _ in range(3):
        op.apply(x, out=y)
        op.apply(x32, out=y32)
    reps = max(10, min(args.steps, 50))
    ms = time_events(lambda: op.apply(x, out=y), reps, stream)
    ms32 = time_events(lambda: op.apply(x32, out=y32), reps, stream)
    lam_q = torch.cat([torch.tensor(_lam_points(m), device="cuda") for m in meshes])

    def src(X):
        v = torch.sin(math.pi * X[:, 0]) * torch.sin(math.pi * X[:, 1]) * torch.sin(math.pi * X[:, 2])
        return (lam_q + 3 * math.pi ** 2) * v
    b = op.rhs(src, _zero)
    b64 = sum(algorithmic_bytes(inspect_mesh(m), 3, 8) for m in meshes)
    b32 = sum(algorithmic_bytes(inspect_mesh(m), 3, 4) for m in meshes)
    cg = {}
    for mode in ("f64", "f32_ir"):
        op.cg_solve(b, tol=1e-10, mode=mode, maxit=50, raise_on_fail=False)
        torch.cuda.synchronize()
        _, info = op.cg_solve(b, tol=1e-10, mode=mode, maxit=getattr(args, "cg_iters", 100000), raise_on_fail=False)
        cg[mode] = solve_record(info, op.n_dofs, b64 if mode == "f64" else b32, 8 if mode == "f64" else 4)
    res = {"workload": synth.WORKLOADS[4], "problems": len(meshes), "n_dofs": op.n_dofs, "variant": op.variant,
           "autotune_ms": tuned, "apply_ms": ms, "gdofs": op.n_dofs / (ms * 1e-3) / 1e9,
           "roofline_frac": b64 / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
           "apply_fp32_ms": ms32, "gdofs_fp32": op.n_dofs / (ms32 * 1e-3) / 1e9, "cg": cg}
    op.close()
    return res


def bench_workload5(args, stream):
    """The 24^3 differentiation workload (orders 3..5, per-element lambda):
    the FP64 application, its transpose, the parameter gradients (the
    backward of the autograd application) and the FP64 PCG solve."""
    import torch

    import synth
    from paper_2504_03573_amd import SipdgOperator, inspect_mesh
    m = synth.workload(5)
    op = SipdgOperator(m)
    op.autotune(20)
    x = torch.tensor(synth.random_coefficients(m, 4005), device="cuda")
    y = torch.empty_like(x)
    for _ in range(5):
        op.apply(x, out=y)
    reps = max(20, min(args.steps, 100))
    ms = time_events(lambda: op.apply(x, out=y), reps, stream)
    mst = time_events(lambda: op.apply_transpose(x, out=y), reps, stream)
    msg = time_events(lambda: op.param_grad(x, y), reps, stream)
    lam_q = torch.tensor(_lam_points(m), device="cuda")

    def src(X):
        v = torch.sin(math.pi * X[:, 0]) * torch.sin(math.pi * X[:, 1]) * torch.sin(math.pi * X[:, 2])
        return (lam_q + 3 * math.pi ** 2) * v
    b = op.rhs(src, _zero)
    op.cg_solve(b, tol=1e-10, maxit=50, raise_on_fail=False)
    torch.cuda.synchronize()
    _, info = op.cg_solve(b, tol=1e-10, maxit=getattr(args, "cg_iters", 100000), raise_on_fail=False)
    res = {"workload": synth.WORKLOADS[5], "n_dofs": op.n_dofs, "variant": op.variant,
           "apply_us": ms * 1e3, "gdofs": op.n_dofs / (ms * 1e-3) / 1e9, "apply_transpose_us": mst * 1e3,
           "param_grad_us": msg * 1e3,
           "cg_f64": solve_record(info, op.n_dofs, algorithmic_bytes(inspect_mesh(m), 3, 8), 8)}
    op.close()
    return res


def bench_sweep(stream, reps=30):
    """FP64 application throughput against problem size and order (the
    paper's size study, Sec. 5.2): perturbed hex meshes N^3 with one order p
    on every element (conforming), N chosen so that N_dof spans about 1e4 to
    1e8; default kernel structure, no autotuning."""
    import torch

    import synth
    from paper_2504_03573_amd import SipdgOperator
    rows = []
    for p in (3, 4, 5, 6):
        for N in (4, 8, 16, 32, 48, 64):
            ndof = N ** 3 * (p + 1) ** 3
            if ndof > 1.1e8:
                continue
            m = synth.structured_mesh(3, N, 0.1, seed=7000 + N, order=p, lam=10.0)
            op = SipdgOperator(m)
            x = torch.randn(op.n_dofs, dtype=torch.float64, device="cuda")
            y = torch.empty_like(x)
            for _ in range(5):
                op.apply(x, out=y)
            ms = time_events(lambda: op.apply(x, out=y), reps, stream)
            rows.append({"p": p, "N": N, "n_dofs": op.n_dofs, "ms": ms, "gdofs": op.n_dofs / (ms * 1e-3) / 1e9})
            op.close()
            del x, y
            torch.cuda.empty_cache()
    return rows


def oracle_cg_times(gpu_2d):
    """The oracle's Jacobi-PCG (plain FP64, OpenMP applications): to 1e-10 on
    the 2-D 4^2 workload; bounded runs on the 2-D 64^2 workload (200
    iterations; its full solve takes about a minute) and on the 3-D 24^3
    workload (10 iterations; many minutes), reported per iteration and as
    the time of the GPU solve's iteration count at that rate."""
    import numpy as np

    import oracle
    import synth
    oracle.build(force=False)
    res = {}
    for k in (1, 2):
        m = synth.workload(k)
        om = oracle.prepare(m)
        b = om.rhs_from(lambda X: (1.0 + 2 * math.pi ** 2) * np.sin(math.pi * X[:, 0]) * np.sin(math.pi * X[:, 1]),
                        lambda X: np.zeros(len(X)))
        gpu = (gpu_2d or {}).get("workload_%d" % k, {}).get("cg_f64", {})
        t0 = time.perf_counter()
        if k == 1:
            _, it, rel = om.cg(b, tol=1e-10)
            dt = time.perf_counter() - t0
            res["workload_1"] = {"time_s": dt, "iters": it, "true_rel_resid": rel, "gpu_time_s": gpu.get("time_s")}
        else:
            _, it, _ = om.cg(b, tol=1e-30, maxit=200)
            dt = time.perf_counter() - t0
            per = dt / it
            res["workload_2"] = {"iters_timed": it, "time_s": dt, "ms_per_iter": per * 1e3,
                                 "projected_time_s": per * gpu["iters"] if gpu.get("iters") else None,
                                 "gpu_time_s": gpu.get("time_s"),
                                 "note": "bounded sample: 200 iterations of the oracle's PCG; projected to the "
                                         "GPU solve's iteration count"}
    m = synth.workload(5)
    om = oracle.prepare(m)
    rng = np.random.default_rng(5)
    b = rng.standard_normal(om.n_dofs)
    t0 = time.perf_counter()
    om.diagonal()
    t_diag = time.perf_counter() - t0
    t0 = time.perf_counter()
    _, it, _ = om.cg(b, tol=1e-30, maxit=10)
    dt = time.perf_counter() - t0
    res["workload_5"] = {"iters_timed": it, "time_s": dt, "diagonal_s": t_diag,
                         "ms_per_iter": max(dt - 2 * t_diag, 0.0) / it * 1e3,
                         "note": "bounded sample: 10 iterations of the oracle's PCG (its Jacobi diagonal and "
                                 "final residual application taken out of the per-iteration time)"}
    res["threads"] = oracle.num_threads()
    return res


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cg", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-probe", action="store_true",
                    help="kept for the profiling commands (the 1 GiB copy always runs)")
    ap.add_argument("--variant", default=None,
                    help="kernel structure to use instead of the autotuner's choice (profiling runs)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="skip the autotuner on the 32^3 workload: default tile shapes (profiling runs, where "
                         "counter collection distorts its timing)")
    ap.add_argument("--no-modal", action="store_true",
                    help="skip the apply in the modified C0 modal basis")
    ap.add_argument("--no-gauss", action="store_true",
                    help="skip the apply with Gauss volume points")
    ap.add_argument("--no-p2p", action="store_true",
                    help="skip the apply with the point-to-point interpolation flux")
    ap.add_argument("--no-map", action="store_true",
                    help="skip the apply with geometry derived from the element maps")
    ap.add_argument("--no-2d", action="store_true",
                    help="skip the 2-D workloads (4^2 p=3 and 64^2 checkerboard 4/5)")
    ap.add_argument("--no-sweep", action="store_true",
                    help="skip the throughput sweep over problem size and order")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the 64-problem batch and the 24^3 differentiation workload")
    ap.add_argument("--cg-iters", type=int, default=100000,
                    help="iteration cap of every CG solve (profiling runs: a bounded number of iterations; "
                         "solves that stop at the cap report converged false)")
    ap.add_argument("--traffic", default=os.path.join(ROOT, "profiles", "traffic_hex32_p3to6.json"))
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    from paper_2504_03573_amd import SipdgOperator, inspect_mesh

    torch.cuda.set_device(0)
    mesh = synth.workload(WORKLOAD)
    st = inspect_mesh(mesh)
    op = SipdgOperator(mesh)
    tuned = None if args.no_autotune else op.autotune(20)
    if args.variant:
        # profiling runs pin the kernel structure (counters distort the autotuner's timing)
        op.variant = args.variant
    stream = torch.cuda.current_stream()
    x_np = synth.random_coefficients(mesh, 4000 + WORKLOAD)
    x = torch.tensor(x_np, device="cuda")
    y = torch.empty_like(x)
    x32 = x.float()
    y32 = torch.empty_like(x32)

    # measured streaming bandwidth: a 1 GiB device-to-device copy (read + write)
    a = torch.empty(1 << 27, dtype=torch.float64, device="cuda").fill_(1.0)
    bcp = torch.empty_like(a)
    bcp.copy_(a)
    torch.cuda.synchronize()
    copy_ms = time_events(lambda: bcp.copy_(a), 10, stream)
    copy_gbs = 2 * a.numel() * 8 / (copy_ms * 1e-3) / 1e9
    del a, bcp

    for _ in range(args.warmup):
        op.apply(x, out=y)
        op.apply(x32, out=y32)
    torch.cuda.synchronize()
    # timed region: exactly K FP64 applications
    torch.cuda.synchronize()
    t_wall0 = time.perf_counter()
    ms = time_events(lambda: op.apply(x, out=y), args.steps, stream)
    torch.cuda.synchronize()
    t_wall = time.perf_counter() - t_wall0
    ms32 = time_events(lambda: op.apply(x32, out=y32), args.steps, stream)
    # per-stage times (stage 1: trace kernels, stage 2: flux/volume kernels)
    op.apply_stage(x, 1)
    ms_s1 = time_events(lambda: op.apply_stage(x, 1), args.steps, stream)
    ms_s2 = time_events(lambda: op.apply_stage(x, 2, out=y), args.steps, stream)

    # per-launch durations of one application, HIP events around every launch
    launches = op.apply_timed(x, y, reps=max(10, min(args.steps, 100)), stream=stream)

    ndof = op.n_dofs
    b64 = algorithmic_bytes(st, 3, 8)
    b32 = algorithmic_bytes(st, 3, 4)
    flops = algorithmic_flops(mesh, st)
    achieved = b64 / (ms * 1e-3) / 1e9
    apply_launches = [L for L in launches if L["stage"] == 2]
    dom = max(apply_launches, key=lambda L: L["ms"])
    tuning = op.tuning()
    dom_name = kernel_name(op.variant, dom["order"], tuning=tuning)
    traffic = traffic_app = None
    if os.path.exists(args.traffic):
        try:
            tr = json.load(open(args.traffic))
            if tr.get("source_hash") == source_hash() and tr.get("variant") == op.variant:
                traffic_app = tr.get("bytes_per_apply")
                traffic = tr.get("bytes_per_dispatch", {}).get(dom_name)
        except (OSError, ValueError):
            traffic = traffic_app = None
    out = {
        "metric": METRIC,
        "value": ndof / (ms * 1e-3) / 1e9,
        "unit": "GDOF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "3-D hex 32^3 perturbed (+-0.1h) on [0,1]^3, order U{3..6} per element "
                        "(seed 2003), lambda=10, Legendre modes, GLL p+2, sigma=1",
            "n_dofs": ndof, "n_elems": op.n_elems,
            "n_interior_faces": st["n_interior_faces"],
            "n_nonconforming_faces": st["n_nonconforming_faces"],
        },
        "roofline": {
            "bound": "hbm", "achieved": dom["alg_bytes"] / (dom["ms"] * 1e-3) / 1e9, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": dom["alg_bytes"] / (dom["ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "traffic": traffic,
            "frac_measured_copy": dom["alg_bytes"] / (dom["ms"] * 1e-3) / 1e9 / copy_gbs,
            "kernel": dom_name,
            "launch_ms": dom["ms"], "elements": dom["elements"], "algorithmic_bytes": dom["alg_bytes"],
            "unit_bytes": "per element of order p: 8*(2(p+1)^3 + 7(p+2)^3 + 1) plus its share of its faces' "
                          "factors (boundary: 4 n_F^2 values + 32 B; interior: half of 7 n_F^2 values + 32 B)",
        },
        "hbm_copy_measured_gbs": copy_gbs,
        "roofline_application": {
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "frac_measured_copy": achieved / copy_gbs,
            "traffic": traffic_app, "algorithmic_bytes": b64,
            "kernels": "all launches of one application (kernel structure: %s)" % op.variant,
        },
        "launches": [{"kernel": kernel_name(op.variant, L["order"], L["stage"], tuning=tuning), "ms": L["ms"],
                      "elements": L["elements"],
                      "gbs": (L["alg_bytes"] / (L["ms"] * 1e-3) / 1e9) if L["alg_bytes"] else None}
                     for L in launches],
        "check_algorithmic_bytes": sum(L["alg_bytes"] for L in apply_launches),
        "fp32_apply": {
            "value": ndof / (ms32 * 1e-3) / 1e9, "unit": "GDOF/s", "ms": ms32,
            "roofline_frac": b32 / (ms32 * 1e-3) / 1e9 / HBM_PEAK_GBS,
        },
        "stages_ms": {"trace": ms_s1, "flux_volume": ms_s2},
        "variant": op.variant,
        "tile_shapes": {str(p): [tuning["tile"][p], tuning["budget"][p]] for p in range(1, 9)},
        "autotune_ms": tuned,
        "flops": {"algorithmic_per_apply": flops,
                  "tflops": flops / (ms * 1e-3) / 1e12,
                  "frac_fp64_peak": flops / (ms * 1e-3) / 1e12 / FP64_PEAK_TFLOPS},
        "wall_timed_s": t_wall,
    }
    if not args.no_cg:
        lam = 10.0
        k = math.pi

        def src(X):
            return (lam + 3 * k * k) * torch.sin(k * X[:, 0]) * torch.sin(k * X[:, 1]) * torch.sin(k * X[:, 2])

        bvec = op.rhs(src, lambda X: torch.zeros(X.shape[0], dtype=torch.float64, device=X.device))
        cg = {}
        # f64: FP64 PCG; f32_ir: FP32 PCG inside FP64 iterative refinement;
        # f32_ru: FP32 PCG with FP64 reliable updates (residual replaced every 10x)
        for mode in ("f64", "f32_ir", "f32_ru"):
            op.cg_solve(bvec, tol=1e-10, mode=mode, maxit=50, raise_on_fail=False)  # graph capture
            torch.cuda.synchronize()
            xs, info = op.cg_solve(bvec, tol=1e-10, mode=mode, maxit=args.cg_iters, raise_on_fail=False)
            cg[mode] = solve_record(info, ndof, b64 if mode == "f64" else b32, 8 if mode == "f64" else 4)
        out["cg"] = cg
    if not args.no_map:
        # the same operator with deformed elements' geometric factors derived at
        # every point from their trilinear maps (not the stored factors that the
        # metric's method reads): reported beside the metric, never as `value`
        keep = op.variant
        op.variant = "gather_fold"
        op.geometry = "map"
        for _ in range(args.warmup):
            op.apply(x, out=y)
            op.apply(x32, out=y32)
        ms_m = time_events(lambda: op.apply(x, out=y), args.steps, stream)
        ms_m32 = time_events(lambda: op.apply(x32, out=y32), args.steps, stream)
        lm = op.apply_timed(x, y, reps=max(10, min(args.steps, 100)), stream=stream)
        gm = {"value": ndof / (ms_m * 1e-3) / 1e9, "unit": "GDOF/s", "ms": ms_m,
              "fp32_value": ndof / (ms_m32 * 1e-3) / 1e9, "fp32_ms": ms_m32,
              "launches": [{"kernel": kernel_name("gather_fold", L["order"], L["stage"], geo_map=True,
                                                  tuning=tuning),
                            "ms": L["ms"]} for L in lm]}
        if not args.no_cg:
            for mode in ("f64", "f32_ir"):
                op.cg_solve(bvec, tol=1e-10, mode=mode, maxit=50, raise_on_fail=False)
                torch.cuda.synchronize()
                _, info = op.cg_solve(bvec, tol=1e-10, mode=mode, maxit=args.cg_iters, raise_on_fail=False)
                gm["cg_" + mode] = solve_record(info, ndof, b64 if mode == "f64" else b32,
                                                8 if mode == "f64" else 4)
        out["geometry_map"] = gm
        op.geometry = "stored"
        op.variant = keep
    if not args.no_p2p:
        # the point-to-point interpolation flux (the paper's alternative to the
        # shared trace space; a different, nonsymmetric operator): application
        # only, reported beside the metric
        op.flux = "p2p"
        for _ in range(args.warmup):
            op.apply(x, out=y)
            op.apply(x32, out=y32)
        ms_p = time_events(lambda: op.apply(x, out=y), args.steps, stream)
        ms_p32 = time_events(lambda: op.apply(x32, out=y32), args.steps, stream)
        lp = op.apply_timed(x, y, reps=max(10, min(args.steps, 100)), stream=stream)
        out["p2p"] = {"value": ndof / (ms_p * 1e-3) / 1e9, "unit": "GDOF/s", "ms": ms_p,
                      "fp32_value": ndof / (ms_p32 * 1e-3) / 1e9, "fp32_ms": ms_p32,
                      "variant": op.variant,
                      "launches": [{"kernel": p2p_kernel_name(op.variant, L["order"], L["stage"]), "ms": L["ms"]}
                                   for L in lp]}
        op.flux = "shared"
    if not args.no_modal:
        # the modified C0 modal basis (Table 1 "Modal"): a congruent operator,
        # on the default gather-fold path; reported beside the metric
        keep = op.variant
        op.basis = "modal"
        for _ in range(args.warmup):
            op.apply(x, out=y)
            op.apply(x32, out=y32)
        ms_b = time_events(lambda: op.apply(x, out=y), args.steps, stream)
        ms_b32 = time_events(lambda: op.apply(x32, out=y32), args.steps, stream)
        out["modal"] = {"value": ndof / (ms_b * 1e-3) / 1e9, "unit": "GDOF/s", "ms": ms_b,
                        "fp32_value": ndof / (ms_b32 * 1e-3) / 1e9, "fp32_ms": ms_b32, "variant": op.variant}
        op.basis = "legendre"
        op.variant = keep
    if not args.no_gauss:
        # Gauss volume points (point sets without the element boundary,
        # Sec. 3.2): volume terms at p+2 Gauss points with geometry from the
        # maps, faces from the trace stage lifted to the modes; another
        # quadrature of the same form, reported beside the metric
        keep = op.variant
        op.points = "gauss"
        for _ in range(args.warmup):
            op.apply(x, out=y)
            op.apply(x32, out=y32)
        ms_g = time_events(lambda: op.apply(x, out=y), args.steps, stream)
        ms_g32 = time_events(lambda: op.apply(x32, out=y32), args.steps, stream)
        lg = op.apply_timed(x, y, reps=max(10, min(args.steps, 100)), stream=stream)
        gs = {"value": ndof / (ms_g * 1e-3) / 1e9, "unit": "GDOF/s", "ms": ms_g,
              "fp32_value": ndof / (ms_g32 * 1e-3) / 1e9, "fp32_ms": ms_g32,
              "launches": [{"kernel": kernel_name("gather_fold", L["order"], 1) if L["stage"] == 1
                            else "sipdg::g3::k3g<double, %d, 3, 2>" % L["order"], "ms": L["ms"]} for L in lg]}
        if not args.no_cg:
            op.cg_solve(bvec, tol=1e-10, mode="f64", maxit=50, raise_on_fail=False)
            torch.cuda.synchronize()
            _, info = op.cg_solve(bvec, tol=1e-10, mode="f64", maxit=args.cg_iters, raise_on_fail=False)
            gs["cg_f64"] = solve_record(info, ndof, b64, 8)
        out["gauss"] = gs
        op.points = "gll"
        op.variant = keep
    if not args.no_2d:
        out["workloads_2d"] = bench_2d(args, stream)
    if not args.no_batch:
        out["workload_4_batched"] = bench_batched(args, stream)
        out["workload_5"] = bench_workload5(args, stream)
    if not args.no_sweep:
        out["sweep"] = bench_sweep(stream)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(mesh, x_np)
        if not args.no_cg:
            out["cpu_baseline"]["cg"] = oracle_cg_times(out.get("workloads_2d"))
    print(json.dumps(out))


if __name__ == "__main__":
    main()
