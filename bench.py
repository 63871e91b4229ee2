"""Benchmark: HIF-IE factor + solve throughput on one MI355X.

Workload (the 512 x 512 configuration): 2D second-kind Laplace volume IE on
the unit square, uniform 512 x 512 cell-centred grid (N = 262144, h = 1/512),
a = b = c = 1 (K_ij = -log|x_i - x_j| h^2 / (2 pi), closed-form diagonal),
eps = 1e-6, leaf boxes of 64 points, 8 standard-normal right-hand sides,
FP64 with the second-kind modification.  One step = hif_factor + hif_solve of
all 8 right-hand sides (+ releasing the factors); inputs are resident in HBM
before the timed region starts.

Printed: one JSON line with the metric (unknowns/s = N / step time), the
accuracy gate (error of the solution against the exact solution of the
discretized system, estimated by one step of refinement with the exact
on-the-fly matvec), a roofline entry for the dominant kernel and the CPU
oracle's throughput on a bounded sample.

``--workload batch48`` times 48 independent problems of uneven sizes (sides 64 to
256, 4 right-hand sides each) factored concurrently by hif_factor_batch and
solved one by one; one step = the batch factorization + every solve.

``--workload diff256`` times the differentiated solve instead: 256 x 256 grid,
a = 1 + 64 Gaussian bumps, one right-hand side, L = |u - u_target|^2 / 2; one
step = forward (factor + solve) + backward (adjoint solve + dL/da, dL/df).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_VECTOR_TFLOPS = 78.6  # MI355X: 256 CUs x 128 FP64 flop/clk x 2.4 GHz
HBM_PEAK_GBS = 8000.0
# HBM bytes per factorization moved by the pivoted-QR kernels (k_bq_init,
# k_bq_piv, k_bq_cols, k_bq_update, k_id_reg, k_id) on this workload, from
# rocprofv3 FETCH_SIZE + WRITE_SIZE runs of `bench.py --steps 1 --warmup 0
# --no-cpu-baseline --no-refine --calib-copy`, each scaled by what the counter
# reads for a 256 MiB copy kernel (159.5 GB read + 5.9 GB written; taken again
# after the last change to k_bq_piv and k_bq_cols).  Valid for these kernels as
# they stand; set to None when they change.
ID_STEP_TRAFFIC_BYTES = 1.655e+11


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=3)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--workload", default="sq512")
    p.add_argument("--eps", type=float, default=None)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-sample", default="sq128")
    p.add_argument("--calib-copy", action="store_true",
                   help="after the timed region, run one plain 256 MiB device copy kernel (scale for HBM counters)")
    p.add_argument("--no-refine", action="store_true",
                   help="skip the FP64 vs FP32-mixed comparison with GMRES refinement")
    p.add_argument("--no-extras", action="store_true",
                   help="skip the short runs of the differentiated-solve and batch workloads")
    return p.parse_args()


def cpu_baseline(sample: str, eps: float):
    """The oracle as it stands (FP64 NumPy/SciPy, one BLAS thread), factor + solve of 8 RHS."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle.factor import factorize
    from oracle.kernels import Operator
    from workloads import grid_points, rhs

    n = int(sample.replace("sq", ""))
    pts = grid_points(n, 2)
    N = pts.shape[0]
    op = Operator.uniform(pts, 1.0 / n, a=np.ones(N))
    F8 = rhs(N, 8, 1)
    with threadpool_limits(1):
        t0 = time.perf_counter()
        F = factorize(op, eps, 64)
        F.solve(F8)
        dt = time.perf_counter() - t0
    return {"value": N / dt, "unit": "unknowns/s", "cores": 1, "kind": "oracle",
            "sample": f"oracle hifie2x factor + 8-RHS solve of the {n}x{n} grid (N={N}, same kernel, "
                      f"leaf 64, eps {eps:g}), {dt:.1f} s on 1 host core"}


def refinement(hif, P, a, Fr, wl, tol=1e-10):
    """FP64 vs FP32-mixed factorization as GMRES preconditioner, to a true relative
    residual of ``tol`` against the exact FP64 operator (hif_gmres).  Total time =
    factor + GMRES (each iteration one solve and one exact matvec, plus the final
    residual check), best over eps in {1e-3, 1e-6} for each precision; one warm run
    per configuration, the second one timed."""
    import torch

    runs = []
    for prec, pname, sk in ((hif.HIF_FP64, "fp64", -1), (hif.HIF_FP32_MIXED, "fp32_mixed", -1),
                            (hif.HIF_FP32_MIXED, "fp32_mixed_x", 1)):
        for e in (1e-3, 1e-6):
            if pname == "fp32_mixed_x" and e != 1e-3:
                continue
            for rep in range(2):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                F = hif.factor(P, e, wl.leaf, a=a, h=wl.h, precision=prec, second_kind=sk)
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                _, its, rr = F.gmres(Fr, tol=tol, maxit=40)
                torch.cuda.synchronize()
                t2 = time.perf_counter()
                F.free()
            runs.append({"precision": pname, "eps": e, "factor_s": t1 - t0, "gmres_s": t2 - t1,
                         "total_s": t2 - t0, "iterations": max(its), "rel_residual_max": max(rr),
                         "converged": bool(max(rr) <= 1.5 * tol)})
    ok = [r for r in runs if r["converged"]]
    best = {}
    for pname in ("fp64", "fp32_mixed"):
        cand = [r for r in ok if r["precision"].startswith(pname)]
        if cand:
            best[pname] = min(cand, key=lambda r: r["total_s"])
    speedup = (best["fp64"]["total_s"] / best["fp32_mixed"]["total_s"]
               if "fp64" in best and "fp32_mixed" in best else None)
    return {"target_residual": tol, "runs": runs, "best": best, "mixed_vs_fp64_speedup": speedup}


def id_roofline(st, ph):
    """Roofline entry of the pivoted-QR kernel family from a factorization's statistics."""
    import numpy as np

    id_bytes = float(np.sum(st["sub_id_bytes"]))
    id_ms = ph["id"]
    achieved = id_bytes / (id_ms * 1e-3) / 1e9 if id_ms > 0 else 0.0
    return {"kernel": "k_bq_piv + k_bq_cols + k_bq_update + k_id_reg + k_id (column-pivoted QR of "
                      "the IDs, all launches of a step)",
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": None, "bytes_per_step": id_bytes, "ms_per_step": id_ms}


def cpu_baseline_diff(n: int, eps: float):
    """The oracle as it stands (one BLAS thread): factor + solve + transposed solve + dL/da
    of the differentiated-solve problem on an n x n grid."""
    from threadpoolctl import threadpool_limits

    from oracle.factor import factorize
    from oracle.kernels import Operator
    from workloads import diff_problem

    p = diff_problem(n)
    op = Operator.uniform(p.points, p.h, a=p.a)
    with threadpool_limits(1):
        t0 = time.perf_counter()
        F = factorize(op, eps, 64)
        u = F.solve(p.f)
        lam = F.solve_T(u - p.u_target)
        _ = -(lam * u)
        dt = time.perf_counter() - t0
    N = p.points.shape[0]
    return {"value": N / dt, "unit": "unknowns/s", "cores": 1, "kind": "oracle",
            "sample": f"oracle hifie2x factor + solve + transposed solve of the {n}x{n} differentiated-solve "
                      f"problem (N={N}, leaf 64, eps {eps:g}), {dt:.1f} s on 1 host core"}


def cpu_baseline_batch(prob, eps: float):
    """The oracle as it stands (one BLAS thread): factor + 4-RHS solve of one problem of the batch."""
    from threadpoolctl import threadpool_limits

    from oracle.factor import factorize
    from oracle.kernels import Operator

    op = Operator.uniform(prob["points"], prob["h"], a=prob["a"])
    with threadpool_limits(1):
        t0 = time.perf_counter()
        F = factorize(op, eps, prob["leaf"])
        F.solve(prob["f"])
        dt = time.perf_counter() - t0
    N = prob["points"].shape[0]
    return {"value": N / dt, "unit": "unknowns/s", "cores": 1, "kind": "oracle",
            "sample": f"oracle hifie2x factor + 4-RHS solve of one {prob['n']}x{prob['n']} problem of the batch "
                      f"(N={N}, leaf {prob['leaf']}, eps {eps:g}), {dt:.1f} s on 1 host core"}


def bench_batch(args, quiet=False):
    """48 independent problems: concurrent factorization (4 worker streams), then every solve."""
    import numpy as np
    import torch

    import paper_1307_2666_amd as hif
    from workloads import batch_problems

    dev = "cuda:0"
    torch.cuda.set_device(0)
    probs = batch_problems()
    Ntot = sum(p["points"].shape[0] for p in probs)
    dp = [dict(points=torch.tensor(p["points"], device=dev), a=torch.tensor(p["a"], device=dev), h=p["h"],
               eps=p["eps"], leaf=p["leaf"]) for p in probs]
    fs = [torch.tensor(p["f"], device=dev) for p in probs]
    nw = 4

    def step(nworkers=nw, lat=None):
        facs, st = hif.factor_batch(dp, nworkers=nworkers)
        if any(x != 0 for x in st):
            raise RuntimeError(f"batch factorization failed: {st}")
        us = []
        for F, f in zip(facs, fs):
            if lat is not None:
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                us.append(F.solve(f))
                e1.record()
                lat.append((e0, e1))
            else:
                us.append(F.solve(f))
        return facs, us

    for _ in range(args.warmup):
        facs, _ = step()
        for F in facs:
            F.free()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = []
    for _ in range(args.steps):
        facs, us = step()
        torch.cuda.synchronize()
        stats.append([F.stats() for F in facs])
        for F in facs:
            F.free()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    # one worker (one factorization at a time) for comparison, and per-solve latency
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    lat = []
    facs, us = step(nworkers=1, lat=lat)
    torch.cuda.synchronize()
    dt1 = time.perf_counter() - t1
    lat_ms = np.array([e0.elapsed_time(e1) for e0, e1 in lat])
    err = 0.0
    for F, u, f in zip(facs, us, fs):
        y, _ = F.apply_A(u)
        err = max(err, (torch.linalg.norm(y - f, dim=1) / torch.linalg.norm(f, dim=1)).max().item())
    st = stats[-1]
    id_bytes = float(sum(np.sum(s["sub_id_bytes"]) for s in st))
    id_ms = float(sum(s["t_phase_ms"]["id"] for s in st))
    for F in facs:
        F.free()
    achieved = id_bytes / (id_ms * 1e-3) / 1e9 if id_ms > 0 else 0.0
    line = {
        "metric": "batch factor+solve unknowns/s (48 uneven problems)",
        "value": Ntot / dt, "unit": "unknowns/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"batch48: 48 independent 2D second-kind Laplace volume IEs, sides from "
                               f"{{64, 96, 128, 192, 256}} (N total {Ntot}), a = 1 + scaled Gaussian bumps, "
                               f"4 RHS each, eps 1e-6, leaves 36 or 64 points, FP64; hif_factor_batch with "
                               f"{nw} worker streams, then every 4-RHS solve", "N_total": Ntot, "problems": 48},
        "accuracy": {"rel_residual_max": err},
        "one_worker_ms_per_step": dt1 * 1e3,
        "solve_latency_ms": {"p50": float(np.percentile(lat_ms, 50)), "p99": float(np.percentile(lat_ms, 99)),
                             "max": float(lat_ms.max())},
        "roofline": {"kernel": "k_bq_piv + k_bq_cols + k_bq_update + k_id_reg + k_id (column-pivoted QR of "
                               "the IDs); per-problem HIP-event times summed, so concurrent problems overlap",
                     "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None, "bytes_per_step": id_bytes,
                     "ms_per_step": id_ms},
    }
    if not args.no_cpu_baseline:
        small = min(probs, key=lambda p: p["n"])
        line["cpu_baseline"] = cpu_baseline_batch(small, 1e-6)
    if quiet:
        return line
    print(json.dumps(line), flush=True)


def bench_diff(args, quiet=False):
    """Forward + backward of the differentiated solve on the 256 x 256 problem."""
    import numpy as np
    import torch

    import paper_1307_2666_amd as hif
    from workloads import diff_problem

    eps = args.eps if args.eps is not None else 1e-6
    dev = "cuda:0"
    torch.cuda.set_device(0)
    p = diff_problem(256)
    N = p.points.shape[0]
    P = torch.tensor(p.points, device=dev)
    a0 = torch.tensor(p.a, device=dev)
    f0 = torch.tensor(p.f, device=dev)
    t = torch.tensor(p.u_target, device=dev)

    def step(prec=hif.HIF_FP64, refine=False):
        a = a0.clone().requires_grad_(True)
        f = f0.clone().requires_grad_(True)
        u = hif.diff.solve(P, a, f, eps, 64, h=p.h, precision=prec, refine=refine, tol=1e-12)
        st = u.grad_fn.fac.stats()
        (0.5 * torch.sum((u - t) ** 2)).backward()
        return a.grad, f.grad, st

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    stats = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ga, gf, st = step()
        stats.append(st)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    modes = {}
    ref = None
    for name, prec, refine in (("fp64_refined", hif.HIF_FP64, True), ("fp32_mixed_refined", hif.HIF_FP32_MIXED, True)):
        step(prec, refine)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        g = step(prec, refine)
        torch.cuda.synchronize()
        modes[name] = {"ms_per_step": (time.perf_counter() - t1) * 1e3}
        if ref is None:
            ref = g
        else:
            modes[name]["grad_a_rel_diff_vs_fp64_refined"] = (torch.linalg.norm(g[0] - ref[0]) /
                                                              torch.linalg.norm(ref[0])).item()
    ga_err = (torch.linalg.norm(ga - ref[0]) / torch.linalg.norm(ref[0])).item()
    gf_err = (torch.linalg.norm(gf - ref[1]) / torch.linalg.norm(ref[1])).item()
    ph = {k: float(np.mean([s["t_phase_ms"][k] for s in stats])) for k in stats[0]["t_phase_ms"]}
    line = {
        "metric": "differentiated solve (forward + backward) unknowns/s",
        "value": N / dt, "unit": "unknowns/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"diff256: 2D Laplace second-kind volume IE, 256x256 grid (N={N}), a = 1 + 64 "
                               f"Gaussian bumps, 1 RHS, L = |u - u_target|^2/2, eps={eps:g}, leaf 64, FP64, "
                               f"gradients of the factored map", "N": N, "eps": eps},
        "accuracy": {"grad_a_rel_err_vs_refined": ga_err, "grad_f_rel_err_vs_refined": gf_err},
        "factor_ms": float(np.mean([s["t_factor_ms"] for s in stats])),
        "phase_ms": ph,
        "modes": modes,
        "roofline": id_roofline(stats[-1], ph),
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline_diff(128, eps)
    if quiet:
        return line
    print(json.dumps(line), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "bench.py runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    if args.workload == "diff256":
        return bench_diff(args)
    if args.workload == "batch48":
        return bench_batch(args)
    import numpy as np
    import torch

    import paper_1307_2666_amd as hif
    from workloads import workload

    wl = workload(args.workload)
    eps = args.eps if args.eps is not None else wl.eps
    dev = "cuda:0"
    torch.cuda.set_device(0)
    P = torch.tensor(wl.points(), device=dev)
    N = wl.N
    a = torch.ones(N, dtype=torch.float64, device=dev)
    Fr = torch.tensor(wl.rhs(), device=dev)
    nrhs = Fr.shape[0]

    def step():
        F = hif.factor(P, eps, wl.leaf, a=a, h=wl.h)
        U = F.solve(Fr)
        return F, U

    for _ in range(args.warmup):
        F, U = step()
        F.free()
    torch.cuda.synchronize()
    stats = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        F, U = step()
        stats.append(F.stats())
        F.free()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps

    # Separate timing of the solve alone (factors kept) and the accuracy gate.
    F, U = step()
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    U = F.solve(Fr)
    ev1.record()
    torch.cuda.synchronize()
    t_solve = ev0.elapsed_time(ev1) * 1e-3
    R = Fr - hif.matvec(P, U, a=a, h=wl.h)
    D = F.solve(R)
    err = (torch.linalg.norm(D, dim=1) / torch.linalg.norm(U + D, dim=1)).max().item()
    res = (torch.linalg.norm(R, dim=1) / torch.linalg.norm(Fr, dim=1)).max().item()
    st = F.stats()
    F.free()

    # Dominant kernel family: the pivoted QR of the IDs (blocked: k_bq_piv +
    # k_bq_cols per pivot step over all large classes, k_bq_update per block of
    # 32 reflectors; k_id for many small classes).  Every step streams the
    # trailing block, so it is bound by HBM; algorithmic bytes from the
    # realized rows, columns and ranks of every class (sub_id_bytes), time from
    # the HIP events the library records on its own stream around the launches.
    ph = {k: float(np.mean([s["t_phase_ms"][k] for s in stats])) for k in stats[0]["t_phase_ms"]}
    id_flops = float(np.sum(st["sub_id_flops"]))
    id_bytes = float(np.sum(st["sub_id_bytes"]))
    id_ms = ph["id"]
    el_flops = float(np.sum(st["sub_elim_flops"]))
    rq_flops = float(np.sum(st["sub_rowqr_flops"]))
    achieved = id_bytes / (id_ms * 1e-3) / 1e9 if id_ms > 0 else 0.0
    line = {
        "metric": "factor+solve unknowns/s at rel.err <=1e-6 vs oracle",
        "value": N / dt,
        "unit": "unknowns/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{wl.name}: 2D Laplace second-kind volume IE, {wl.n}x{wl.n} grid (N={N}), "
                               f"{nrhs} RHS, eps={eps:g}, leaf {wl.leaf}, HIF-IE with second-kind "
                               f"modification, FP64", "N": N, "nrhs": nrhs, "eps": eps, "leaf": wl.leaf},
        "accuracy": {"rel_err_est_max": err, "rel_residual_max": res, "gate_1e-6": bool(err <= 1e-6)},
        "solve_ms": t_solve * 1e3,
        "solve_unknowns_per_s": N * nrhs / t_solve,
        "factor_ms": float(np.mean([s["t_factor_ms"] for s in stats])),
        "phase_ms": ph,
        "sub_ms": [{k: round(v, 3) for k, v in d.items() if v > 0} for d in st["sub_t_ms"]],
        "top_size": st["top_size"],
        "factor_bytes": st["factor_bytes"],
        "roofline": {"kernel": "k_bq_piv + k_bq_cols + k_bq_update + k_id_reg + k_id (column-pivoted QR of "
                               "the IDs, all launches of a step)",
                     "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": (ID_STEP_TRAFFIC_BYTES if ID_STEP_TRAFFIC_BYTES and wl.name == "sq512"
                                 and abs(eps - 1e-6) < 1e-12 else None),
                     "bytes_per_step": id_bytes, "ms_per_step": id_ms,
                     "flops_per_step": id_flops,
                     "fp64_tflops": id_flops / (id_ms * 1e-3) / 1e12 if id_ms > 0 else 0.0},
        "row_compression": {"flops_per_step": rq_flops, "ms_per_step": ph["rowqr"],
                            "tflops": rq_flops / (ph["rowqr"] * 1e-3) / 1e12 if ph["rowqr"] > 0 else 0.0,
                            "fp64_peak_tflops": PEAK_FP64_VECTOR_TFLOPS},
        "elimination": {"flops_per_step": el_flops, "ms_per_step": ph["elimination"],
                        "tflops": el_flops / (ph["elimination"] * 1e-3) / 1e12 if ph["elimination"] > 0 else 0.0},
        "paper_context": {"hifie2x_512sq_eps1e-6": {"t_f_s": 470.0, "t_as_s": 1.0, "unknowns_per_s_f8": 548,
                                                    "hardware": "MATLAB R2010b, 1 core Xeon E7-4820 2.0 GHz, "
                                                                "FP64, adaptive leaf"}},
    }
    if args.calib_copy:  # 256 MiB read + 256 MiB written by one elementwise kernel
        src = torch.ones(32 << 20, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        torch.neg(src, out=dst)
        torch.cuda.synchronize()
        del src, dst
    if not args.no_refine:
        line["refinement"] = refinement(hif, P, a, Fr, wl)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(args.cpu_sample, eps)
    if not args.no_extras and wl.name == "sq512":
        # the two other workloads, briefly (their own bench lines: --workload diff256 / batch48)
        class _A:
            steps, warmup, eps, no_cpu_baseline = 2, 1, None, True
        keep = ("metric", "value", "unit", "ms_per_step", "accuracy", "modes", "one_worker_ms_per_step",
                "solve_latency_ms")
        line["other_workloads"] = {
            "diff256": {k: v for k, v in bench_diff(_A, quiet=True).items() if k in keep},
            "batch48": {k: v for k, v in bench_batch(_A, quiet=True).items() if k in keep},
        }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
