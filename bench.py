"""Benchmark: HIF-IE factor + solve throughput on one MI355X.

Workload (the 512 x 512 configuration): 2D second-kind Laplace volume IE on
the unit square, uniform 512 x 512 cell-centred grid (N = 262144, h = 1/512),
a = b = c = 1 (K_ij = -log|x_i - x_j| h^2 / (2 pi), closed-form diagonal),
eps = 1e-6, leaf boxes of 64 points, 8 standard-normal right-hand sides,
FP64 with the second-kind modification.  One step = hif_factor + hif_solve of
all 8 right-hand sides (+ releasing the factors); inputs are resident in HBM
before the timed region starts.

Printed: one JSON line with
* the metric (unknowns/s = N / step time);
* accuracy of the step's solution through the library's own exact operator
  (relative residual with the pair-by-pair matvec, and the forward error
  estimated by one refinement step); the element-by-element parity with the
  CPU oracle (sampled oracle rows at this size) is the job of the tests;
* e_a ~ |A - F| / |A| and e_s ~ |I - A F^{-1}| by power iteration as in
  Section 5 of the paper (uniform random start, 1e-2 relative change), with
  the library's apply / solve sweeps and its exact operator;
* ``roofline``: the dominant step, the interpolative decompositions (row
  compression + column-pivoted QR), against the FP64 ALU peak, from the
  phase times the library measures with HIP events on its own stream;
  ``phases``: the same for every phase with its own bound;
* the FP64 vs FP32-mixed comparison with GMRES refinement to a true residual
  of 1e-10, with the exact pair-by-pair operator (and, labelled apart, with
  the FFT form of the same operator);
* ``cpu_baseline``: the CPU oracle on a bounded sample of the workload.

``--workload batch48`` times 48 independent problems of uneven sizes (sides 64 to
256, 4 right-hand sides each); ``--workload diff256`` the differentiated solve
(256 x 256 grid, a = 1 + 64 Gaussian bumps, L = |u - u_target|^2 / 2; one
step = forward (factor + solve) + backward (adjoint solve + dL/da, dL/df)).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published peaks: FP64 vector and FP64 matrix 78.6 TFLOP/s
# (256 CUs x 128 FP64 flop/clk x 2.4 GHz), FP32 matrix 157.3 TFLOP/s, HBM3E
# 8 TB/s.
PEAK_FP64_TFLOPS = 78.6
PEAK_FP32_MFMA_TFLOPS = 157.3
HBM_PEAK_GBS = 8000.0
# HBM bytes per factorization moved by the kernels of the IDs on this
# workload (row compression and pivoted QR), from rocprofv3 FETCH_SIZE and
# WRITE_SIZE runs scaled by what the counters read for a 256 MiB copy kernel
# (see the profile summaries); None until taken for the kernels as they stand.
# 267 GB read + 73 GB written per factorization (profiles/hbm_traffic_id_sq512.md).
ID_STEP_TRAFFIC_BYTES = 340.50e9
# ALU roof of the exact pair-by-pair product (2D, 8 right-hand sides, two
# targets per thread): its inner loop issues 110 vector instructions per
# source for two targets, 55 per pair (log, distance, select, 8 FMAs); a
# wave64 vector instruction takes 4 cycles of a 16-lane SIMD, so the chip
# issues 256 CUs x 64 lanes x 2.4 GHz lane-operations per second.
MATVEC_VALU_PER_PAIR = 55
VALU_LANE_OPS_PER_S = 256 * 64 * 2.4e9


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=3)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--workload", default="sq512")
    p.add_argument("--eps", type=float, default=None)
    p.add_argument("--precision", choices=("fp64", "fp32_mixed"), default="fp64",
                   help="precision of the timed factorization (fp32_mixed: FP32 entries and matrix-core GEMMs)")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-sample", type=int, default=256, help="grid side of the oracle's sample (2D)")
    p.add_argument("--calib-copy", action="store_true",
                   help="after the timed region, run one plain 256 MiB device copy kernel (scale for HBM counters)")
    p.add_argument("--no-refine", action="store_true",
                   help="skip the FP64 vs FP32-mixed comparison with GMRES refinement")
    p.add_argument("--no-errors", action="store_true", help="skip the power-iteration estimates of e_a, e_s")
    p.add_argument("--no-extras", action="store_true",
                   help="skip the short runs of the differentiated-solve and batch workloads")
    return p.parse_args()


def host_info():
    """CPU model, core count and BLAS library of this host (for the CPU baseline)."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    blas = []
    try:
        from threadpoolctl import threadpool_info

        blas = [{k: d.get(k) for k in ("internal_api", "version", "num_threads")} for d in threadpool_info()
                if d.get("user_api") == "blas"]
    except Exception:
        pass
    return {"cpu_model": model, "os_cpu_count": os.cpu_count(), "blas": blas}


def cpu_baseline(n: int, eps: float):
    """The oracle as it stands (FP64 NumPy/SciPy), factor + solve of 8 right-hand sides on an
    n x n sample of the workload, plus the 64 x 64 case (the setting closest to the paper's
    single-core timings).  One BLAS thread: the oracle works on blocks of tens to a few
    hundred rows, where BLAS threads cost more than they save (128 x 128: 8.9 s on one
    thread, 49 s on eight, in the build container)."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle.factor import factorize
    from oracle.kernels import Operator
    from workloads import grid_points, rhs

    def run(side):
        pts = grid_points(side, 2)
        N = pts.shape[0]
        op = Operator.uniform(pts, 1.0 / side, a=np.ones(N))
        F8 = rhs(N, 8, 1)
        t0 = time.perf_counter()
        F = factorize(op, eps, 64)
        F.solve(F8)
        return N, time.perf_counter() - t0

    with threadpool_limits(1):
        N, dt = run(n)
        N1, dt1 = run(64)
    return {"value": N / dt, "unit": "unknowns/s", "cores": 1, "kind": "oracle",
            "sample": f"oracle hifie2x factor + 8-RHS solve of the {n}x{n} grid (N={N}; same kernel, leaf 64, "
                      f"eps {eps:g}), {dt:.1f} s on 1 host core (1 BLAS thread)",
            "sample_64x64": {"value": N1 / dt1, "seconds": dt1},
            "host": host_info()}


def power_errors(hif_F, N, seed=0, rtol=1e-2, maxit=60):
    """e_a ~ |A - F| / |A| and e_s ~ |I - A F^{-1}| by power iteration (Section 5): uniform
    random start, stop at a relative change below rtol; A is the handle's exact operator
    (pair by pair), F and F^{-1} the factored sweeps.  Returns (e_a, e_s, products used)."""
    import torch

    gen = torch.Generator().manual_seed(seed)
    count = [0]

    def A(x, T=False):
        count[0] += 1
        return hif_F.apply_A(x, transpose=T)[0]

    def norm2(op, opT):
        v = torch.rand(N, generator=gen, dtype=torch.float64).cuda()
        v /= torch.linalg.norm(v)
        est = 0.0
        for _ in range(maxit):
            w = opT(op(v))
            nw = torch.linalg.norm(w).item()
            if nw == 0.0:
                return 0.0
            new = nw ** 0.5
            v = w / nw
            if est > 0.0 and abs(new - est) <= rtol * new:
                return new
            est = new
        return est

    num = norm2(lambda x: A(x) - hif_F.apply(x), lambda y: A(y, True) - hif_F.apply_T(y))
    den = norm2(lambda x: A(x), lambda y: A(y, True))
    es = norm2(lambda x: x - A(hif_F.solve(x)), lambda y: y - hif_F.solve_T(A(y, True)))
    return num / den, es, count[0]


def refinement(hif, P, a, Fr, wl, fft, tol=1e-10):
    """FP64 vs FP32-mixed factorization as GMRES preconditioner, to a true relative
    residual of ``tol`` against the exact FP64 operator (hif_gmres), applied pair by pair
    (``fft`` False) or by FFT convolution on the uniform grid.  Total time = factor +
    GMRES (each iteration one solve and one product with A, plus the final residual
    check), best over eps in {1e-3, 1e-6} for each precision; one warm run per
    configuration, the second one timed."""
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
                F = hif.factor(P, e, wl.leaf, a=a, h=wl.h, precision=prec, second_kind=sk,
                               fft_matvec=1 if fft else 0)
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
    return {"operator": "fft convolution" if fft else "pair by pair (exact on-the-fly matvec)",
            "target_residual": tol, "runs": runs, "best": best, "mixed_vs_fp64_speedup": speedup}


def id_flops_ms(st, ph):
    import numpy as np

    return float(np.sum(st["sub_id_flops"])), ph["id"] + ph["rowqr"]


def id_roofline(st, ph, traffic=None):
    """Roofline entry of the interpolative decompositions (row compression + pivoted QR):
    algorithmic flops of the ID (Householder QR to rank k, 4 m n k - 2 k^2 (m + n) + 4 k^3 / 3,
    plus k^2 r for T) over the time of both phases, against the FP64 peak."""
    fl, ms = id_flops_ms(st, ph)
    achieved = fl / (ms * 1e-3) / 1e12 if ms > 0 else 0.0
    return {"kernel": "interpolative decompositions: row compression (k_tsqr_*) + column-pivoted QR "
                      "(k_bq_*, k_id_reg, k_id, k_idm_T_block), all launches of a step",
            "bound": "alu", "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP64_TFLOPS, "traffic": traffic, "flops_per_step": fl, "ms_per_step": ms}


def phase_rooflines(st, ph, solve_ms, nrhs, mv_ms, mv_rhs):
    """Per-phase rooflines: the algorithmic work of each phase (from the realized group
    sizes and ranks) over its time, against the bound of that phase."""
    import numpy as np

    out = {}
    fl, ms = id_flops_ms(st, ph)
    out["id (a4)"] = {"bound": "alu FP64", "work": fl, "unit": "flop", "ms": ms,
                      "achieved": fl / ms * 1e-9, "peak": PEAK_FP64_TFLOPS, "achieved_unit": "TFLOP/s"}
    el = float(np.sum(st["sub_elim_flops"]))
    out["elimination (a6)"] = {"bound": "mfma FP64", "work": el, "unit": "flop", "ms": ph["elimination"],
                               "achieved": el / ph["elimination"] * 1e-9, "peak": PEAK_FP64_TFLOPS,
                               "achieved_unit": "TFLOP/s"}
    top = float(st["top_size"])
    tf = 2.0 / 3.0 * top ** 3
    out["top LU (a8)"] = {"bound": "mfma FP64", "work": tf, "unit": "flop", "ms": ph["top"],
                          "achieved": tf / ph["top"] * 1e-9 if ph["top"] > 0 else 0.0, "peak": PEAK_FP64_TFLOPS,
                          "achieved_unit": "TFLOP/s"}
    # sweeps: the stored factors once, plus gathering and scattering every
    # record's entries of all right-hand sides (2 (k + r) doubles per record
    # and right-hand side; sum of k + r over a sub-level <= its active DOFs)
    vec = 8.0 * nrhs * 2.0 * (float(np.sum(st["sub_active"])) + top)
    sb = float(st["factor_bytes"]) + vec
    out["solve (a10)"] = {"bound": "hbm", "work": sb, "unit": "byte", "ms": solve_ms,
                          "achieved": sb / solve_ms * 1e-6, "peak": HBM_PEAK_GBS, "achieved_unit": "GB/s"}
    pairs = float(st["n"]) ** 2 * mv_rhs
    out["matvec (a11)"] = {"bound": "alu (log per pair)", "work": pairs, "unit": "pair x rhs", "ms": mv_ms,
                           "achieved": pairs / mv_ms * 1e-6, "achieved_unit": "Gpair/s"}
    if mv_rhs == 8 and st.get("dim", 2) == 2:
        out["matvec (a11)"]["peak"] = VALU_LANE_OPS_PER_S / MATVEC_VALU_PER_PAIR * mv_rhs * 1e-9
    for v in out.values():
        if "peak" in v:
            v["frac"] = v["achieved"] / v["peak"]
    return out


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
    """48 independent problems: one step = the level-synchronous batch factorization
    (hif_factor_batch, nworkers = 0: every sub-level one launch sequence over all
    problems) + every problem's 4-RHS solve.  Per-solve latency p50 / p99 from replays
    of graph-captured solves (hif_solve_graph) and from eager solves; the factorization
    on 4 concurrent worker threads for comparison."""
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

    def factor(nworkers=0):
        facs, st = hif.factor_batch(dp, nworkers=nworkers)
        if any(x != 0 for x in st):
            raise RuntimeError(f"batch factorization failed: {st}")
        return facs

    def step(nworkers=0):
        facs = factor(nworkers)
        return facs, [F.solve(f) for F, f in zip(facs, fs)]

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
        stats.append(facs[0].stats())
        for F in facs:
            F.free()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    # the same factorizations on 4 concurrent worker threads, for comparison
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    facs4 = factor(4)
    torch.cuda.synchronize()
    dt4 = time.perf_counter() - t1
    for F in facs4:
        F.free()
    # per-solve latency: eager solves, and replays of graph-captured solves
    facs, us = step()
    torch.cuda.synchronize()
    err = 0.0
    for F, u, f in zip(facs, us, fs):
        y, _ = F.apply_A(u)
        err = max(err, (torch.linalg.norm(y - f, dim=1) / torch.linalg.norm(f, dim=1)).max().item())

    def latencies(run):
        out = []
        for i in range(len(facs)):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            run(i)
            e1.record()
            out.append((e0, e1))
        torch.cuda.synchronize()
        return np.array([a.elapsed_time(b) for a, b in out])

    outs = [torch.empty_like(f) for f in fs]
    graphs = [F.solve_graph(f, o) for F, f, o in zip(facs, fs, outs)]
    for g in graphs:  # one warm replay each
        g.launch()
    lat_eager = np.concatenate([latencies(lambda i: facs[i].solve(fs[i], out=outs[i])) for _ in range(3)])
    lat_graph = np.concatenate([latencies(lambda i: graphs[i].launch()) for _ in range(3)])
    same = all(torch.equal(o, u) for o, u in zip(outs, us))
    for g in graphs:
        g.free()
    for F in facs:
        F.free()
    ph = stats[-1]["t_phase_ms"]  # phase times of the whole batch

    def pct(x):
        return {"p50": float(np.percentile(x, 50)), "p99": float(np.percentile(x, 99)), "max": float(x.max())}

    line = {
        "metric": "batch factor+solve unknowns/s (48 uneven problems)",
        "value": Ntot / dt, "unit": "unknowns/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"batch48: 48 independent 2D second-kind Laplace volume IEs, sides from "
                               f"{{64, 96, 128, 192, 256}} (N total {Ntot}), a = 1 + scaled Gaussian bumps, "
                               f"4 RHS each, eps 1e-6, leaves 36 or 64 points, FP64; level-synchronous "
                               f"hif_factor_batch, then every 4-RHS solve", "N_total": Ntot, "problems": 48},
        "accuracy": {"rel_residual_max": err, "graph_replay_equals_eager": bool(same)},
        "factor_ms_4_worker_threads": dt4 * 1e3,
        "solve_latency_ms": {"graph_replay": pct(lat_graph), "eager": pct(lat_eager)},
        "phase_ms": ph,
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
    mixed = args.precision == "fp32_mixed"
    prec = hif.HIF_FP32_MIXED if mixed else hif.HIF_FP64

    def step():
        F = hif.factor(P, eps, wl.leaf, a=a, h=wl.h, precision=prec)
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

    # Separate timings of the solve alone (factors kept) and of one exact
    # product with A, on the stream the library launches on (torch's current
    # stream), then the accuracy of the solution through the exact operator.
    F, U = step()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    ev[0].record()
    U = F.solve(Fr)
    ev[1].record()
    AU = hif.matvec(P, U, a=a, h=wl.h)
    ev[2].record()
    torch.cuda.synchronize()
    solve_ms = ev[0].elapsed_time(ev[1])
    mv_ms = ev[1].elapsed_time(ev[2])
    R = Fr - AU
    D = F.solve(R)
    err = (torch.linalg.norm(D, dim=1) / torch.linalg.norm(U + D, dim=1)).max().item()
    res = (torch.linalg.norm(R, dim=1) / torch.linalg.norm(Fr, dim=1)).max().item()
    st = F.stats()
    errors = None
    if not args.no_errors:
        t1 = time.perf_counter()
        ea, es, nprod = power_errors(F, N, seed=0)
        errors = {"e_a": ea, "e_s": es, "products_with_A": nprod, "seconds": time.perf_counter() - t1,
                  "method": "power iteration, uniform random start, 1e-2 relative change (Section 5); A pair "
                            "by pair, F by the factored sweeps"}
    F.free()

    ph = {k: float(np.mean([s["t_phase_ms"][k] for s in stats])) for k in stats[0]["t_phase_ms"]}
    line = {
        "metric": "factor+solve unknowns/s at rel.err \u22641e-6 vs oracle; FP32-mixed vs FP64 speedup",
        "value": N / dt,
        "unit": "unknowns/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32/f64" if mixed else "f64",
        "data": "synthetic",
        "config": {"workload": f"{wl.name}: {wl.d}D Laplace second-kind volume IE, "
                               f"{'x'.join([str(wl.n)] * wl.d)} grid (N={N}), "
                               f"{nrhs} RHS, eps={eps:g}, leaf {wl.leaf}, " +
                               ("HIF-IE without the second-kind modification, FP32 entries and matrix-core "
                                "GEMMs, FP64 IDs, LU and sweeps" if mixed else
                                "HIF-IE with second-kind modification, FP64"),
                   "N": N, "nrhs": nrhs, "eps": eps, "leaf": wl.leaf, "precision": args.precision},
        "accuracy": {"rel_residual_max": res, "rel_err_est_max": err, "gate_1e-6": bool(err <= 1e-6 and res <= 1e-6),
                     "how": "residual f - A u with the exact pair-by-pair operator; error by one refinement "
                            "step F^{-1}(f - A u); oracle parity at this size is checked by the tests"},
        "errors_section5": errors,
        "solve_ms": solve_ms,
        "solve_unknowns_per_s": N * nrhs / (solve_ms * 1e-3),
        "matvec_ms": mv_ms,
        "factor_ms": float(np.mean([s["t_factor_ms"] for s in stats])),
        "phase_ms": ph,
        "sub_ms": [{k: round(v, 3) for k, v in d.items() if v > 0} for d in st["sub_t_ms"]],
        "top_size": st["top_size"],
        "factor_bytes": st["factor_bytes"],
        "roofline": id_roofline(st, ph, ID_STEP_TRAFFIC_BYTES if wl.name == "sq512" and abs(eps - 1e-6) < 1e-12
                                else None),
        "phases": phase_rooflines(st, ph, solve_ms, nrhs, mv_ms, nrhs),
        "paper_context": {"hifie2x_512sq_eps1e-6": {"t_f_s": 470.0, "t_as_s": 1.0, "unknowns_per_s_f8": 548,
                                                    "e_a": 5.9e-7, "e_s": 6.7e-7,
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
        line["refinement"] = refinement(hif, P, a, Fr, wl, fft=False)
        line["refinement_fft_operator"] = refinement(hif, P, a, Fr, wl, fft=True)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(args.cpu_sample, eps)
    if not args.no_extras and wl.name == "sq512":
        # the two other workloads, briefly (their own bench lines: --workload diff256 / batch48)
        class _A:
            steps, warmup, eps, no_cpu_baseline = 2, 1, None, True
        keep = ("metric", "value", "unit", "ms_per_step", "accuracy", "modes", "factor_ms_4_worker_threads",
                "solve_latency_ms")
        line["other_workloads"] = {
            "diff256": {k: v for k, v in bench_diff(_A, quiet=True).items() if k in keep},
            "batch48": {k: v for k, v in bench_batch(_A, quiet=True).items() if k in keep},
        }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
