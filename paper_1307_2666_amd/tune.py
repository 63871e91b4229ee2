"""Autotuner of the launch shapes the factorization picks by problem size.

Buckets and candidates (``hif_tuning`` in ``include/hif.h``):

* ``id_reg_waves[b]``: waves per problem of the register-resident pivoted QR
  of the IDs (a wave holds 64 (b + 1) / waves rows of every column), for
  problems of at most 64, 128, 192 columns.  Timed with ``hif_id_batched`` on
  batches shaped like the factorization's IDs after row compression: square
  blocks of n_c rows and columns (the n_c x n_c R factor of the row
  compression), n_c in the upper half of the bucket, and column scales
  decaying so that about half the columns are skeletons at eps 1e-6.
* ``lu_panel_threads[b]``: threads of the register-resident LU panel for
  panels of at most 512 and 1024 rows.  Timed with ``hif_lu_batched`` on
  batches of well-conditioned n x n blocks with r = n / 2 eliminated columns
  (the redundant part of a transformed group block), n in the bucket.
* ``rowqr_update_waves`` / ``rowqr_update_kind``: the shape of the row
  compression's trailing update beside the next panel.  It competes with the
  panel factorization for the CUs, so it is timed on whole factorizations:
  ``hif_factor`` of the second-kind 2D problem on a 384 x 384 grid (eps 1e-6,
  leaf 64), the row-compression phase time of the library's own events.
* ``sweep_many_threads``: threads per record of the solve on sub-levels of many
  small records, timed by 8-RHS solves with one factorization of that
  problem (HIP events, median of 5).

Every candidate is timed with HIP events over 5 runs after a warm run, on the
same inputs (the inputs are restored before each run); the fastest median
wins.  ``python -m paper_1307_2666_amd.tune --write`` rewrites
``csrc/tuning_gfx950.h`` with the chosen table and the measured medians; the
library then needs a rebuild to use it as its built-in table.  Without
``--write`` it prints the table as JSON.
"""
from __future__ import annotations

import argparse
import json
import os

import numpy as np
import torch

from . import _binding as B

HEADER = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc", "tuning_gfx950.h")

ID_BUCKETS = [(33, 64, 4096), (97, 128, 2048), (161, 192, 1024)]  # (n_c lo, n_c hi, problems)
ID_CANDIDATES = [(4, 8, 16), (4, 8, 16), (8, 16)]
LU_BUCKETS = [(257, 512, 256), (513, 1024, 64)]  # (n lo, n hi, problems)
LU_CANDIDATES = [(256, 512, 1024), (512, 1024)]
ROWQR_CANDIDATES = [(4, 0), (8, 0), (4, 1), (8, 1), (4, 2), (8, 2)]  # (waves, kind)
ROWQR_GRID = 384
SWEEP_CANDIDATES = [64, 128, 256]


def _median_ms(run, reps=5):
    run()  # warm (and the first use of every code path)
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        run()
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    return float(np.median(ts))


def _id_batch(lo, hi, count, seed):
    rng = np.random.default_rng(seed)
    mats = []
    for _ in range(count):
        n = int(rng.integers(lo, hi + 1))
        scale = 10.0 ** (-12.0 * np.arange(n) / n)
        mats.append(np.triu(rng.standard_normal((n, n))) * scale[rng.permutation(n)])
    return mats


def _time_id(mats, tol=1e-6):
    lib = B.load_library()
    shapes = [m.shape for m in mats]
    src = torch.cat([torch.tensor(m, device="cuda").reshape(-1) for m in mats])
    work = torch.empty_like(src)
    offs, poffs, o, po = [], [], 0, 0
    for (m, n) in shapes:
        offs.append(o)
        poffs.append(po)
        o += m * n
        po += n
    dev = dict(device="cuda")
    off = torch.tensor(offs, dtype=torch.int64, **dev)
    rows = torch.tensor([s[0] for s in shapes], dtype=torch.int32, **dev)
    cols = torch.tensor([s[1] for s in shapes], dtype=torch.int32, **dev)
    tl = torch.full((len(mats),), tol, dtype=torch.float64, **dev)
    rank = torch.zeros(len(mats), dtype=torch.int32, **dev)
    perm = torch.zeros(po, dtype=torch.int32, **dev)
    poff = torch.tensor(poffs, dtype=torch.int64, **dev)
    maxc = max(s[1] for s in shapes)
    stream = B._stream()

    def run():
        work.copy_(src)
        B._check(lib.hif_id_batched(B._ptr(work), B._ptr(off), B._ptr(rows), B._ptr(cols), B._ptr(tl), len(mats),
                                    maxc, B._ptr(rank), B._ptr(perm), B._ptr(poff), None, None, stream))

    return _median_ms(run)


def _lu_batch(lo, hi, count, seed):
    rng = np.random.default_rng(seed)
    mats = []
    for _ in range(count):
        n = int(rng.integers(lo, hi + 1))
        mats.append(rng.standard_normal((n, n)) + n * np.eye(n))
    return mats


def _time_lu(mats):
    lib = B.load_library()
    ns = [m.shape[0] for m in mats]
    src = torch.cat([torch.tensor(m, device="cuda").reshape(-1) for m in mats])
    work = torch.empty_like(src)
    offs, poffs = [0], [0]
    for n in ns:
        offs.append(offs[-1] + n * n)
        poffs.append(poffs[-1] + n // 2)
    dev = dict(device="cuda")
    off = torch.tensor(offs[:-1], dtype=torch.int64, **dev)
    poff = torch.tensor(poffs[:-1], dtype=torch.int64, **dev)
    n_t = torch.tensor(ns, dtype=torch.int32, **dev)
    r_t = torch.tensor([n // 2 for n in ns], dtype=torch.int32, **dev)
    piv = torch.zeros(poffs[-1], dtype=torch.int32, **dev)
    status = torch.zeros(1, dtype=torch.int32, **dev)
    stream = B._stream()

    def run():
        work.copy_(src)
        B._check(lib.hif_lu_batched(B._ptr(work), B._ptr(off), B._ptr(n_t), B._ptr(r_t), B._ptr(piv), B._ptr(poff),
                                    len(mats), max(ns), max(ns) // 2, B._ptr(status), stream))

    return _median_ms(run)


def _time_rowqr(reps=3):
    factor = B.factor
    pts, a, h = _grid_problem()
    F = factor(pts, 1e-6, 64, a=a, h=h)  # warm
    F.free()
    ts = []
    for _ in range(reps):
        F = factor(pts, 1e-6, 64, a=a, h=h)
        ts.append(F.stats()["t_phase_ms"]["rowqr"])
        F.free()
    return float(np.median(ts))


def _grid_problem():
    n = ROWQR_GRID
    g = (torch.arange(n, dtype=torch.float64, device="cuda") + 0.5) / n
    pts = torch.stack([g.repeat(n), g.repeat_interleave(n)], dim=1).contiguous()
    return pts, torch.ones(n * n, dtype=torch.float64, device="cuda"), 1.0 / n


def _time_sweep(F, f):
    return _median_ms(lambda: F.solve(f))


def tune(seed=0):
    """Time every candidate of every bucket; returns (table, timings)."""
    base = B.tuning_get()
    table = {k: (list(v) if isinstance(v, list) else v) for k, v in base.items()}
    timings = {"id_reg_waves": [], "lu_panel_threads": []}
    for b, ((lo, hi, cnt), cands) in enumerate(zip(ID_BUCKETS, ID_CANDIDATES)):
        mats = _id_batch(lo, hi, cnt, seed + b)
        res = {}
        for w in cands:
            t = {k: (list(v) if isinstance(v, list) else v) for k, v in table.items()}
            t["id_reg_waves"][b] = w
            B.tuning_set(t)
            res[w] = _time_id(mats)
        table["id_reg_waves"][b] = min(res, key=res.get)
        timings["id_reg_waves"].append({"columns": [lo, hi], "problems": cnt, "ms": res})
    for b, ((lo, hi, cnt), cands) in enumerate(zip(LU_BUCKETS, LU_CANDIDATES)):
        mats = _lu_batch(lo, hi, cnt, seed + 10 + b)
        res = {}
        for th in cands:
            t = {k: (list(v) if isinstance(v, list) else v) for k, v in table.items()}
            t["lu_panel_threads"][b] = th
            B.tuning_set(t)
            res[th] = _time_lu(mats)
        table["lu_panel_threads"][b] = min(res, key=res.get)
        timings["lu_panel_threads"].append({"rows": [lo, hi], "problems": cnt, "ms": res})
    res = {}
    for w, lds in ROWQR_CANDIDATES:
        t = {k: (list(v) if isinstance(v, list) else v) for k, v in table.items()}
        t["rowqr_update_waves"], t["rowqr_update_kind"] = w, lds
        B.tuning_set(t)
        res[(w, lds)] = _time_rowqr()
    best = min(res, key=res.get)
    table["rowqr_update_waves"], table["rowqr_update_kind"] = best
    B.tuning_set(dict(table, rowqr_update_waves=best[0], rowqr_update_kind=best[1]))
    pts, a, h = _grid_problem()
    F = B.factor(pts, 1e-6, 64, a=a, h=h)
    f = torch.randn(8, pts.shape[0], dtype=torch.float64, device="cuda",
                    generator=torch.Generator("cuda").manual_seed(seed))
    sres = {}
    for th in SWEEP_CANDIDATES:
        t = {k: (list(v) if isinstance(v, list) else v) for k, v in table.items()}
        t["sweep_many_threads"] = th
        B.tuning_set(t)
        sres[th] = _time_sweep(F, f)
    F.free()
    table["sweep_many_threads"] = min(sres, key=sres.get)
    timings["sweep_many_threads"] = {"grid": ROWQR_GRID, "rhs": 8, "ms": sres}
    kinds = {0: "", 1: " + LDS", 2: " rows split"}
    timings["rowqr_update"] = {"grid": ROWQR_GRID, "ms": {f"{w} waves{kinds[k]}": v for (w, k), v in res.items()}}
    B.tuning_set(table)
    return table, timings


def write_header(table, timings, path=HEADER):
    lines = ["// Built-in launch shapes for gfx950 (MI355X): the table hif_tuning_get",
             "// returns until hif_tuning_set replaces it.  Written by",
             "// paper_1307_2666_amd/tune.py from timings on one MI355X; see that script for",
             "// the candidates and the problem sizes of each bucket.", "//", "// Medians (ms):"]
    for e in timings["id_reg_waves"]:
        lines.append(f"//   ID, {e['problems']} problems of {e['columns'][0]}-{e['columns'][1]} columns: " +
                     ", ".join(f"{k} waves {v:.3f}" for k, v in e["ms"].items()))
    for e in timings["lu_panel_threads"]:
        lines.append(f"//   LU, {e['problems']} blocks of {e['rows'][0]}-{e['rows'][1]} rows: " +
                     ", ".join(f"{k} threads {v:.3f}" for k, v in e["ms"].items()))
    sw = timings.get("sweep_many_threads")
    if sw:
        lines.append(f"//   8-RHS solve of a {sw['grid']} x {sw['grid']} factorization: " +
                     ", ".join(f"{k} threads {v:.3f}" for k, v in sw["ms"].items()))
    ru = timings.get("rowqr_update")
    if ru:
        lines.append(f"//   row compression of a {ru['grid']} x {ru['grid']} factorization (eps 1e-6): " +
                     ", ".join(f"{k} {v:.2f}" for k, v in ru["ms"].items()))
    lines += ["#pragma once", "",
              "// waves per problem of the register-resident pivoted QR, problems of at most",
              "// 64, 128 and 192 columns",
              "#define HIF_TUNED_ID_REG_WAVES {" + ", ".join(str(x) for x in table["id_reg_waves"]) + "}",
              "// threads of the register-resident LU panel, panels of at most 512 and 1024 rows",
              "#define HIF_TUNED_LU_PANEL_THREADS {" + ", ".join(str(x) for x in table["lu_panel_threads"]) + "}",
              "// waves (16 columns each) per workgroup of the row compression's trailing",
              "// update beside the next panel",
              f"#define HIF_TUNED_ROWQR_UPDATE_WAVES {table['rowqr_update_waves']}",
              "// 0: Y in registers, 1: the chunk reflectors staged in LDS, 2: rows split over two waves",
              f"#define HIF_TUNED_ROWQR_UPDATE_KIND {table['rowqr_update_kind']}",
              "// threads per record of the sweeps on sub-levels of at least 1024 records",
              f"#define HIF_TUNED_SWEEP_MANY_THREADS {table['sweep_many_threads']}", ""]
    with open(path, "w") as fh:
        fh.write("\n".join(lines))


def main():
    p = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    p.add_argument("--write", action="store_true", help="rewrite csrc/tuning_gfx950.h")
    p.add_argument("--out", default=None, help="also write the table and timings as JSON to this file")
    args = p.parse_args()
    table, timings = tune()
    print(json.dumps({"table": table, "timings": timings}))
    if args.out:
        with open(args.out, "w") as fh:
            json.dump({"table": table, "timings": timings}, fh)
    if args.write:
        write_header(table, timings)


if __name__ == "__main__":
    main()
