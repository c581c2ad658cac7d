"""Benchmark of the DPG per-cell local solve on one MI355X.

A step is one full local-solve pass (geometry, formation of G, B_f, l,
Jacobi-scaled blocked Cholesky, triangular solves, K_e = W^H W, l_e, eta) over
every cell of the workload, inputs already resident in HBM.  Prints one JSON
line (see the keys below).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c2]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_2609_03155_amd import workloads as W  # noqa: E402

METRIC = "DPG local-solve elements/s (B^H G^{-1} B + eta) mixed-prec vs FP64; rel err"
PEAK_FP64_TFLOPS = 78.6      # MI355X dense FP64 matrix peak
PEAK_HBM_GBS = 8000.0
STREAM_CELLS = 8192          # cells per range when the outputs are streamed


def algorithmic_flops(p: int, dp: int) -> dict:
    """Structure-aware algorithmic flop counts per cell: formation of the real
    S, M, C, D, R, T contractions, complex Cholesky of the n_v x n_v Gram
    matrix, triangular solves (half cost on the real trace columns), HERK and
    the two GEMVs (l_e, eta)."""
    s, r = p + dp + 1, p + 1
    n1 = p + dp + 2
    N = 3 * s * (s + 1) ** 2
    nv = 2 * N
    m1 = (p + 1) ** 3
    nq = n1 ** 3
    nu, nt = 6 * m1, 24 * r * r
    k = nu + nt
    return dict(form=12 * N * N * nq + 12 * N * m1 * nq + 48 * N * r * (r + 1) * n1 * n1,
                chol=4.0 / 3.0 * nv ** 3, trsm=4 * nv * nv * nu + 2 * nv * nv * nt, herk=4 * k * k * nv,
                vec=32 * nv * k)


def measured_traffic(workload: str, precision: str, kernel: str):
    """HBM bytes per launch of the dominant kernel class from the committed
    rocprofv3 counter summaries (profiles/*.md), or None when none matches or
    the kernel source has changed since the counters were taken."""
    import glob
    import hashlib
    src = os.path.join(ROOT, "paper_2609_03155_amd", "csrc", "dpg_kernels.hip")
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        kv = {}
        for line in open(path):
            line = line.strip()
            if line.startswith("traffic_") and " = " in line:
                k, v = line.split(" = ", 1)
                kv[k] = v.strip()
        if (kv.get("traffic_workload") == workload and kv.get("traffic_precision") == precision
                and kv.get("traffic_kernel") == kernel and kv.get("traffic_source_sha256_prefix") == sha):
            return float(kv["traffic_bytes_per_launch"])
    return None


def trace_system_timings(w, plan, prob, xd, K, l, eta, info, solve, stream, reps: int = 5, mv_reps: int = 50,
                         cg_iters: int = 200):
    """Condensation (A_K, b_K), gather assembly, complex CSR matvec, a fixed
    number of CG iterations (no preconditioner), the trace scatter and the
    reconstruction of the interior unknowns on the workload, timed with HIP
    events."""
    import torch
    from paper_2609_03155_amd import dpg
    solve(dpg.DPG_FP64)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ts = dpg.TraceSystem(plan, w.cells, w.face_kind)
    build_s = time.perf_counter() - t0
    print(f"[bench] trace system: {ts.n_dofs} unknowns, {ts.nnz} nonzeros, built in {build_s:.1f} s",
          file=sys.stderr, flush=True)

    def timed_ms(fn, n):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(n):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / n

    out = {}
    cond = {}

    def do_cond():
        cond["r"] = plan.condense(K, l, stream=stream)
    cond_ms = timed_ms(do_cond, reps)
    A, b, cinfo = cond["r"]
    asm = {}

    def do_asm():
        asm["r"] = ts.assemble(A, b, stream=stream)
    asm_ms = timed_ms(do_asm, reps)
    vals, rhs = asm["r"]
    x = torch.ones(ts.n_dofs, dtype=torch.complex128, device="cuda")
    y = torch.empty_like(x)
    mv_ms = timed_ms(lambda: ts.matvec(vals, x, y, stream=stream), mv_reps)
    fl = 0.0
    contrib = 0
    for p in sorted(set(int(v) for v in w.degree)):
        cnt = int(np.sum(w.degree == p))
        nu, nt = 6 * (p + 1) ** 3, 24 * (p + 1) ** 2
        fl += cnt * (4.0 / 3.0 * nu ** 3 + 4.0 * nu * nu * nt + 4.0 * nt * nt * nu)
        contrib += cnt * nt * nt
    mv_bytes = ts.nnz * (16 + 4) + (ts.n_dofs + 1) * 8 + 2 * ts.n_dofs * 16
    # CG: cg_iters iterations from zero (tolerance 0, so all of them run)
    t = torch.zeros(ts.n_dofs, dtype=torch.complex128, device="cuda")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    cg_it, cg_rr = ts.solve(vals, rhs, t, 0.0, cg_iters, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    cg_ms = e0.elapsed_time(e1) / max(cg_it, 1)
    # the true residual of the last iterate, against the recursively updated one
    ts.matvec(vals, t, y, stream=stream)
    torch.cuda.synchronize()
    cg_true = float(torch.linalg.vector_norm(rhs[:ts.n_dofs] - y[:ts.n_dofs]) / torch.linalg.vector_norm(rhs[:ts.n_dofs]))
    # per iteration: the matvec, x, p, r, q read and x, r written by the update, r, p read and p written
    cg_bytes = mv_bytes + 9 * 16 * ts.n_dofs
    tl = ts.scatter(t, stream=stream)
    rec_out = {}

    def do_rec():
        rec_out["r"] = plan.reconstruct(K, l, tl, stream=stream)
    rec_ms = timed_ms(do_rec, reps)
    rinfo = rec_out["r"][1]
    # power dissipation of the reconstructed fields
    xr = rec_out["r"][0]
    pw = {}

    def do_pw():
        pw["r"] = plan.power_dissipation(prob, xr, stream=stream)
    pw_ms = timed_ms(do_pw, reps)
    # Doerfler marking of the workload's eta (sort, scans, flags; synchronous, allocates)
    ev = eta[:w.n_cells].contiguous()
    dpg.dorfler_mark(ev, stream=stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        dpg.dorfler_mark(ev, stream=stream)
    mark_ms = (time.perf_counter() - t0) / reps * 1e3
    rfl = 0.0
    for p in sorted(set(int(v) for v in w.degree)):
        cnt = int(np.sum(w.degree == p))
        nu, nt = 6 * (p + 1) ** 3, 24 * (p + 1) ** 2
        rfl += cnt * (4.0 / 3.0 * nu ** 3 + 8.0 * nu * nt + 8.0 * nu * nu)
    out.update({
        "n_dofs": ts.n_dofs, "nnz": ts.nnz, "build_s": build_s,
        "condense_ms": cond_ms, "condense_tflops": fl / (cond_ms * 1e-3) / 1e12,
        "condense_failed_cells": int(np.sum(cinfo.cpu().numpy()[:w.n_cells] != 0)),
        "assemble_ms": asm_ms,
        "assemble_GBps": (contrib * 24 + ts.nnz * 24) / (asm_ms * 1e-3) / 1e9,
        "spmv_ms": mv_ms, "spmv_nnz_per_s": ts.nnz / (mv_ms * 1e-3),
        "spmv_GBps": mv_bytes / (mv_ms * 1e-3) / 1e9,
        "spmv_frac_hbm": mv_bytes / (mv_ms * 1e-3) / 1e9 / PEAK_HBM_GBS,
        "spmv_bytes_note": "algorithmic: 16 B value + 4 B column per nonzero, row pointers, x and y once",
        "cg_iterations": cg_it, "cg_relres": cg_rr, "cg_true_relres": cg_true, "cg_ms_per_iteration": cg_ms,
        "cg_GBps": cg_bytes / (cg_ms * 1e-3) / 1e9,
        "cg_frac_hbm": cg_bytes / (cg_ms * 1e-3) / 1e9 / PEAK_HBM_GBS,
        "cg_bytes_note": "per iteration: the matvec's algorithmic bytes plus 9 complex vectors of n (update, direction)",
        "reconstruct_ms": rec_ms, "reconstruct_tflops": rfl / (rec_ms * 1e-3) / 1e12,
        "reconstruct_failed_cells": int(np.sum(rinfo.cpu().numpy()[:w.n_cells] != 0)),
        "dorfler_mark_ms": mark_ms,
        "power_dissipation_ms": pw_ms,
    })
    ts.close()
    del A, b, vals, rhs, t, tl, rec_out, pw, xr
    return out


def cpu_baseline(w, budget_s: float = 20.0):
    """The oracle, as it stands, on a bounded seeded sample of the workload's
    cells; returns (record, per-cell oracle outputs)."""
    from oracle import dpg_oracle as O
    try:
        from threadpoolctl import threadpool_info
        cores = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    except Exception:
        cores = os.cpu_count() or 1
    om = O.omega_dimensionless(w.freq_hz)
    pt = w.port
    pm = O.PortMode(pt["a"], pt["b"], pt["m"], pt["n"], om, pt["eps"], pt["mu"])
    x, off = W.random_coefficients(w)
    rng = np.random.default_rng(W.SEED_BASE + 77)
    order = rng.permutation(w.n_cells)
    outs = {}
    t0 = time.perf_counter()
    for c in order:
        c = int(c)
        cp = O.CellProblem(X=w.cell_vertices(c), p=int(w.degree[c]), dp=w.dp, eps=complex(w.eps[c]),
                           mu=complex(w.mu[c]), omega=om, face_kind=tuple(int(k) for k in w.face_kind[c]),
                           zinv=tuple(complex(z) for z in w.zinv[c]), port=pm)
        G, Bf, l = O.cell_forms(cp)
        K, le, eta = O.local_solve(G, Bf, l, x[off[c]:off[c + 1]])
        outs[c] = (K, le, eta)
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    rec = {"value": len(outs) / dt, "unit": "elements/s", "cores": int(cores), "kind": "oracle",
           "sample": f"{len(outs)} seeded cells of {w.name} ({dt:.1f} s, numpy/LAPACK FP64, LU solves)"}
    return rec, outs


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c2", choices=["c1", "c2", "c3", "c4", "c5"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--precision", default="both", choices=["both", "fp64", "split"])
    ap.add_argument("--copy-calib-mib", type=int, default=0,
                    help="run one device-to-device copy of this many MiB first (calibrates HBM byte counters)")
    ap.add_argument("--no-graph", action="store_true", help="time eager solves instead of HIP-graph replays")
    ap.add_argument("--no-autotune", action="store_true", help="skip the batching autotuner")
    ap.add_argument("--sequential", action="store_true", help="degree groups one after the other (no branches)")
    ap.add_argument("--no-trace-system", action="store_true",
                    help="skip the condensation / assembly / CSR matvec measurement")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (requested --gpus {args.gpus}); the per-cell local solve needs no "
              "communication: each GPU would run the same plan on its own contiguous, cost-balanced share of the cells.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2609_03155_amd import dpg

    w = W.CONFIGS[int(args.workload[1])]()
    x, off = W.random_coefficients(w)
    plan = dpg.Plan(w.degree, w.dp)
    prob = dpg.DeviceProblem.from_workload(w)
    xd = torch.from_numpy(x).cuda()
    stream = torch.cuda.current_stream()
    # Outputs that do not fit in 80% of the memory left after the plan's
    # workspace are streamed: the step solves consecutive ranges of
    # STREAM_CELLS cells into one reused output buffer (eta and info for all
    # cells stay resident).
    free_b, _ = torch.cuda.mem_get_info()
    streaming = int(plan.K_off[-1]) * 16 > 0.8 * free_b
    if streaming:
        ranges = [(a, min(STREAM_CELLS, w.n_cells - a)) for a in range(0, w.n_cells, STREAM_CELLS)]
        nK = max(plan.range_sizes(a, n)[0] for a, n in ranges)
        nv = max(plan.range_sizes(a, n)[1] for a, n in ranges)
        K = torch.empty(nK, dtype=torch.complex128, device="cuda")
        l = torch.empty(nv, dtype=torch.complex128, device="cuda")
        eta = torch.empty(w.n_cells, dtype=torch.float64, device="cuda")
        info = torch.empty(w.n_cells, dtype=torch.int32, device="cuda")
        args.no_graph = True
        args.no_autotune = True
    else:
        K, l, eta, info = plan.alloc_outputs()

    def solve(precision):
        if not streaming:
            plan.local_solve(prob, xd, K, l, eta, info, precision=precision, stream=stream)
            return
        for a, n in ranges:
            plan.local_solve_range(prob, a, n, xd[int(off[a]):], K, l, eta[a:], info[a:], precision=precision,
                                   stream=stream)

    if args.copy_calib_mib > 0:
        n = args.copy_calib_mib * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.sequential:
        plan.set_concurrency(False)

    def timed(precision):
        """(ms per step, per-class kernel profile of eager steps, outputs, replay stats)."""
        if not args.no_autotune:
            t_at = plan.autotune(prob, xd, K, l, eta, info, precision=precision, stream=stream)
            print(f"[bench] precision {precision}: autotuned, solve {t_at:.1f} ms", file=sys.stderr, flush=True)
        # eager steps with per-launch HIP events: kernel classes and the roofline
        for _ in range(args.warmup):
            solve(precision)
        torch.cuda.synchronize()
        plan.profile()                       # discard
        # per-launch durations are taken on the sequential schedule, where
        # kernels of different degree groups do not share the device
        conc = plan.tuning(int(w.degree[0]))[1]
        plan.set_concurrency(False)
        plan.set_profiling(True)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(args.steps):
            solve(precision)
        e1.record(stream)
        torch.cuda.synchronize()
        plan.set_profiling(False)
        plan.set_concurrency(conc)
        eager_ms = e0.elapsed_time(e1) / args.steps
        prof = plan.profile()
        print(f"[bench] precision {precision}: eager {eager_ms:.1f} ms/step", file=sys.stderr, flush=True)
        rep = None
        ms = eager_ms
        if not args.no_graph:
            # the headline: K replays of the captured solve, bracketed by synchronisation
            g = plan.graph(prob, xd, K, l, eta, info, precision)
            for _ in range(args.warmup):
                g.launch(stream)
            torch.cuda.synchronize()
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
            ev[0].record(stream)
            for k in range(args.steps):
                g.launch(stream)
                ev[k + 1].record(stream)
            torch.cuda.synchronize()
            per = [ev[k].elapsed_time(ev[k + 1]) for k in range(args.steps)]
            ms = ev[0].elapsed_time(ev[-1]) / args.steps
            rep = {"median_ms": float(np.median(per)), "min_ms": float(np.min(per)), "max_ms": float(np.max(per)),
                   "eager_ms_per_step": eager_ms}
            g.close()
        return ms, prof, precision, rep

    def cell_outputs(precision, c):
        """(K_e, l_e, eta) of cell c from the last solve, or from a one-cell range solve when streaming."""
        k = int(off[c + 1] - off[c])
        if not streaming:
            Kc = K[int(plan.K_off[c]):int(plan.K_off[c + 1])].cpu().numpy().reshape(k, k).T
            return Kc, l[int(off[c]):int(off[c + 1])].cpu().numpy(), float(eta[c])
        Kc = torch.empty(k * k, dtype=torch.complex128, device="cuda")
        lc = torch.empty(k, dtype=torch.complex128, device="cuda")
        ec = torch.empty(1, dtype=torch.float64, device="cuda")
        ic = torch.empty(1, dtype=torch.int32, device="cuda")
        plan.local_solve_range(prob, c, 1, xd[int(off[c]):], Kc, lc, ec, ic, precision=precision, stream=stream)
        torch.cuda.synchronize()
        return Kc.cpu().numpy().reshape(k, k).T, lc.cpu().numpy(), float(ec[0])

    precisions = {"fp64": dpg.DPG_FP64, "split": dpg.DPG_SPLIT_FP32}
    if args.precision != "both":
        precisions = {args.precision: precisions[args.precision]}
    runs = {name: timed(code) for name, code in precisions.items()}
    head = "split" if "split" in runs else "fp64"
    ms_step, prof, _, _ = runs[head]
    info_h = info.cpu().numpy()
    value = w.n_cells / (ms_step * 1e-3)

    # roofline of the dominant kernel class, from the live per-launch event timings
    fl = {}
    for p in sorted(set(int(v) for v in w.degree)):
        cnt = int(np.sum(w.degree == p))
        for key, v in algorithmic_flops(p, w.dp).items():
            fl[key] = fl.get(key, 0.0) + v * cnt
    form_keys = ("scale", "form_SM", "form_IF", "form_pad", "form_B", "form_load")
    classes = {k: v for k, v in prof.items() if v[1] > 0}
    dominant = max(classes, key=lambda k: classes[k][0])
    dom_key = dominant
    if dominant in ("chol_diag", "chol_panel"):
        dom_key = "chol_diag+chol_panel"
        dom_name = "chol_diag+chol_panel (blocked Cholesky + TRSM sweep, FP64)"
        dom_flops = (fl["chol"] + fl["trsm"]) * args.steps
        dom_ms = prof["chol_diag"][0] + prof["chol_panel"][0]
        dom_launches = prof["chol_diag"][1] + prof["chol_panel"][1]
    elif dominant == "herk":
        dom_name = "herk (K_e = W^H W, l_e)"
        dom_flops = (fl["herk"] + fl["vec"]) * args.steps
        dom_ms, dom_launches = prof["herk"]
    else:
        dom_name = "formation"
        dom_flops = fl["form"] * args.steps
        dom_ms = sum(prof[k][0] for k in form_keys)
        dom_launches = sum(prof[k][1] for k in form_keys)
    achieved = dom_flops / (dom_ms * 1e-3) / 1e12
    total_alg = sum(fl.values())
    rec = {
        "metric": METRIC, "value": value, "unit": "elements/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64+bf16x3" if head == "split" else "f64", "data": "synthetic",
        "config": {"workload": w.name, "cells": w.n_cells, "degrees": sorted(set(int(v) for v in w.degree)),
                   "dp": w.dp, "freq_hz": w.freq_hz, "precision": head, "parallelism": "single-gpu"},
        "roofline": {"bound": "mfma", "kernel": dom_name, "achieved": achieved, "peak": PEAK_FP64_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_TFLOPS,
                     "traffic": measured_traffic(w.name, head, dom_key), "traffic_unit": "HBM bytes per launch",
                     "launches_per_step": dom_launches / args.steps,
                     "avg_launch_ms": dom_ms / max(1, dom_launches)},
        "whole_step_tflops": total_alg / (ms_step * 1e-3) / 1e12,
        "kernel_ms_per_step": {k: v[0] / args.steps for k, v in prof.items() if v[1]},
        "failed_cells": int(np.sum(info_h != 0)),
    }
    for name, (ms_n, prof_n, _, rep_n) in runs.items():
        rec[f"{name}_path"] = {"value": w.n_cells / (ms_n * 1e-3), "ms_per_step": ms_n,
                               "kernel_ms_per_step": {k: v[0] / args.steps for k, v in prof_n.items() if v[1]}}
        if rep_n:
            rec[f"{name}_path"]["graph_replays"] = rep_n
    degs = sorted(set(int(v) for v in w.degree))
    rec["batching"] = {"timed": "eager" if args.no_graph else "hip-graph replays",
                       "concurrent_degree_branches": plan.tuning(degs[0])[1],
                       "cells_per_launch": {str(p): plan.tuning(p)[0] for p in degs}}
    if "split" in runs and "fp64" in runs:
        rec["speedup_split_vs_fp64"] = runs["fp64"][0] / runs["split"][0]
    if not args.no_trace_system and not streaming:
        rec["trace_system"] = trace_system_timings(w, plan, prob, xd, K, l, eta, info, solve, stream)
    if not args.no_cpu_baseline:
        base, outs = cpu_baseline(w, args.cpu_budget)
        rec["cpu_baseline"] = base
        errs = {}
        for name, (_, _, code, _) in runs.items():
            eK, el, ee = [], [], []
            if not streaming:
                solve(code)                  # outputs of this precision
                torch.cuda.synchronize()
            for c, (Ko, lo, eo) in outs.items():
                Kg, lg, eg = cell_outputs(code, c)
                eK.append(np.linalg.norm(Kg - Ko) / np.linalg.norm(Ko))
                if np.linalg.norm(lo) > 0:
                    el.append(np.linalg.norm(lg - lo) / np.linalg.norm(lo))
                ee.append(abs(eg - eo) / eo)
            errs[name] = {"cells": len(outs), "K_e_max": float(np.max(eK)), "K_e_median": float(np.median(eK)),
                          "l_e_max": float(np.max(el)) if el else None, "l_e_cells": len(el),
                          "eta_max": float(np.max(ee))}
        rec["rel_err_vs_oracle"] = errs
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
