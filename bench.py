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


def formation_flops_sf(p: int, dp: int) -> float:
    """Flops per cell of the sum-factorised formation as the kernels compute
    it (k_form_SM: per component pair a >= b and (i2, j2) block, the q2 pass
    over five terms, the q1 pass and the (term, q0) GEMM; k_form_Bsf: the
    same per (a, c) with three terms and the DG factors on the trial side;
    G_IF from its tables, 8 flops per complex entry).  Lower triangles only,
    no padding."""
    Q1, P1 = p + dp + 2, p + 1
    S = Q1 - 1

    def n(comp, d):
        return S if comp == d else Q1
    f = 0.0
    for a in range(3):
        for b in range(a + 1):
            R, ncb = n(a, 0) * n(b, 0), n(a, 1) * n(b, 1)
            nblk = n(a, 2) * (n(a, 2) + 1) // 2 if a == b else n(a, 2) * n(b, 2)
            f += nblk * (15 * Q1 ** 3 + 10 * ncb * Q1 * Q1 + 10 * R * ncb * Q1)
        for c in range(3):
            R, ncb, nblk = n(a, 0) * P1, n(a, 1) * P1, n(a, 2) * P1
            f += nblk * (9 * Q1 ** 3 + 6 * ncb * Q1 * Q1 + 6 * R * ncb * Q1)
    N = 3 * S * Q1 * Q1
    return f + 8.0 * N * N


def algorithmic_flops(p: int, dp: int) -> dict:
    """Algorithmic flop counts per cell: the sum-factorised formation
    (formation_flops_sf), complex Cholesky of the n_v x n_v Gram matrix,
    triangular solves (half cost on the real trace columns), HERK and the two
    GEMVs (l_e, eta).  form_dense is the count of the same formation summed
    over all quadrature points (the structure-aware count without sum
    factorisation), kept for reference and not part of the totals."""
    s, r = p + dp + 1, p + 1
    n1 = p + dp + 2
    N = 3 * s * (s + 1) ** 2
    nv = 2 * N
    m1 = (p + 1) ** 3
    nq = n1 ** 3
    nu, nt = 6 * m1, 24 * r * r
    k = nu + nt
    return dict(form=formation_flops_sf(p, dp),
                chol=4.0 / 3.0 * nv ** 3, trsm=4 * nv * nv * nu + 2 * nv * nv * nt, herk=4 * k * k * nv,
                vec=32 * nv * k)


def formation_flops_dense(p: int, dp: int) -> float:
    s, r = p + dp + 1, p + 1
    n1 = p + dp + 2
    N = 3 * s * (s + 1) ** 2
    m1 = (p + 1) ** 3
    return 12 * N * N * n1 ** 3 + 12 * N * m1 * n1 ** 3 + 48 * N * r * (r + 1) * n1 * n1


PEAK_BF16_TFLOPS = 2500.0    # MI355X dense bf16 matrix peak
BF16_FLOPS_PER_TILE_STAGE = 4 * 96 * 2 * 16 * 16 * 32   # k_herk_split: 4 waves x 96 MFMA 16x16x32 per 32-column stage


def split_herk_executed_flops(p: int, dp: int) -> float:
    """bf16 MFMA flops k_herk_split executes per cell: 6.3 MF per 64x64 output
    tile and 32-column stage, over the tiles of the lower triangle of
    K_aug; a tile whose row block of W^H is zero in the F test columns skips
    their stages (the kernel's herk_k0)."""
    s, r = p + dp + 1, p + 1
    N = 3 * s * (s + 1) ** 2
    Np = (N + 31) // 32 * 32
    nvp = 2 * Np
    m1 = (p + 1) ** 3
    nu, nt1 = 6 * m1, 12 * r * r
    k = nu + 2 * nt1
    kp = (k + 2 + 63) // 64 * 64

    def zero_rows(r0, nr=32):
        eh0, hh0, lr0 = nvp + nu, nvp + nu + nt1, nvp + k
        pad0, r1 = lr0 + 2, r0 + nr
        if r0 < eh0 or (r0 < pad0 and r1 > lr0):
            return False                        # complex rows
        return not (r0 < lr0 and r1 > hh0)      # zero unless real (H-hat) rows

    def zero_f(blk):
        r0 = nvp + 64 * blk
        return zero_rows(r0) and zero_rows(r0 + 32)
    kb = kp // 64
    stages = 0
    for a in range(kb):
        for b in range(a + 1):
            k0 = (Np // 64) * 64 if (zero_f(a) or zero_f(b)) else 0
            stages += (nvp - k0) // 32
    return float(stages) * BF16_FLOPS_PER_TILE_STAGE


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
    # Doerfler marking of the workload's eta (sort, scans, flags) with its
    # temporaries in a workspace kept across calls
    ev = eta[:w.n_cells].contiguous()
    mark_ws = torch.empty(dpg.dorfler_mark_workspace_size(w.n_cells), dtype=torch.uint8, device=ev.device)

    def do_mark():
        dpg.dorfler_mark(ev, stream=stream, workspace=mark_ws)
    mark_ms = timed_ms(do_mark, reps)
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


def _oracle_cells(args):
    """Worker of the CPU baseline: forms and solves the given cells with the
    oracle, one thread (returns the number of cells done)."""
    wname, cells = args
    import threadpoolctl
    from oracle import dpg_oracle as O
    w = W.CONFIGS[int(wname[1])]()
    om = O.omega_dimensionless(w.freq_hz)
    pt = w.port
    pm = O.PortMode(pt["a"], pt["b"], pt["m"], pt["n"], om, pt["eps"], pt["mu"])
    x, off = W.random_coefficients(w)
    with threadpoolctl.threadpool_limits(1):
        for c in cells:
            cp = O.CellProblem(X=w.cell_vertices(c), p=int(w.degree[c]), dp=w.dp, eps=complex(w.eps[c]),
                               mu=complex(w.mu[c]), omega=om, face_kind=tuple(int(k) for k in w.face_kind[c]),
                               zinv=tuple(complex(z) for z in w.zinv[c]), port=pm)
            G, Bf, l = O.cell_forms(cp)
            O.local_solve(G, Bf, l, x[off[c]:off[c + 1]])
    return len(cells)


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(wname: str, budget_s: float = 20.0):
    """The oracle, as it stands (numpy forms + LAPACK LU per cell, FP64), on
    the GPU machine's host: a seeded sample of the workload's cells solved by a
    pool of single-threaded worker processes (the cell loop parallelised, one
    process per core used), then by one process on one core; each leg runs
    for about budget_s / 2 seconds.  Returns the cpu_baseline record."""
    import concurrent.futures as cf
    import multiprocessing as mp
    w = W.CONFIGS[int(wname[1])]()
    rng = np.random.default_rng(W.SEED_BASE + 77)
    order = [int(c) for c in rng.permutation(w.n_cells)]
    ncores = min(16, len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1))
    half = budget_s / 2.0
    # all cores: chunks of 2 cells handed to the pool until the time is up
    ctx = mp.get_context("spawn")
    with cf.ProcessPoolExecutor(max_workers=ncores, mp_context=ctx) as ex:
        list(ex.map(_oracle_cells, [(wname, order[:1])] * ncores))   # start-up and imports, not timed
        t0 = time.perf_counter()
        pending, done, pos = set(), 0, 0
        while True:
            while len(pending) < 2 * ncores and time.perf_counter() - t0 < half:
                pending.add(ex.submit(_oracle_cells, (wname, order[pos:pos + 2])))
                pos += 2
            if not pending:
                break
            fin, pending = cf.wait(pending, return_when=cf.FIRST_COMPLETED)
            done += sum(f.result() for f in fin)
        t_par = time.perf_counter() - t0
    # one core
    t0 = time.perf_counter()
    n1 = 0
    while time.perf_counter() - t0 < half:
        n1 += _oracle_cells((wname, order[n1:n1 + 1]))
    t_one = time.perf_counter() - t0
    return {"value": done / t_par, "unit": "elements/s", "cores": ncores, "kind": "oracle",
            "one_core_value": n1 / t_one, "cpu_model": cpu_model(), "nproc": os.cpu_count(),
            "sample": (f"seeded cells of {w.name}: {done} cells on {ncores} single-threaded worker processes "
                       f"in {t_par:.1f} s, {n1} cells on one core in {t_one:.1f} s (numpy forms, LAPACK LU, FP64)")}


def accuracy_report(w, cells, outputs):
    """Element-wise errors of the GPU outputs of the sampled cells against the
    oracle (tests/_oracle_cases.OracleRef: scale sqrt(K_aa K_bb), the oracle's
    own FP64 floor e_or and formation floor s_form).  outputs: {precision:
    {cell: (K_e, l_e, eta)}}."""
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from _oracle_cases import OracleRef
    x, off = W.random_coefficients(w)
    rows = {name: [] for name in outputs}
    floors = []
    for c in cells:
        ref = OracleRef(w, c, x[off[c]:off[c + 1]])
        floors.append(ref)
        for name, out in outputs.items():
            rows[name].append(ref.errors(*out[c]))
    rec = {"cells": [int(c) for c in cells], "metric": "max_ab |dK_ab| / sqrt(K_aa K_bb); max_a |dl_a| / "
           "(sqrt(K_aa) ||y||); |d eta| / eta; against the oracle's FP64 LU solve",
           "oracle_floor": {q: float(max(r.e_or[q] for r in floors)) for q in ("K", "l", "eta")},
           "formation_floor": {q: float(max(r.s_form[q] for r in floors)) for q in ("K", "l", "eta")},
           "fp64_bar_min": {q: float(min(r.fp64_bar(q) for r in floors)) for q in ("K", "l", "eta")}}
    for name, es in rows.items():
        d = {}
        for q in ("K", "l", "eta", "K_x", "K_frob"):
            v = [e[q] for e in es if q in e]
            d[q + "_max"] = float(max(v))
            d[q + "_median"] = float(np.median(v))
        d["blocks_max"] = {b: float(max(e["blocks"][b] for e in es)) for b in es[0]["blocks"]}
        d["within_bars"] = bool(all(e["K"] <= r.fp64_bar("K") + (1e-6 if name == "split" else 0) and
                                    e["l"] <= r.fp64_bar("l") + (1e-6 if name == "split" else 0) and
                                    e.get("eta", 0) <= r.fp64_bar("eta") for e, r in zip(es, floors)))
        d["robin_null_rows_exact"] = bool(all(e["null_exact"] for e in es))
        rec[name] = d
    return rec


FORM_KEYS = ("scale", "form_SM", "form_IF", "form_pad", "form_B", "form_load")


def sub_record(wname: str, steps: int = 2, warmup: int = 1, err_cells=None, tune: bool = False):
    """A smaller measurement of another workload for the same JSON line: both
    precisions, default batching (concurrent degree branches, whole chunks)
    or, with `tune`, the autotuner's choice (chunking, formation tile shape
    and schedule per degree, tuned once on the split path); one profiled
    eager solve on the sequential schedule for the kernel-class times, then
    `steps` timed graph replays after `warmup`; element-wise errors of
    `err_cells(w)` against the oracle if given."""
    import torch
    from paper_2609_03155_amd import dpg
    torch.cuda.empty_cache()
    w = W.CONFIGS[int(wname[1])]()
    x, off = W.random_coefficients(w)
    plan = dpg.Plan(w.degree, w.dp)
    prob = dpg.DeviceProblem.from_workload(w)
    xd = torch.from_numpy(x).cuda()
    K, l, eta, info = plan.alloc_outputs()
    stream = torch.cuda.current_stream()
    degs = sorted(set(int(v) for v in w.degree))
    if tune:
        plan.autotune(prob, xd, K, l, eta, info, precision=dpg.DPG_SPLIT_FP32, stream=stream)
        torch.cuda.synchronize()
    rec = {"workload": w.name, "cells": w.n_cells, "degrees": degs, "dp": w.dp,
           "batching": ("autotuned (split path): cells per launch sequence, formation tile shape, schedule"
                        if tune else "concurrent degree branches, whole chunks (default plan, not autotuned)"),
           "concurrent_degree_branches": plan.tuning(degs[0])[1],
           "cells_per_launch": {str(p): plan.tuning(p)[0] for p in degs},
           "formation_col_tiles": {str(p): plan.tiles(p) for p in degs}}
    cells = err_cells(w) if err_cells else []
    outs = {}
    for name, code in (("fp64", dpg.DPG_FP64), ("split", dpg.DPG_SPLIT_FP32)):
        plan.local_solve(prob, xd, K, l, eta, info, precision=code, stream=stream)   # first touch
        torch.cuda.synchronize()
        plan.profile()
        plan.set_concurrency(False)
        plan.set_profiling(True)
        plan.local_solve(prob, xd, K, l, eta, info, precision=code, stream=stream)
        torch.cuda.synchronize()
        plan.set_profiling(False)
        plan.set_concurrency(rec["concurrent_degree_branches"])
        prof = plan.profile()
        if cells:
            outs[name] = {}
            for c in cells:
                k = int(off[c + 1] - off[c])
                outs[name][c] = (K[int(plan.K_off[c]):int(plan.K_off[c + 1])].cpu().numpy().reshape(k, k).T,
                                 l[int(off[c]):int(off[c + 1])].cpu().numpy(), float(eta[c]))
        g = plan.graph(prob, xd, K, l, eta, info, code)
        for _ in range(warmup):
            g.launch(stream)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            g.launch(stream)
        e1.record(stream)
        torch.cuda.synchronize()
        g.close()
        ms = e0.elapsed_time(e1) / steps
        assert int((info != 0).sum()) == 0
        rec[name] = {"value": w.n_cells / (ms * 1e-3), "unit": "elements/s", "ms_per_step": ms,
                     "formation_ms": sum(prof[k][0] for k in FORM_KEYS),
                     "sweep_ms": prof["chol_diag"][0] + prof["chol_panel"][0], "herk_ms": prof["herk"][0],
                     "eager_sequential_ms": sum(v[0] for v in prof.values())}
        print(f"[bench] {w.name} {name}: {rec[name]['value']:.0f} elements/s", file=sys.stderr, flush=True)
    rec["speedup_split_vs_fp64"] = rec["fp64"]["ms_per_step"] / rec["split"]["ms_per_step"]
    del K, l, eta, info, xd
    plan.close()
    torch.cuda.empty_cache()
    if cells:
        rec["rel_err_vs_oracle"] = accuracy_report(w, cells, outs)
    return rec


def _c2_cells(w):
    """WR340 cells: port face with two PEC walls (0, 15), the outlet corner,
    the last cell and two seeded interior ones."""
    rng = np.random.default_rng(W.SEED_BASE + 22)
    return sorted(set([0, 15, 4992, w.n_cells - 1] + [int(c) for c in rng.choice(w.n_cells, 2, replace=False)]))


def _c3_cells(w):
    """One cell of each degree of the mixed workload."""
    return [int(np.nonzero(w.degree == p)[0][0]) for p in sorted(set(int(v) for v in w.degree))]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c2", choices=["c1", "c2", "c3", "c4", "c5"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--precision", default="both", choices=["both", "fp64", "split"])
    ap.add_argument("--mfma-calib", type=int, default=0,
                    help="run three n x n FP64 GEMMs (torch) before the solve, to calibrate the MFMA-busy counter")
    ap.add_argument("--copy-calib-mib", type=int, default=0,
                    help="run one device-to-device copy of this many MiB first (calibrates HBM byte counters)")
    ap.add_argument("--no-graph", action="store_true", help="time eager solves instead of HIP-graph replays")
    ap.add_argument("--no-autotune", action="store_true", help="skip the batching autotuner")
    ap.add_argument("--sequential", action="store_true", help="degree groups one after the other (no branches)")
    ap.add_argument("--no-trace-system", action="store_true",
                    help="skip the condensation / assembly / CSR matvec measurement")
    ap.add_argument("--no-sub", action="store_true",
                    help="skip the mixed-degree (c3) and high-order (c4) sub-records of the default workload")
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

    if args.mfma_calib > 0:
        # a vendor FP64 GEMM of known size: its duration (kernel trace) and
        # flops give its matrix-core utilisation, against which the MFMA-busy
        # counter of the same run is normalised
        n = args.mfma_calib
        a = torch.ones((n, n), dtype=torch.float64, device="cuda")
        b = torch.ones((n, n), dtype=torch.float64, device="cuda")
        for _ in range(3):
            c = a @ b
        torch.cuda.synchronize()
        del a, b, c
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
        "flop_counts_per_step": {"formation_sum_factorised": fl["form"], "cholesky": fl["chol"], "trsm": fl["trsm"],
                                 "herk": fl["herk"], "gemv": fl["vec"],
                                 "formation_dense_reference": sum(formation_flops_dense(int(p), w.dp)
                                                                  for p in w.degree)},
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
                       "cells_per_launch": {str(p): plan.tuning(p)[0] for p in degs},
                       "formation_col_tiles": {str(p): plan.tiles(p) for p in degs}}
    if "split" in runs and "fp64" in runs:
        rec["speedup_split_vs_fp64"] = runs["fp64"][0] / runs["split"][0]
    if not args.no_trace_system and not streaming:
        rec["trace_system"] = trace_system_timings(w, plan, prob, xd, K, l, eta, info, solve, stream)
    if "split" in runs:
        # the split HERK against its own (bf16) MFMA peak, and its FP64-equivalent work
        ms_h, n_h = runs["split"][1]["herk"]
        ex = sum(int(np.sum(w.degree == p)) * split_herk_executed_flops(p, w.dp)
                 for p in sorted(set(int(v) for v in w.degree))) * args.steps
        alg = (fl["herk"] + fl["vec"]) * args.steps
        rec["roofline_split_herk"] = {
            "kernel": "k_herk_split (K_aug = W^H W from bf16x3 splits on v_mfma_f32_16x16x32_bf16)",
            "bound": "mfma", "achieved": ex / (ms_h * 1e-3) / 1e12, "peak": PEAK_BF16_TFLOPS, "unit": "TFLOP/s",
            "frac": ex / (ms_h * 1e-3) / 1e12 / PEAK_BF16_TFLOPS,
            "fp64_equivalent_achieved": alg / (ms_h * 1e-3) / 1e12,
            "fp64_equivalent_frac": alg / (ms_h * 1e-3) / 1e12 / PEAK_FP64_TFLOPS,
            "avg_launch_ms": ms_h / max(1, n_h), "launches_per_step": n_h / args.steps,
            "note": "executed: 6 bf16 products per real product, 64x64 tiles of the lower triangle of K_aug "
                    "incl. padding; FP64-equivalent: 4 k^2 n_v + 32 n_v k per cell"}
    if not args.no_cpu_baseline:
        if not streaming and w.name.startswith("c2"):
            cells = _c2_cells(w)
        else:
            rng = np.random.default_rng(W.SEED_BASE + 77)
            cells = sorted(int(c) for c in rng.choice(w.n_cells, 2, replace=False))
        outs = {}
        for name, (_, _, code, _) in runs.items():
            if not streaming:
                solve(code)                  # outputs of this precision
                torch.cuda.synchronize()
            outs[name] = {c: cell_outputs(code, c) for c in cells}
        rec["rel_err_vs_oracle"] = accuracy_report(w, cells, outs)
        rec["cpu_baseline"] = cpu_baseline(args.workload, args.cpu_budget)
    if not args.no_sub and args.workload == "c2":
        del K, l, eta, info
        plan.close()
        torch.cuda.empty_cache()
        rec["sub_records"] = {"c3_mixed_degrees": sub_record("c3", err_cells=_c3_cells, tune=True),
                              "c4_p4_dp2": sub_record("c4", steps=1, warmup=1)}
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
