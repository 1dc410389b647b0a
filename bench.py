"""Benchmark: preconditioned Legendre-Galerkin PCG on one MI355X.

Default workload `3d_N256_T6_mixed` (the largest single-GPU configuration):
3D, N = 256 (255^3 = 16,581,375 unknowns), a = 2 + sum_{j,k,l<=6} c_jkl
L_j L_k L_l (c = 0.3 2^-(j+k+l) U(-1,1), seed 3), b = 1 + |x|^2, f from the
manufactured u* = prod sin(pi x_i) e^{x_i}, preconditioner truncation T = 6
with the ILU(0) factorisation in FP64 and the factor kept in FP32 only (the
FP64 factor, 306 GB, does not fit in HBM), mixed-precision solve: FP32 inner
PCG (products on the matrix cores, inner tolerance 1e-4) inside FP64
iterative refinement to a true relative residual of 1e-10. Other workloads:
--workload 2d_N32_T4 | 2d_N1024_T8 | 3d_N128_T6 (FP64).

One timed step = one request end to end on the device, inputs (nodal a, b,
f) resident in HBM: build the operator, assemble and factor the
preconditioner, form the load vector, solve (true FP64 residual checked).
`value` is requests per second. Also reported: solve-only rates (FP64 and /
or FP32 and BF16 inner), matvec TFLOP/s in FP64, FP32 and BF16 against the
matrix-core peaks, substitution bandwidth, the dominant kernel's roofline,
and the oracle on the host CPU (bounded sample).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
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

HBM_PEAK_GBS = 8000.0
PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3, "bf16": 2500.0}   # dense matrix-core peaks
FP64_VECTOR_TFLOPS = 78.6


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def matvec_flops(d, N):
    n1, q = N - 1, N + 1
    if d == 1:
        return 4.0 * n1 * q
    if d == 2:
        return 8.0 * n1 * n1 * q + 12.0 * q * q * n1
    return 8.0 * q * n1 ** 3 + 12.0 * q * q * n1 * n1 + 16.0 * q ** 3 * n1


def _range_count(n1, a, b, lo=0, hi=None):
    """Number of x in [lo, hi) with x, x + a, x + b all in [0, n1) (arrays)."""
    hi = n1 if hi is None else hi
    start = np.maximum(lo, np.maximum(0, np.maximum(-a, -b)))
    stop = np.minimum(hi, n1 - np.maximum(0, np.maximum(a, b)))
    return np.maximum(0, stop - start)


def lower_entries(d, n1, offsets):
    """In-grid strictly lower entries of L (sum over lower offsets of the rows
    whose column stays in the grid)."""
    offs = np.array([list(o[:d]) + [0] * (3 - d) for o in offsets], dtype=np.int64)
    lower = np.array([tuple(reversed(o[:d])) < tuple([0] * d) for o in offsets])
    tot = np.ones(lower.sum(), dtype=np.float64)
    for k in range(d):
        tot *= _range_count(n1, offs[lower, k], 0 * offs[lower, k])
    return float(tot.sum())


def _offset_cube(offs):
    """Membership of offset vectors in the pattern: a boolean cube over
    [-2h, 2h]^3 (differences of two offsets stay inside)."""
    h = int(np.abs(offs).max())
    R = 2 * h
    cube = np.zeros((2 * R + 1,) * 3, dtype=bool)
    cube[offs[:, 2] + R, offs[:, 1] + R, offs[:, 0] + R] = True
    return cube, R


def _rows_count(d, n1, a, b, yrange, zrange):
    c = np.ones(len(b))
    for ax in range(d):
        lo, hi = 0, n1
        if ax == 1 and yrange is not None:
            lo, hi = yrange
        if ax == 2 and zrange is not None:
            lo, hi = zrange
        c *= _range_count(n1, np.full(len(b), a[ax]), b[:, ax], lo, hi)
    return c


def ilu_pairs(d, n1, offsets, yrange=None, zrange=None):
    """Left-looking ILU(0) work: number of (row, j, l) with L(i, i+d_j) and
    L(i+d_j, i+d_j+d_l) both in the grid, d_j and d_l lower, d_j + d_l in
    the pattern (each such triple is one multiply-add of Alg. 2 with
    U = D L^T). Optionally rows restricted to y, z ranges."""
    offs = np.array([list(o[:d]) + [0] * (3 - d) for o in offsets], dtype=np.int64)
    cube, R = _offset_cube(offs)
    diag = [tuple(o) for o in offs.tolist()].index((0, 0, 0))
    lower = offs[:diag]
    tot = 0.0
    for dj in lower:
        dk = lower + dj                          # d_j + d_l for every lower l
        inS = cube[dk[:, 2] + R, dk[:, 1] + R, dk[:, 0] + R]
        if inS.any():
            tot += _rows_count(d, n1, dj, dk[inS], yrange, zrange).sum()
    return tot


def oracle_c_work(d, n1, offsets, yrange=None, zrange=None):
    """Inner-loop iterations of the oracle's Alg. 2 (C, IKJ order): per row,
    per lower offset k in the grid, per later offset j with j - k in the
    pattern and j in the grid."""
    offs = np.array([list(o[:d]) + [0] * (3 - d) for o in offsets], dtype=np.int64)
    cube, R = _offset_cube(offs)
    diag = [tuple(o) for o in offs.tolist()].index((0, 0, 0))
    tot = 0.0
    for ok in range(diag):
        a = offs[ok]
        later = offs[ok + 1:]
        df = later - a
        inS = cube[df[:, 2] + R, df[:, 1] + R, df[:, 0] + R]
        if inS.any():
            tot += _rows_count(d, n1, a, later[inS], yrange, zrange).sum()
    return tot


def cpu_baseline(cfg, sample_lines, iters):
    """The oracle (plain FP64 numpy + single-threaded C) on the same
    workload, timed on a bounded sample of rows and scaled by the oracle's
    own operation counts:
      * stencil rows of M for the first z-plane (3D) or all rows (2D);
      * Alg. 2 on the first `sample_lines` grid lines of rows, scaled to the
        whole grid by the count of the C loop's inner iterations (rows near
        the faces have fewer terms, so the count, not the row count, scales);
      * Alg. 3 on the same rows, scaled by the in-grid entries of L; Alg. 4
        taken equal to Alg. 3 (same entries, one division more per row);
      * one sum-factorised FP64 matvec over the whole grid;
    total = setup + factorisation + `iters` x (matvec + both substitutions)."""
    import synth
    from oracle import galerkin as gk
    from oracle import ilu as oilu
    from oracle import precond as pc
    from oracle import workload as owl
    d, N, n1 = cfg.d, cfg.N, cfg.N - 1
    t0 = time.perf_counter()
    B = gk.Basis(N)
    c = synth.coefficient_draws(d, cfg.J, cfg.seed)
    a = owl.coefficient_a(c, B.x)
    b = owl.coefficient_b(d, B.x)
    F = gk.load_vector(d, N, owl.rhs_f(c, B.x), B)
    ah, bh = pc.series_pair(a, b, B, cfg.T, cfg.T)
    offs = pc.stencil_offsets(ah, bh)
    t_series = time.perf_counter() - t0
    t1 = time.perf_counter()
    H = pc.stencil_rows(d, n1, ah, bh, offs, nplanes=1 if d == 3 else None)
    t_rows = time.perf_counter() - t1
    rows_in_H = H.shape[0]
    t_rows_full = t_rows * (n1 ** d / rows_in_H)
    lines = min(sample_lines, n1)
    nrows = lines * n1
    st = oilu.StencilILU(d, n1, offs, H)
    t1 = time.perf_counter()
    st.factor(nrows=nrows)
    t_fac_s = time.perf_counter() - t1
    yr = (0, lines)
    zr = (0, 1) if d == 3 else None
    w_s = oracle_c_work(d, n1, offs, yrange=yr, zrange=zr)
    w_full = oracle_c_work(d, n1, offs)
    t_fac = t_fac_s * (w_full / max(w_s, 1.0))
    r = np.ascontiguousarray(F[:rows_in_H]) if d == 3 else F
    t1 = time.perf_counter()
    st.forward_prefix(r, nrows)
    t_fw_s = time.perf_counter() - t1
    e_s = lower_entries_prefix(d, n1, offs, lines)
    e_full = lower_entries(d, n1, offs)
    t_sweeps = 2.0 * t_fw_s * (e_full / max(e_s, 1.0))
    u = np.random.default_rng(0).uniform(0.0, 1.0, size=n1 ** d)
    t1 = time.perf_counter()
    gk.matvec_sumfact(d, N, a, b, u, B)
    t_mv = time.perf_counter() - t1
    total = t_series + t_rows_full + t_fac + iters * (t_mv + t_sweeps)
    sample = ("oracle on %s: series and offsets %.1f s; stencil rows of M for %d rows %.1f s, scaled to all rows "
              "%.0f s; Alg. 2 on the first %d lines (%d rows) %.2f s, scaled by the C loop's inner iterations "
              "(%.3g of %.3g) to %.0f s; Alg. 3 on those rows %.3f s, scaled by in-grid L entries and doubled for "
              "Alg. 4: %.1f s per application; one full FP64 matvec %.2f s; total over %d iterations"
              % (cfg.name, t_series, rows_in_H, t_rows, t_rows_full, lines, nrows, t_fac_s, w_s, w_full, t_fac,
                 t_fw_s, t_sweeps, t_mv, iters))
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or os.cpu_count()
    return dict(total=total, sample=sample, threads=threads)


def fast_dlt_section(log):
    """The product of Sec. 4.3 through the fast discrete Legendre transforms
    (lgp_matvec_fast) against the dense contractions on the matrix cores
    (lgp_matvec), at 2D N = 1024 (config 1's grid), and one batch of 1D
    transforms (all 1025 lines of the grid) each way. Events on the stream
    the library runs on."""
    import torch

    import synth
    from paper_2004_13961_amd.solver import FastTransforms, Problem
    from paper_2004_13961_amd.workload import family_nodal
    cfg = synth.WORKLOADS["2d_N1024_T8"]
    d, N = cfg.d, cfg.N
    a, b, _, _ = family_nodal(d, N, cfg.J, cfg.seed, with_rhs=False)
    dev = lambda v: torch.from_numpy(np.ascontiguousarray(v).reshape(-1)).cuda()
    P = Problem(d, N, dev(a), dev(b))
    T = FastTransforms(P)
    u = torch.rand(P.n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(u)
    yd = torch.empty_like(u)
    c = torch.rand(P.nq, dtype=torch.float64, device="cuda")
    f = torch.empty_like(c)

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    fast = timed(lambda: T.matvec(u, y), 3)
    dense = timed(lambda: P.matvec(u, yd), 10)
    bwd = timed(lambda: T.lines(c, forward=False, out=f), 3)
    fwd = timed(lambda: T.lines(c, forward=True, out=f), 3)
    diff = float(torch.max(torch.abs(y - yd)) / torch.max(torch.abs(yd)))
    log("fast DLT (2D N=1024): product %.2f ms (dense %.3f ms), 1025 BDLTs %.2f ms, FDLTs %.2f ms, %d blocks" % (
        fast, dense, bwd, fwd, T.blocks()))
    return {"workload": "2d_N1024_T8", "fast_product_ms": round(fast, 3), "dense_product_ms": round(dense, 4),
            "bdlt_1025_lines_ms": round(bwd, 3), "fdlt_1025_lines_ms": round(fwd, 3), "expansion_blocks": T.blocks(),
            "max_rel_diff_fast_vs_dense": diff}


def cpu_full(cfg, log):
    """The oracle on the whole workload, end to end, nothing sampled or
    scaled: coefficients, load vector, truncated series and pattern, the
    stencil rows of M for every row, Alg. 2 on every row, then PCG (Alg. 1)
    with the oracle's sum-factorised product and its Alg. 3/4 to the
    workload's tolerance; the residual checked by the oracle's product."""
    import platform

    import synth
    from oracle import galerkin as gk
    from oracle import ilu as oilu
    from oracle import pcg as opcg
    from oracle import precond as pc
    from oracle import workload as owl
    d, N, n1 = cfg.d, cfg.N, cfg.N - 1
    tt = {}
    t0 = time.perf_counter()
    B = gk.Basis(N)
    c = synth.coefficient_draws(d, cfg.J, cfg.seed)
    a = owl.coefficient_a(c, B.x)
    b = owl.coefficient_b(d, B.x)
    F = gk.load_vector(d, N, owl.rhs_f(c, B.x), B)
    ah, bh = pc.series_pair(a, b, B, cfg.T, cfg.T)
    offs = pc.stencil_offsets(ah, bh)
    tt["setup_s"] = time.perf_counter() - t0
    log("cpu full: setup %.1f s" % tt["setup_s"])
    t1 = time.perf_counter()
    H = pc.stencil_rows(d, n1, ah, bh, offs)
    tt["stencil_rows_s"] = time.perf_counter() - t1
    log("cpu full: stencil rows %.1f s" % tt["stencil_rows_s"])
    t1 = time.perf_counter()
    st = oilu.StencilILU(d, n1, offs, H).factor()
    tt["ilu0_s"] = time.perf_counter() - t1
    log("cpu full: ILU(0) %.1f s" % tt["ilu0_s"])
    mv = lambda v: gk.matvec_sumfact(d, N, a, b, v, B)
    t1 = time.perf_counter()
    x, iters, hist = opcg.pcg(mv, st.apply, F, cfg.tol)
    tt["pcg_s"] = time.perf_counter() - t1
    total = time.perf_counter() - t0
    relres = float(np.linalg.norm(F - mv(x)) / np.linalg.norm(F))
    log("cpu full: PCG %d iterations %.1f s, residual %.2e" % (iters, tt["pcg_s"], relres))
    model = platform.processor()
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count()
    return {"workload": cfg.name, "kind": "oracle", "mode": "full run, nothing sampled",
            "seconds": round(total, 2), "requests_per_sec": 1.0 / total,
            "phases_s": {k: round(v, 2) for k, v in tt.items()}, "pcg_iterations": iters,
            "relres_oracle": relres, "cpu_model": model, "cores_available": cores,
            "threads": {"oracle C loops": 1,
                        "numpy BLAS": os.environ.get("OMP_NUM_THREADS", "library default")}}


def lower_entries_prefix(d, n1, offsets, lines):
    """In-grid lower entries of L in the rows of the first `lines` grid lines
    (z = 0 plane in 3D)."""
    offs = np.array([list(o[:d]) + [0] * (3 - d) for o in offsets], dtype=np.int64)
    lower = np.array([tuple(reversed(o[:d])) < tuple([0] * d) for o in offsets])
    lo = offs[lower]
    tot = _range_count(n1, lo[:, 0], 0 * lo[:, 0]).astype(np.float64)
    if d >= 2:
        tot *= _range_count(n1, lo[:, 1], 0 * lo[:, 1], 0, lines)
    if d == 3:
        tot *= _range_count(n1, lo[:, 2], 0 * lo[:, 2], 0, 1)
    return float(tot.sum())


KERNEL_SOURCES = {"factor": ("paper_2004_13961_amd/csrc/ilu.hip", "paper_2004_13961_amd/csrc/ilu3d.hip"),
                  "sweep": ("paper_2004_13961_amd/csrc/ilu.hip", "paper_2004_13961_amd/csrc/ilu3d.hip"),
                  "matvec": ("paper_2004_13961_amd/csrc/gemm.hip",)}


def measured_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` from the committed counter figures
    (profiles/traffic_<kernel>_<workload>.json), or None when there are none
    or the kernel's sources changed since they were taken."""
    path = os.path.join(ROOT, "profiles", "traffic_%s_%s.json" % (kernel, workload))
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    h = hashlib.sha256()
    for src in KERNEL_SOURCES[kernel]:
        with open(os.path.join(ROOT, src), "rb") as fh:
            h.update(fh.read())
    if rec.get("sources_sha256") != h.hexdigest():
        return None
    return rec.get("bytes_per_launch")


def batched_throughput(count, log):
    """`count` requests of the 2D N = 1024, T = 8 family (coefficient seeds 1,
    2, ...): end to end one after another (each: operator, factor, load
    vector, PCG to 1e-10), against the same requests with their PCG solves
    run together as one batch (factors built one after another, then
    lgp_pcg_solve_batched). Every batched result is checked equal, bit for
    bit, to its solve alone."""
    import torch

    import synth
    from paper_2004_13961_amd.solver import Factor, Problem, pcg_solve, pcg_solve_batched
    from paper_2004_13961_amd.workload import family_nodal
    cfg = synth.WORKLOADS["2d_N1024_T8"]
    d, N, T = cfg.d, cfg.N, cfg.T
    dev = lambda v: torch.from_numpy(np.ascontiguousarray(v).reshape(-1)).cuda()
    inputs = []
    for k in range(count):
        a, b, f, _ = family_nodal(d, N, cfg.J, cfg.seed + k)
        inputs.append((dev(a), dev(b), dev(f)))
    torch.cuda.synchronize()

    def build(k):
        a, b, f = inputs[k]
        P = Problem(d, N, a, b)
        M = Factor(P, T)
        return P, M, P.load_vector(f)

    # warm (tile choices, first launches)
    P0, M0, F0 = build(0)
    pcg_solve(P0, M0, F0, rtol=cfg.tol)
    pcg_solve_batched([P0], [M0], [F0], rtol=cfg.tol)
    del P0, M0, F0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    alone = []
    for k in range(count):
        P, M, F = build(k)
        x, info = pcg_solve(P, M, F, rtol=cfg.tol)
        alone.append((x, info))
        del P, M, F
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    t0 = time.perf_counter()
    reqs = [build(k) for k in range(count)]
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    t1 = time.perf_counter()
    xs, infos = pcg_solve_batched([r[0] for r in reqs], [r[1] for r in reqs], [r[2] for r in reqs], rtol=cfg.tol)
    torch.cuda.synchronize()
    t_solve = time.perf_counter() - t1
    t_batch = time.perf_counter() - t0
    same = all(torch.equal(xb, xa[0]) and ib["iters"] == xa[1]["iters"] for xb, ib, xa in zip(xs, infos, alone))
    # solve-only, one at a time on the same factors
    t1 = time.perf_counter()
    for P, M, F in reqs:
        pcg_solve(P, M, F, rtol=cfg.tol)
    torch.cuda.synchronize()
    t_solve_seq = time.perf_counter() - t1
    log("batch of %d (2d_N1024_T8): one by one %.1f ms, batched %.1f ms (setup %.1f + solves %.1f), "
        "solves one by one %.1f ms, identical %s" % (count, t_seq * 1e3, t_batch * 1e3, t_setup * 1e3,
                                                     t_solve * 1e3, t_solve_seq * 1e3, same))
    del reqs, xs, alone, inputs
    torch.cuda.empty_cache()
    return {"workload": "2d_N1024_T8", "requests": count, "requests_per_sec_one_by_one": round(count / t_seq, 3),
            "requests_per_sec_batched": round(count / t_batch, 3),
            "solves_per_sec_one_by_one": round(count / t_solve_seq, 3),
            "solves_per_sec_batched": round(count / t_solve, 3), "setup_ms": round(t_setup * 1e3, 2),
            "batched_equal_to_alone": bool(same), "iters": [i["iters"] for i in infos]}


def serving_run(count, log):
    """The serving mix (synth.serving_requests: 70 % 2D with N log-uniform in
    [64, 1024], 30 % 3D with N log-uniform in [32, 192], T in {4, 6, 8},
    tolerance in {1e-8, 1e-10, 1e-12}), its first `count` requests: once all
    arriving at time 0 (closed loop, the saturation throughput C), then as a
    Poisson stream at 0.8 C (seed 4), with an HBM budget of 160 GiB and 8
    slots per batch. Reports p50 / p99 latency and solves per second."""
    import torch

    import synth
    from paper_2004_13961_amd.serving import Server, latency_summary, poisson_arrivals
    reqs = synth.serving_requests()[:count]
    budget = 160 << 30
    recs = Server(budget, slots_per_batch=8, step_iters=2).serve(reqs, [0.0] * count)
    closed = latency_summary(recs)
    del recs
    torch.cuda.empty_cache()
    rate = 0.8 * closed["solves_per_sec"]
    recs = Server(budget, slots_per_batch=8, step_iters=2).serve(reqs, list(poisson_arrivals(count, rate)))
    opened = latency_summary(recs)
    shapes = len({(r["d"], r["N"], r["T"]) for r in reqs})
    log("serving %d requests: closed loop %.2f solves/s; Poisson %.2f/s: p50 %.3f s, p99 %.3f s" % (
        count, closed["solves_per_sec"], rate, opened["p50_s"], opened["p99_s"]))
    del recs
    torch.cuda.empty_cache()
    return {"stream": "first %d of the 4096-request serving mix (%d distinct (d, N, T))" % (count, shapes),
            "solve": "FP64 PCG, batched per (d, N, pattern)", "budget_bytes": budget,
            "closed_loop_solves_per_sec": round(closed["solves_per_sec"], 3),
            "poisson_rate_per_sec": round(rate, 3), "solves_per_sec": round(opened["solves_per_sec"], 3),
            "p50_latency_s": round(opened["p50_s"], 4), "p99_latency_s": round(opened["p99_s"], 4),
            "all_ok": bool(closed["all_ok"] and opened["all_ok"])}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="3d_N256_T6_mixed",
                    help="3d_N256_T6_mixed (default), 3d_N128_T6, 2d_N1024_T8 or 2d_N32_T4")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-lines", type=int, default=64)
    ap.add_argument("--batch", type=int, default=8, help="requests of the batched-throughput section (0: skip)")
    ap.add_argument("--serve", type=int, default=24, help="requests of the serving section (0: skip)")
    ap.add_argument("--only-extras", action="store_true", help="skip the main workload (batch / serving only)")
    ap.add_argument("--no-fast-dlt", action="store_true", help="skip the fast-transform product section")
    ap.add_argument("--cpu-full", action="store_true",
                    help="run the oracle on the whole workload on the host CPU (no GPU) and print its timing")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="finish with one device-to-device copy of this many bytes (a reference "
                         "for hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the solver runs each request on a single GPU "
              "and has no multi-GPU path (requested --gpus %d)" % args.gpus)
        sys.exit(2)

    if args.cpu_full:
        import synth
        print(json.dumps(cpu_full(synth.WORKLOADS[args.workload], log)), flush=True)
        return

    import torch

    import synth
    from paper_2004_13961_amd import lgpcg
    from paper_2004_13961_amd.solver import Factor, Problem, pcg_solve
    from paper_2004_13961_amd.workload import family_nodal

    if args.only_extras:
        extras = {}
        if args.batch > 0:
            extras["batched"] = batched_throughput(args.batch, log)
        if args.serve > 0:
            extras["serving"] = serving_run(args.serve, log)
        if not args.no_fast_dlt:
            extras["fast_dlt"] = fast_dlt_section(log)
        print(json.dumps(extras), flush=True)
        return

    cfg = synth.WORKLOADS[args.workload]
    d, N, T = cfg.d, cfg.N, cfg.T
    mixed = cfg.mixed
    # the FP64 factor of the 3D mixed workload does not fit in HBM: FP32 only
    store = ("f32only" if d == 3 else "f32") if mixed else "f64"
    inner = "f32" if mixed else "f64"
    inner_rtol = 1e-4 if mixed else 0.0
    lgpcg.lib()
    a, b, f, _ = family_nodal(d, N, cfg.J, cfg.seed)
    dev = lambda v: torch.from_numpy(np.ascontiguousarray(v).reshape(-1)).cuda()
    a_d, b_d, f_d = dev(a), dev(b), dev(f)
    del a, b, f
    torch.cuda.synchronize()

    state = {}

    def one_request():
        state.clear()   # the previous request's buffers go before the next is built
        P = Problem(d, N, a_d, b_d)
        M = Factor(P, T, store=store)
        F = P.load_vector(f_d)
        x, info = pcg_solve(P, M, F, rtol=cfg.tol, inner=inner, inner_rtol=inner_rtol)
        state.update(P=P, M=M, F=F, x=x, info=info)
        return info

    log("config %s: inputs resident; factor store %s, solve %s" % (cfg.name, store, inner))
    for _ in range(args.warmup):
        one_request()
    torch.cuda.synchronize()
    log("warmup done")
    t0 = time.perf_counter()
    infos, fac_ms_list = [], []
    for k in range(args.steps):
        infos.append(one_request())
        fac_ms_list.append(float(state["M"].describe()["factor_kernel_ms"]))
        log("step %d done" % k)
    torch.cuda.synchronize()
    t_e2e = (time.perf_counter() - t0) / args.steps
    log("timed steps: %.3f ms/step" % (t_e2e * 1e3))
    for inf in infos:
        assert inf["relres_true"] <= cfg.tol, inf
    P, M, F, x = state["P"], state["M"], state["F"], state["x"]
    desc = M.describe()
    n = P.n

    # solve only (factors built)
    solve = {}
    for inn in (("f32", "bf16") if mixed else ("f64",)):
        xs = torch.zeros_like(F)
        rt = inner_rtol if inn == "f32" else 0.0
        pcg_solve(P, M, F, x=xs, rtol=cfg.tol, inner=inn, inner_rtol=rt)
        torch.cuda.synchronize()
        reps = 2 if d == 3 else max(3, args.steps)
        t0 = time.perf_counter()
        for _ in range(reps):
            xs.zero_()
            _, info_s = pcg_solve(P, M, F, x=xs, rtol=cfg.tol, inner=inn, inner_rtol=rt)
        torch.cuda.synchronize()
        ts = (time.perf_counter() - t0) / reps
        err = float(torch.linalg.norm(xs - x) / torch.linalg.norm(x))
        solve[inn] = dict(solves_per_sec=round(1.0 / ts, 4), ms=round(ts * 1e3, 3), iters=info_s["iters"],
                          outer=info_s["outer"], relres_true=info_s["relres_true"],
                          rel_diff_vs_step_solution=err)
        log("solve only (%s): %.3f ms, %s" % (inn, ts * 1e3, info_s))
        del xs

    # matvec in each precision, substitutions, with events on the library's stream
    def timed(fn, reps):
        for _ in range(2):
            fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    mv = {}
    u64 = torch.rand(n, dtype=torch.float64, device="cuda")
    y64 = torch.empty_like(u64)
    mv["f64"] = timed(lambda: P.matvec(u64, y64), 10)
    del y64
    u32 = u64.float()
    del u64
    y32 = torch.empty_like(u32)
    mv["f32"] = timed(lambda: P.matvec(u32, y32, prec="f32"), 10)
    mv["bf16"] = timed(lambda: P.matvec(u32, y32, prec="bf16"), 10)
    mv_tf = {k: matvec_flops(d, N) / (v * 1e-3) / 1e12 for k, v in mv.items()}
    if desc["L"] is not None:
        sd = "f64"
        uu = torch.rand(n, dtype=torch.float64, device="cuda")
        yy = torch.empty_like(uu)
        sw_ms = timed(lambda: M.forward(uu, yy), 3)
        swb_ms = timed(lambda: M.backward(uu, yy), 3)
        s_L = 8
    else:
        sd = "f32"
        sw_ms = timed(lambda: M.forward32(u32, y32), 3)
        swb_ms = timed(lambda: M.backward32(u32, y32), 3)
        s_L = 4
    torch.cuda.synchronize()
    offsets = desc["offsets"]
    nnz = lower_entries(d, N - 1, offsets)
    sweep_bytes = nnz * s_L + 2 * n * s_L
    sw_gbs = sweep_bytes / (sw_ms * 1e-3) / 1e9
    fac_ms = float(np.median(fac_ms_list))
    log("matvec %s ms; sweeps %.3f / %.3f ms (%s); factor kernel %.1f ms" % (
        {k: round(v, 4) for k, v in mv.items()}, sw_ms, swb_ms, sd, fac_ms))

    # dominant kernel of the timed step, by time share
    info = infos[-1]
    it = info["iters"]
    sweeps_per_step = 2 * it
    share = {"factor": fac_ms, "sweep": sweeps_per_step * (sw_ms + swb_ms) / 2,
             "matvec": (it + 2 * max(1, info["outer"])) * mv[inner if inner != "f64" else "f64"]}
    dominant = max(share, key=share.get)
    if dominant == "factor":
        flops = 2.0 * ilu_pairs(d, N - 1, offsets) + 3.0 * nnz + 2.0 * n
        ach = flops / (fac_ms * 1e-3) / 1e12
        fk = {3: "ilu3d_factor_kernel", 2: "ilu_factor2_kernel", 1: "ilu_factor_kernel"}.get(
            desc["factor_kernel"], "ilu_factor_kernel")
        # a factorisation may take several launches (the 3D kernel: one per
        # window of z-planes); per launch = per factorisation / launches,
        # and the event span covers all launches of the factorisation
        nl = max(1, int(desc.get("factor_launches", 1)))
        roof = dict(kernel=fk + " (ILU(0), Alg. 2, FP64)", bound="alu", achieved=round(ach, 4),
                    peak=FP64_VECTOR_TFLOPS, unit="TFLOP/s", frac=round(ach / FP64_VECTOR_TFLOPS, 6),
                    flops_per_factorisation=flops, launches_per_factorisation=nl,
                    flops_per_launch=flops / nl, launch_ms=round(fac_ms / nl, 3),
                    factorisation_ms=round(fac_ms, 3), bytes_written=nnz * (4 if store == "f32only" else 8))
    elif dominant == "sweep":
        sk = "sweep3d_kernel" if d == 3 else "sweep2d_pair_kernel"
        roof = dict(kernel=sk + " (forward substitution, Alg. 3, %s)" % sd, bound="hbm",
                    achieved=round(sw_gbs, 2), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(sw_gbs / HBM_PEAK_GBS, 5), bytes_per_launch=sweep_bytes,
                    launch_ms=round(sw_ms, 4))
    else:
        pm = inner if inner != "f64" else "f64"
        roof = dict(kernel="gemm_k4_kernel (sum-factorised matvec, %s)" % pm, bound="mfma",
                    achieved=round(mv_tf[pm], 3), peak=PEAK_TFLOPS[pm], unit="TFLOP/s",
                    frac=round(mv_tf[pm] / PEAK_TFLOPS[pm], 5), flops_per_launch=matvec_flops(d, N),
                    launch_ms=round(mv[pm], 4))
    roof["traffic"] = measured_traffic(dominant, cfg.name)
    roof["time_share_ms"] = {k: round(v, 3) for k, v in share.items()}

    out = {
        "metric": "PCG solves/sec + matvec TFLOP/s at rel. residual 1e-10, mixed vs FP64",
        "value": round(1.0 / t_e2e, 5),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(t_e2e * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if not mixed else "f64+f32",
        "data": "synthetic",
        "config": {"workload": cfg.name, "d": d, "N": N, "T": T, "unknowns": n, "tol": cfg.tol,
                   "coefficients": "a = 2 + sum_{j<=%d} c_j L_j..., seed %d; b = 1+|x|^2" % (cfg.J, cfg.seed),
                   "factor_store": store, "solve": inner if not mixed else "FP64 refinement, FP32 inner (1e-4)",
                   "step": "build operator + factor M (ILU(0) in FP64) + load vector + solve to 1e-10"},
        "pcg_iterations": it,
        "outer": info["outer"],
        "relres_true": info["relres_true"],
        "factor_kernel_ms": round(fac_ms, 3),
        "solve_only": solve,
        "matvec_ms": {k: round(v, 4) for k, v in mv.items()},
        "matvec_tflops": {k: round(v, 3) for k, v in mv_tf.items()},
        "matvec_frac_peak": {k: round(mv_tf[k] / PEAK_TFLOPS[k], 5) for k in mv_tf},
        "sweep_ms": round(sw_ms, 4),
        "sweep_backward_ms": round(swb_ms, 4),
        "sweep_dtype": sd,
        "sweep_gbs": round(sw_gbs, 2),
        "roofline": {k: roof[k] for k in ("bound", "achieved", "peak", "unit", "frac", "traffic")},
        "roofline_detail": roof,
    }
    # release the main workload's buffers (the closure above still holds
    # `state`, and the descriptor holds views of the factor's buffer)
    state.clear()
    del P, M, F, x, u32, y32, desc
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    log("main workload released: %.1f GiB still allocated" % (torch.cuda.memory_allocated() / 2**30))
    if args.batch > 0:
        out["batched"] = batched_throughput(args.batch, log)
    if args.serve > 0:
        out["serving"] = serving_run(args.serve, log)
    if not args.no_fast_dlt:
        out["fast_dlt"] = fast_dlt_section(log)
    if not args.no_cpu_baseline:
        log("oracle on the host CPU (bounded sample)")
        cb = cpu_baseline(cfg, args.cpu_sample_lines, max(1, it))
        out["cpu_baseline"] = {"value": float("%.4g" % (1.0 / cb["total"])), "unit": "solves/s",
                               "cores": cb["threads"], "kind": "oracle", "sample": cb["sample"]}
    print(json.dumps(out), flush=True)
    if args.copy_probe > 0:
        src = torch.ones(args.copy_probe // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log("copy probe: %d bytes" % (src.numel() * 8))


if __name__ == "__main__":
    main()
