"""Benchmark: preconditioned Legendre-Galerkin PCG on one MI355X.

Workload (default): 2D, N = 1024 ((N-1)^2 = 1,046,529 unknowns), coefficient
a = 2 + sum_{j,k<=12} c_jk L_j(x) L_k(y) (c_jk = 0.3 2^-(j+k) U(-1,1), seed 1),
b = 1 + x^2 + y^2, f from the manufactured u* = sin(pi x) sin(pi y) e^{x+y},
preconditioner truncation T = 8, FP64, PCG from x0 = 0 to relative residual
1e-10. Inputs (nodal a, b, f) are resident in HBM before timing starts.

One timed step = one request end to end on the device: build the operator
from the nodal coefficients, assemble and factor the preconditioner
(ILU(0) in FP64), form the load vector, and run PCG to 1e-10 (true FP64
residual checked). `value` is steps per second. Also reported: solve-only
rate (factors built), the FP64 matvec rate against the matrix-core peak, the
forward-sweep bandwidth, mixed-precision (FP32 and BF16 inner) solves, and the
oracle on the host CPU (bounded sample).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload 2d_N1024_T8]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6


def matvec_flops(d, N):
    n1, q = N - 1, N + 1
    if d == 2:
        return 8.0 * n1 * n1 * q + 12.0 * q * q * n1
    return 8.0 * q * n1 ** 3 + 12.0 * q * q * n1 * n1 + 16.0 * q ** 3 * n1


def nnz_lower(d, n1, offsets):
    """In-grid strictly lower entries of L: sum over lower offsets of the
    number of rows whose column stays in the grid."""
    tot = 0
    for o in offsets:
        key = tuple(reversed(o[:d]))
        if key < tuple([0] * d):
            cnt = 1
            for k in range(d):
                cnt *= max(0, n1 - abs(o[k]))
            tot += cnt
    return tot


def cpu_baseline(cfg, sample_rows):
    """The oracle (plain FP64 numpy + single-threaded C) timed on the same
    workload, as a bounded sample: coefficient series, 1D factors and the
    stencil rows of M in full; Alg. 2 on the first `sample_rows` rows (rows
    depend only on earlier rows, so the prefix costs what it costs inside the
    full factorisation), scaled to all rows; one PCG iteration (sum-factorised
    matvec + both substitutions with the prefix-factored rows completed by
    the sample scaling), scaled to the iteration count of the GPU solve."""
    import synth
    from oracle import galerkin as gk
    from oracle import ilu as oilu
    from oracle import pcg as opcg
    from oracle import precond as pc
    from oracle import workload as owl
    t0 = time.perf_counter()
    B = gk.Basis(cfg.N)
    c = synth.coefficient_draws(cfg.d, cfg.J, cfg.seed)
    a = owl.coefficient_a(c, B.x)
    b = owl.coefficient_b(cfg.d, B.x)
    F = gk.load_vector(cfg.d, cfg.N, owl.rhs_f(c, B.x), B)
    ah, bh = pc.series_pair(a, b, B, cfg.T, cfg.T)
    offs = pc.stencil_offsets(ah, bh)
    H = pc.stencil_rows(cfg.d, cfg.n1, ah, bh, offs)
    t_rows = time.perf_counter() - t0
    st = oilu.StencilILU(cfg.d, cfg.n1, offs, H)
    rows = min(sample_rows, cfg.n)
    t1 = time.perf_counter()
    st.factor(nrows=rows)
    t_fac = (time.perf_counter() - t1) * (cfg.n / rows)
    mv = lambda v: gk.matvec_sumfact(cfg.d, cfg.N, a, b, v, B)
    t1 = time.perf_counter()
    z = st.apply(F)
    w = mv(z)
    t_it = time.perf_counter() - t1
    sample = ("oracle on %s: operator data + stencil rows %.1f s (full), Alg. 2 on %d of %d rows "
              "scaled to %.1f s, one PCG iteration (matvec + Alg. 3 + Alg. 4) %.2f s"
              % (cfg.name, t_rows, rows, cfg.n, t_fac, t_it))
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or os.cpu_count()
    return dict(setup=t_rows + t_fac, t_iter=t_it, sample=sample, threads=threads)


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


KERNEL_SOURCES = {"factor": "paper_2004_13961_amd/csrc/ilu.hip", "sweep": "paper_2004_13961_amd/csrc/ilu.hip",
                  "matvec": "paper_2004_13961_amd/csrc/gemm.hip"}


def measured_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` from the committed counter figures
    (profiles/traffic_<kernel>_<workload>.json: FETCH_SIZE and WRITE_SIZE per
    dispatch, scaled by what the same counters read for a copy of known
    size). None when there are none or the kernel's source file changed since
    they were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic_%s_%s.json" % (kernel, workload))
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    with open(os.path.join(ROOT, KERNEL_SOURCES[kernel]), "rb") as fh:
        digest = hashlib.sha256(fh.read()).hexdigest()
    if rec.get("source_sha256") != digest:
        return None
    return rec.get("bytes_per_launch")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="2d_N1024_T8", help="2d_N32_T4, 2d_N1024_T8, 3d_N128_T6 or 3d_N256_T6_mixed")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-rows", type=int, default=100000)
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="finish with one device-to-device copy of this many bytes (a reference "
                         "for hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the solver runs each request on a single GPU "
              "and has no multi-GPU path (requested --gpus %d)" % args.gpus)
        sys.exit(2)

    import torch

    import synth
    from paper_2004_13961_amd import lgpcg
    from paper_2004_13961_amd.solver import Factor, Problem, pcg_solve
    from paper_2004_13961_amd.workload import family_nodal

    cfg = synth.WORKLOADS[args.workload]
    d, N, T = cfg.d, cfg.N, cfg.T
    lgpcg.lib()
    a, b, f, _ = family_nodal(d, N, cfg.J, cfg.seed)
    dev = lambda v: torch.from_numpy(np.ascontiguousarray(v).reshape(-1)).cuda()
    a_d, b_d, f_d = dev(a), dev(b), dev(f)
    torch.cuda.synchronize()

    def one_request():
        P = Problem(d, N, a_d, b_d)
        M = Factor(P, T)
        F = P.load_vector(f_d)
        x, info = pcg_solve(P, M, F, rtol=cfg.tol)
        return P, M, F, x, info

    log("config %s: inputs resident" % cfg.name)
    for _ in range(args.warmup):
        one_request()
    torch.cuda.synchronize()
    log("warmup done")
    t0 = time.perf_counter()
    infos = []
    for _ in range(args.steps):
        P, M, F, x, info = one_request()
        infos.append(info)
    torch.cuda.synchronize()
    t_e2e = (time.perf_counter() - t0) / args.steps
    log("timed steps: %.3f ms/step" % (t_e2e * 1e3))
    for inf in infos:
        assert inf["relres_true"] <= cfg.tol, inf

    # solve only (factors built)
    ws = torch.empty(lgpcg.lib().lgp_solve_workspace_bytes(P.handle, 0), dtype=torch.uint8, device="cuda")
    x = torch.zeros_like(F)
    pcg_solve(P, M, F, x=x, rtol=cfg.tol, ws=ws)
    torch.cuda.synchronize()
    reps = max(3, args.steps)
    t0 = time.perf_counter()
    for _ in range(reps):
        x.zero_()
        _, info_s = pcg_solve(P, M, F, x=x, rtol=cfg.tol, ws=ws)
    torch.cuda.synchronize()
    t_solve = (time.perf_counter() - t0) / reps
    log("solve only: %.3f ms" % (t_solve * 1e3))

    # matvec and sweep timing with events on the library's stream
    u = torch.rand(P.n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(u)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(6)]
    for _ in range(3):
        P.matvec(u, y)
    nmv = 20
    ev[0].record()
    for _ in range(nmv):
        P.matvec(u, y)
    ev[1].record()
    nsw = 10
    for _ in range(2):
        M.forward(u, y)
    ev[2].record()
    for _ in range(nsw):
        M.forward(u, y)
    ev[3].record()
    for _ in range(2):
        M.backward(u, y)
    ev[4].record()
    for _ in range(nsw):
        M.backward(u, y)
    ev[5].record()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    M_t = Factor(P, T)
    torch.cuda.synchronize()
    t_factor = time.perf_counter() - t0
    mv_ms = ev[0].elapsed_time(ev[1]) / nmv
    sw_ms = ev[2].elapsed_time(ev[3]) / nsw
    swb_ms = ev[4].elapsed_time(ev[5]) / nsw
    mv_tflops = matvec_flops(d, N) / (mv_ms * 1e-3) / 1e12
    desc = M.describe()
    fac_ms = float(M_t.describe()["factor_kernel_ms"])   # ILU(0) kernel, HIP events on the library's stream
    nnz = nnz_lower(d, N - 1, desc["offsets"])
    n = P.n
    sweep_bytes = nnz * 8 + 2 * n * 8      # L entries in the grid, r read, y written
    sw_gbs = sweep_bytes / (sw_ms * 1e-3) / 1e9
    # ILU(0): every in-grid entry of L and every pivot written once, and each
    # row of L read at least once by the rows that use it
    factor_bytes = 2 * (nnz + n) * 8

    iters = info_s["iters"]
    # time of each candidate kernel inside one step
    share = {"factor": fac_ms, "sweep": iters * (sw_ms + swb_ms), "matvec": (iters + 2) * mv_ms}
    dominant = max(share, key=share.get)
    if dominant == "factor":
        ach = factor_bytes / (fac_ms * 1e-3) / 1e9
        fk = "ilu_factor2_kernel" if desc.get("factor_kernel") == 2 else "ilu_factor_kernel"
        roof = dict(kernel=fk + " (ILU(0), Alg. 2)", bound="hbm", achieved=round(ach, 2),
                    peak=HBM_PEAK_GBS, unit="GB/s", frac=round(ach / HBM_PEAK_GBS, 6),
                    bytes_per_launch=factor_bytes, launch_ms=round(fac_ms, 3))
    elif dominant == "sweep":
        sk = "sweep2d_pair_kernel" if d == 2 else "sweep_kernel"
        roof = dict(kernel=sk + " (forward substitution, Alg. 3)", bound="hbm",
                    achieved=round(sw_gbs, 2), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(sw_gbs / HBM_PEAK_GBS, 5), bytes_per_launch=sweep_bytes,
                    launch_ms=round(sw_ms, 4))
    else:
        roof = dict(kernel="gemm_k4_kernel<double> (sum-factorised matvec)", bound="mfma",
                    achieved=round(mv_tflops, 3), peak=FP64_PEAK_TFLOPS, unit="TFLOP/s",
                    frac=round(mv_tflops / FP64_PEAK_TFLOPS, 5), flops_per_matvec=matvec_flops(d, N),
                    launch_ms=round(mv_ms, 4))
    roof["traffic"] = measured_traffic(dominant, cfg.name)
    roof["time_share_ms"] = {k: round(v, 3) for k, v in share.items()}

    log("matvec %.4f ms, sweeps %.4f / %.4f ms, factor %.1f ms (kernel %.1f ms)" % (mv_ms, sw_ms, swb_ms,
                                                                                   t_factor * 1e3, fac_ms))
    mixed = {}
    if not args.no_mixed:
        xd = x.clone()
        M32 = Factor(P, T, store="f32")
        for inner in ("f32", "bf16"):
            xm = torch.zeros_like(F)
            pcg_solve(P, M32, F, x=xm, rtol=cfg.tol, inner=inner)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(2):
                xm.zero_()
                _, im = pcg_solve(P, M32, F, x=xm, rtol=cfg.tol, inner=inner)
            torch.cuda.synchronize()
            tm = (time.perf_counter() - t0) / 2
            log("mixed %s: %.3f ms, %s" % (inner, tm * 1e3, im))
            err = float(torch.linalg.norm(xm - xd) / torch.linalg.norm(xd))
            mixed[inner] = dict(solves_per_sec=round(1.0 / tm, 3), inner_iters=im["iters"], outer=im["outer"],
                                relres_true=im["relres_true"], rel_err_vs_fp64=err)

    out = {
        "metric": "PCG solves/sec + matvec TFLOP/s at rel. residual 1e-10, mixed vs FP64",
        "value": round(1.0 / t_e2e, 4),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(t_e2e * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": cfg.name, "d": d, "N": N, "T": T, "unknowns": n, "tol": cfg.tol,
                   "coefficients": "a = 2 + sum_{j,k<=%d} c_jk L_j L_k, seed %d; b = 1+|x|^2" % (cfg.J, cfg.seed),
                   "step": "build operator + factor M (ILU(0), FP64) + load vector + PCG to 1e-10"},
        "solve_only_per_sec": round(1.0 / t_solve, 3),
        "solve_only_ms": round(t_solve * 1e3, 3),
        "pcg_iterations": iters,
        "relres_true": info_s["relres_true"],
        "factor_ms": round(t_factor * 1e3, 3),
        "matvec_ms": round(mv_ms, 4),
        "matvec_tflops": round(mv_tflops, 3),
        "matvec_frac_fp64_peak": round(mv_tflops / FP64_PEAK_TFLOPS, 4),
        "sweep_ms": round(sw_ms, 4),
        "sweep_backward_ms": round(swb_ms, 4),
        "factor_kernel_ms": round(fac_ms, 3),
        "sweep_gbs": round(sw_gbs, 2),
        "sweep_levels": desc["levels"],
        "mixed": mixed,
        "roofline": {k: roof[k] for k in ("bound", "achieved", "peak", "unit", "frac", "traffic")},
        "roofline_detail": roof,
    }
    if not args.no_cpu_baseline:
        log("oracle on the host CPU (bounded sample)")
        cb = cpu_baseline(cfg, args.cpu_sample_rows)
        total = cb["setup"] + cb["t_iter"] * iters
        out["cpu_baseline"] = {"value": round(1.0 / total, 6), "unit": "solves/s", "cores": cb["threads"],
                               "kind": "oracle",
                               "sample": cb["sample"] + "; total scaled to the GPU's %d iterations" % iters}
    print(json.dumps(out))
    if args.copy_probe > 0:
        src = torch.ones(args.copy_probe // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log("copy probe: %d bytes" % (src.numel() * 8))


if __name__ == "__main__":
    main()
