#!/usr/bin/env python3
"""Benchmark of the FMM-BEM hot path on one MI355X.

Workload (default): the crowded protein-solution system, 512 blobby
molecules of 20,480 flat panels on an 8x8x8 lattice, 10,485,760 panels and
512,000 charges, eps 4/80, p = 10, theta = 0.5, ncrit = 64 -- the largest
configuration that one GPU holds.

One step = one pass of the whole hot path over it, inputs already resident
in HBM: build the octree (geometry, Morton sort, cells, lists) -> solve
A x = f B q to a 1e-6 relative residual with FP32-FMM GMRES inside FP64
iterative refinement -> solvation energy -> BIBEE/CFA energy -> adjoint
gradient (d dG/dq and d dG/dr).  K steps are timed after W warm-up steps.

`value` is the metric's quantity: FP32 A-matvec panels per second on the
last step's tree, N / median(t), with t the HIP-event time of one
bemfmm_fmm_matvec(A, FP32) (median of --matvec-reps after 3 warm-ups).
Also reported: the FP64 A-matvec rate, the plain FP64 and FP32-refined
times to a 1e-6 residual, the step throughput, sampled-row errors against
the FP64 dense oracle, the roofline of the dominant kernel from HIP events
on the stream it runs on (inside the timed steps), the BIBEE energy of the
1.31M-panel blobby surface against the oracle's full dense BIBEE, and the
oracle's own speed on the host cores (a reported baseline).

The JSON line also carries `extensions`: on the 1.31M-panel blobby surface,
the FP32 and FP64 A products with and without near quadrature (exact
close-pair integrals, nu = 2), and the linearised Poisson-Boltzmann
(screened solvent, kappa = 0.125/A) product, solve to 1e-6 and energy, with
the screened energy's parity against the dense oracle on the Kirkwood
sphere (5,120 panels).

Usage: python bench.py [--steps K] [--warmup W] [--config crowded|blobby|kirkwood|differentiation]
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

import numpy as np

METRIC = "BEM-FMM matvec panels/s + solve time to 1e-6 rel residual, FP32 vs FP64"
# MI355X published FP32 vector peak, the near field's roofline: a wave64
# FMA every 2 clocks per SIMD, 1024 SIMDs, 2.4 GHz.  An FP32 instruction that
# reads an SGPR issues at half that rate (78.6), reported beside it.
PEAK_FP32_VALU = 157.3e12
PEAK_FP32_ISSUE_MODEL = 78.6e12
PEAK_FP32_MFMA = 157.3e12    # dense FP32 MFMA
PEAK_HBM = 8.0e12            # MI355X HBM3E
P2P_FLOPS_PER_PAIR = 18      # K' monopole pair: 3 sub, 5 for r^2, 1 rsq, 3 mul, 6 for 3 FMA
M2L_FLOPS_PER_PAIR = 2 * 100 * 100   # dense p^2 x p^2 contraction at p = 10
# M2L pair at p = 10: the p^2 FP32 source coefficients in, the p^2 result
# coefficients out (its row of the pair-ordered output), two int32 indices
M2L_BYTES_PER_PAIR = 400 + 400 + 8
# library sources whose code decides the kernels' memory traffic
TRAFFIC_SOURCES = ("fmm.hip", "tree_build.hip", "common.h")


def kernel_source_hash(*paths):
    """SHA-256 of source files' code: comments and whitespace removed, so
    that only a change of the code itself invalidates measured figures."""
    import hashlib
    import re
    h = hashlib.sha256()
    for path in paths:
        text = open(path).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        text = re.sub(r"//[^\n]*", "", text)
        text = re.sub(r"\s+", "", text)
        h.update(text.encode())
    return h.hexdigest()


def library_source_hash():
    here = os.path.dirname(os.path.abspath(__file__))
    return kernel_source_hash(*[os.path.join(here, "paper_1007_4591_amd", "csrc", f) for f in TRAFFIC_SOURCES])


def pmc_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` from the committed hardware-counter
    summary of `workload`, or None when the library's code changed since it
    was taken."""
    here = os.path.dirname(os.path.abspath(__file__))
    path = os.path.join(here, "profiles", f"pmc_traffic_{workload}.md")
    if not os.path.exists(path):
        return None
    sha = library_source_hash()
    for line in open(path):
        if line.startswith("| `" + kernel + "`"):
            cells = [c.strip() for c in line.strip().strip("|").split("|")]
            # | kernel | fetch bytes | write bytes | total bytes | code sha256 | launches |
            if cells[4] == sha:
                return float(cells[3])
    return None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="crowded")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-rows", type=int, default=1024)
    ap.add_argument("--matvec-reps", type=int, default=20)
    ap.add_argument("--no-standalone", action="store_true", help="skip the standalone (near field in line) tree")
    ap.add_argument("--no-bibee-check", action="store_true",
                    help="skip the 1.31M-panel blobby BIBEE against the oracle's full dense BIBEE")
    ap.add_argument("--no-rows", action="store_true",
                    help="skip the near-quadrature and linearised Poisson-Boltzmann measurements")
    ap.add_argument("--calib-copy-mb", type=int, default=256,
                    help="size of a plain device copy run before the matvecs, the reference kernel for "
                         "hardware byte counters")
    return ap.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _event_ms(torch, fn, reps):
    """Median HIP-event time (ms) of fn() on the current stream over reps calls."""
    times = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        e1.synchronize()
        times.append(e0.elapsed_time(e1))
    return statistics.median(times)


def extension_rows(B, torch, synth, params, dev, no_oracle):
    """Near quadrature and linearised Poisson-Boltzmann on the blobby surface
    (1.31M panels), with their parity against the oracle on small cases."""
    import dataclasses
    pb = synth.config("blobby")
    N = pb.n_panels
    x = torch.as_tensor(np.random.default_rng(3).normal(size=N), device=dev)
    y = torch.empty_like(x)
    out = {"workload": f"blobby-L8: {N} panels, {pb.n_charges} charges, p=10, theta=0.5, ncrit=64"}
    # near quadrature: the same tree with and without the close-pair corrections
    nu = 2.0
    t0 = B.build_tree(pb.verts, pb.tris, pb.charge_pos, params)
    tq = B.build_tree(pb.verts, pb.tris, pb.charge_pos, dataclasses.replace(params, near_quad=nu))
    nq = {"nu": nu, "close_pairs": tq.info["n_nearquad_pairs"]}
    for prec, name in ((B.FP32, "fp32"), (B.FP64, "fp64")):
        for t, key in ((t0, "A_ms_one_point"), (tq, "A_ms_near_quad")):
            for _ in range(3):
                B.fmm_matvec(t, B.OP_A, prec, x, y)
            nq[f"{name}_{key}"] = _event_ms(torch, lambda: B.fmm_matvec(t, B.OP_A, prec, x, y), 10)
    if not no_oracle:
        # 64 sampled rows of the near-quadrature A against the dense oracle's
        # rows plus the corrections of those rows
        import oracle
        from oracle import panel_integrals as opi
        g = oracle.geometry(pb.verts, pb.tris)
        rows = np.sort(np.random.default_rng(5).choice(N, size=64, replace=False))
        xh = x.cpu().numpy()
        f = 1.0 - pb.eps_in / pb.eps_out
        corr = opi.kprime_correction_of(g, pb.verts, pb.tris, nu, rows, side="row")
        want = oracle.apply_A(g, f, xh, rows=rows) - f * opi.apply_correction(corr, xh, N)[rows]
        for prec, name in ((B.FP32, "fp32"), (B.FP64, "fp64")):
            B.fmm_matvec(tq, B.OP_A, prec, x, y)
            got = y.cpu().numpy()[rows]
            nq[f"{name}_rel_err_vs_oracle_64_rows"] = float(np.linalg.norm(got - want) / np.linalg.norm(want))
    B.tree_destroy(tq)
    out["near_quad"] = nq
    # linearised Poisson-Boltzmann, 150 mM (kappa = 0.125 / A)
    kappa = 0.125
    q = torch.as_tensor(pb.q, device=dev)
    uv = torch.as_tensor(np.random.default_rng(4).normal(size=2 * N), device=dev)
    yy = torch.empty_like(uv)
    s0 = time.perf_counter()
    B.lpb_matvec(t0, kappa, uv, yy)  # first call: per-level operators, lists, self integrals
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - s0
    mv_ms = _event_ms(torch, lambda: B.lpb_matvec(t0, kappa, uv, yy), 5)
    c0 = time.perf_counter()
    sol, info = B.lpb_solve(t0, q, kappa, tol=1e-6, maxit=300, restart=50)
    torch.cuda.synchronize()
    solve_s = time.perf_counter() - c0
    dG = B.lpb_energy(t0, q, sol)
    xs, _ = B.solve_bem(t0, q, tol=1e-6, maxit=300, precision=B.FP64)
    dG0 = B.solvation_energy(t0, q, xs, precision=B.FP64)
    B.tree_destroy(t0)
    lpb = {"kappa_per_A": kappa, "setup_s": setup_s, "matvec_ms": mv_ms, "unknowns": 2 * N,
           "unknowns_per_s": 2 * N / (mv_ms / 1e3), "solve_s": solve_s, "iters": info.iters,
           "rel_residual": info.rel_residual, "dG_kcal_mol": dG, "dG_unscreened_kcal_mol": dG0}
    if not no_oracle:
        # parity on a case the dense oracle solves: Kirkwood sphere L4, 100 charges
        import oracle
        from oracle import lpb as olpb
        pk = synth.kirkwood(4)
        g = oracle.geometry(pk.verts, pk.tris)
        S = olpb.LPB(g, pk.verts, pk.tris, pk.eps_in, pk.eps_out, kappa)
        o0 = time.perf_counter()
        want = S.energy(pk.charge_pos, pk.q, S.solve(pk.charge_pos, pk.q))
        o_s = time.perf_counter() - o0
        tk = B.build_tree(pk.verts, pk.tris, pk.charge_pos, params)
        qk = torch.as_tensor(pk.q, device=dev)
        sk, _ = B.lpb_solve(tk, qk, kappa, tol=1e-10, maxit=400, restart=60)
        got = B.lpb_energy(tk, qk, sk)
        B.tree_destroy(tk)
        lpb["parity_kirkwood_L4"] = {"gpu_kcal_mol": got, "oracle_kcal_mol": want, "rel_err": abs(got - want) / abs(want),
                                     "oracle_dense_solve_s": o_s}
    out["lpb"] = lpb
    return out


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build runs on one GPU only (the multi-GPU design is documented, not built); "
              "use --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch
    import synth
    import paper_1007_4591_amd as B

    if not torch.cuda.is_available():
        print("bench.py: no GPU", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    prob = synth.config(args.config)
    N, Q = prob.n_panels, prob.n_charges
    log(f"config={args.config} N={N} Q={Q}")
    verts = torch.as_tensor(prob.verts, device=dev)
    tris = torch.as_tensor(prob.tris, device=dev)
    cpos = torch.as_tensor(prob.charge_pos, device=dev)
    q = torch.as_tensor(prob.q, device=dev)
    params = B.Params(p=10, ncrit=64, theta=0.5, mac=B.MAC_THETA, eps_in=prob.eps_in, eps_out=prob.eps_out)
    TOL = 1e-6

    live = {"p2p": [0.0, 0], "m2l": [0.0, 0]}   # FP32 A products inside the timed steps

    build_ms = []   # build_tree wall time in the timed steps (it returns synchronised)

    def step(record=False, count=True):
        tb = time.perf_counter()
        t = B.build_tree(verts, tris, cpos, params)
        if count:
            build_ms.append(1000.0 * (time.perf_counter() - tb))
        if record:
            B.profile(t, True, True)
            B.profile_select(t, B.OP_A, B.FP32)  # other products record nothing
        x, info = B.solve_bem(t, q, tol=TOL, maxit=300, restart=30, precision=B.FP32_REFINED)
        dG = B.solvation_energy(t, q, x, precision=B.FP64)
        bib = B.bibee_energy(t, q, kind=B.BIBEE_CFA, precision=B.FP32)
        dq, dpos, ainfo = B.adjoint_grad(t, q, x, tol=TOL, maxit=300, restart=30, precision=B.FP32_REFINED)
        if record:
            for k in live:
                ms, n = B.profile_get(t, f"{k}/{B.OP_A}/{B.FP32}")
                if count:
                    live[k][0] += ms
                    live[k][1] += n
            B.profile(t, False, False)
        return t, x, info, ainfo, dG, bib

    last = None
    for _ in range(args.warmup):
        last = None
        last = step(record=True, count=False)  # the same work as a timed step, event records included
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    each = []
    for _ in range(args.steps):
        ts = time.perf_counter()
        # the previous step's tree is destroyed before the next is built, as
        # in the warm-up steps, so its device blocks return to the cache
        last = None
        last = step(record=True)
        torch.cuda.synchronize()  # a step ends in host reads already; this only closes its interval
        each.append(1000.0 * (time.perf_counter() - ts))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_per_step = 1000.0 * dt / args.steps
    tree, x, sinfo, ainfo, dG, bib = last
    log(f"step {ms_per_step:.2f} ms (each: {', '.join(f'{v:.1f}' for v in each)}) dG={dG:.6f} "
        f"bibee={bib:.6f} solve iters={sinfo.iters} outer={sinfo.outer_iters} adjoint iters={ainfo.iters}")

    # ---- a plain copy of known size (reference for FETCH_SIZE / WRITE_SIZE)
    if args.calib_copy_mb > 0:
        nel = args.calib_copy_mb * (1 << 20) // 4
        src = torch.ones(nel, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    # ---- matvec throughput (HIP events on the stream the product runs on)
    rng = np.random.default_rng(1)
    xv = torch.as_tensor(rng.normal(size=N), device=dev)
    yv = torch.empty(N, dtype=torch.float64, device=dev)
    mv = {}
    for prec, name in ((B.FP32, "fp32"), (B.FP64, "fp64")):
        for _ in range(3):
            B.fmm_matvec(tree, B.OP_A, prec, xv, yv)
        times = []
        for _ in range(args.matvec_reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            B.fmm_matvec(tree, B.OP_A, prec, xv, yv)
            e1.record()
            e1.synchronize()
            times.append(e0.elapsed_time(e1) / 1000.0)
        mv[name] = {"median_ms": 1000 * statistics.median(times), "panels_per_s": N / statistics.median(times),
                    "min_ms": 1000 * min(times), "max_ms": 1000 * max(times)}
    log(f"matvec {mv}")
    # per-stage times of the FP32 matvec
    B.profile(tree, True, True)
    nprof = 5
    for _ in range(nprof):
        B.fmm_matvec(tree, B.OP_A, B.FP32, xv, yv)
    stages = {s: B.profile_get(tree, s) for s in ("p2m", "m2m", "m2l", "l2l", "p2p", "l2p", "other")}
    B.profile(tree, False, True)
    log(f"stages(ms, count)={stages}")
    info = tree.info

    # ---- solve time to 1e-6: plain FP64 vs FP32-refined
    solves = {}
    for prec, name in ((B.FP64, "fp64"), (B.FP32_REFINED, "fp32_refined")):
        B.solve_bem(tree, q, tol=TOL, maxit=300, precision=prec)
        torch.cuda.synchronize()
        s0 = time.perf_counter()
        xs, si = B.solve_bem(tree, q, tol=TOL, maxit=300, precision=prec)
        torch.cuda.synchronize()
        solves[name] = {"seconds": time.perf_counter() - s0, "iters": si.iters, "outer": si.outer_iters,
                        "rel_residual": si.rel_residual,
                        "dG_kcal_mol": B.solvation_energy(tree, q, xs, precision=B.FP64)}
    solves["dG_rel_diff_refined_vs_fp64"] = abs(solves["fp32_refined"]["dG_kcal_mol"] - solves["fp64"]["dG_kcal_mol"]) \
        / abs(solves["fp64"]["dG_kcal_mol"])
    log(f"solves {solves}")

    # ---- error vs the FP64 dense oracle on sampled rows, and the oracle's speed
    err = {}
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        g = oracle.geometry(prob.verts, prob.tris)
        rows = np.sort(np.random.default_rng(2).choice(N, size=min(args.cpu_rows, N), replace=False))
        xh = xv.cpu().numpy()
        c0 = time.perf_counter()
        want = oracle.apply_A(g, 1.0 - prob.eps_in / prob.eps_out, xh, rows=rows)
        cpu_s = time.perf_counter() - c0
        for prec, name in ((B.FP32, "fp32"), (B.FP64, "fp64")):
            got = B.fmm_matvec(tree, B.OP_A, prec, xv).cpu().numpy()[rows]
            err[name] = float(np.linalg.norm(got - want) / np.linalg.norm(want))
        t_row = cpu_s / len(rows)
        cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
        omp = int(os.environ.get("OMP_NUM_THREADS", cores))
        cpu = {"value": 1.0 / t_row, "unit": "panels/s", "cores": min(cores, omp), "kind": "oracle",
               "sample": (f"{len(rows)} random rows of the dense FP64 A x (oracle, C + OpenMP) at N={N}: "
                          f"{cpu_s:.2f} s; value = rows/s = N / projected dense matvec time "
                          f"({t_row * N:.0f} s per product)")}
        del g
        log(f"sampled-row error vs oracle {err}; cpu {cpu}")

    # ---- roofline of the dominant kernels from the HIP events of the timed steps
    p2p_ms = live["p2p"][0] / max(live["p2p"][1], 1)
    m2l_ms = live["m2l"][0] / max(live["m2l"][1], 1)
    p2p_flops = info["p2p_pairs_panels"] * P2P_FLOPS_PER_PAIR
    m2l_flops = info["n_m2l_panel_pairs"] * M2L_FLOPS_PER_PAIR
    wl = args.config
    roof_p2p = {"bound": "alu", "kernel": "k_p2p_near<float,0,0,1> (near field of A, FP32, second stream)",
                "achieved": p2p_flops / (p2p_ms / 1e3) / 1e12, "peak": PEAK_FP32_VALU / 1e12, "unit": "TFLOP/s",
                "avg_ms": p2p_ms, "launches": live["p2p"][1],
                "traffic": pmc_traffic("k_p2p_near<float, 0, 0, 1>", wl)}
    roof_p2p["frac"] = roof_p2p["achieved"] / roof_p2p["peak"]
    roof_p2p["frac_of_issue_model"] = roof_p2p["achieved"] / (PEAK_FP32_ISSUE_MODEL / 1e12)
    # the M2L runs on the bf16 matrix cores (FP32 accuracy from split
    # operands), which are busy for a small part of its launch: it is bound
    # by the pair rows it streams, so its roofline is HBM; its useful FP32
    # flops are reported beside
    m2l_bytes = info["n_m2l_panel_pairs"] * M2L_BYTES_PER_PAIR
    roof_m2l = {"bound": "hbm", "kernel": "k_m2l_bf<7,25> (M2L, FP32 by split-bf16 MFMA, persistent)",
                "achieved": m2l_bytes / (m2l_ms / 1e3) / 1e9, "peak": PEAK_HBM / 1e9, "unit": "GB/s",
                "bytes_per_pair": M2L_BYTES_PER_PAIR, "avg_ms": m2l_ms, "launches": live["m2l"][1],
                "traffic": pmc_traffic("k_m2l_bf<7, 25>", wl),
                "useful_tflops": m2l_flops / (m2l_ms / 1e3) / 1e12}
    roof_m2l["frac"] = roof_m2l["achieved"] / roof_m2l["peak"]
    roof_m2l["useful_frac_of_fp32_mfma"] = roof_m2l["useful_tflops"] / (PEAK_FP32_MFMA / 1e12)
    roofline = roof_p2p if p2p_ms >= m2l_ms else roof_m2l
    tree_sizes = {k: info[k] for k in ("leaf_level", "n_cells", "n_leaves", "n_near_pairs", "n_far_pairs",
                                       "n_m2l_panel_pairs", "n_offsets", "p2p_pairs_panels")}
    # the timed tree goes before the next one is built (two trees of the
    # crowded system would not fit together)
    del tree, last, x
    torch.cuda.synchronize()

    # ---- the same kernels alone on the chip (near field not concurrent): a
    # second tree built with the concurrent near field switched off (the
    # library reads the switch at a tree's first product)
    if not args.no_standalone:
        os.environ["BEMFMM_CONCURRENT_P2P"] = "0"
        tree_alone = B.build_tree(verts, tris, cpos, params)
        for _ in range(3):
            B.fmm_matvec(tree_alone, B.OP_A, B.FP32, xv, yv)
        del os.environ["BEMFMM_CONCURRENT_P2P"]
        B.profile(tree_alone, True, True)
        for _ in range(nprof):
            B.fmm_matvec(tree_alone, B.OP_A, B.FP32, xv, yv)
        for r, stage, work, unit in ((roof_p2p, "p2p", p2p_flops, 1e12), (roof_m2l, "m2l", m2l_bytes, 1e9)):
            ms, n = B.profile_get(tree_alone, f"{stage}/{B.OP_A}/{B.FP32}")
            r["standalone_avg_ms"] = ms / max(n, 1)
            r["standalone_frac"] = work / (r["standalone_avg_ms"] / 1e3) / unit / r["peak"]
        B.profile(tree_alone, False, True)
        B.tree_destroy(tree_alone)
        del tree_alone
    del verts, tris, cpos, q, xv, yv
    torch.cuda.synchronize()

    # ---- BIBEE of the 1.31M-panel blobby surface against the oracle's full
    # dense BIBEE (B q and C x, N x Q sums each), and the oracle's time
    bibee_check = None
    if not args.no_bibee_check and not args.no_cpu_baseline:
        import oracle
        pb = synth.config("blobby")
        tb = B.build_tree(pb.verts, pb.tris, pb.charge_pos, params)
        qb = torch.as_tensor(pb.q, device=dev)
        g32 = B.bibee_energy(tb, qb, kind=B.BIBEE_CFA, precision=B.FP32)
        g64 = B.bibee_energy(tb, qb, kind=B.BIBEE_CFA, precision=B.FP64)
        B.tree_destroy(tb)
        gb = oracle.geometry(pb.verts, pb.tris)
        c0 = time.perf_counter()
        want = oracle.bibee_energy(gb, pb.charge_pos, pb.q, pb.eps_in, pb.eps_out, "cfa")
        ob_s = time.perf_counter() - c0
        bibee_check = {"workload": f"blobby-L8: {pb.n_panels} panels, {pb.n_charges} charges", "oracle_kcal_mol": want,
                       "oracle_seconds": ob_s, "fp32_kcal_mol": g32, "fp64_kcal_mol": g64,
                       "fp32_rel_err": abs(g32 - want) / abs(want), "fp64_rel_err": abs(g64 - want) / abs(want)}
        log(f"bibee check {bibee_check}")

    # ---- the extensions on the 1.31M-panel blobby surface: near quadrature
    # (exact close-pair integrals) and the linearised Poisson-Boltzmann solve
    rows = None
    if not args.no_rows:
        rows = extension_rows(B, torch, synth, params, dev, args.no_cpu_baseline)
        log(f"extension rows {rows}")

    out = {
        "metric": METRIC, "value": mv["fp32"]["panels_per_s"], "unit": "panels/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "ms_each_step": [round(v, 2) for v in each], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{prob.name}: {N} panels, {Q} charges, eps 4/80, p=10, theta=0.5, ncrit=64; "
                               "value = N / t(FP32 A matvec); step = tree build + FP32-refined solve to 1e-6 + "
                               "energy + BIBEE + adjoint",
                   "panels": N, "charges": Q},
        "step_panels_per_s": N / (ms_per_step / 1e3),
        "matvec": {k: {"panels_per_s": v["panels_per_s"], "ms": v["median_ms"], "min_ms": v["min_ms"],
                       "max_ms": v["max_ms"], "rel_err_vs_oracle": err.get(k)} for k, v in mv.items()},
        "solve_to_1e-6": solves,
        "energies": {"dG_kcal_mol": dG, "bibee_cfa_kcal_mol": bib},
        "bibee_vs_dense_oracle": bibee_check,
        "stages_ms_per_matvec_fp32": {k: v[0] / max(v[1], 1) for k, v in stages.items()},
        "tree": tree_sizes,
        "build_tree": ({"median_ms": statistics.median(build_ms), "min_ms": min(build_ms), "max_ms": max(build_ms),
                        "steps": len(build_ms), "note": "bemfmm_build_tree wall time inside the timed steps (it "
                        "returns synchronised); part of ms_per_step"} if build_ms else None),
        "roofline": roofline,
        "roofline_other": roof_m2l if roofline is roof_p2p else roof_p2p,
        "cpu_baseline": cpu,
        "extensions": rows,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
