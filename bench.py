"""Benchmark: QB time-to-tolerance of randQB_FP on one MI355X.

Workload (synthetic, seeded): dense FP64 A = U diag(sigma) V^T + noise, 20000 x 15000,
sigma_j = exp(-j/150) on 3000 Haar columns, iid N(0, (1e-8)^2) noise, block size b = 64,
relative Frobenius tolerance 1e-3.  One step is one full call of the library's randQB_FP
(||A||^2, Omega, G = A Omega, H = A^T G, block loop to the tolerance, restarts) with A
already resident in HBM.  The headline uses the adaptive chunk schedule (l_tilde = -1:
8 b Omega columns first, later chunks sized from the decay of E, at most 50 b); the
paper's fixed l~ = 50 b rule (Section 5.4) and randQB_EI are timed beside it on the same
matrix, and so is trQRCP (randomized QR with column pivoting) stopped by the same
indicator (Remark 3.2).

Precision form (reported beside the headline, in "precision"): the 32768 x 32768 matrix
with sigma_j = j^-1.5 (b = 128, tol 1e-2) factorised once from its binary64 storage by the
FP64 path and once from its bfloat16 storage by the precision form (bfloat16 sketch
products on MFMA with FP32 accumulation, binary64 block loop), same Omega and schedule;
both times and both achieved errors against the binary64 matrix, and the roofline of the
bfloat16 sketch GEMMs against the 2.5 PFLOP/s dense BF16 peak.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] [--no-precision]

Prints one JSON line.  value = median time-to-tolerance in seconds (lower is better).
roofline: the dominant kernel (the larger of the two FP64 MFMA sketch GEMMs, G = A Omega
or H = A^T G) -- algorithmic flops 2 m n l~ per launch over its average launch time,
measured with HIP events recorded by the library on the stream the GEMM runs on;
MI355X FP64 matrix peak 78.6 TFLOP/s.  Its traffic (HBM bytes per launch) and MFMA busy
percentage come from three rocprofv3 counter passes (FETCH_SIZE, WRITE_SIZE, MfmaUtil) over
one call of the same workload in a child process, each counter scaled by what it reads for a
library kernel of exactly 1 GiB of traffic (skip with --no-counters).  cpu_baseline: the
FP64 oracle (NumPy/OpenBLAS) on the same workload on the host cores, median of 5 runs, with
the oracle's times on the other workloads beside it.
"""
from __future__ import annotations

import argparse
import json

import numpy as np
import os
import re
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6
FP32_PEAK_TFLOPS = 157.3
BF16_PEAK_TFLOPS = 2500.0
FP8_PEAK_TFLOPS = 5000.0
HBM_PEAK_GBPS = 8000.0


def block_loop_work(m, n, b, rank, blocks, ei=False):
    """Algorithmic flops and HBM bytes of the block loop (FP64, without the products with A).
    Block i starts at rank k_i = i b (the last block may stop early).  randQB_FP per block:
    W = B Omega_J and S = H_J^T - D^T B read B (k x n) twice; Y = G_J - Q W, D = Q^T Y,
    Z = Q^T Q_i and Q_i - Q Z read Q (m x k) four times: 8 m k b + 4 n k b flops, plus the
    b-column CholeskyQR pair and B_i = S R_i^{-1} (8 m b^2 + 2 n b^2).  randQB_EI drops D and
    S: Q is read three times and B once."""
    flops = bytes_ = 0.0
    for i in range(blocks):
        k = min(i * b, rank)
        if ei:
            flops += 6.0 * m * k * b + 2.0 * n * k * b + 8.0 * m * b * b
            bytes_ += 8.0 * (3.0 * m * k + n * k)
        else:
            flops += 8.0 * m * k * b + 4.0 * n * k * b + 8.0 * m * b * b + 2.0 * n * b * b
            bytes_ += 8.0 * (4.0 * m * k + 2.0 * n * k)
    return flops, bytes_


def end_to_end_roofline(m, n, b, r):
    """Sum over the phases of a dense randQB_FP call of the time each would take at its
    roofline (||A||^2 and Omega at HBM speed, the sketch GEMMs and the block loop at the FP64
    matrix peak or HBM, whichever binds), divided by the call's device time."""
    w_tot = r.gemm_flops[0] / (2.0 * m * n)
    t = 8.0 * m * n / (HBM_PEAK_GBPS * 1e9)                                  # ||A||^2
    t += 8.0 * n * w_tot / (HBM_PEAK_GBPS * 1e9)                             # Omega
    t += (r.gemm_flops[0] + r.gemm_flops[1]) / (FP64_PEAK_TFLOPS * 1e12)     # G, H
    f, by = block_loop_work(m, n, b, r.rank, r.blocks)
    t += max(f / (FP64_PEAK_TFLOPS * 1e12), by / (HBM_PEAK_GBPS * 1e9))      # block loop
    return round(t / (r.ms[5] * 1e-3), 4) if r.ms[5] > 0 else None


def block_loop_roofline(m, n, b, r, ei=False):
    """Achieved rates of the block loop against the FP64 matrix and HBM peaks (the loop's
    Q and B sweeps sit near the ridge point: about b / 4 flops per byte)."""
    f, by = block_loop_work(m, n, b, r.rank, r.blocks, ei)
    t = r.ms[4] * 1e-3
    if t <= 0:
        return None
    return {"flops": f, "bytes": by, "TFLOPs": round(f / t / 1e12, 2), "GBps": round(by / t / 1e9, 1),
            "frac_fp64": round(f / t / 1e12 / FP64_PEAK_TFLOPS, 4),
            "frac_hbm": round(by / t / 1e9 / HBM_PEAK_GBPS, 4)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-ei", action="store_true")
    ap.add_argument("--no-precision", action="store_true")
    ap.add_argument("--no-diff", action="store_true")
    ap.add_argument("--no-sparse", action="store_true")
    ap.add_argument("--no-power", action="store_true")
    ap.add_argument("--no-trqrcp", action="store_true")
    ap.add_argument("--no-onepass", action="store_true")
    ap.add_argument("--onepass-only", action="store_true",
                    help="only one call of each sketch sweep (two-pass, single-pass) at l = 1024, for counters")
    ap.add_argument("--sparse-only", action="store_true",
                    help="run only the CSR block and print its JSON (for profiling runs)")
    ap.add_argument("--precision-only", action="store_true",
                    help="run only the precision-form block and print its JSON (for profiling runs)")
    ap.add_argument("--no-counters", action="store_true",
                    help="skip the rocprofv3 counter passes (HBM traffic, MFMA busy) of the dominant kernel")
    ap.add_argument("--counter-probe", action="store_true",
                    help=argparse.SUPPRESS)   # the program the counter passes run
    ap.add_argument("--gen-device", default="cuda", choices=["cuda", "cpu"],
                    help="where the seeded test matrix is generated (cpu keeps the GPU QR of the "
                         "generator out of counter-collection runs)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run one plain 1 GiB device copy first (scale for HBM counter runs)")
    ap.add_argument("--l-tilde", type=int, default=-1,
                    help="headline chunk schedule (-1: adaptive, 0: paper rule 50 b, >0: fixed)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); this build has no "
              "multi-GPU path", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1606_09402_amd as qb
    import workloads as W

    if args.counter_probe:
        counter_probe(qb, W, torch, args.l_tilde)
        return
    if args.sparse_only:
        print(json.dumps({"sparse": sparse_block(qb, W, torch)}), flush=True)
        return
    if args.precision_only:
        print(json.dumps({"precision": precision_block(qb, W, torch, max(1, min(args.steps, 5)), args.l_tilde,
                                                       args.gen_device)}), flush=True)
        return
    wl = W.C2
    seed = W.SEED_OMEGA | 2
    dev = torch.device("cuda:0")
    t0 = time.time()
    A = wl.make(device=dev if args.gen_device == "cuda" else "cpu").to(dev)
    torch.cuda.synchronize()
    print(f"# generated {wl.name} on the GPU in {time.time() - t0:.1f} s", file=sys.stderr, flush=True)
    if args.onepass_only:
        ows = torch.empty(qb.qb_sketch_onepass_bytes_for(A, 1024), dtype=torch.uint8, device=dev)
        torch.cuda.synchronize()
        qb.qb_sketch_dense(A, seed, 0, 1024)
        torch.cuda.synchronize()
        qb.qb_sketch_onepass(A, seed, 0, 1024, ws=ows)
        torch.cuda.synchronize()
        print(json.dumps({"onepass_only": {"l": 1024, "calls": 1}}), flush=True)
        return
    m, n = A.shape
    l_max = min(m, n)
    Qs = torch.empty((l_max, m), dtype=torch.float64, device=dev)
    Bs = torch.empty((l_max, n), dtype=torch.float64, device=dev)
    need = max(qb.qb_workspace_bytes(qb.QB_ALGO_FP, False, m, n, 0, wl.tol, wl.b, l_max, args.l_tilde),
               qb.qb_workspace_bytes(qb.QB_ALGO_FP, False, m, n, 0, wl.tol, wl.b, l_max, args.l_tilde, 1),
               qb.qb_workspace_bytes(qb.QB_ALGO_EI, False, m, n, 0, wl.tol, wl.b, l_max))
    ws = torch.empty(need, dtype=torch.uint8, device=dev)

    def fp(l_tilde=args.l_tilde, power=0):
        return qb.qb_fp_dense(A, wl.tol, wl.b, seed, l_max=l_max, l_tilde=l_tilde,
                              Q_store=Qs, B_store=Bs, ws=ws, power=power)

    def ei():
        return qb.qb_ei_dense(A, wl.tol, wl.b, seed, l_max=l_max, Q_store=Qs, B_store=Bs, ws=ws)

    if args.calib_copy:   # 2^27 doubles read and written once: 1 GiB each way
        src = torch.ones(2 ** 27, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    for i in range(args.warmup):
        r = fp()
        print(f"# warmup {i}: rank {r.rank} E {r.E:.4e} {r.ms[5]:.1f} ms", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    times, results = [], []
    t_all = time.perf_counter()
    for i in range(args.steps):
        t = time.perf_counter()
        r = fp()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t)
        results.append(r)
        print(f"# step {i}: {times[-1] * 1e3:.2f} ms rank {r.rank}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_all
    r = results[-1]
    med = statistics.median(times)

    # dominant kernel: the sketch GEMM with the larger share of device time.  Per launch:
    # 2 m n w algorithmic flops over the launch's device time (HIP events the library
    # records on the stream the GEMM runs on); averaged over the chunks of a call.
    g_ms = statistics.median(x.ms[2] for x in results) / max(1, r.chunks)
    h_ms = statistics.median(x.ms[3] for x in results) / max(1, r.chunks)
    flops_per_launch = r.gemm_flops[0] / max(1, r.chunks)
    dom_ms, dom_name = (h_ms, "gemm_f64 H=A^T G") if h_ms >= g_ms else (g_ms, "gemm_f64 G=A Omega")
    achieved = flops_per_launch / (dom_ms * 1e-3) / 1e12
    schedule = {-1: "adaptive (8b first, <= 50b)", 0: "paper rule 50b"}.get(args.l_tilde,
                                                                          str(args.l_tilde))

    # accuracy of the returned factorisation (verification, not timed)
    Q = r.Q
    Bm = r.B
    res2 = float(torch.linalg.matrix_norm(A - Q @ Bm) ** 2)
    true_rel = (res2 / r.normA2) ** 0.5

    # eq. (3) on the returned factorisation: the SVD of B and U = Q U~ (not part of the
    # time-to-tolerance)
    svd_ws = torch.empty(qb.qb_svd_workspace_bytes(m, n, r.rank), dtype=torch.uint8, device=dev)
    sv_t = []
    for _ in range(2):
        t = time.perf_counter()
        sv = qb.svd_from_qb(Q, Bm, ws=svd_ws)
        torch.cuda.synchronize()
        sv_t.append(time.perf_counter() - t)
    svd_entry = {"time_s": round(min(sv_t), 6), "k": r.rank, "sweeps": sv.sweeps,
                 "s_top5": [round(float(x), 6) for x in sv.s[:5].cpu()]}
    del svd_ws, sv
    print(f"# svd from QB: {min(sv_t) * 1e3:.1f} ms (k {r.rank}, {svd_entry['sweeps']} sweeps)",
          file=sys.stderr, flush=True)

    out = {
        "metric": "QB time-to-tol (s)",
        "value": round(med, 6),
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 3),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": wl.name, "m": m, "n": n, "b": wl.b, "tol": wl.tol,
                   "l_tilde": schedule, "algo": "randQB_FP", "power": 0},
        "rank": r.rank,
        "E_rel": (max(r.E, 0.0) / r.normA2) ** 0.5,
        "true_rel_err": true_rel,
        "passes": r.passes,
        "chunks": r.chunks,
        "blocks": r.blocks,
        "phase_ms": {"normA2": r.ms[0], "omega": r.ms[1], "G": r.ms[2], "H": r.ms[3],
                     "block_loop": r.ms[4], "total": r.ms[5]},
        "sketch_tflops": (r.gemm_flops[0] + r.gemm_flops[1]) / ((r.ms[2] + r.ms[3]) * 1e-3) / 1e12,
        "block_loop_roofline": block_loop_roofline(m, n, wl.b, r),
        "end_to_end_roofline_frac": end_to_end_roofline(m, n, wl.b, r),
        "svd_from_qb": svd_entry,
        "roofline": {"bound": "mfma", "kernel": dom_name, "achieved": round(achieved, 3),
                     "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(achieved / FP64_PEAK_TFLOPS, 4), "traffic": None},
    }
    if not args.no_counters:
        # HBM bytes and MFMA busy of the same kernel, from rocprofv3 counter passes over one
        # call of the same workload run as a child process (measure_counters)
        cnt = measure_counters(args.l_tilde)
        out["counters"] = cnt
        key = "H" if dom_name.startswith("gemm_f64 H") else "G"
        # algorithmic bytes per launch, 8 (m n + (m + n) w) for the mean chunk width w
        w_mean = r.gemm_flops[0] / (2.0 * m * n) / max(1, r.chunks)
        alg = 8.0 * (m * n + (m + n) * w_mean)
        cnt["algorithmic_bytes_per_launch"] = int(alg)
        if cnt.get("traffic_bytes", {}).get(key) is not None:
            out["roofline"]["traffic"] = int(cnt["traffic_bytes"][key])
            out["roofline"]["traffic_over_algorithmic"] = round(cnt["traffic_bytes"][key] / alg, 3)
        if cnt.get("mfma_util_pct", {}).get(key) is not None:
            out["roofline"]["mfma_busy_pct"] = cnt["mfma_util_pct"][key]
    if args.l_tilde != 0:   # the paper's fixed l~ = 50 b beside the headline schedule
        fp(0)
        pt = []
        for _ in range(max(1, min(args.steps, 3))):
            t = time.perf_counter()
            rp = fp(0)
            torch.cuda.synchronize()
            pt.append(time.perf_counter() - t)
        out["paper_rule"] = {"time_to_tol_s": round(statistics.median(pt), 6), "rank": rp.rank,
                             "l_tilde": 50 * wl.b, "passes": rp.passes,
                             "sketch_tflops": (rp.gemm_flops[0] + rp.gemm_flops[1])
                             / ((rp.ms[2] + rp.ms[3]) * 1e-3) / 1e12,
                             "phase_ms": {"G": rp.ms[2], "H": rp.ms[3], "block_loop": rp.ms[4],
                                          "total": rp.ms[5]}}
        print(f"# paper rule: {statistics.median(pt) * 1e3:.1f} ms rank {rp.rank}", file=sys.stderr,
              flush=True)
    if not args.no_power:   # Algorithm 4's power scheme, P = 1, same schedule
        fp(power=1)
        torch.cuda.synchronize()
        pw = []
        for _ in range(max(1, min(args.steps, 3))):
            t = time.perf_counter()
            rq = fp(power=1)
            torch.cuda.synchronize()
            pw.append(time.perf_counter() - t)
        res2 = float(torch.linalg.matrix_norm(A - rq.Q @ rq.B) ** 2)
        out["power1"] = {"time_to_tol_s": round(statistics.median(pw), 6), "rank": rq.rank,
                         "true_rel_err": (res2 / rq.normA2) ** 0.5, "passes": rq.passes,
                         "chunks": rq.chunks, "fallbacks": rq.fallbacks,
                         "phase_ms": {"power_rounds": rq.ms[6], "G": rq.ms[2], "H": rq.ms[3],
                                      "block_loop": rq.ms[4], "total": rq.ms[5]}}
        print(f"# power 1: {statistics.median(pw) * 1e3:.1f} ms rank {rq.rank} passes {rq.passes}",
              file=sys.stderr, flush=True)
    # the 1000 x 800 matrix (sigma_j = j^-2, b = 20, tol 1e-2): latency-bound, wall time only
    c1 = W.C1.make().to(dev)
    s1 = W.SEED_OMEGA | 1
    c1_ws = torch.empty(max(qb.qb_workspace_bytes(qb.QB_ALGO_FP, False, W.C1.m, W.C1.n, 0, W.C1.tol, W.C1.b,
                                                  min(W.C1.m, W.C1.n)),
                            qb.qb_workspace_bytes(qb.QB_ALGO_EI, False, W.C1.m, W.C1.n, 0, W.C1.tol, W.C1.b,
                                                  min(W.C1.m, W.C1.n))), dtype=torch.uint8, device=dev)
    c1_out = {"workload": W.C1.name}
    for nm, fn in (("fp", lambda: qb.qb_fp_dense(c1, W.C1.tol, W.C1.b, s1, ws=c1_ws)),
                   ("ei", lambda: qb.qb_ei_dense(c1, W.C1.tol, W.C1.b, s1, ws=c1_ws))):
        fn()
        torch.cuda.synchronize()
        tt = []
        for _ in range(20):
            t = time.perf_counter()
            rc1 = fn()
            torch.cuda.synchronize()
            tt.append(time.perf_counter() - t)
        c1_out[nm] = {"time_to_tol_s": round(statistics.median(tt), 6), "rank": rc1.rank,
                      "E_rel": (max(rc1.E, 0.0) / rc1.normA2) ** 0.5, "passes": rc1.passes, "runs": 20}
    out["c1"] = c1_out
    print(f"# 1000x800: fp {c1_out['fp']['time_to_tol_s'] * 1e3:.2f} ms, ei {c1_out['ei']['time_to_tol_s'] * 1e3:.2f} ms",
          file=sys.stderr, flush=True)
    del c1, c1_ws
    if not args.no_ei:
        ei()
        torch.cuda.synchronize()
        et = []
        for _ in range(max(1, min(args.steps, 3))):
            t = time.perf_counter()
            re_ = ei()
            torch.cuda.synchronize()
            et.append(time.perf_counter() - t)
        ei_tf = re_.gemm_flops[1] / (re_.ms[3] * 1e-3) / 1e12 if re_.ms[3] > 0 else None
        out["ei"] = {"time_to_tol_s": round(statistics.median(et), 6), "rank": re_.rank,
                     "passes": re_.passes, "blocks": re_.blocks,
                     "roofline": {"bound": "mfma", "kernel": "gemm_f64 A^T Q_i (all blocks)",
                                  "achieved": ei_tf, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                                  "frac": ei_tf / FP64_PEAK_TFLOPS if ei_tf else None},
                     "phase_ms": {"A_Omega_i": re_.ms[2], "At_Q_i": re_.ms[3], "total": re_.ms[5]}}
        print(f"# ei: {statistics.median(et) * 1e3:.1f} ms rank {re_.rank} passes {re_.passes}",
              file=sys.stderr, flush=True)
    if not args.no_trqrcp:   # trQRCP driven by the same indicator (Remark 3.2), same matrix
        def qrcp():
            return qb.qb_trqrcp_dense(A, wl.tol, wl.b, seed, oversample=8, Q_store=Qs, B_store=Bs)
        qrcp()
        torch.cuda.synchronize()
        qt = []
        for _ in range(max(1, min(args.steps, 3))):
            t = time.perf_counter()
            rc = qrcp()
            torch.cuda.synchronize()
            qt.append(time.perf_counter() - t)
        res3 = float(torch.linalg.matrix_norm(A - rc.Q @ rc.B) ** 2)
        out["trqrcp"] = {"time_to_tol_s": round(statistics.median(qt), 6), "rank": rc.rank,
                         "true_rel_err": (res3 / rc.normA2) ** 0.5, "oversample": 8,
                         "passes": rc.passes, "blocks": rc.blocks,
                         "bi_gemm_tflops": rc.gemm_flops[1] / (rc.ms[3] * 1e-3) / 1e12 if rc.ms[3] > 0 else None,
                         "roofline": {"bound": "mfma", "kernel": "gemm_f64 B_i = Q_i^T A (all blocks)",
                                      "achieved": rc.gemm_flops[1] / (rc.ms[3] * 1e-3) / 1e12 if rc.ms[3] > 0 else None,
                                      "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                                      "frac": rc.gemm_flops[1] / (rc.ms[3] * 1e-3) / 1e12 / FP64_PEAK_TFLOPS
                                      if rc.ms[3] > 0 else None},
                         "phase_ms": {"sketch": rc.ms[2], "At_Q_i": rc.ms[3],
                                      "pivots_and_blocks": rc.ms[4], "total": rc.ms[5]}}
        print(f"# trqrcp: {statistics.median(qt) * 1e3:.1f} ms rank {rc.rank} passes {rc.passes} "
              f"phases {rc.ms[2]:.2f}/{rc.ms[3]:.2f}/{rc.ms[4]:.2f}", file=sys.stderr, flush=True)

    if not args.no_onepass:   # the single-pass sketch sweep (Remark 4.2) beside the two-pass one
        w1 = 1024
        tp, to = [], []
        ows = torch.empty(qb.qb_sketch_onepass_bytes_for(A, w1), dtype=torch.uint8, device=dev)
        for it in range(4):
            torch.cuda.synchronize()
            t = time.perf_counter()
            qb.qb_sketch_dense(A, seed, 0, w1)
            torch.cuda.synchronize()
            tp.append(time.perf_counter() - t)
            t = time.perf_counter()
            qb.qb_sketch_onepass(A, seed, 0, w1, ws=ows)
            torch.cuda.synchronize()
            to.append(time.perf_counter() - t)
        del ows
        out["onepass"] = {"l": w1, "two_pass_s": round(statistics.median(tp[1:]), 6),
                          "one_pass_s": round(statistics.median(to[1:]), 6)}
        print(f"# sketch sweep l={w1}: two-pass {statistics.median(tp[1:]) * 1e3:.2f} ms, "
              f"one-pass {statistics.median(to[1:]) * 1e3:.2f} ms", file=sys.stderr, flush=True)

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(A, wl, seed, args.l_tilde)
    if not args.no_precision:
        del A, Qs, Bs, ws
        torch.cuda.empty_cache()
        out["precision"] = precision_block(qb, W, torch, max(1, min(args.steps, 5)), args.l_tilde,
                                           args.gen_device)
    if not args.no_diff:
        out["diff"] = diff_block(qb, W, torch, max(1, min(args.steps, 5)))
    if not args.no_sparse:
        out["sparse"] = sparse_block(qb, W, torch)
    print(json.dumps(out), flush=True)


def precision_block(qb, W, torch, steps, l_tilde, gen_device="cuda"):
    """BF16 precision form against the FP64 path on the 32768 x 32768 workload."""
    import statistics

    wl = W.C4
    seed = W.SEED_OMEGA | 4
    dev = torch.device("cuda:0")
    t0 = time.time()
    A64 = wl.make(device=dev if gen_device == "cuda" else "cpu").to(dev)
    Aq = W.to_bf16(A64)
    torch.cuda.synchronize()
    print(f"# generated {wl.name} in {time.time() - t0:.1f} s", file=sys.stderr, flush=True)
    m, n = A64.shape
    l_max = min(m, n)
    Qs = torch.empty((l_max, m), dtype=torch.float64, device=dev)
    Bs = torch.empty((l_max, n), dtype=torch.float64, device=dev)
    need = max(qb.qb_dense_workspace_bytes(qb.QB_ALGO_FP, X, wl.tol, wl.b, l_max, l_tilde)
               for X in (A64, Aq))
    ws = torch.empty(need, dtype=torch.uint8, device=dev)
    a64_norm = float(torch.linalg.matrix_norm(A64))
    A8, e8, _ = W.to_e4m3_rows(A64)
    res = {}
    # e4m3 storage: its rounding error (2.6e-2 of ||A||) lies above tol 1e-2, so it runs at
    # tol 5e-2 and the FP64 path is timed again at the error the e4m3 run achieved
    for name, X, tol, rexp in (("f64", A64, wl.tol, None), ("bf16", Aq, wl.tol, None),
                               ("fp8_e4m3", A8, 5e-2, e8), ("f64_at_fp8_error", A64, None, None)):
        if tol is None:
            tol = res["fp8_e4m3"]["true_rel_err"]
        run = lambda: qb.qb_fp_dense(X, tol, wl.b, seed, l_max=l_max, l_tilde=l_tilde,
                                     Q_store=Qs, B_store=Bs, ws=ws, row_exp=rexp)
        run()
        torch.cuda.synchronize()
        ts, rs = [], []
        for _ in range(steps):
            t = time.perf_counter()
            r = run()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t)
            rs.append(r)
        r = rs[-1]
        true_rel = float(torch.linalg.matrix_norm(A64 - r.Q @ r.B)) / a64_norm
        g_ms = statistics.median(x.ms[2] for x in rs) / max(1, r.chunks)
        h_ms = statistics.median(x.ms[3] for x in rs) / max(1, r.chunks)
        per_launch = r.gemm_flops[0] / max(1, r.chunks)
        peak = FP64_PEAK_TFLOPS if name.startswith("f64") else BF16_PEAK_TFLOPS
        dom_ms = max(g_ms, h_ms)
        achieved = per_launch / (dom_ms * 1e-3) / 1e12
        gemms = None
        if name == "fp8_e4m3":
            # G on the 8-bit matrix cores (e4m3 x e4m3, 5.0 PFLOP/s dense), H on bfloat16 ones
            gemms = {"G": {"kernel": "gemm_f8 (MFMA 32x32x64 f8f6f4, e4m3 A and Omega_q, FP32 acc)",
                           "ms_per_launch": g_ms, "tflops": round(per_launch / (g_ms * 1e-3) / 1e12, 2),
                           "peak_tflops": FP8_PEAK_TFLOPS,
                           "frac": round(per_launch / (g_ms * 1e-3) / 1e12 / FP8_PEAK_TFLOPS, 4)},
                     "H": {"kernel": "gemm_bf16 (MFMA 32x32x16 bf16, e4m3 A widened on load)",
                           "ms_per_launch": h_ms, "tflops": round(per_launch / (h_ms * 1e-3) / 1e12, 2),
                           "peak_tflops": BF16_PEAK_TFLOPS,
                           "frac": round(per_launch / (h_ms * 1e-3) / 1e12 / BF16_PEAK_TFLOPS, 4)}}
        elif name == "bf16":
            gemms = {k: {"ms_per_launch": t_, "tflops": round(per_launch / (t_ * 1e-3) / 1e12, 2),
                         "peak_tflops": BF16_PEAK_TFLOPS,
                         "frac": round(per_launch / (t_ * 1e-3) / 1e12 / BF16_PEAK_TFLOPS, 4)}
                     for k, t_ in (("G", g_ms), ("H", h_ms))}
        res[name] = {"tol": tol, "time_to_tol_s": round(statistics.median(ts), 6), "rank": r.rank,
                     "true_rel_err": true_rel, "E_rel": (max(r.E, 0.0) / r.normA2) ** 0.5,
                     "passes": r.passes, "chunks": r.chunks,
                     "phase_ms": {"normA2": r.ms[0], "omega": r.ms[1], "G": r.ms[2], "H": r.ms[3],
                                  "block_loop": r.ms[4], "total": r.ms[5]},
                     "sketch_gemm": {"kernel": "gemm_f64 (MFMA 16x16x4 f64)" if name.startswith("f64")
                                     else "gemm_bf16 (MFMA 32x32x16 bf16, FP32 acc)"
                                     if name == "bf16" else "G: gemm_f8 (MFMA 32x32x64 e4m3), "
                                     "H: gemm_bf16 (e4m3 A widened on load); rate of the slower launch "
                                     "against the BF16 peak",
                                     "G_ms_per_launch": g_ms, "H_ms_per_launch": h_ms,
                                     "achieved_tflops": round(achieved, 2), "peak_tflops": peak,
                                     "frac": round(achieved / peak, 4)}}
        if gemms is not None:
            res[name]["sketch_gemms"] = gemms
        print(f"# precision {name}: {statistics.median(ts) * 1e3:.2f} ms rank {r.rank} "
              f"true rel {true_rel:.4e}", file=sys.stderr, flush=True)
    res["workload"] = wl.name
    res["schedule"] = {-1: "adaptive (8b first, <= 50b)", 0: "paper rule 50b"}.get(l_tilde, str(l_tilde))
    res["speedup_bf16_vs_f64"] = round(res["f64"]["time_to_tol_s"] / res["bf16"]["time_to_tol_s"], 3)
    res["speedup_fp8_vs_f64_at_fp8_error"] = round(
        res["f64_at_fp8_error"]["time_to_tol_s"] / res["fp8_e4m3"]["time_to_tol_s"], 3)
    res["note"] = ("all runs factorise the same binary64 matrix (bf16 / fp8_e4m3: its bfloat16 / "
                   "row-scaled e4m3 storage); true_rel_err is ||A - QB||_F / ||A||_F against the "
                   "binary64 A; f64_at_fp8_error runs the FP64 path at the error the e4m3 run achieved")
    del A64, Aq, A8, e8, Qs, Bs, ws
    torch.cuda.empty_cache()
    return res


def diff_block(qb, W, torch, steps):
    """Differentiation form: fixed-rank randQB_FP forward and the hand-written backward on
    the 64 x 2048 x 1024 binary32 batch (k = 128, b = 32), with fixed random adjoints."""
    import statistics

    wl = W.C5
    seed = W.SEED_OMEGA | 5
    dev = torch.device("cuda:0")
    A = wl.make(device=dev)
    g = torch.Generator(device=dev)
    g.manual_seed(5)
    dQ = torch.randn((wl.batch, wl.m, wl.k), generator=g, device=dev, dtype=torch.float32)
    dB = torch.randn((wl.batch, wl.k, wl.n), generator=g, device=dev, dtype=torch.float32)
    ws = torch.empty(qb.qb_fixed_rank_workspace_bytes(A, wl.k, wl.b), dtype=torch.uint8, device=dev)
    flag = torch.zeros(1, dtype=torch.int32, device=dev)
    Q, B = qb.qb_fixed_rank_fwd(A, wl.k, wl.b, seed, ws=ws, breakdown=flag)
    qb.qb_fixed_rank_bwd(A, wl.k, wl.b, seed, Q, dQ, dB, ws=ws)
    torch.cuda.synchronize()
    tf, tb = [], []
    for _ in range(steps):
        t = time.perf_counter()
        Q, B = qb.qb_fixed_rank_fwd(A, wl.k, wl.b, seed, ws=ws, breakdown=flag)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        qb.qb_fixed_rank_bwd(A, wl.k, wl.b, seed, Q, dQ, dB, ws=ws)
        torch.cuda.synchronize()
        tb.append(time.perf_counter() - t1)
        tf.append(t1 - t)
    bt, m, n, k, b = wl.batch, wl.m, wl.n, wl.k, wl.b
    sk = b * (k // b) * (k // b - 1) // 2            # sum of the ranks before each block
    f_fwd = bt * (4.0 * m * n * k + 2.0 * (4 * m + 2 * n) * b * sk + 2.0 * (4 * m + n) * b * k
                  + 4.0 * b * b * k)
    f_bwd = bt * (8.0 * m * n * k + 8.0 * m * k * k)
    mf, mb = statistics.median(tf), statistics.median(tb)
    res = {"workload": wl.name, "dtype": "f32", "forward_ms": round(mf * 1e3, 3),
           "backward_ms": round(mb * 1e3, 3), "step_ms": round((mf + mb) * 1e3, 3),
           "forward_tflops": round(f_fwd / mf / 1e12, 2), "backward_tflops": round(f_bwd / mb / 1e12, 2),
           "peak_tflops": FP32_PEAK_TFLOPS,
           "frac_fwd_bwd": round((f_fwd + f_bwd) / (mf + mb) / 1e12 / FP32_PEAK_TFLOPS, 4),
           "breakdown": bool(flag.item()),
           "note": "forward enqueued without a host wait (CholeskyQR breakdown flag returned on the "
                   "device, checked after the timed steps); backward recomputes G = A Omega and R = Q^T G"}
    print(f"# diff: forward {mf * 1e3:.2f} ms, backward {mb * 1e3:.2f} ms", file=sys.stderr, flush=True)
    del A, dQ, dB, ws, Q, B
    torch.cuda.empty_cache()
    return res


def sparse_block(qb, W, torch, steps=1):
    """CSR workload: randQB_FP (paper rule and adaptive) and randQB_EI on the 500000 x 200000
    power-law matrix (nnz 5e6, b = 50, tol 0.6), with the SpMM sweep rate.  Each variant
    runs once untimed (allocation) and once timed: a run takes seconds (rank ~13000; the
    block loop's 4 (m + n) l^2 flops dominate)."""
    import statistics

    import numpy as np

    wl = W.C3
    seed = W.SEED_OMEGA | 3
    dev = torch.device("cuda:0")
    t0 = time.time()
    c = wl.make()
    print(f"# generated {wl.name} in {time.time() - t0:.1f} s", file=sys.stderr, flush=True)
    rowptr = torch.from_numpy(c.rowptr).to(dev)
    colind = torch.from_numpy(c.colind).to(dev)
    val = torch.from_numpy(c.val).to(dev)
    l_max = 16384   # capacity of Q / B (P = 0 needs about 2.8x the optimal rank, ~4800)
    Qs = torch.empty((l_max, c.m), dtype=torch.float64, device=dev)
    Bs = torch.empty((l_max, c.n), dtype=torch.float64, device=dev)
    need = max(qb.qb_workspace_bytes(qb.QB_ALGO_FP, True, c.m, c.n, c.nnz, wl.tol, wl.b, l_max, 0),
               qb.qb_workspace_bytes(qb.QB_ALGO_FP, True, c.m, c.n, c.nnz, wl.tol, wl.b, l_max, 0, 1),
               qb.qb_workspace_bytes(qb.QB_ALGO_EI, True, c.m, c.n, c.nnz, wl.tol, wl.b, l_max))
    ws = torch.empty(need, dtype=torch.uint8, device=dev)
    res = {"workload": wl.name, "l_max": l_max}
    runs = (("fp_paper_rule", lambda: qb.qb_fp_csr(c.m, c.n, rowptr, colind, val, wl.tol, wl.b, seed,
                                                    l_max=l_max, l_tilde=0, Q_store=Qs, B_store=Bs, ws=ws)),
            ("fp_adaptive", lambda: qb.qb_fp_csr(c.m, c.n, rowptr, colind, val, wl.tol, wl.b, seed,
                                                  l_max=l_max, l_tilde=-1, Q_store=Qs, B_store=Bs, ws=ws)),
            ("ei", lambda: qb.qb_ei_csr(c.m, c.n, rowptr, colind, val, wl.tol, wl.b, seed, l_max=l_max,
                                        Q_store=Qs, B_store=Bs, ws=ws)),
            ("fp_power1", lambda: qb.qb_fp_csr(c.m, c.n, rowptr, colind, val, wl.tol, wl.b, seed,
                                                l_max=l_max, l_tilde=0, Q_store=Qs, B_store=Bs, ws=ws,
                                                power=1)))
    for name, fn in runs:
        torch.cuda.synchronize()
        ts, rs = [], []
        for _ in range(steps):
            t = time.perf_counter()
            r = fn()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t)
            rs.append(r)
        r = rs[-1]
        entry = {"time_to_tol_s": round(statistics.median(ts), 6), "rank": r.rank,
                 "E_rel": (max(r.E, 0.0) / r.normA2) ** 0.5, "status": r.status, "passes": r.passes,
                 "blocks": r.blocks, "chunks": r.chunks,
                 "phase_ms": {"normA2_and_csc": r.ms[0], "omega": r.ms[1], "A_X": r.ms[2],
                              "At_X": r.ms[3], "block_loop": r.ms[4], "power_rounds": r.ms[6],
                              "total": r.ms[5]}}
        entry["block_loop_roofline"] = block_loop_roofline(c.m, c.n, wl.b, r, ei=name == "ei")
        if name.startswith("fp"):
            # algorithmic bytes of the two SpMM passes per chunk: CSR arrays once, the dense
            # operand once, the dense result once
            w_tot = r.gemm_flops[0] / (2.0 * c.m * c.n) if r.gemm_flops[0] else 0.0
            csr_b = c.nnz * 12 + (c.m + 1) * 8
            bytes_g = r.chunks * csr_b + 8.0 * w_tot * (c.n + c.m)
            bytes_h = r.chunks * (c.nnz * 12 + (c.n + 1) * 8) + 8.0 * w_tot * (c.m + c.n)
            entry["spmm_GBps"] = {"A_X": round(bytes_g / (r.ms[2] * 1e-3) / 1e9, 1) if r.ms[2] else None,
                                  "At_X": round(bytes_h / (r.ms[3] * 1e-3) / 1e9, 1) if r.ms[3] else None,
                                  "peak": 8000.0}
        res[name] = entry
        print(f"# sparse {name}: {statistics.median(ts) * 1e3:.1f} ms rank {r.rank} passes {r.passes}",
              file=sys.stderr, flush=True)
    # COO input: the same matrix as shuffled triplets, turned into CSR by the library
    coo = c.to_scipy().tocoo()
    perm = np.random.default_rng(7).permutation(coo.nnz)
    tr = [torch.from_numpy(np.ascontiguousarray(a[perm])).to(dev)
          for a in (coo.row.astype(np.int32), coo.col.astype(np.int32), coo.data)]
    del coo, perm
    qb.coo_to_csr(c.m, c.n, *tr)
    torch.cuda.synchronize()
    t = time.perf_counter()
    rp2, ci2, va2 = qb.coo_to_csr(c.m, c.n, *tr)
    torch.cuda.synchronize()
    t_coo = time.perf_counter() - t
    same = bool(torch.equal(rp2, rowptr) and torch.equal(ci2, colind) and torch.equal(va2, val))
    res["coo_to_csr"] = {"time_s": round(t_coo, 6), "nnz": int(c.nnz), "equals_csr": same}
    print(f"# sparse coo -> csr: {t_coo * 1e3:.1f} ms (identical CSR: {same})", file=sys.stderr, flush=True)
    del tr, rp2, ci2, va2
    del Qs, Bs, ws, rowptr, colind, val
    torch.cuda.empty_cache()
    return res


def counter_probe(qb, W, torch, l_tilde):
    """The program the counter passes run (bench.py --counter-probe): two calibration kernels
    of known traffic -- ||X||^2 of a 1 GiB matrix (sumsq_dense_partial reads exactly 2^30
    bytes) and 2^27 Gaussian entries (gauss_fill_kernel writes exactly 2^30 bytes) -- then the
    headline randQB_FP call twice (warm-up, measured) on the same matrix, generated on the
    host so that no library QR of the generator runs under the counters."""
    dev = torch.device("cuda:0")
    X = torch.full((8192, 16384), 0.5, dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    qb.qb_sumsq_dense(X)
    del X
    g = qb.qb_gaussian_fill(1, 8192, 16384)
    torch.cuda.synchronize()
    del g
    wl = W.C2
    seed = W.SEED_OMEGA | 2
    A = wl.make(device="cpu").to(dev)
    m, n = A.shape
    l_max = min(m, n)
    for _ in range(2):
        qb.qb_fp_dense(A, wl.tol, wl.b, seed, l_max=l_max, l_tilde=l_tilde)
        torch.cuda.synchronize()


def _read_counters(csv_path):
    """rocprofv3 counter-collection CSV -> list of (dispatch id, kernel name, counter, value)."""
    import csv
    out = []
    with open(csv_path) as f:
        for row in csv.DictReader(f):
            out.append((int(row["Dispatch_Id"]), row["Kernel_Name"], row["Counter_Name"], float(row["Counter_Value"])))
    out.sort()
    return out


def measure_counters(l_tilde, timeout=300):
    """Counter passes over counter_probe (each its own rocprofv3 run: FETCH_SIZE, WRITE_SIZE,
    then the MfmaUtil metric): the dominant sketch GEMMs' HBM bytes per launch of the measured
    call (each counter scaled by what it reads for its calibration kernel of exactly 1 GiB)
    and their MFMA busy percentage.  Returns {} fields as None when a pass fails."""
    import glob
    import shutil
    import subprocess
    import tempfile

    res = {"traffic_bytes": {"G": None, "H": None}, "mfma_util_pct": {"G": None, "H": None}, "passes": {}}
    tmp = tempfile.mkdtemp(prefix="qb_counters_", dir="/tmp")
    env = dict(os.environ, TMPDIR="/tmp")
    prof = shutil.which("rocprofv3") or "/opt/rocm/bin/rocprofv3"
    per = {}
    for name in ("FETCH_SIZE", "WRITE_SIZE", "MfmaUtil"):
        d = os.path.join(tmp, name)
        cmd = [prof, "--pmc", name, "--output-format", "csv", "-d", d, "-o", "run", "--",
               sys.executable, os.path.join(ROOT, "bench.py"), "--counter-probe", "--l-tilde", str(l_tilde)]
        print(f"# counters: {name} pass ...", file=sys.stderr, flush=True)
        try:
            r = subprocess.run(cmd, cwd="/tmp", env=env, stdout=subprocess.DEVNULL, stderr=subprocess.PIPE,
                               timeout=timeout)
            rc = r.returncode
        except subprocess.TimeoutExpired:
            rc = "timeout"
        files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
        res["passes"][name] = {"rc": rc, "csv": bool(files)}
        if files:
            per[name] = _read_counters(files[0])
    # the sketch GEMMs: gemm_f64_kernel<128, 128, ...> with A layout 0 (G = A Omega) or
    # 1 (H = A^T G); the measured call's launches are the last half of each
    def launches(rows, counter, al):
        tag = re.compile(rf"gemm_f64_kernel<128, 128, \d+, 4, 2, {al}, 0,")
        vals = [v for _, k, c, v in rows if c == counter and tag.search(k)]
        return vals[len(vals) // 2:]

    def first(rows, counter, kname):
        for _, k, c, v in rows:
            if c == counter and kname in k:
                return v
        return None

    try:
        fetch, write = per.get("FETCH_SIZE"), per.get("WRITE_SIZE")
        if fetch and write:
            cal_f = first(fetch, "FETCH_SIZE", "sumsq_dense_partial")
            cal_w = first(write, "WRITE_SIZE", "gauss_fill_kernel")
            f_scale = 2.0 ** 30 / (cal_f * 1024.0)
            w_scale = 2.0 ** 30 / (cal_w * 1024.0)
            res["scale"] = {"FETCH_SIZE": round(f_scale, 4), "WRITE_SIZE": round(w_scale, 4)}
            for key, al in (("G", 0), ("H", 1)):
                fl, wr = launches(fetch, "FETCH_SIZE", al), launches(write, "WRITE_SIZE", al)
                if fl and wr and len(fl) == len(wr):
                    res["traffic_bytes"][key] = float(np.mean([a * 1024 * f_scale + b * 1024 * w_scale
                                                               for a, b in zip(fl, wr)]))
                    res["launches"] = len(fl)
        mf = per.get("MfmaUtil")
        if mf:
            for key, al in (("G", 0), ("H", 1)):
                u = launches(mf, "MfmaUtil", al)
                if u:
                    res["mfma_util_pct"][key] = round(float(np.mean(u)), 2)
    except Exception as e:  # a malformed file leaves the fields at None
        res["error"] = repr(e)
    shutil.rmtree(tmp, ignore_errors=True)
    return res


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(A, wl, seed, l_tilde, runs=5):
    """The FP64 oracle's randQB_FP on the same matrix and schedule on the host cores: the
    median of `runs` runs (matrix generation excluded), with the host's core count and CPU
    model, and the oracle's times on the other workloads' instances (randQB_FP and randQB_EI
    on the 1000 x 800 matrix, the 4096 x 4096 precision-form parity instance in bfloat16,
    and a bounded sample of the CSR workload)."""
    import numpy as np
    import torch

    import workloads as W
    from oracle import randqb as R
    try:
        from threadpoolctl import threadpool_info
        threads = max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
    except Exception:  # pragma: no cover
        threads = os.cpu_count() or 1
    An = A.cpu().numpy()
    print("# cpu baseline: oracle randQB_FP on the full workload ...", file=sys.stderr, flush=True)
    ts = []
    for _ in range(runs):
        t = time.perf_counter()
        ora = R.randqb_fp(An, wl.tol, wl.b, seed, l_tilde=l_tilde)
        ts.append(time.perf_counter() - t)
    dt = statistics.median(ts)
    print(f"# cpu baseline: median {dt:.2f} s of {runs} (rank {ora.rank})", file=sys.stderr, flush=True)
    others = {}
    # 1000 x 800 (sigma_j = j^-2, b = 20, tol 1e-2): randQB_FP and randQB_EI
    c1 = W.C1.make().numpy()
    s1 = W.SEED_OMEGA | 1
    for name, fn in (("fp", lambda: R.randqb_fp(c1, W.C1.tol, W.C1.b, s1)),
                     ("ei", lambda: R.randqb_ei(c1, W.C1.tol, W.C1.b, s1))):
        tt = []
        for _ in range(runs):
            t = time.perf_counter()
            r = fn()
            tt.append(time.perf_counter() - t)
        others[f"{W.C1.name}_{name}"] = {"median_s": round(statistics.median(tt), 4), "rank": r.rank,
                                          "E_rel": (max(r.E, 0.0) / r.normA2) ** 0.5}
    # precision-form parity instance, 4096 x 4096 bfloat16 (paper chunk rule)
    c4 = W.to_bf16(W.C4_SMALL.make()).double().numpy()
    tt = []
    for _ in range(3):
        t = time.perf_counter()
        r = R.randqb_fp(c4, W.C4_SMALL.tol, W.C4_SMALL.b, W.SEED_OMEGA | 4, precision="bf16")
        tt.append(time.perf_counter() - t)
    others[f"{W.C4_SMALL.name}_bf16"] = {"median_s": round(statistics.median(tt), 4), "rank": r.rank, "runs": 3}
    # CSR workload, bounded sample: the first 250 rows of the factorisation (one chunk of 250
    # columns, l_max = 250), once; SciPy's sparse products are single-threaded
    csr = W.C3.make().to_scipy()
    t = time.perf_counter()
    r = R.randqb_fp(csr, W.C3.tol, W.C3.b, W.SEED_OMEGA | 3, l_max=250, l_tilde=250)
    others[f"{W.C3.name}_sample"] = {"time_s": round(time.perf_counter() - t, 3), "rank": r.rank,
                                      "sample": "l_max = 250 (one chunk of 250 columns, 5 blocks), "
                                                "not converged; SciPy sparse products single-threaded"}
    print(f"# cpu baseline others: {json.dumps(others)}", file=sys.stderr, flush=True)
    return {"value": round(dt, 3), "unit": "s", "cores": threads, "kind": "oracle",
            "sample": f"full {wl.name} workload, randQB_FP with the same chunk schedule "
                      f"(NumPy/OpenBLAS FP64), median of {runs} runs",
            "runs_s": [round(x, 3) for x in ts], "rank": ora.rank, "nproc": os.cpu_count(),
            "cpu_model": _cpu_model(), "others": others}


if __name__ == "__main__":
    main()
