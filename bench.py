#!/usr/bin/env python3
"""Benchmark: blocked randomized QB (randQB_pb) to a relative Frobenius
tolerance of 1e-8 on one MI355X.

One step = one complete factorisation (every row of the hot path: sketch,
sampling product, orth, power iteration, re-projection, B = Q^T A, downdate,
stopping rule) of a 20000 x 16000 float64 matrix A = U diag(1/j) V^T
(U, V: Q factors of seeded Gaussian matrices), block b = 256, P = 0, with
the input already resident in HBM.  At eps = 1e-8 ||A||_F the run needs
every column: k = 16000 in 63 blocks.  `value` is nominal GFLOP/s,
(6 + 4P) m n k + 2 m k^2 over the measured seconds (the paper's cost model,
Sections 4.4 and 5.3, with two flops per multiply-add).

The JSON line also carries
  roofline        the dominant kernel's algorithmic rate, timed with HIP
                  events on its launch stream over one extra profiled
                  factorisation (kept out of the timed steps), against MI355X
                  peak
  cpu_baseline    the CPU oracle timed on the host on a bounded sample of the
                  same factorisation (its first blocks, same matrix), and the
                  GPU's first blocks compared with it
  mixed           the mixed-precision form on the same matrix and
                  tolerance: the sample as the exact-range int8 product
                  (QB_SAMPLE_INT8X8), its seconds, error, stop reason and
                  speed-up over the float64 line
  variants        mixed-precision sampling on the same matrix (exact int8,
                  FP32, bf16x3; then P + 1 power iterations in float64,
                  FP32 and bf16x3 with the last product of each block in
                  float64); the spectral-gap matrix of the same size; the
                  10000 x 10000 j^-2 workload at P = 0 and 1
  small_workload  the 2000 x 1000 exp(-j/40) workload: GPU and oracle medians
                  of 3, the oracle also on one thread
"""
from __future__ import annotations

import argparse
import ctypes
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "QB solve s & GFLOP/s at 1e-8 rel. Frobenius err: plain FP64 vs mixed prec"
PEAK = {"f64_mfma": 78.6, "f32_mfma": 157.3, "hbm_gbs": 8000.0}


def nominal_flops(m, n, k, P):
    return (6 + 4 * P) * m * n * k + 2 * m * k * k


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def profile_snapshot(lib):
    out = {}
    for i in range(lib.qb_profile_count()):
        ms, fl, by = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        la = ctypes.c_int64()
        lib.qb_profile_read(i, ctypes.byref(ms), ctypes.byref(la), ctypes.byref(fl), ctypes.byref(by))
        if la.value:
            out[lib.qb_profile_name(i).decode()] = {"ms": ms.value, "launches": la.value,
                                                    "flops": fl.value, "bytes": by.value}
    return out


def run_variant(qbmi, lib, torch, A, eps, wl, P, sample, steps, warmup, bufs, profile,
                power_orth=True):
    Q, B, ws = bufs

    def one():
        return qbmi.qb_factor(A, eps, wl.b, P, wl.seed_omega, sample=sample, workspace=ws,
                              Q=Q, B=B, power_orth=power_orth)

    for _ in range(warmup):
        one()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    res = None
    for _ in range(steps):
        res = one()
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    prof = None
    if profile:
        # per-kernel event timing brackets every launch with two events, which
        # lengthens the gaps between launches: it runs on one extra step of
        # its own, outside the timed ones
        lib.qb_profile_enable(1)
        one()
        torch.cuda.synchronize()
        prof = profile_snapshot(lib)
        lib.qb_profile_enable(0)
    return res, ms, prof


def committed_traffic(kernel, run):
    """HBM bytes per launch of `kernel` from a committed rocprofv3 counter
    summary under profiles/ (FETCH_SIZE + WRITE_SIZE, copy-kernel scaled),
    for the run configuration `run` ("<workload>/P<power iterations>/<sample
    precision>": a class's launches differ in shape between configurations).
    None unless the summary holds a line for this kernel and run, and the
    SHA-256 of every source file the line names matches the current file:
    counters taken on an older kernel say nothing about this one."""
    import glob
    import hashlib
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        with open(path) as f:
            for line in f:
                parts = line.split()
                if len(parts) < 2 or parts[0] != "traffic":
                    continue
                kv = dict(p.split("=", 1) for p in parts[1:] if "=" in p)
                if kv.get("kernel") != kernel or kv.get("run") != run:
                    continue
                srcs = kv.get("source", "").split(",")
                shas = kv.get("sha256", "").split(",")
                if len(srcs) != len(shas) or not srcs[0]:
                    continue
                ok = True
                for src, sha in zip(srcs, shas):
                    fp = os.path.join(ROOT, src)
                    if not os.path.isfile(fp):
                        ok = False
                        break
                    with open(fp, "rb") as g:
                        if hashlib.sha256(g.read()).hexdigest() != sha:
                            ok = False
                            break
                if ok:
                    return float(kv["bytes_per_launch"]), os.path.relpath(path, ROOT)
    return None, None


def residual_rel(torch, A, res):
    # independent check of ||A - Q B||_F / ||A||_F (verification only)
    R = A - res.Q @ res.B
    return float(torch.linalg.norm(R) / torch.linalg.norm(A))


def skip_reorth_experiment():
    """Section 6.3 / Figure 8 on the GPU: Matrix 1 (800 x 600, singular values
    from 0.59 down to 1e-18), error of the single pass (randQB_p, l columns)
    and of the blocked scheme (b = 10), with and without orthonormalisation
    between applications of A and A^T.  Prints one JSON line."""
    import numpy as np
    import torch
    import paper_1503_07157_amd as qbmi
    import synth

    A = synth.paper_matrix1(800, 600, seed=1)
    s = np.linalg.svd(A, compute_uv=False)
    nA = float(np.linalg.norm(A))
    Ad = qbmi.colmajor(torch.from_numpy(np.ascontiguousarray(A)).cuda())
    tau = 2.0 ** -20

    def err(res):
        R = Ad - res.Q @ res.B
        return float(torch.linalg.norm(R)) / float(s[0])

    rows = []
    for P in (1, 2):
        for l in (20, 40, 60, 80):
            ey = float(np.sqrt(np.sum(s[l:] ** 2))) / float(s[0])
            row = {"P": P, "l": l, "eckart_young": ey}
            for orth in (True, False):
                r = qbmi.qb_factor(Ad, 0.0, l, P, 7, kmax=l, power_orth=orth, single_block=True)
                row["single_" + ("orth" if orth else "no_orth")] = {"err": err(r), "k": r.k}
            rows.append(row)
        for orth in (True, False):
            r = qbmi.qb_factor(Ad, 1e-13 * nA, 10, P, 7, power_orth=orth)
            rows.append({"P": P, "blocked_b10": "orth" if orth else "no_orth", "err": err(r),
                         "k": r.k, "stop": r.stop_reason})
    print(json.dumps({"experiment": "skip-reorth", "matrix": "paper Matrix 1, 800x600, seed 1",
                      "sigma1": float(s[0]), "tau": tau,
                      "floor_single_no_orth": {str(P): tau ** (1 / (2 * P + 1)) for P in (1, 2)},
                      "floor_single_orth": tau, "rows": rows}), flush=True)


def post_experiment():
    """Section 3.3 on the GPU: time the low-rank SVD and the partial pivoted
    QR computed from the QB factors, for the 2000 x 1000 exp(-j/40) workload
    (eps = 1e-6 ||A||) and the 10000 x 10000 j^-2 workload at eps = 1e-5
    ||A||.  Prints one JSON line."""
    import numpy as np
    import torch
    import paper_1503_07157_amd as qbmi
    import synth

    out = []
    for name, eps_rel, P in (("exp40_2000x1000", 1e-6, 0), ("pow2_10000x10000", 1e-5, 1)):
        wl = synth.workload(name)
        if wl.m * wl.n > 4e7:
            A = synth.workload_matrix_gpu(name)
        else:
            A = qbmi.colmajor(torch.from_numpy(np.ascontiguousarray(
                synth.workload_matrix(name))).cuda())
        nA = float(torch.linalg.norm(A))
        res = qbmi.qb_factor(A, eps_rel * nA, wl.b, P, wl.seed_omega)
        Q, B = res.Q, res.B
        times = {}
        for what, fn in (("svd", lambda: qbmi.svd(Q, B)), ("pivoted_qr", lambda: qbmi.pivoted_qr(Q, B))):
            fn()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = fn()
            torch.cuda.synchronize()
            times[what] = time.perf_counter() - t0
            if what == "svd":
                U, S, V, sweeps = r
                k = min(int((S > 1e-14 * S[0]).sum()), S.numel())
                err = float(torch.linalg.norm(A - (U[:, :k] * S[:k]) @ V[:, :k].t())) / nA
                times["svd_sweeps"] = sweeps
                times["svd_rel_err"] = err
            else:
                Qh, R, perm = r
                err = float(torch.linalg.norm(A[:, perm] - Qh @ R)) / nA
                times["qr_rel_err"] = err
        out.append({"workload": name, "eps_rel": eps_rel, "power_iters": P, "k": res.k,
                    "n": wl.n, "m": wl.m, **times})
        log(f"[bench] post {name}: k={res.k} svd {times['svd']*1e3:.1f} ms "
            f"({times['svd_sweeps']} sweeps), pivoted qr {times['pivoted_qr']*1e3:.1f} ms")
        del A, Q, B, res
        torch.cuda.empty_cache()
    print(json.dumps({"experiment": "post", "rows": out}), flush=True)


def batched_experiment(steps, warmup, no_cpu, tune=True):
    """Many matrices of uneven sizes: 512 float32 matrices, m uniform in
    [256, 4096], n uniform in [128, min(m, 2048)], s_j = r^j with r uniform
    in [0.9, 0.995], b in {16, 32, 64}, eps = 1e-5 ||A||_F, P = 0, all
    factorised by one qb_factor_batched call.  Reports seconds per batch,
    matrices/s and nominal GFLOP/s (sum of 6 m n k + 2 m k^2), the same 512
    problems run one by one through qb_factor for comparison, sampled parity
    against the oracle and the oracle's own rate on those samples.  Prints
    one JSON line."""
    import numpy as np
    import torch
    import paper_1503_07157_amd as qbmi
    from paper_1503_07157_amd import _lib
    import synth

    lib = _lib.load()
    specs = synth.batch_specs()
    t0 = time.perf_counter()
    As = []
    for i, sp in enumerate(specs):
        As.append(synth.batch_matrix_gpu(sp))
        if i % 128 == 127:
            torch.cuda.synchronize()
            log(f"[bench] batched: generated {i + 1}/{len(specs)} matrices "
                f"({time.perf_counter() - t0:.1f} s)")
    nA = [float(torch.linalg.norm(A, dtype=torch.float64)) for A in As]
    eps = [1e-5 * v for v in nA]
    bs = [sp.b for sp in specs]
    seeds = [sp.seed_omega for sp in specs]

    def one():
        return qbmi.qb_factor_batched(As, eps, bs, seeds)

    def timed():
        for _ in range(warmup):
            one()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            r = one()
        torch.cuda.synchronize()
        return r, (time.perf_counter() - t0) / steps

    default_tiles = qbmi.batched_tiles()
    res, sec_default = timed()
    log(f"[bench] batched: {sec_default * 1e3:.1f} ms per batch with the default tiles")
    sec = sec_default
    sub, tune_s, trials, sub_before, sub_after = [], 0.0, 0, None, None
    if tune:
        # tile classes tuned on every fourth problem of the batch, then the
        # whole batch timed again with the tuned table
        from paper_1503_07157_amd.autotune import tune_batched
        sub = list(range(0, len(specs), 4))
        t0 = time.perf_counter()
        tuned, sub_before, sub_after, trials = tune_batched(
            [As[i] for i in sub], [eps[i] for i in sub], [bs[i] for i in sub],
            [seeds[i] for i in sub])
        tune_s = time.perf_counter() - t0
        log(f"[bench] batched: tuned on {len(sub)} problems in {tune_s:.1f} s ({trials} trials): "
            f"{sub_before * 1e3:.1f} -> {sub_after * 1e3:.1f} ms")
        res, sec = timed()
        if sec_default < sec:  # keep whichever table ran the whole batch faster
            qbmi.set_batched_tiles(default_tiles)
            res, sec = timed()
    ks = [r.k for r in res]
    nblk = [r.blocks for r in res]
    active = [sum(1 for v in nblk if v > it) for it in range(max(nblk))]
    flops = sum(nominal_flops(sp.m, sp.n, r.k, 0) for sp, r in zip(specs, res))
    bad = [i for i, r in enumerate(res) if r.status < 0]
    log(f"[bench] batched: {sec * 1e3:.1f} ms per batch of {len(specs)}, "
        f"{flops / sec / 1e9:.0f} GFLOP/s, k in [{min(ks)}, {max(ks)}], errors {len(bad)}")
    lib.qb_profile_enable(1)
    one()
    torch.cuda.synchronize()
    prof = profile_snapshot(lib)
    lib.qb_profile_enable(0)
    kern = {name: {"ms": round(v["ms"], 3), "launches": v["launches"],
                   **({"tflops": round(v["flops"] / v["ms"] / 1e9, 2)} if v["flops"] else {}),
                   **({"gbs": round(v["bytes"] / v["ms"] / 1e6, 1)} if v["bytes"] else {})}
            for name, v in prof.items()}
    # the largest kernel class: the downdate, a stream over R (HBM-bound)
    dom_name = max((k for k in prof if k.startswith("batch_")), key=lambda k: prof[k]["ms"])
    dom = prof[dom_name]
    gbs = dom["bytes"] / dom["ms"] / 1e6 if dom["bytes"] else None
    roofline = {"bound": "hbm", "kernel": dom_name, "achieved": gbs, "peak": PEAK["hbm_gbs"],
                "unit": "GB/s", "frac": gbs / PEAK["hbm_gbs"] if gbs else None,
                "tflops": dom["flops"] / dom["ms"] / 1e9 if dom["flops"] else None,
                "note": "algorithmic bytes (8 (MK + KN + 2MN) per product) over the summed "
                        "launch durations, HIP events, one extra profiled batch"}
    # critical path: the problem that needs the most block iterations, alone
    slow = max(range(len(specs)), key=lambda i: nblk[i])
    qbmi.qb_factor_batched([As[slow]], [eps[slow]], [bs[slow]], [seeds[slow]])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    qbmi.qb_factor_batched([As[slow]], [eps[slow]], [bs[slow]], [seeds[slow]])
    torch.cuda.synchronize()
    tail = time.perf_counter() - t0
    log(f"[bench] batched: the {nblk[slow]}-iteration problem alone ({specs[slow].m}x{specs[slow].n}, "
        f"b={bs[slow]}) takes {tail * 1e3:.1f} ms")
    # the same problems one by one through the single-matrix path (float64 input)
    seq = 0.0
    same_k = 0
    for i, (sp, A) in enumerate(zip(specs, As)):
        A64 = qbmi.colmajor(A.to(torch.float64))
        torch.cuda.synchronize()
        ts = time.perf_counter()
        r1 = qbmi.qb_factor(A64, eps[i], sp.b, 0, sp.seed_omega)
        torch.cuda.synchronize()
        seq += time.perf_counter() - ts
        same_k += int(r1.k == res[i].k)
        del A64, r1
    log(f"[bench] batched: one by one {seq * 1e3:.1f} ms, same k {same_k}/{len(specs)}")
    # parity on sampled problems against the oracle, which is also timed
    cpu = None
    parity = []
    if not no_cpu:
        from oracle import randqb_pb
        import threadpoolctl
        order = sorted(range(len(specs)), key=lambda i: specs[i].m * specs[i].n * max(ks[i], 1))
        picks = [order[len(order) // 8], order[len(order) // 4], order[len(order) // 2]]
        cpu_s = 0.0
        cpu_fl = 0.0
        for i in picks:
            sp = specs[i]
            Ah = As[i].cpu().numpy().astype(np.float64)
            tc = time.perf_counter()
            o = randqb_pb(Ah, eps[i], sp.b, 0, sp.seed_omega)
            cpu_s += time.perf_counter() - tc
            cpu_fl += nominal_flops(sp.m, sp.n, o.k, 0)
            Qg, Bg = res[i].Q.cpu().numpy(), res[i].B.cpu().numpy()
            d = float(np.linalg.norm(Qg @ Bg - o.Q @ o.B)) / nA[i]
            parity.append({"index": i, "m": sp.m, "n": sp.n, "b": sp.b, "r": round(sp.r, 5),
                           "k_gpu": res[i].k, "k_oracle": o.k, "qb_rel_diff": d})
            log(f"[bench] batched parity #{i} {sp.m}x{sp.n} b={sp.b}: k {res[i].k}/{o.k} "
                f"rel diff {d:.2e}")
        info = threadpoolctl.threadpool_info()
        cores = max([d.get("num_threads", 1) for d in info if d.get("user_api") == "blas"] or [1])
        cpu = {"value": cpu_fl / cpu_s / 1e9, "unit": "GFLOP/s", "cores": int(cores),
               "kind": "oracle", "seconds": cpu_s,
               "sample": f"{len(picks)} of the 512 problems (the 1/8, 1/4 and 1/2 quantiles by "
                         f"m n k), float64 numpy/OpenBLAS on the host"}
    print(json.dumps({"experiment": "batched", "problems": len(specs),
                      "seconds_per_batch": sec, "matrices_per_s": len(specs) / sec,
                      "seconds_per_batch_default_tiles": sec_default,
                      "tiles": qbmi.batched_tiles(), "default_tiles": default_tiles,
                      "tuning": {"problems": len(sub), "seconds": tune_s, "trials": trials,
                                 "sub_batch_before_s": sub_before,
                                 "sub_batch_after_s": sub_after},
                      "gflops": flops / sec / 1e9, "nominal_flops": flops,
                      "k_min": min(ks), "k_max": max(ks), "k_total": sum(ks),
                      "errors": len(bad), "iterations": len(active), "active_per_iteration": active,
                      "longest_problem_alone_seconds": tail,
                      "one_by_one_seconds": seq,
                      "one_by_one_same_k": same_k, "roofline": roofline, "kernels": kern,
                      "parity": parity,
                      "cpu_baseline": cpu, "dtype": "f32 input, f64 arithmetic",
                      "data": "synthetic"}), flush=True)


def adjoint_experiment(steps, warmup, no_cpu):
    """The fixed-sketch QB map and its hand-written adjoint on a 4096 x 2048
    float32 matrix with s_j = exp(-j/100), b = 64, 4 blocks (k = 256), P in
    {0, 1}, loss L = <G, Q B> with G ~ N(0, 1): seconds for the forward
    (qb_fixed) and for the backward (qb_adjoint), the backward's GEMM rate
    from the per-kernel profile, its error against the float64 oracle
    gradient, and the oracle's own time for the same gradient.  Prints one
    JSON line."""
    import numpy as np
    import torch
    import paper_1503_07157_amd as qbmi
    from paper_1503_07157_amd import _lib
    import synth

    lib = _lib.load()
    m, n, b, s, seed = 4096, 2048, 64, 4, 77
    A32 = synth.prescribed_svd(m, n, np.exp(-np.arange(1, n + 1) / 100.0), 31, 32).astype(np.float32)
    A64 = A32.astype(np.float64)
    G = np.random.default_rng(5).standard_normal((m, n))
    Ad = qbmi.colmajor(torch.from_numpy(A64).cuda())
    Gd = qbmi.colmajor(torch.from_numpy(G).cuda())
    rows = []
    for P in (0, 1):
        Q, B = qbmi.qb_fixed(Ad, b, s, P, seed)
        dQ = qbmi.colmajor(Gd @ B.t())
        dB = qbmi.colmajor(Q.t() @ Gd)
        for _ in range(warmup):
            qbmi.qb_fixed(Ad, b, s, P, seed)
            qbmi.qb_adjoint(Ad, Q, B, dQ, dB, b, s, P, seed)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            qbmi.qb_fixed(Ad, b, s, P, seed)
        torch.cuda.synchronize()
        t_fwd = (time.perf_counter() - t0) / steps
        t0 = time.perf_counter()
        for _ in range(steps):
            dA = qbmi.qb_adjoint(Ad, Q, B, dQ, dB, b, s, P, seed)
        torch.cuda.synchronize()
        t_bwd = (time.perf_counter() - t0) / steps
        lib.qb_profile_enable(1)
        qbmi.qb_adjoint(Ad, Q, B, dQ, dB, b, s, P, seed)
        torch.cuda.synchronize()
        prof = profile_snapshot(lib)
        lib.qb_profile_enable(0)
        gemm_fl = sum(v["flops"] for k, v in prof.items() if k.startswith("gemm"))
        gemm_ms = sum(v["ms"] for k, v in prof.items() if k.startswith("gemm"))
        row = {"power_iters": P, "forward_s": t_fwd, "backward_s": t_bwd,
               "backward_gemm_flops": gemm_fl, "backward_gemm_tflops": gemm_fl / gemm_ms / 1e9,
               "backward_gflops": gemm_fl / t_bwd / 1e9,
               "roofline": {"bound": "mfma", "kernel": "backward GEMMs (all classes)",
                            "achieved": gemm_fl / gemm_ms / 1e9, "peak": PEAK["f64_mfma"],
                            "unit": "TFLOP/s",
                            "frac": gemm_fl / gemm_ms / 1e9 / PEAK["f64_mfma"]},
               "kernels": {k: {"ms": round(v["ms"], 3), "launches": v["launches"]}
                           for k, v in prof.items()}}
        if not no_cpu:
            from oracle.adjoint import qb_fixed_vjp
            Qn, Bn = Q.cpu().numpy(), B.cpu().numpy()
            tc = time.perf_counter()
            _, _, dAo = qb_fixed_vjp(A64, G @ Bn.T, Qn.T @ G, b, s, P, seed)
            row["oracle_s"] = time.perf_counter() - tc
            row["rel_err_vs_oracle"] = float(np.linalg.norm(dA.cpu().numpy() - dAo) / np.linalg.norm(dAo))
        log(f"[bench] adjoint P={P}: forward {t_fwd * 1e3:.1f} ms, backward {t_bwd * 1e3:.1f} ms "
            f"({row['backward_gflops']:.0f} GFLOP/s), oracle {row.get('oracle_s', float('nan')):.2f} s")
        rows.append(row)
    import threadpoolctl
    info = threadpoolctl.threadpool_info()
    cores = max([d.get("num_threads", 1) for d in info if d.get("user_api") == "blas"] or [1])
    print(json.dumps({"experiment": "adjoint", "workload": "exp100_4096x2048_f32, b=64, 4 blocks",
                      "rows": rows, "oracle": "torch CPU float64 autograd", "oracle_cores": cores,
                      "dtype": "f32 input, f64 arithmetic", "data": "synthetic"}), flush=True)


def precision_experiment():
    """The precision sweep: 20000 x 16000 matrices with s_j = 1/j and with a
    spectral gap (s_j = 1 for j <= 500, 1e-6 after), b = 256,
    eps = 1e-8 ||A||_F.  At P = 0: the sampling product in float64, as the
    exact-range int8 product, in FP32 and in bf16x3, and B_i in FP32 and
    bf16x3; at P = 1: float64, FP32 and bf16x3 sampling (the last product of
    each block in float64).  Reports per variant the seconds, rank, stop
    reason and the true error ||A - Q B||_F / ||A||_F (computed on the GPU).
    The oracle is pinned to these paths through the first blocks
    (tests/test_gpu_fullsize.py, tests/test_gpu_exact_sample.py).  Prints
    one JSON line."""
    import torch
    import paper_1503_07157_amd as qbmi
    import synth

    rows = []
    variants = [(0, "f64", "f64"), (0, "int8x8", "f64"), (0, "f32", "f64"), (0, "bf16x3", "f64"),
                (0, "f64", "f32"), (0, "f64", "bf16x3"), (1, "f64", "f64"), (1, "f32", "f64"),
                (1, "bf16x3", "f64")]
    for name in ("inv1_20000x16000", "gap_20000x16000"):
        wl = synth.workload(name)
        log(f"[bench] precision: generating {name}")
        A = synth.workload_matrix_gpu(name)
        nA = float(torch.linalg.norm(A))
        eps = wl.eps_rel * nA
        ws = None
        for P, sample, bgemm in variants:
            res = qbmi.qb_factor(A, eps, wl.b, P, wl.seed_omega, sample=sample, bgemm=bgemm,
                                 workspace=ws)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            res = qbmi.qb_factor(A, eps, wl.b, P, wl.seed_omega, sample=sample, bgemm=bgemm,
                                 workspace=ws)
            torch.cuda.synchronize()
            sec = time.perf_counter() - t0
            err = residual_rel(torch, A, res)
            fl = nominal_flops(wl.m, wl.n, res.k, P)
            rows.append({"workload": name, "power_iters": P, "sample": sample, "bgemm": bgemm,
                         "k": res.k, "stop": res.stop_reason, "status": res.status,
                         "seconds": sec, "gflops": fl / sec / 1e9, "rel_err": err})
            log(f"[bench] precision {name} P={P} sample={sample} B={bgemm}: k={res.k} "
                f"{res.stop_reason} {sec * 1e3:.0f} ms rel_err={err:.2e}")
            del res
            torch.cuda.empty_cache()
        del A
        torch.cuda.empty_cache()
    print(json.dumps({"experiment": "precision", "eps_rel": 1e-8, "b": 256,
                      "rows": rows, "data": "synthetic"}), flush=True)


def host_cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def blas_threads():
    import threadpoolctl
    info = threadpoolctl.threadpool_info()
    return max([d.get("num_threads", 1) for d in info if d.get("user_api") == "blas"] or [1])


def small_workload_timing(qbmi, torch, no_cpu):
    """The 2000 x 1000 exp(-j/40) workload (b = 50, P = 0, eps = 1e-6 ||A||):
    median of 3 GPU runs (HIP events around each call), the oracle's median
    of 3 on all host threads and one run on one thread, same input bytes;
    k and Q B compared between the two."""
    import numpy as np
    import synth

    wl = synth.workload("exp40_2000x1000")
    Ah = synth.workload_matrix(wl.name)
    A = qbmi.colmajor(torch.from_numpy(np.ascontiguousarray(Ah)).cuda())
    nA = float(np.linalg.norm(Ah))
    eps = wl.eps_rel * nA
    r = min(wl.m, wl.n)
    Q = torch.empty((r, wl.m), dtype=torch.float64, device="cuda").t()
    B = torch.empty((wl.n, r), dtype=torch.float64, device="cuda").t()
    ws = torch.empty(qbmi.workspace_bytes(wl.m, wl.n, wl.b, r) + 512, dtype=torch.uint8,
                     device="cuda")
    stream = torch.cuda.current_stream()
    gpu_ms = []
    res = None
    for i in range(4):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        res = qbmi.qb_factor(A, eps, wl.b, 0, wl.seed_omega, workspace=ws, Q=Q, B=B)
        e1.record(stream)
        torch.cuda.synchronize()
        if i > 0:                         # the first call is a warm-up
            gpu_ms.append(e0.elapsed_time(e1))
    gpu_ms.sort()
    out = {"workload": wl.name, "m": wl.m, "n": wl.n, "b": wl.b, "power_iters": 0,
           "eps_rel": wl.eps_rel, "k": res.k, "stop": res.stop_reason,
           "gpu_s_median3": gpu_ms[1] / 1e3, "gpu_s_runs": [v / 1e3 for v in gpu_ms],
           "gpu_gflops": nominal_flops(wl.m, wl.n, res.k, 0) / (gpu_ms[1] * 1e-3) / 1e9}
    if not no_cpu:
        import threadpoolctl
        from oracle import randqb_pb
        times = []
        o = None
        for _ in range(3):
            t0 = time.perf_counter()
            o = randqb_pb(Ah, eps, wl.b, 0, wl.seed_omega)
            times.append(time.perf_counter() - t0)
        times.sort()
        with threadpoolctl.threadpool_limits(limits=1, user_api="blas"):
            t0 = time.perf_counter()
            randqb_pb(Ah, eps, wl.b, 0, wl.seed_omega)
            one = time.perf_counter() - t0
        d = float(np.linalg.norm(res.Q.cpu().numpy() @ res.B.cpu().numpy() - o.Q @ o.B)) / nA
        out.update({"oracle_k": o.k, "qb_rel_diff_vs_oracle": d,
                    "oracle_s_median3": times[1], "oracle_threads": int(blas_threads()),
                    "oracle_s_one_thread": one, "host_cpu": host_cpu_model()})
    log(f"[bench] {wl.name}: k={res.k} GPU {gpu_ms[1]:.2f} ms (median of 3)"
        + ("" if no_cpu else f", oracle {out['oracle_s_median3']:.2f} s "
                             f"({out['oracle_threads']} threads), {out['oracle_s_one_thread']:.2f} s "
                             f"(1 thread), k {out['oracle_k']}, QB diff {out['qb_rel_diff_vs_oracle']:.1e}"))
    del A, Q, B, ws
    torch.cuda.empty_cache()
    return out


def cpu_baseline_parity(qbmi, torch, A, eps, wl, P, blocks, sample="f64"):
    """The oracle on the first `blocks` blocks of the same factorisation
    (timed on all host threads), and the GPU's first blocks compared with
    it element by element: the oracle's Q B moved to the GPU and subtracted
    from the GPU's own Q B for the same kmax."""
    import numpy as np
    from oracle import randqb_pb

    m, n = wl.m, wl.n
    kmax = min(blocks * wl.b, min(m, n))
    A_host = A.cpu().numpy()
    t0 = time.perf_counter()
    o = randqb_pb(A_host, eps, wl.b, P, wl.seed_omega, kmax=kmax)
    dt = time.perf_counter() - t0
    del A_host
    g = qbmi.qb_factor(A, eps, wl.b, P, wl.seed_omega, kmax=kmax, sample=sample)
    Qo = torch.from_numpy(np.ascontiguousarray(o.Q)).cuda()
    Bo = torch.from_numpy(np.ascontiguousarray(o.B)).cuda()
    nA = float(torch.linalg.norm(A))
    diff = float(torch.linalg.norm(g.Q @ g.B - Qo @ Bo)) / nA
    del Qo, Bo, g
    torch.cuda.empty_cache()
    fl = nominal_flops(m, n, o.k, P)
    return {"value": fl / dt / 1e9, "unit": "GFLOP/s", "cores": int(blas_threads()),
            "kind": "oracle", "seconds": dt, "k": o.k, "host_cpu": host_cpu_model(),
            "qb_rel_diff_vs_gpu": diff,
            "sample": f"first {o.blocks} blocks (k={o.k}) of the same {m}x{n} factorisation, "
                      f"b={wl.b}, P={P}, float64 numpy/OpenBLAS on the host; GFLOP/s by the "
                      f"same nominal count as the GPU value; the GPU's first {o.blocks} blocks "
                      f"differ from it by qb_rel_diff_vs_gpu relative to ||A||_F"}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="inv1_20000x16000")
    ap.add_argument("--power-iters", type=int, default=0)
    ap.add_argument("--sample", default="f64", choices=["f64", "f32", "bf16x3", "int8x8"])
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-tune", action="store_true",
                    help="batched experiment: keep the default tile table (no tuning pass)")
    ap.add_argument("--cpu-blocks", type=int, default=3)
    ap.add_argument("--variant-steps", type=int, default=2,
                    help="timed steps per variant (at most --steps)")
    ap.add_argument("--experiment", default=None, choices=["skip-reorth", "post", "batched", "adjoint", "precision"],
                    help="run one of the side experiments instead of the benchmark")
    ap.add_argument("--matrix", default="workload", choices=["workload", "gaussian"],
                    help="gaussian: i.i.d. N(0, 1/m) entries of the workload's shape instead of "
                         "the prescribed spectrum (no QR in the process; used for hardware-counter "
                         "passes, where only the launch shapes matter)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU; --gpus {args.gpus} is not supported "
              f"(the library has no multi-GPU path)", file=sys.stderr)
        sys.exit(2)
    if args.experiment == "skip-reorth":
        skip_reorth_experiment()
        return
    if args.experiment == "post":
        post_experiment()
        return
    if args.experiment == "batched":
        batched_experiment(args.steps, args.warmup, args.no_cpu, tune=not args.no_tune)
        return
    if args.experiment == "adjoint":
        adjoint_experiment(args.steps, args.warmup, args.no_cpu)
        return
    if args.experiment == "precision":
        precision_experiment()
        return

    import torch
    import paper_1503_07157_amd as qbmi
    import synth

    lib = qbmi.load()

    def make_matrix(name):
        w = synth.workload(name)
        if args.matrix == "gaussian":
            log(f"[bench] generating a Gaussian {w.m}x{w.n} matrix on the GPU")
            gen = torch.Generator(device="cuda")
            gen.manual_seed(w.seed_u)
            X = torch.randn((w.n, w.m), generator=gen, dtype=torch.float64, device="cuda").t()
            X.mul_(1.0 / math.sqrt(w.m))
        else:
            log(f"[bench] generating {w.name} on the GPU")
            X = synth.workload_matrix_gpu(w.name)
        torch.cuda.synchronize()
        return w, X

    def buffers(w):
        r = min(w.m, w.n)
        Qb = torch.empty((r, w.m), dtype=torch.float64, device="cuda").t()
        Bb = torch.empty((w.n, r), dtype=torch.float64, device="cuda").t()
        need = max(qbmi.workspace_bytes(w.m, w.n, w.b, r, sample=sm)
                   for sm in ("f64", "int8x8"))
        wsb = torch.empty(need + 512, dtype=torch.uint8, device="cuda")
        return Qb, Bb, wsb

    wl, A = make_matrix(args.workload)
    m, n = wl.m, wl.n
    nA2, bad = qbmi.frob2(A)
    assert not bad
    eps = wl.eps_rel * math.sqrt(nA2)
    bufs = buffers(wl)

    P = args.power_iters
    log(f"[bench] timing {wl.name} P={P} sample={args.sample}: warmup {args.warmup}, steps {args.steps}")
    res, ms, prof = run_variant(qbmi, lib, torch, A, eps, wl, P, args.sample, args.steps,
                                args.warmup, bufs, profile=True)
    k = res.k
    flops = nominal_flops(m, n, k, P)
    gflops = flops / (ms * 1e-3) / 1e9
    rel = residual_rel(torch, A, res)
    log(f"[bench] k={k} stop={res.stop_reason} {ms:.1f} ms/step {gflops:.0f} GFLOP/s rel_err={rel:.3e}")

    # dominant kernel by total time inside the profiled step
    dom_name, dom = max(prof.items(), key=lambda kv: kv[1]["ms"])
    dom_tflops = dom["flops"] / (dom["ms"] * 1e-3) / 1e12 if dom["ms"] > 0 else 0.0
    traffic, traffic_src = committed_traffic(dom_name, f"{wl.name}/P{P}/{args.sample}")
    roofline = {"bound": "mfma", "kernel": dom_name, "achieved": dom_tflops,
                "peak": PEAK["f64_mfma"], "unit": "TFLOP/s", "frac": dom_tflops / PEAK["f64_mfma"],
                "traffic": traffic, "traffic_source": traffic_src,
                "algorithmic_bytes": dom["bytes"] / dom["launches"],
                "avg_launch_ms": dom["ms"] / dom["launches"],
                "launches": dom["launches"],
                "note": "achieved = algorithmic flops of this kernel class (2 x rows x cols x depth "
                        "per product) over its summed launch durations, HIP events on the launch "
                        "stream, measured on one extra profiled factorisation after the timed steps"}
    kernels = {name: {"ms_per_step": v["ms"], "launches_per_step": v["launches"],
                      "tflops": (v["flops"] / (v["ms"] * 1e-3) / 1e12) if v["ms"] > 0 else None,
                      "gbs": (v["bytes"] / (v["ms"] * 1e-3) / 1e9) if v["ms"] > 0 else None}
               for name, v in prof.items()}

    vsteps = max(1, min(args.steps, args.variant_steps))
    variants = []

    def variant(w, X, e, vp, vs, vbufs, vo=True, ref=None):
        try:
            vres, vms, _ = run_variant(qbmi, lib, torch, X, e, w, vp, vs, vsteps, 1, vbufs,
                                       profile=False, power_orth=vo)
        except qbmi.QBError as ex:
            variants.append({"workload": w.name, "power_iters": vp, "sample": vs,
                             "power_orth": vo, "error": str(ex)})
            return None
        vfl = nominal_flops(w.m, w.n, vres.k, vp)
        row = {"workload": w.name, "power_iters": vp, "sample": vs, "power_orth": vo,
               "k": vres.k, "solve_s": vms / 1e3, "gflops": vfl / (vms * 1e-3) / 1e9,
               "rel_err": residual_rel(torch, X, vres), "stop": vres.stop_reason,
               "status": vres.status}
        if ref is not None:
            row["qb_rel_diff_vs_f64"] = float(torch.linalg.norm(vres.Q @ vres.B - ref)) / \
                float(torch.linalg.norm(X))
        variants.append(row)
        log(f"[bench] variant {w.name} P={vp} {vs}{'' if vo else ' no-orth'}: k={vres.k} "
            f"{vms:.1f} ms rel_err={row['rel_err']:.2e} {vres.stop_reason}")
        return vres

    mixed = None
    if not args.no_variants:
        # mixed-precision sampling on the same matrix, read against the float64
        # run: the exact-range int8 sample first (the mixed form that reaches
        # the float64 tolerance at k = min(m, n) < m), then the rounded f32 and
        # bf16x3 samples; then P + 1 power iterations, where the last product
        # of each block runs in float64 in every mode
        ref = (res.Q @ res.B) if args.sample == "f64" else None
        for vs in ("int8x8", "f32", "bf16x3"):
            if vs != args.sample:
                vr = variant(wl, A, eps, P, vs, bufs, ref=ref)
                if vs == "int8x8" and vr is not None and args.sample == "f64":
                    row = variants[-1]
                    mixed = {"sample": vs, "power_iters": P, "solve_s": row["solve_s"],
                             "gflops": row["gflops"], "k": row["k"], "stop": row["stop"],
                             "rel_err": row["rel_err"], "reaches_eps": row["status"] == 0,
                             "speedup_vs_f64": (ms / 1e3) / row["solve_s"],
                             "f64_solve_s": ms / 1e3}
                del vr
        del ref
        torch.cuda.empty_cache()
        r64 = variant(wl, A, eps, P + 1, "f64", bufs)
        ref = (r64.Q @ r64.B) if r64 is not None else None
        del r64
        for vs in ("f32", "bf16x3"):
            variant(wl, A, eps, P + 1, vs, bufs, ref=ref)
        del ref
        torch.cuda.empty_cache()
    cpu = None
    if not args.no_cpu:
        log(f"[bench] timing the CPU oracle on the first {args.cpu_blocks} blocks")
        cpu = cpu_baseline_parity(qbmi, torch, A, eps, wl, P, args.cpu_blocks, args.sample)
        log(f"[bench] cpu oracle: {cpu['seconds']:.1f} s, {cpu['value']:.1f} GFLOP/s on "
            f"{cpu['cores']} threads; GPU first blocks differ by {cpu['qb_rel_diff_vs_gpu']:.1e}")
    if not args.no_variants:
        # the other workloads of the sweep: the gap matrix at the same size,
        # the square 10^4 workload at P = 0 and 1
        for name, ps in (("gap_20000x16000", (0,)), ("pow2_10000x10000", (0, 1))):
            if name == wl.name:
                continue
            del bufs
            torch.cuda.empty_cache()
            w2, X2 = make_matrix(name)
            e2 = w2.eps_rel * float(torch.linalg.norm(X2))
            bufs = buffers(w2)
            for vp in ps:
                r64 = variant(w2, X2, e2, vp, "f64", bufs)
                ref = (r64.Q @ r64.B) if r64 is not None else None
                del r64
                for vs in ("int8x8", "f32", "bf16x3"):
                    variant(w2, X2, e2, vp, vs, bufs, ref=ref)
                del ref
                torch.cuda.empty_cache()
            del X2
            torch.cuda.empty_cache()
    small = small_workload_timing(qbmi, torch, args.no_cpu) if not args.no_variants else None

    line = {
        "metric": METRIC, "value": gflops, "unit": "GFLOP/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if args.sample == "f64" else f"f64+{args.sample}-sampling",
        "data": "synthetic",
        "config": {"workload": wl.name if args.matrix == "workload" else f"gaussian_{m}x{n}",
                   "m": m, "n": n, "b": wl.b, "power_iters": P,
                   "eps_rel": wl.eps_rel, "sample": args.sample, "k": k, "solve_s": ms / 1e3,
                   "rel_err": rel, "stop": res.stop_reason, "blocks": res.blocks,
                   "seeds": {"U": wl.seed_u, "V": wl.seed_v, "omega": wl.seed_omega}},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "mixed": mixed,
        "variants": variants,
        "small_workload": small,
        "kernels": kernels,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
