#!/usr/bin/env python3
"""Rank-1 SVD updates per second on one MI355X.

Workload (default): m = n = 8192, A = U diag(sigma) V^T with Haar U, V (seeded
Gaussian QR), sigma ~ U[1e-3, 1] sorted descending, a, b ~ N(0, 1/n); plain
FP64 path with the direct product. One step is one complete update through the
C ABI (projections, 2x2 splits, four eigen-updates with secular solves and
Cauchy weights, sign pairing, four products X C~), with its inputs resident in
HBM; every step gets its own (a, b).

Prints one JSON line. `roofline` describes the product kernel (the dominant
one): algorithmic FP64 flops per launch over its mean launch time, measured
with HIP events recorded on the launch stream by the library's timing ring.
One launch computes the products of one level, U C~_L+ and V C~_R+ (or
U~ C~_L- and V~ C~_R-): 2 m^3 + 2 n^3 flops. `forms` adds the precision forms
(exact-slice INT8, split FP32), the FMM path, the serving form and the batched
form (512 uneven problems in one captured graph) measured on the same box;
`configs` the other workloads (m = n = 256 latency, m = n = 4096 direct vs FMM
with its clustered / zeroed variants, m = 4096 n = 8192 precision forms, and
the FMM error against the expansion order). `cpu_baseline` times one CPU
oracle update of the benchmark workload (see cpu_baseline()). `traffic` comes from the rocprofv3 counter summary under
profiles/ when it was taken on the current product-kernel source, else null.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_MFMA_PEAK_TFLOPS = 78.6
CSRC = os.path.join(ROOT, "paper_1707_08369_amd", "csrc")
GEMM_SRCS = [os.path.join(CSRC, f) for f in ("k_gemm_f64.hip", "cauchy_tile.h", "device_util.h", "jobs.h")]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "gemm_cauchy_f64_traffic.json")


def gemm_source_hash() -> str:
    """Hash of the product kernel's source and the headers it includes."""
    h = hashlib.sha256()
    for f in GEMM_SRCS:
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def load_traffic(m: int, n: int):
    """HBM bytes per product launch from the committed counter runs, or None."""
    try:
        rec = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_sha256_16") != gemm_source_hash():
        return None
    if rec.get("m") != m or rec.get("n") != n:
        return None
    return rec.get("bytes_per_launch")


def host_info():
    """CPU threads this process may use, and the CPU model."""
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return cores, model


def cpu_baseline(U, sigma, V, a, b):
    """The CPU oracle (as it stands) on one update of the benchmark workload.

    Sample: one complete oracle update at the benchmark's size on host copies of
    the inputs of the timed GPU steps (the first timed step's a, b), timed
    wall-clock. The oracle's dense products and the dense A^ of its sign
    pairing run in numpy's BLAS on the host's threads; its secular solves,
    weights and eigenvector columns are single-threaded numpy.
    """
    import threadpoolctl

    import oracle.svdu_oracle as OS
    Uh, sh, Vh, ah, bh = (x.cpu().numpy() for x in (U, sigma, V, a, b))
    orig = OS.rank_one_update
    done = [0]

    def staged(*args, **kw):      # reports each of the oracle's four eigen-updates as it completes
        r = orig(*args, **kw)
        done[0] += 1
        print(f"[bench] oracle eigen-update {done[0]}/4 done at {time.perf_counter() - t0:.1f} s",
              file=sys.stderr, flush=True)
        return r
    t0 = time.perf_counter()
    OS.rank_one_update = staged
    try:
        OS.svd_rank1_update(Uh, sh, Vh, ah, bh)
    finally:
        OS.rank_one_update = orig
    secs = time.perf_counter() - t0
    info = threadpoolctl.threadpool_info()
    blas = max([i.get("num_threads", 1) for i in info] + [1])
    cores, model = host_info()
    m, n = Uh.shape[0], Vh.shape[0]
    return {
        "value": 1.0 / secs,
        "unit": "updates/s",
        "cores": int(max(blas, 1)),
        "kind": "oracle",
        "sample": (f"one full oracle update at m={m} n={n} on the benchmark's inputs: {secs:.1f} s wall-clock "
                   f"({blas} BLAS threads for the dense products; the O(n^2) phases single-threaded); "
                   f"host: {cores} usable CPUs, {model}"),
        "seconds_per_update": secs,
        "host_cpus": cores,
        "cpu_model": model,
    }


INT8_PEAK_TOPS = 5000.0


def _recon_orth(torch, U, sigma, V, a, b, Uo, so, Vo):
    m, n = U.shape[0], V.shape[0]
    Ah = (U * sigma[None, :]) @ V[:, :m].T + torch.outer(a, b)
    rec = ((Uo * so[None, :]) @ Vo[:, :m].T - Ah).norm().item() / Ah.norm().item()
    ou = (Uo.T @ Uo - torch.eye(m, dtype=Uo.dtype, device=Uo.device)).abs().max().item()
    ov = (Vo.T @ Vo - torch.eye(n, dtype=Vo.dtype, device=Vo.device)).abs().max().item()
    return rec, ou, ov


def measure_forms(svdu, torch, U, sigma, V, A_vecs, B_vecs, Uo, so, Vo, stream, fp64_ms, check, steps=4,
                  fmm=True):
    """The precision forms (exact-slice INT8 with 6, 7 and 8 slices; split FP32)
    and the FMM path on the same inputs: updates/s, speedup over the plain FP64
    path, and reconstruction / orthogonality error against the inputs. For the
    INT8 form also the product phases from the context's timing ring (slicing
    plus slice products, per level) and the slice products' INT8 rate against
    the 5.0 POPS dense peak."""
    res = {}
    m, n = U.shape[0], V.shape[0]
    k_ref = steps % A_vecs.shape[0]
    ref = svdu.rank1_update(U, sigma, V, A_vecs[k_ref], B_vecs[k_ref], want_defl=False, stream=stream) \
        if check else None
    forms = [("int8_slices7", svdu.SVDU_PREC_SLICED_INT8, svdu.SVDU_PATH_DIRECT, 7),
             ("int8_slices6", svdu.SVDU_PREC_SLICED_INT8, svdu.SVDU_PATH_DIRECT, 6),
             ("int8_slices8", svdu.SVDU_PREC_SLICED_INT8, svdu.SVDU_PATH_DIRECT, 8),
             ("split32", svdu.SVDU_PREC_SPLIT32, svdu.SVDU_PATH_DIRECT, 7)]
    if fmm:
        forms.append(("fmm_eps1e-10", svdu.SVDU_PREC_FP64, svdu.SVDU_PATH_FMM, 7))
    for name, prec, path, slices in forms:
        ctx = svdu.Context()
        ctx.set_option(svdu.SVDU_OPT_SLICES, slices)
        wsf = svdu.new_workspace(svdu.svdu_workspace_bytes(m, n, path, prec), U.device)

        def run(k):
            svdu.rank1_update(U, sigma, V, A_vecs[k], B_vecs[k], eps=1e-10, path=path, precision=prec,
                              out=(Uo, so, Vo), workspace=wsf, want_defl=False, stream=stream, check=False, ctx=ctx)
        for _ in range(3):   # a fresh context and workspace: the first calls of a form run slower
            run(0)
        torch.cuda.synchronize()
        ctx.set_option(svdu.SVDU_OPT_TIMING, 1)
        t0 = time.perf_counter()
        for k in range(1, steps + 1):
            run(k % A_vecs.shape[0])
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / steps
        ph = svdu.timing_read(steps, ctx=ctx)
        ctx.close()
        rec = dict(updates_per_s=1e3 / ms, ms_per_update=ms, speedup_vs_fp64=fp64_ms / ms)
        if prec == svdu.SVDU_PREC_SLICED_INT8:
            lev_ms = [sum(p[2] for p in ph) / len(ph), sum(p[3] for p in ph) / len(ph)]
            pairs = slices * (slices + 1) // 2
            ops = 2.0 * pairs * (m ** 3 + n ** 3)          # slice-product integer ops of one level
            rec["slices"] = slices
            rec["product_level_ms"] = lev_ms
            rec["int8_tops_per_level"] = ops / (sum(lev_ms) / 2 * 1e-3) / 1e12
            rec["int8_frac_of_peak"] = rec["int8_tops_per_level"] / INT8_PEAK_TOPS
            rec["fp64_equivalent_tflops"] = 2.0 * (m ** 3 + n ** 3) / (sum(lev_ms) / 2 * 1e-3) / 1e12
        if check:
            k = steps % A_vecs.shape[0]
            r, ou, ov = _recon_orth(torch, U, sigma, V, A_vecs[k], B_vecs[k], Uo, so, Vo)
            rec.update(recon=r, orth_U=ou, orth_V=ov, bound=1e-10 if path == svdu.SVDU_PATH_DIRECT else 1e-9)
            rec["sigma_bitwise_fp64"] = bool(torch.equal(so, ref[1]))
            if path == svdu.SVDU_PATH_FMM:
                rec["max_abs_diff_vs_direct_U"] = (Uo - ref[0]).abs().max().item()
                rec["max_abs_diff_vs_direct_V"] = (Vo - ref[2]).abs().max().item()
        res[name] = rec
        del wsf
    return res


def haar_inputs(torch, S, m, n, seed, kind="uniform01"):
    import numpy as np
    rng = np.random.default_rng(seed)
    U = S.haar_torch(m, seed=seed + 1, device="cuda")
    V = S.haar_torch(n, seed=seed + 2, device="cuda")
    sig = S.sigma_geometric(m) if kind == "geometric" else S.sigma_uniform(m, 1e-3, 1.0, rng)
    a = rng.standard_normal(m) / np.sqrt(n)
    b = rng.standard_normal(n) / np.sqrt(n)
    d = lambda x: torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")
    return U, d(sig), V, d(a), d(b)


def _time_update(svdu, torch, args, reps=3, **kw):
    out = svdu.rank1_update(*args, want_defl=False, **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        out = svdu.rank1_update(*args, want_defl=False, check=False, **kw)
    torch.cuda.synchronize()
    return 1e3 * (time.perf_counter() - t0) / reps, out


def measure_config_small(svdu, torch, reps=200):
    """m = n = 256, sigma ~ U[0.1, 10], Haar factors: latency of one update,
    called eagerly (enqueue + wait each time) and as a captured graph replay
    (a batch of one problem)."""
    import numpy as np

    import synth_inputs as S
    P = S.make_problem(256, 256, "uniform", seed=1001)
    d = lambda x: torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")
    args = (d(P.U), d(P.sigma), d(P.V), d(P.a), d(P.b))
    outs = (torch.empty((256, 256), dtype=torch.float64, device="cuda"),
            torch.empty(256, dtype=torch.float64, device="cuda"),
            torch.empty((256, 256), dtype=torch.float64, device="cuda"))
    ws = svdu.new_workspace(svdu.svdu_workspace_bytes(256, 256), "cuda")
    eager = []
    for i in range(reps + 10):
        t0 = time.perf_counter()
        svdu.rank1_update(*args, out=outs, workspace=ws, want_defl=False, check=False)
        torch.cuda.synchronize()
        if i >= 10:
            eager.append(1e3 * (time.perf_counter() - t0))
    b = svdu.Batch([args])
    b.launch(use_graph=True)
    torch.cuda.synchronize()
    graph = []
    for i in range(reps + 10):
        t0 = time.perf_counter()
        b.launch(use_graph=True)
        torch.cuda.synchronize()
        if i >= 10:
            graph.append(1e3 * (time.perf_counter() - t0))
    b.close()
    pct = lambda v, q: float(np.percentile(np.asarray(v), q))
    return {"workload": "m=n=256, sigma~U[0.1,10], haar U,V, a,b~N(0,1/n), fp64 direct",
            "eager_ms": {"p50": pct(eager, 50), "p99": pct(eager, 99)},
            "graph_ms": {"p50": pct(graph, 50), "p99": pct(graph, 99)},
            "graph_updates_per_s": 1e3 / pct(graph, 50)}


def measure_config_4096(svdu, torch):
    """m = n = 4096 geometric spectrum sigma_i = 10^(-6 i / m): direct vs FMM at
    eps = 1e-10; and the variant with 32 close pairs (relative spacing 1e-11)
    and 5 % of a's projected components zeroed, in both readings (p zeroed
    alone; p and q zeroed at the same indices)."""
    import synth_inputs as S
    res = {}
    U, sig, V, a, b = haar_inputs(torch, S, 4096, 4096, 4096, "geometric")
    cases = [("geometric", (U, sig, V, a, b))]
    Uh, Vh = U.cpu().numpy(), V.cpu().numpy()
    d = lambda x: torch.as_tensor(x, dtype=torch.float64, device="cuda")
    for name, zq in (("clustered_zero_p", False), ("clustered_zero_p_and_q", True)):
        P = S.make_problem(4096, 4096, "clustered", seed=4097, zero_frac=0.05, zero_q=zq, U=Uh, V=Vh)
        cases.append((name, (U, d(P.sigma), V, d(P.a), d(P.b))))
    for name, args in cases:
        md, od = _time_update(svdu, torch, args)
        mf, of = _time_update(svdu, torch, args, path=svdu.SVDU_PATH_FMM, eps=1e-10)
        r, ou, ov = _recon_orth(torch, *args, *of[:3])
        res[name] = {"direct_ms": md, "fmm_ms": mf, "fmm_speedup": md / mf,
                     "fmm_vs_direct_max_abs": max((of[0] - od[0]).abs().max().item(),
                                                  (of[2] - od[2]).abs().max().item()),
                     "fmm_recon": r, "fmm_orth": max(ou, ov)}
    return res


def measure_config_3a(svdu, torch):
    """m = 4096, n = 8192, sigma ~ U[1e-3, 1]: the precision forms against the
    plain FP64 path."""
    import synth_inputs as S
    args = haar_inputs(torch, S, 4096, 8192, 3000)
    res = {}
    mf, of = _time_update(svdu, torch, args)
    res["fp64"] = {"ms_per_update": mf}
    for name, prec, sl in (("int8_slices7", svdu.SVDU_PREC_SLICED_INT8, 7),
                           ("int8_slices6", svdu.SVDU_PREC_SLICED_INT8, 6),
                           ("split32", svdu.SVDU_PREC_SPLIT32, 7)):
        ctx = svdu.Context()
        ctx.set_option(svdu.SVDU_OPT_SLICES, sl)
        ms, o = _time_update(svdu, torch, args, precision=prec, ctx=ctx)
        ctx.close()
        r, ou, ov = _recon_orth(torch, *args, *o[:3])
        res[name] = {"ms_per_update": ms, "speedup_vs_fp64": mf / ms, "recon": r, "orth_U": ou, "orth_V": ov,
                     "bound": 1e-10, "sigma_bitwise_fp64": bool(torch.equal(o[1], of[1]))}
    return res


def measure_fmm_order_sweep(svdu, torch, sizes=((4096, "geometric"), (8192, "uniform01"))):
    """FMM error against the direct product as the expansion order p runs from
    8 to 16 (eps = 1.5 * 5^-p, so that ceil(log_5(1/eps)) = p): the largest
    difference of U^ and V^ from the direct path's, and the time per update.
    The Chebyshev far field converges like (3 + sqrt(8))^-p."""
    import synth_inputs as S
    res = {}
    for N, kind in sizes:
        args = haar_inputs(torch, S, N, N, 5000 + N, kind)
        md, od = _time_update(svdu, torch, args, reps=1)
        rows = []
        for p in range(8, 17):
            eps = 1.5 * 5.0 ** (-p)
            mf, of = _time_update(svdu, torch, args, reps=1, path=svdu.SVDU_PATH_FMM, eps=eps)
            err = max((of[0] - od[0]).abs().max().item(), (of[2] - od[2]).abs().max().item())
            rows.append({"p": p, "eps": eps, "max_abs_diff_vs_direct": err, "ms": mf,
                         "rate_bound": (3.0 + 8.0 ** 0.5) ** (-p)})
        res[f"n{N}_{kind}"] = {"direct_ms": md, "orders": rows}
    return res


def measure_secular_far_field(svdu, torch, reps=20):
    """The secular solve alone (poles sigma^2, sigma ~ U[1e-3, 1]; z ~ N(0, 1/K);
    rho = 2.6) with the direct sums and with the far field from per-leaf
    interpolants (SVDU_OPT_SECULAR_FMM 0 and 2), and the m = n = 8192 update on
    both product paths with the direct sums and with the default (the far field
    at this order)."""
    import numpy as np

    import synth_inputs as S
    ctxs = {}
    for name, mode in (("direct_sums", 0), ("far_field", 2)):
        ctxs[name] = svdu.Context()
        ctxs[name].set_option(svdu.SVDU_OPT_SECULAR_FMM, mode)
    res = {"workload": "secular roots: d = sigma^2, sigma~U[1e-3,1], z~N(0,1/K), rho=2.6; updates m=n=8192"}
    for K in (1024, 4096, 8192):
        rng = np.random.default_rng(K)
        d = torch.as_tensor(np.sort(rng.uniform(1e-3, 1.0, K) ** 2), device="cuda")
        z = torch.as_tensor(rng.standard_normal(K) / np.sqrt(K), device="cuda")
        row = {}
        for name, ctx in ctxs.items():
            for _ in range(3):
                svdu.secular(d, z, 2.6, ctx=ctx, check=False)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                svdu.secular(d, z, 2.6, ctx=ctx, check=False)
            e1.record()
            torch.cuda.synchronize()
            _, _, its = svdu.secular(d, z, 2.6, ctx=ctx)
            row[name] = {"ms": e0.elapsed_time(e1) / reps, "mean_iterations": float(its.float().mean())}
        res[f"secular_K{K}"] = row
    args = haar_inputs(torch, S, 8192, 8192, 8192)
    for path, pname in ((svdu.SVDU_PATH_FMM, "fmm"), (svdu.SVDU_PATH_DIRECT, "direct")):
        md, od = _time_update(svdu, torch, args, reps=3, path=path, eps=1e-10, ctx=ctxs["direct_sums"])
        mf, of = _time_update(svdu, torch, args, reps=3, path=path, eps=1e-10)
        res[f"update_8192_{pname}_path"] = {
            "direct_sums_ms": md, "far_field_ms": mf,
            "sigma_max_abs_diff": (of[1] - od[1]).abs().max().item(),
            "vectors_max_abs_diff": max((of[0] - od[0]).abs().max().item(), (of[2] - od[2]).abs().max().item())}
        del od, of
    for c in ctxs.values():
        c.close()
    return res


def measure_fmm_crossover(svdu, torch, sizes=(256, 512, 1024, 2048, 4096, 8192)):
    """Direct against FMM product path (eps = 1e-10) as the order grows (the
    analogue of the paper's comparison of the direct and the fast product):
    m = n, sigma ~ U[1e-3, 1], Haar factors; time per update on each path,
    their ratio, and the FMM result's largest difference from the direct one.
    The crossover is the smallest order from which the FMM path is faster."""
    import synth_inputs as S
    rows = []
    for N in sizes:
        args = haar_inputs(torch, S, N, N, 7000 + N)
        reps = 20 if N <= 1024 else (5 if N <= 4096 else 3)
        md, od = _time_update(svdu, torch, args, reps=reps)
        mf, of = _time_update(svdu, torch, args, reps=reps, path=svdu.SVDU_PATH_FMM, eps=1e-10)
        err = max((of[0] - od[0]).abs().max().item(), (of[2] - od[2]).abs().max().item())
        rows.append({"n": N, "direct_ms": md, "fmm_ms": mf, "fmm_speedup": md / mf, "fmm_vs_direct_max_abs": err})
        del args, od, of
    faster = [r["n"] for r in rows if r["fmm_speedup"] > 1.0]
    return {"workload": "m=n, sigma~U[1e-3,1], haar U,V, a,b~N(0,1/n), fp64, direct vs fmm eps=1e-10",
            "orders": rows, "fmm_faster_from_n": min(faster) if faster else None}


def batched_workload(torch, count=512, seed=4):
    """512 independent problems: m log-uniform in [64, 1024], n = m + U{0..m},
    sigma ~ U[0.01, 10] descending, Haar U and V, a, b ~ N(0, 1/n)."""
    import numpy as np

    import synth_inputs as S
    ms, ns = S.batched_sizes(count, seed=seed)
    rng = np.random.default_rng(seed + 100)
    items = []
    for i, (m, n) in enumerate(zip(ms.tolist(), ns.tolist())):
        U = S.haar_torch(m, seed=10_000 + 2 * i, device="cuda")
        V = S.haar_torch(n, seed=10_001 + 2 * i, device="cuda")
        sig = torch.as_tensor(S.sigma_uniform(m, 0.01, 10.0, rng), device="cuda")
        a = torch.as_tensor(rng.standard_normal(m) / np.sqrt(n), device="cuda")
        b = torch.as_tensor(rng.standard_normal(n) / np.sqrt(n), device="cuda")
        items.append((U, sig, V, a, b))
    return items


def measure_batched(svdu, torch, reps=5, check=True,
                    modes=("fp64_graph", "fp64_graph_persistent", "fp64_eager", "int8_graph", "split32_graph"),
                    table=None, one_by_one=True):
    """The batched form: the 512-problem workload as one batch, launched as one
    captured graph (or eagerly), against the same problems updated one call at
    a time through svdu_rank1_update. Tile shapes come from the autotuner."""
    import numpy as np
    items = batched_workload(torch)
    count = len(items)
    flops = float(sum(4.0 * (it[0].shape[0] ** 3 + it[2].shape[0] ** 3) for it in items))
    res = {"workload": "512 problems, m log-uniform [64,1024], n = m + U{0..m}, sigma~U[0.01,10], haar U,V, "
                       "a,b~N(0,1/n)", "count": count, "product_flops_per_batch": flops}
    tuned = {}
    if table is not None:   # a given FP64 table instead of tuning (profiling runs)
        svdu.tile_table(svdu.SVDU_PREC_FP64, table)
        tuned["fp64"] = {"table": table, "ms": None}
    else:
        for prec in (svdu.SVDU_PREC_FP64, svdu.SVDU_PREC_SPLIT32):   # the INT8 product has one tile shape
            tab, times = svdu.autotune(prec, max_n=2048)
            tuned["fp64" if prec == 0 else "split32"] = {"table": tab, "ms": [[round(t, 4) for t in row]
                                                                             for row in times[:6]]}
    res["autotune"] = tuned
    for mode in modes:
        prec = (svdu.SVDU_PREC_SPLIT32 if mode.startswith("split32") else
                svdu.SVDU_PREC_SLICED_INT8 if mode.startswith("int8") else svdu.SVDU_PREC_FP64)
        b = svdu.Batch(items, precision=prec, persistent="persistent" in mode)
        graph = "graph" in mode
        b.launch(use_graph=graph)                 # warm-up (and capture)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        times = []
        for _ in range(reps):
            e0.record()
            b.launch(use_graph=graph)
            e1.record()
            e1.synchronize()
            times.append(e0.elapsed_time(e1))
        st = b.status()
        ms = float(np.median(times))
        rec = {"ms_per_batch": ms, "ms_min": float(min(times)), "updates_per_s": count / (ms * 1e-3),
               "product_tflops_effective": flops / (ms * 1e-3) / 1e12, "status_ok": all(c == 0 for c in st)}
        if check and prec != svdu.SVDU_PREC_SPLIT32:
            worst = 0.0
            for it, o in zip(items[:64], b.outs[:64]):
                U, sg, V, a, bb = it
                mm = U.shape[0]
                Ah = (U * sg[None, :]) @ V[:, :mm].T + torch.outer(a, bb)
                worst = max(worst, ((o[0] * o[1][None, :]) @ o[2][:, :mm].T - Ah).norm().item() / Ah.norm().item())
            rec["recon_max_first64"] = worst
        res[mode] = rec
        b.close()
        del b
    if not one_by_one:
        return res
    # the same problems one call at a time (eager single-problem path)
    outs = [(torch.empty_like(it[0]), torch.empty_like(it[1]), torch.empty_like(it[2])) for it in items]
    wss = [svdu.new_workspace(svdu.svdu_workspace_bytes(it[0].shape[0], it[2].shape[0]), "cuda") for it in items]
    for it, o, w in zip(items, outs, wss):
        svdu.rank1_update(*it, out=o, workspace=w, want_defl=False, check=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for it, o, w in zip(items, outs, wss):
        svdu.rank1_update(*it, out=o, workspace=w, want_defl=False, check=False)
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0)
    res["one_call_per_problem"] = {"ms_per_batch": ms, "updates_per_s": count / (ms * 1e-3)}
    best = min(res[mo]["ms_per_batch"] for mo in modes if mo.startswith("fp64"))
    res["speedup_batched_vs_one_call_per_problem"] = ms / best
    return res


def measure_serving(svdu, torch, arrival_s=4.0, rate=2000.0, workers=3, sustain_s=6.0, seed=5):
    """The serving form: 64 resident matrices (m = n drawn from {256, 1024,
    2048, 4096, 8192}), Poisson arrivals targeting matrices uniformly, memory
    admission and continuous batching in the library's server. First at the
    stated rate for `arrival_s` seconds (the offered load far exceeds the
    device, so the backlog grows; requests still queued when arrivals end are
    dropped), then at 70 % of the throughput measured there, drained, so that
    latency is interpretable; both again with requests for orders >= 4096 on
    the FMM path. Factors: one Haar pair per size; every matrix of
    that size gets its own orthogonal factors from it by a random permutation
    of rows and of columns and random column signs; sigma ~ U[0.1, 10]
    descending; a, b ~ N(0, 1/n) from a pool of 16 pairs per size."""
    import numpy as np

    import synth_inputs as S
    sizes = S.serving_sizes(64, seed=seed).tolist()
    rng = np.random.default_rng(seed + 1)
    haar = {n: (S.haar_torch(n, seed=20_000 + n, device="cuda"), S.haar_torch(n, seed=30_000 + n, device="cuda"))
            for n in sorted(set(sizes))}
    pool = {n: [(torch.as_tensor(rng.standard_normal(n) / np.sqrt(n), device="cuda"),
                 torch.as_tensor(rng.standard_normal(n) / np.sqrt(n), device="cuda")) for _ in range(16)]
            for n in haar}
    factors = []

    def scrambled(Q):
        n = Q.shape[0]
        pr = torch.as_tensor(rng.permutation(n), device="cuda")
        pc = torch.as_tensor(rng.permutation(n), device="cuda")
        sg = torch.as_tensor(rng.choice([-1.0, 1.0], n), device="cuda")
        return (Q[pr][:, pc] * sg[None, :]).contiguous()

    for n in sizes:
        sig = torch.as_tensor(np.sort(rng.uniform(0.1, 10.0, n))[::-1].copy(), device="cuda")
        factors.append((scrambled(haar[n][0]), sig, scrambled(haar[n][1])))
    resident = sum(2 * (2 * n * n + n) * 8 for n in sizes)

    def run(rate_, span, drain, fmm_min_n=0):
        srv = svdu.Server(arena_bytes=24 << 30, workers=workers, max_batch=64, fmm_min_n=fmm_min_n,
                          min_batch_cost=2e10)
        for U, sg, V in factors:
            srv.add_matrix(U, sg, V)
        r = np.random.default_rng(seed + 7)
        t, reqs = 0.0, []
        while True:
            t += r.exponential(1.0 / rate_)
            if t > span:
                break
            reqs.append((int(r.integers(0, 64)), t))
        srv.start()
        for k, (i, tr) in enumerate(reqs):
            a, b = pool[sizes[i]][k % 16]
            srv.submit(i, a, b, tr)
        done = []
        while srv.now() < span:
            time.sleep(0.05)
            done += srv.poll()
        backlog = srv.stats()["queued"]
        if drain:
            srv.drain(600.0)
        done += srv.poll()
        st = srv.stats()
        srv.close()
        ok = [c for c in done if c["status"] == 0]
        in_window = [c for c in ok if c["t_done"] <= span]
        lat = np.array([c["t_done"] - c["t_release"] for c in (ok if drain else in_window)]) * 1e3
        by_n, svc_n = {}, {}
        for c in ok:
            by_n.setdefault(sizes[c["matrix"]], []).append(1e3 * (c["t_done"] - c["t_release"]))
            svc_n.setdefault(sizes[c["matrix"]], []).append(1e3 * (c["t_done"] - c["t_start"]))
        return {"offered_per_s": rate_, "arrivals": len(reqs), "window_s": span,
                "completed": len(ok), "completed_in_window": len(in_window),
                "updates_per_s": (len(ok) / max(c["t_done"] for c in ok)) if drain and ok
                else len(in_window) / span,
                "latency_ms": {"p50": float(np.percentile(lat, 50)) if lat.size else None,
                               "p99": float(np.percentile(lat, 99)) if lat.size else None},
                "latency_p50_ms_by_n": {str(n): float(np.percentile(v, 50)) for n, v in sorted(by_n.items())},
                "completed_by_n": {str(n): len(v) for n, v in sorted(by_n.items())},
                "service_ms_mean_by_n": {str(n): float(np.mean(v)) for n, v in sorted(svc_n.items())},
                "backlog_at_end_of_arrivals": int(backlog),
                "mean_batch": (st["updates"] / st["batches"]) if st["batches"] else None,
                "errors": len(done) - len(ok)}

    res = {"workload": "64 resident matrices, m=n from {256,1024,2048,4096,8192}, Poisson arrivals, "
                       "uniform targets, a,b~N(0,1/n)", "sizes_count": {str(n): sizes.count(n) for n in haar},
           "resident_bytes": resident, "workers": workers}
    res["stated_rate"] = run(rate, arrival_s, drain=False)
    sus = 0.7 * res["stated_rate"]["updates_per_s"]
    res["sustainable_rate"] = run(sus, sustain_s, drain=True)
    res["stated_rate_fmm_n_ge_4096"] = run(rate, arrival_s, drain=False, fmm_min_n=4096)
    sus_f = 0.7 * res["stated_rate_fmm_n_ge_4096"]["updates_per_s"]
    res["sustainable_rate_fmm_n_ge_4096"] = run(sus_f, sustain_s, drain=True, fmm_min_n=4096)
    return res


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--m", type=int, default=8192)
    ap.add_argument("--n", type=int, default=8192)
    ap.add_argument("--seed", type=int, default=2026)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--haar", choices=("device", "host"), default="device",
                    help="where the Haar factors are drawn: torch QR on the GPU, or numpy QR on the host "
                         "(no library kernels besides libsvdu's run on the GPU then; for counter runs)")
    ap.add_argument("--no-check", action="store_true", help="skip the reconstruction spot check")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the short measurements of the other forms (precision form) on the same inputs")
    ap.add_argument("--path", choices=("direct", "fmm"), default="direct",
                    help="product path of the timed steps (the metric is the direct path; fmm is for profiling)")
    ap.add_argument("--precision", choices=("fp64", "int8", "split32"), default="fp64",
                    help="arithmetic of the products in the timed steps (the metric is fp64; the others are for "
                         "profiling the precision forms)")
    ap.add_argument("--slices", type=int, default=7, help="slices of the int8 form in the timed steps")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched form")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving form")
    ap.add_argument("--serving-window", type=float, default=50.0,
                    help="seconds of arrivals at the stated rate (50 s: the 100k-request stream at 2000/s)")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the other workloads (m=n=256 latency, m=n=4096 direct vs FMM, m=4096 n=8192 "
                         "precision forms, FMM order sweep, secular far field, direct vs FMM crossover)")
    ap.add_argument("--serving-only", action="store_true", help="measure only the serving form")
    ap.add_argument("--batch-reps", type=int, default=5, help="timed launches of the batched workload")
    ap.add_argument("--batched-only", action="store_true",
                    help="measure only the batched form (for profiling it)")
    ap.add_argument("--tile", type=int, default=-1,
                    help="force the product tile shape of the timed steps (SVDU_TILE_*; -1: tuning table)")
    ap.add_argument("--tile-table", default="",
                    help="with --batched-only: FP64 tile shapes per size bucket (comma list) instead of tuning")
    ap.add_argument("--profile-copy", type=int, default=0,
                    help="run only N plain 1 GiB device copies (counter calibration) and exit")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path "
              "(the update shards by rows with one all-reduce of the projections; not built).",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1707_08369_amd as svdu
    import synth_inputs as S

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")

    if args.profile_copy:
        src = torch.ones(1 << 27, dtype=torch.float64, device=dev)   # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(args.profile_copy):
            torch.mul(src, 1.0, out=dst)      # one elementwise kernel: 1 GiB read, 1 GiB written
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_each": src.numel() * 8, "copies": args.profile_copy}))
        return

    if args.serving_only:
        print(json.dumps(measure_serving(svdu, torch, arrival_s=args.serving_window)))
        return
    if args.batched_only:
        table = [int(x) for x in args.tile_table.split(",")] if args.tile_table else None
        print(json.dumps(measure_batched(svdu, torch, reps=args.batch_reps, check=False, modes=("fp64_graph",),
                                         table=table, one_by_one=False)))
        return

    m, n, K, W = args.m, args.n, args.steps, args.warmup
    rng = np.random.default_rng(args.seed)
    if args.haar == "device":
        U = S.haar_torch(m, seed=args.seed + 1, device="cuda")
        V = S.haar_torch(n, seed=args.seed + 2, device="cuda")
    else:
        U = torch.as_tensor(S.haar(m, S.rng_for(args.seed + 1)), device=dev)
        V = torch.as_tensor(S.haar(n, S.rng_for(args.seed + 2)), device=dev)
    sigma = torch.as_tensor(S.sigma_uniform(m, 1e-3, 1.0, rng), device=dev)
    A_vecs = torch.as_tensor(rng.standard_normal((W + K, m)) / np.sqrt(n), device=dev)
    B_vecs = torch.as_tensor(rng.standard_normal((W + K, n)) / np.sqrt(n), device=dev)
    Uo = torch.empty((m, m), dtype=torch.float64, device=dev)
    so = torch.empty(m, dtype=torch.float64, device=dev)
    Vo = torch.empty((n, n), dtype=torch.float64, device=dev)
    path = svdu.SVDU_PATH_FMM if args.path == "fmm" else svdu.SVDU_PATH_DIRECT
    prec = {"fp64": svdu.SVDU_PREC_FP64, "int8": svdu.SVDU_PREC_SLICED_INT8,
            "split32": svdu.SVDU_PREC_SPLIT32}[args.precision]
    if args.tile >= 0:
        svdu.set_option(svdu.SVDU_OPT_TILE_SHAPE, args.tile)
    svdu.set_option(svdu.SVDU_OPT_SLICES, args.slices)
    ws = svdu.new_workspace(svdu.svdu_workspace_bytes(m, n, path, prec), dev)
    stream = torch.cuda.current_stream()

    def step(k, check=False):
        svdu.rank1_update(U, sigma, V, A_vecs[k], B_vecs[k], eps=1e-10, path=path, precision=prec,
                          out=(Uo, so, Vo), workspace=ws, want_defl=False, stream=stream, check=check)

    for k in range(W):
        step(k, check=(k == 0))
    torch.cuda.synchronize()
    print(f"[bench] m={m} n={n} warmup={W} done", file=sys.stderr, flush=True)

    svdu.set_option(svdu.SVDU_OPT_TIMING, 1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(W, W + K):
        step(k)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    phases = svdu.timing_read(K)
    svdu.set_option(svdu.SVDU_OPT_TIMING, 0)
    status = svdu.svdu_get_status(svdu._aligned(ws)[0], svdu._stream_handle(stream))
    if status != 0:
        print(f"[bench] device status {svdu.svdu_status_string(status)}", file=sys.stderr)
        sys.exit(1)
    print(f"[bench] timed {K} steps in {t1 - t0:.3f} s", file=sys.stderr, flush=True)

    # correctness spot check of the last timed update (not timed)
    recon = None
    if not args.no_check:
        k = W + K - 1
        Ah = (U * sigma[None, :]) @ V[:, :m].T + torch.outer(A_vecs[k], B_vecs[k])
        recon = ((Uo * so[None, :]) @ Vo[:, :m].T - Ah).norm().item() / Ah.norm().item()

    ph = np.asarray(phases)                       # K x 5 ms
    per_update = ph.sum(axis=1)
    gemm_ms = ph[:, 2:4]                          # the two product launches of each update
    mean_flops = 2.0 * m ** 3 + 2.0 * n ** 3      # per launch
    mean_gemm_ms = float(gemm_ms.mean())
    achieved = mean_flops / (mean_gemm_ms * 1e-3) / 1e12
    traffic = load_traffic(m, n)

    value = K / (t1 - t0)
    plain = args.path == "direct" and args.precision == "fp64"
    out = {
        "metric": ("rank-1 SVD updates/s at m=n=8192 (plain FP64 GPU path); p50/p99 update latency" if plain else
                   f"rank-1 SVD updates/s at m=n=8192 ({args.precision} products, {args.path} path; not the metric's "
                   f"plain FP64 path); p50/p99 update latency"),
        "value": value,
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": 1e3 * (t1 - t0) / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "int8": "i8 slices (exact i32 sums, f64 results)", "split32": "f32x3"}[args.precision],
        "data": "synthetic",
        "config": {"workload": f"rank1_svd_update m={m} n={n} sigma~U[1e-3,1] haar U,V a,b~N(0,1/n) "
                               f"{args.precision} {args.path} product", "m": m, "n": n, "path": args.path,
                   "precision": args.precision,
                   "seed": args.seed},
        "latency_ms": {"p50": float(np.percentile(per_update, 50)), "p99": float(np.percentile(per_update, 99)),
                       "mean": float(per_update.mean())},
        "phase_ms_mean": {"projections": float(ph[:, 0].mean()), "eigen_updates_small": float(ph[:, 1].mean()),
                          "products": float(gemm_ms.sum(axis=1).mean()), "flags": float(ph[:, 4].mean())},
        "recon_last": recon,
        # the product-phase times of the FMM path cover a dozen kernels, so the
        # GEMM roofline below only describes the direct path
        "roofline": None if not plain else {
            "bound": "mfma",
            "kernel": "gemm_cauchy_f64_kernel<2, 2, 4, 8> (256x128 tiles on 8 waves, 64-k LDS stages)",
            "achieved": achieved,
            "peak": FP64_MFMA_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / FP64_MFMA_PEAK_TFLOPS,
            "traffic": traffic,
            "flops_per_launch": mean_flops,
            "mean_launch_ms": mean_gemm_ms,
        },
    }
    if not args.no_forms:
        print("[bench] precision forms and FMM at the benchmark size ...", file=sys.stderr, flush=True)
        out["forms"] = measure_forms(svdu, torch, U, sigma, V, A_vecs, B_vecs, Uo, so, Vo, stream,
                                     fp64_ms=1e3 * (t1 - t0) / K, check=not args.no_check)
    del ws
    base_inputs = (U, sigma, V, A_vecs[W], B_vecs[W])
    if not args.no_configs:
        cf = out.setdefault("configs", {})
        print("[bench] m=n=256 latency ...", file=sys.stderr, flush=True)
        cf["m256_latency"] = measure_config_small(svdu, torch)
        print("[bench] m=n=4096 direct vs FMM ...", file=sys.stderr, flush=True)
        cf["m4096_direct_vs_fmm"] = measure_config_4096(svdu, torch)
        print("[bench] m=4096 n=8192 precision forms ...", file=sys.stderr, flush=True)
        cf["m4096_n8192_precision"] = measure_config_3a(svdu, torch)
        print("[bench] FMM order sweep ...", file=sys.stderr, flush=True)
        cf["fmm_order_sweep"] = measure_fmm_order_sweep(svdu, torch)
        print("[bench] secular sums: direct vs far field ...", file=sys.stderr, flush=True)
        cf["secular_far_field"] = measure_secular_far_field(svdu, torch)
        print("[bench] direct vs FMM crossover ...", file=sys.stderr, flush=True)
        cf["fmm_crossover"] = measure_fmm_crossover(svdu, torch)
    if not args.no_serving:
        print("[bench] serving form ...", file=sys.stderr, flush=True)
        out.setdefault("forms", {})["serving"] = measure_serving(svdu, torch, arrival_s=args.serving_window)
    if not args.no_batched:
        print("[bench] batched form ...", file=sys.stderr, flush=True)
        out.setdefault("forms", {})["batched_512"] = measure_batched(svdu, torch, reps=args.batch_reps,
                                                                     check=not args.no_check)
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (one oracle update) ...", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(*base_inputs)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
