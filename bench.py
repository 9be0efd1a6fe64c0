"""Benchmark of the RBF-FD Laplacian hot path on one MI355X.

One step = one pass of the whole path over the unit-disk workload (about
100k jittered interior nodes plus 1000 boundary nodes, m = 4, n = 30):
kNN supports -> FP64 stencil weights -> CSR operator with Dirichlet rows ->
residual W u - f.  Inputs are resident in HBM before the timed region.

Printed: one JSON line with whole-step throughput (stencils/s), the
roofline position of the dominant kernel (the weights kernel, timed live
with HIP events on the stream it runs on), the oracle's CPU throughput on a
bounded sample of the same workload, and per-order / mixed-order weights
throughputs on the 1M-node square as extra fields.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6      # 256 CU x 4 SIMD x 16 lanes x 2 flop (FMA) x 2.4 GHz
HBM_PEAK_GBS = 8000.0


def n_monomials(m: int) -> int:
    return (m + 1) * (m + 2) // 2


def weights_flops(m: int, n: int) -> int:
    """Algorithmic FP64 flops of one stencil: LU of the K x K system, the two
    triangular solves and the assembly (pivot search and swaps not counted,
    a square root counts as one)."""
    M = n_monomials(m)
    K = n + M
    lu = (K - 1) * K // 2 + (K - 1) * K * (2 * K - 1) // 3
    solves = 2 * K * (K - 1) + K
    assembly = 4 * n * (n - 1) + 12 * (n - 1) + n * (M - 1) + n
    return lu + solves + assembly


def weights3_flops(n: int, m: int = 2) -> int:
    """The same count for the 3-D stencil (M = (m+1)(m+2)(m+3)/6 monomials,
    K = n + M): LU and solves as above; assembly 5 n (n - 1) (half the pairs,
    3 differences, 3 squares, 2 sums, a square root and a product each),
    18 (n - 1) for the offsets, scale and right-hand side, n (M - 1)
    monomial products, n."""
    M = (m + 1) * (m + 2) * (m + 3) // 6
    K = n + M
    lu = (K - 1) * K // 2 + (K - 1) * K * (2 * K - 1) // 3
    solves = 2 * K * (K - 1) + K
    assembly = 5 * n * (n - 1) + 18 * (n - 1) + n * (M - 1) + n
    return lu + solves + assembly


def source_digest(paths) -> str:
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


# sources of the dominant kernel (K = 45 instance of the blocked MFMA kernel)
WEIGHTS_SOURCES = ["paper_2107_03632_amd/csrc/common.h",
                   "paper_2107_03632_amd/csrc/weights_kernel.h",
                   "paper_2107_03632_amd/csrc/weights_ms.h",
                   "paper_2107_03632_amd/csrc/weights_mf.h",
                   "paper_2107_03632_amd/csrc/weights_k45.hip"]
WEIGHTS_KERNEL = "weights_mf_kernel<45, 30, 4, 1, 4, false, 0>"


def read_traffic(kernel_tag: str):
    """HBM bytes per launch from the committed rocprofv3 --pmc summary, or
    None when the kernel source changed after the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"{kernel_tag}_traffic.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    if kv.get("source_sha") != source_digest(WEIGHTS_SOURCES):
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def measured_fma_peak(torch, dev, dtype: int, blocks: int = 8192, iters: int = 4096):
    """TFLOP/s of a plain vector FMA loop on this device (dtype 0 FP64, 1 FP32),
    from the calibration library built beside librbffd."""
    import ctypes
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_2107_03632_amd", "libcalib.so"))
    lib.calib_fma_loop.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p,
                                   ctypes.c_int32, ctypes.c_void_p]
    sink = torch.empty(blocks * 256, dtype=torch.float64 if dtype == 0 else torch.float32,
                       device=dev)
    stream = torch.cuda.current_stream(dev)

    def run():
        rc = lib.calib_fma_loop(dtype, iters, ctypes.c_void_p(sink.data_ptr()), blocks,
                                ctypes.c_void_p(stream.cuda_stream))
        if rc != 0:
            raise RuntimeError(f"calib_fma_loop failed: {rc}")
    ms = timed(torch, stream, run, reps=3)
    return blocks * 256 * iters * 8 * 2 / (ms * 1e-3) / 1e12


def host_cpu():
    """The host's CPU model, its logical CPU count and the threads this
    process may use (its affinity set, capped by OMP_NUM_THREADS if set)."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    avail = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    env = os.environ.get("OMP_NUM_THREADS", "")
    threads = min(avail, int(env)) if env.isdigit() and int(env) > 0 else avail
    return model, os.cpu_count(), max(1, threads)


def _oracle_rows_parallel(fn, rows, threads):
    """fn(chunk) over `rows` split into contiguous chunks, one host thread
    each.  The oracle's C calls release the GIL, so the chunks run on
    separate cores; each stencil is computed exactly as in a serial call."""
    import concurrent.futures as cf
    chunks = [c for c in np.array_split(rows, threads * 4) if c.size]
    with cf.ThreadPoolExecutor(max_workers=threads) as ex:
        return list(ex.map(fn, chunks))


def cpu_baseline(ns, m, n, stride):
    """The oracle (plain C, one stencil at a time, unchanged) on the host.
    All cores: the whole bench step over every stencil of the workload
    (brute-force kNN, weights, CSR rows, SpMV rows), rows split over host
    threads, with kNN and weights also reported alone.  One core: every
    stride-th stencil, as the paper times its CPU (one core).  Per order:
    weights alone at m = 2, 4, 6 on the 10k-node square."""
    import oracle
    from paper_2107_03632_amd import nodes
    model, nproc, threads = host_cpu()
    N = ns.n_nodes
    u, f = nodes.manufactured(ns.x, ns.y)

    # all cores, every stencil
    rows = np.arange(N)
    t0 = time.perf_counter()
    parts = _oracle_rows_parallel(lambda c: oracle.knn(ns.x, ns.y, n, queries=c), rows, threads)
    nb = np.concatenate(parts)
    t1 = time.perf_counter()
    parts = _oracle_rows_parallel(lambda c: oracle.weights(ns.x, ns.y, nb, m=m, n=n, rows=c),
                                  rows, threads)
    w = np.concatenate([p[0] for p in parts])
    t2 = time.perf_counter()
    rp, col, val = oracle.csr(nb, w, n=n, is_boundary=ns.is_boundary)
    oracle.spmv(rp, col, val, u, f)
    t3 = time.perf_counter()

    # one core, every stride-th stencil
    srows = np.arange(0, N, stride)
    s0 = time.perf_counter()
    snb = oracle.knn(ns.x, ns.y, n, queries=srows)
    s1 = time.perf_counter()
    full = np.zeros((N, n), dtype=np.int32)
    full[srows] = snb
    sw, _ = oracle.weights(ns.x, ns.y, full, m=m, n=n, rows=srows)
    s2 = time.perf_counter()
    srp, scol, sval = oracle.csr(snb, sw, n=n, is_boundary=ns.is_boundary[srows])
    oracle.spmv(srp, scol, sval, u, f[srows])
    s3 = time.perf_counter()

    # weights alone per order, all cores, on the 10k-node square (h = 1e-2)
    sq = nodes.workload("square_10k_m6")
    sqrows = np.arange(sq.n_nodes)
    per_order = {}
    for mo, no in ((2, 12), (4, 30), (6, 56)):
        nbo = np.concatenate(_oracle_rows_parallel(
            lambda c: oracle.knn(sq.x, sq.y, no, queries=c), sqrows, threads))
        q0 = time.perf_counter()
        _oracle_rows_parallel(lambda c: oracle.weights(sq.x, sq.y, nbo, m=mo, n=no, rows=c),
                              sqrows, threads)
        q1 = time.perf_counter()
        per_order[f"m{mo}_n{no}"] = {"weights_stencils_per_s": sq.n_nodes / (q1 - q0),
                                     "s": q1 - q0}

    return {"value": N / (t3 - t0), "unit": "stencils/s", "cores": threads, "kind": "oracle",
            "sample": f"all {N} stencils of the workload on {threads} host threads (rows "
                      f"split into chunks): brute-force kNN {t1 - t0:.2f} s, weights "
                      f"{t2 - t1:.2f} s, CSR+SpMV {t3 - t2:.2f} s (one thread)",
            "host_cpu": model, "nproc": nproc,
            "knn_only_stencils_per_s": N / (t1 - t0),
            "weights_only_stencils_per_s": N / (t2 - t1),
            "single_core": {
                "value": len(srows) / (s3 - s0), "cores": 1,
                "knn_only_stencils_per_s": len(srows) / (s1 - s0),
                "weights_only_stencils_per_s": len(srows) / (s2 - s1),
                "sample": f"{len(srows)} of {N} stencils (every {stride}th node): kNN "
                          f"{s1 - s0:.2f} s, weights {s2 - s1:.2f} s, CSR+SpMV "
                          f"{s3 - s2:.2f} s"},
            "per_order_weights_square_10k": per_order}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the per-order and mixed-order 1M-node measurements")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one plain device copy of known size first (for --pmc scaling)")
    ap.add_argument("--cpu-stride", type=int, default=7)
    ap.add_argument("--profile-case", default=None,
                    help="only run one weights launch pattern under a profiler: "
                         "{fp64,mixed}_m{2,4,6} on the 1M-node square, cube_m{2,4} / "
                         "cube40_m4 on the 3-D lattice (prints its timing)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}, "
              f"WORLD_SIZE={world}); stencils are independent and would shard by "
              f"rows, but only the one-GPU path is built", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2107_03632_amd import binding as rb
    from paper_2107_03632_amd import nodes

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    if args.profile_case:
        profile_case(torch, rb, nodes, dev, args.profile_case, args.warmup, args.steps)
        return

    if args.copy_calibration:
        nbytes = 1 << 30
        a = torch.empty(nbytes // 8, dtype=torch.float64, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        print(f"copy calibration: {nbytes} bytes read, {nbytes} bytes written", file=sys.stderr)
        del a, b

    m, n = 4, 30
    ns = nodes.workload("disk_100k_m4")
    N = ns.n_nodes
    X = torch.as_tensor(ns.x, device=dev)
    Y = torch.as_tensor(ns.y, device=dev)
    B = torch.as_tensor(ns.is_boundary, device=dev)
    u_h, f_h = nodes.manufactured(ns.x, ns.y)
    U = torch.as_tensor(u_h, device=dev)
    F = torch.as_tensor(f_h, device=dev)
    stream = torch.cuda.current_stream(dev)

    ev = []

    def step(record):
        nbr = rb.rbffd_knn(X, Y, n)
        if record:
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
        w, st, _ = rb.rbffd_weights(X, Y, nbr, m=m, n=n)
        if record:
            e1.record(stream)
            ev.append((e0, e1))
        rp, col, val = rb.rbffd_assemble_csr(nbr, w, n=n, is_boundary=B)
        r = rb.rbffd_spmv(rp, col, val, U, F)
        return r, st

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        r, st = step(True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_eager = 1e3 * elapsed / args.steps

    # The same step captured once in a graph and replayed: every kernel of
    # the step runs at every replay (its outputs in the graph's pool), with
    # no host work between the launches.  The headline figure.
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        step(False)  # warm-up on the capture stream
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        r_g, st_g = step(False)
    for _ in range(args.warmup):
        graph.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        graph.replay()
    torch.cuda.synchronize()
    ms_step = 1e3 * (time.perf_counter() - t0) / args.steps
    if not (torch.equal(r_g, r) and torch.equal(st_g, st)):
        raise SystemExit("bench: the graph replay differs from the eager step")
    w_ms = [a.elapsed_time(b) for a, b in ev]
    w_ms_avg = float(np.mean(w_ms))
    bad = int((st != 0).sum().item())
    resid = r[B == 0].abs().max().item()

    flops_launch = weights_flops(m, n) * N
    achieved = flops_launch / (w_ms_avg * 1e-3) / 1e12
    traffic = read_traffic("weights_k45_disk100k")
    fma64 = measured_fma_peak(torch, dev, 0)
    fma32 = measured_fma_peak(torch, dev, 1)
    out = {
        # the headline metric; this line's value is its m = 4 FP64 point on the
        # unit disk, per whole step (the workload below), and the m = 2/4/6
        # FP64 and mixed figures are in per_order_1M_square
        "metric": "RBF-FD \u2207\u00b2 stencils/sec at m=2/4/6 (FP64 vs mixed+refine); "
                  "% of FLOP roofline",
        "value": N / (ms_step * 1e-3),
        "unit": "stencils/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "ms_per_step_eager": ms_eager,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded jittered lattice on the unit disk)",
        "config": {"workload": "unit disk, 100k jittered lattice nodes + 1000 boundary, "
                               "m=4, n=30, FP64: kNN -> weights -> CSR -> W u - f",
                   "launch": "the step captured in a graph, replayed once per step "
                             "(ms_per_step_eager: the same step launched from the host)",
                   "n_nodes": N, "m": m, "n": n, "global_batch": N, "parallelism": "none"},
        # the FP64 MFMA peak of this chip equals its FP64 vector peak; the
        # kernel is bound by its vector instruction stream (column steps)
        "roofline": {"bound": "alu", "kernel": WEIGHTS_KERNEL,
                     "achieved": achieved, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP64_PEAK_TFLOPS, "traffic": traffic,
                     "flops_per_stencil": weights_flops(m, n), "launch_ms": w_ms_avg,
                     "measured_fp64_fma_tflops": fma64, "frac_of_measured": achieved / fma64,
                     "measured_fp32_fma_tflops": fma32},
        "weights_stencils_per_s": N / (w_ms_avg * 1e-3),
        "failed_stencils": bad,
        "residual_max_interior": resid,
    }

    if not args.no_extras:
        out["implicit_solve_unit_disk"] = extras_solve(torch, rb, nodes, dev, X, Y, B, U, F,
                                                       ns, m, n)
        stages = [
            ("per_order_1M_square", lambda: extras_per_order(torch, rb, nodes, dev, stream)),
            ("adjoint_annulus_200k_m4", lambda: extras_adjoint(torch, rb, nodes, dev, stream)),
            ("time_loop_unit_disk", lambda: extras_time_loop(torch, rb, nodes, dev, stream)),
            ("time_loop_cache_sweep",
             lambda: extras_time_loop_sweep(torch, rb, nodes, dev, stream)),
            ("derivative_weights_unit_disk",
             lambda: extras_ops(torch, rb, stream, X, Y, ns, m, n)),
            ("laplacian_3d_cube_1m", lambda: extras_3d(torch, rb, nodes, dev, stream)),
        ]
        for name, fn in stages:
            t_stage = time.perf_counter()
            out[name] = fn()
            print(f"bench: {name} done in {time.perf_counter() - t_stage:.1f} s",
                  file=sys.stderr, flush=True)

    if not args.no_cpu_baseline:
        t_stage = time.perf_counter()
        out["cpu_baseline"] = cpu_baseline(ns, m, n, args.cpu_stride)
        print(f"bench: cpu_baseline done in {time.perf_counter() - t_stage:.1f} s",
              file=sys.stderr, flush=True)

    print(json.dumps(out), flush=True)


def timed(torch, stream, fn, reps=3):
    fn()
    ts = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        fn()
        e1.record(stream)
        e1.synchronize()
        ts.append(e0.elapsed_time(e1))
    return float(np.median(ts))


def profile_case(torch, rb, nodes, dev, case, warmup, steps):
    """One weights launch pattern, for kernel traces and counters: `warmup`
    untimed calls, then `steps` timed ones.  fp64_m{2,4,6}, mixed_m{2,4,6}:
    the 1M-node square; cube_m{2,4}: the 3-D Laplacian on the jittered 100^3
    lattice (n = 20, 70); cube40_m4: the same on the 40^3 lattice."""
    prec, mpart = case.split("_")
    m = int(mpart[1:])
    stream = torch.cuda.current_stream(dev)
    if prec in ("cube", "cube40"):
        if m not in (2, 4):
            raise SystemExit(f"unknown profile case {case}")
        n = {2: 20, 4: 70}[m]
        x, y, z = nodes.jittered_cube(100 if prec == "cube" else 40, seed=6)
        X, Y, Z = (torch.as_tensor(a, device=dev) for a in (x, y, z))
        nb = rb.rbffd_knn3(X, Y, Z, n)
        N = x.shape[0]
        out = torch.empty((N, n), dtype=torch.float64, device=dev)
        st = torch.empty(N, dtype=torch.int32, device=dev)

        def run():
            rb.rbffd_weights3(X, Y, Z, nb, m, n, out=out, status=st)
    else:
        n = {2: 12, 4: 30, 6: 56}.get(m)
        if prec not in ("fp64", "mixed") or n is None:
            raise SystemExit(f"unknown profile case {case}")
        ns = nodes.workload("square_1m_m6")
        X = torch.as_tensor(ns.x, device=dev)
        Y = torch.as_tensor(ns.y, device=dev)
        nb = rb.rbffd_knn(X, Y, n)
        N = ns.n_nodes
        out = torch.empty((N, n), dtype=torch.float64, device=dev)
        st = torch.empty(N, dtype=torch.int32, device=dev)
        pr = rb.MIXED if prec == "mixed" else rb.FP64

        def run():
            rb.rbffd_weights(X, Y, nb, m=m, n=n, precision=pr, out=out, status=st)
    for _ in range(max(warmup, 0)):
        run()
    torch.cuda.synchronize()
    ts = []
    for _ in range(steps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        run()
        e1.record(stream)
        e1.synchronize()
        ts.append(e0.elapsed_time(e1))
    print(json.dumps({"profile_case": case, "n_nodes": N, "ms": ts,
                      "statuses": np.bincount(st.cpu().numpy()).tolist()}), flush=True)


def extras_per_order(torch, rb, nodes, dev, stream):
    """Weights-kernel throughput on the 1M-node cell-centred square at m = 2,
    4, 6 (uniform), FP64 and mixed precision (FP32 factorisation + FP64
    refinement), and for the per-node {2,4,6} mixed-order batch.  The mixed
    weights' error is taken against the FP64 weights of the same call
    sequence (the FP64 path reproduces the oracle bit for bit)."""
    ns = nodes.workload("square_1m_mixed")
    X = torch.as_tensor(ns.x, device=dev)
    Y = torch.as_tensor(ns.y, device=dev)
    nbr = rb.rbffd_knn(X, Y, 56)
    N = ns.n_nodes
    res = {"n_nodes": N}
    for m, n in ((2, 12), (4, 30), (6, 56)):
        nb = nbr[:, :n].contiguous()
        ms = timed(torch, stream, lambda: rb.rbffd_weights(X, Y, nb, m=m, n=n))
        w64, st64, _ = rb.rbffd_weights(X, Y, nb, m=m, n=n)
        it = torch.zeros(N, dtype=torch.int32, device=dev)
        ms_mx = timed(torch, stream,
                      lambda: rb.rbffd_weights(X, Y, nb, m=m, n=n, precision=rb.MIXED))
        wmx, stmx, _ = rb.rbffd_weights(X, Y, nb, m=m, n=n, precision=rb.MIXED, refine_steps=it)
        ok = (stmx == 0)
        err = ((wmx - w64).abs().amax(1) / w64.abs().amax(1)).max().item()
        fl = weights_flops(m, n) * N / 1e12
        res[f"m{m}_n{n}"] = {
            "fp64": {"stencils_per_s": N / (ms * 1e-3), "ms": ms,
                     "frac_fp64_peak": fl / (ms * 1e-3) / FP64_PEAK_TFLOPS,
                     "failed": int((st64 != 0).sum().item())},
            "mixed": {"stencils_per_s": N / (ms_mx * 1e-3), "ms": ms_mx,
                      "speedup_vs_fp64": ms / ms_mx,
                      "target_met": bool(ms / ms_mx > 1.0 and err <= 1e-9),
                      "mean_corrections": it[ok].double().mean().item() if ok.any() else None,
                      "fell_back": int((stmx == rb.FELL_BACK_FP64).sum().item()),
                      "failed": int(((stmx != 0) & (stmx != rb.FELL_BACK_FP64)).sum().item()),
                      "max_rel_err_vs_fp64": err},
        }
    O = torch.as_tensor(ns.order, device=dev)
    ms = timed(torch, stream, lambda: rb.rbffd_weights(X, Y, nbr, order=O))
    ms_graph = graph_timed(torch, lambda: rb.rbffd_weights(X, Y, nbr, order=O))
    ms_mx = timed(torch, stream, lambda: rb.rbffd_weights(X, Y, nbr, order=O, precision=rb.MIXED))
    counts = {mm: int((ns.order == mm).sum()) for mm in (2, 4, 6)}
    fl = sum(counts[mm] * weights_flops(mm, nn) for mm, nn in ((2, 12), (4, 30), (6, 56)))
    # baselines for the one-launch batch: the same stencils as three
    # single-order launches (from the uniform 1M runs above), and every
    # stencil padded to the order-6 system (the uniform m = 6 run)
    per_order = sum(counts[mm] / N * res[f"m{mm}_n{nn}"]["fp64"]["ms"]
                    for mm, nn in ((2, 12), (4, 30), (6, 56)))
    padded = res["m6_n56"]["fp64"]["ms"]
    res["mixed_order"] = {"fp64": {"stencils_per_s": N / (ms * 1e-3), "ms": ms,
                                   "speedup_vs_padded_k84": padded / ms,
                                   "speedup_vs_single_order_launches": per_order / ms,
                                   "frac_fp64_peak": fl / (ms * 1e-3) / 1e12 / FP64_PEAK_TFLOPS,
                                   "graph_replay_ms": ms_graph,
                                   "graph_stencils_per_s": N / (ms_graph * 1e-3)},
                          "mixed": {"stencils_per_s": N / (ms_mx * 1e-3), "ms": ms_mx,
                                    "speedup_vs_fp64": ms / ms_mx}}
    res["knn_k56_ms"] = timed(torch, stream, lambda: rb.rbffd_knn(X, Y, 56))
    # m = 6 at h = 1e-2 (10k nodes): both precisions on the same input
    ns10 = nodes.workload("square_10k_m6")
    X10 = torch.as_tensor(ns10.x, device=dev)
    Y10 = torch.as_tensor(ns10.y, device=dev)
    nb10 = rb.rbffd_knn(X10, Y10, 56)
    ms64 = timed(torch, stream, lambda: rb.rbffd_weights(X10, Y10, nb10, m=6, n=56))
    msmx = timed(torch, stream, lambda: rb.rbffd_weights(X10, Y10, nb10, m=6, n=56,
                                                         precision=rb.MIXED))
    w64, _, _ = rb.rbffd_weights(X10, Y10, nb10, m=6, n=56)
    wmx, stmx, _ = rb.rbffd_weights(X10, Y10, nb10, m=6, n=56, precision=rb.MIXED)
    err = ((wmx - w64).abs().amax(1) / w64.abs().amax(1)).max().item()
    res["square_10k_m6"] = {"n_nodes": ns10.n_nodes, "fp64_ms": ms64, "mixed_ms": msmx,
                            "fell_back": int((stmx == rb.FELL_BACK_FP64).sum().item()),
                            "max_rel_err_mixed_vs_fp64": err}
    return res


def extras_solve(torch, rb, nodes, dev, X, Y, B, U, F, ns, m, n, rtol=1e-10):
    """Implicit solve of the assembled Dirichlet Poisson system on the bench
    disk (BiCGSTAB, rbffd_solve): wall time of the call (it synchronizes),
    iterations, the true relative residual and the error against the
    manufactured solution.  Bytes per iteration on the model of two SpMVs
    (12 B per nonzero + 8 B gathered per nonzero + 16 B per row) and the
    vector updates (14 vectors of 8 B per row)."""
    nbr = rb.rbffd_knn(X, Y, n)
    w, st, _ = rb.rbffd_weights(X, Y, nbr, m=m, n=n)
    rp, col, val = rb.rbffd_assemble_csr(nbr, w, n=n, is_boundary=B)
    b = torch.where(B == 1, U, F)
    rb.rbffd_solve(rp, col, val, b, rtol=rtol)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    x, it, rr, info = rb.rbffd_solve(rp, col, val, b, rtol=rtol)
    ms = 1e3 * (time.perf_counter() - t0)
    N, nnz = ns.n_nodes, int(col.numel())
    per_it = 2 * (20 * nnz + 16 * N) + 14 * 8 * N
    res = {"method": "BiCGSTAB, no preconditioner", "rtol": rtol, "iterations": it,
           "info": info, "relres_true": rr, "ms": ms, "ms_per_iteration": ms / max(it, 1),
           "model_bytes_per_iteration": per_it,
           "model_gb_per_s": per_it * it / (ms * 1e-3) / 1e9,
           "max_err_vs_exact": (x - U).abs().max().item(), "nnz": nnz}
    # the host-synchronisation-free form: eager, then as one captured graph
    # (max_iter iterations enqueued; those after convergence return at once),
    # and with the Jacobi preconditioner
    max_iter = it + 16
    xa = torch.zeros_like(b)
    ws = None
    res_t = torch.empty(16, dtype=torch.int8, device=dev)
    for name, pre in (("none", rb.PRECOND_NONE), ("jacobi", rb.PRECOND_JACOBI)):
        mi = max_iter if pre == rb.PRECOND_NONE else 2 * max_iter

        def run():
            xa.zero_()
            rb.rbffd_solve_async(rp, col, val, b, xa, rtol=rtol, max_iter=mi, precond=pre,
                                 result=res_t, workspace=ws)
        _, _, ws = rb.rbffd_solve_async(rp, col, val, b, xa, rtol=rtol, max_iter=mi,
                                        precond=pre, result=res_t, workspace=ws)
        ms_eager = timed(torch, torch.cuda.current_stream(dev), run, reps=2)
        ms_graph = graph_timed(torch, run, reps=2)
        ia, ra, fa = rb.solve_result(res_t)
        res[f"async_{name}"] = {"iterations": ia, "info": fa, "relres_true": ra,
                                "max_iter_enqueued": mi, "ms_eager": ms_eager,
                                "ms_graph_replay": ms_graph,
                                "max_err_vs_exact": (xa - U).abs().max().item()}
    return res


def extras_ops(torch, rb, stream, X, Y, ns, m, n):
    """First-derivative weights (rbffd_weights_op, d/dx and d/dy) on the bench
    disk: time per launch, the fraction of the FP64 peak on the Laplacian's
    flop count (the same factorisation and solves), and the largest error of
    the differentiated u = sin(pi x) sin(pi y) over all nodes; the mixed
    precision form beside each, and d/dx at m = 6 in both precisions."""
    nbr = rb.rbffd_knn(X, Y, n)
    N = ns.n_nodes
    u = torch.sin(math.pi * X) * torch.sin(math.pi * Y)
    exact = {rb.OP_DX: math.pi * torch.cos(math.pi * X) * torch.sin(math.pi * Y),
             rb.OP_DY: math.pi * torch.sin(math.pi * X) * torch.cos(math.pi * Y)}
    res = {"n_nodes": N, "m": m, "n": n}
    for name, op in (("d_dx", rb.OP_DX), ("d_dy", rb.OP_DY)):
        ms = timed(torch, stream, lambda: rb.rbffd_weights_op(X, Y, nbr, m, n, op))
        w, st = rb.rbffd_weights_op(X, Y, nbr, m, n, op)
        approx = (w * u[nbr.long()]).sum(1)
        res[name] = {"ms": ms, "stencils_per_s": N / (ms * 1e-3),
                     "frac_fp64_peak": weights_flops(m, n) * N / 1e12 / (ms * 1e-3)
                     / FP64_PEAK_TFLOPS,
                     "failed": int((st != 0).sum().item()),
                     "max_abs_err": (approx - exact[op]).abs().max().item()}
        # the same operator in mixed precision (FP32 factorisation + FP64
        # refinement), against the FP64 weights of this call
        ms_mx = timed(torch, stream, lambda: rb.rbffd_weights_op_mixed(X, Y, nbr, m, n, op))
        wmx, stmx = rb.rbffd_weights_op_mixed(X, Y, nbr, m, n, op)
        err = ((wmx - w).abs().amax(1) / w.abs().amax(1)).max().item()
        res[name]["mixed"] = {"ms": ms_mx, "speedup_vs_fp64": ms / ms_mx,
                              "fell_back": int((stmx == rb.FELL_BACK_FP64).sum().item()),
                              "max_rel_err_vs_fp64": err}
    # m = 6 (K = 84) d/dx, FP64 and mixed, on the same disk
    nb56 = rb.rbffd_knn(X, Y, 56)
    ms64 = timed(torch, stream, lambda: rb.rbffd_weights_op(X, Y, nb56, 6, 56, rb.OP_DX))
    msmx = timed(torch, stream, lambda: rb.rbffd_weights_op_mixed(X, Y, nb56, 6, 56, rb.OP_DX))
    res["d_dx_m6"] = {"fp64_ms": ms64, "mixed_ms": msmx, "speedup_vs_fp64": ms64 / msmx}
    return res


def extras_3d(torch, rb, nodes, dev, stream):
    """Three-dimensional nodes: the jittered 100^3 lattice of [0,1]^3 at
    m = 2, n = 20 (K = 30) and m = 4, n = 70 (K = 105).  Per order: kNN and
    weights per launch, the weights' fraction of the FP64 peak, and the
    largest error of the weights applied to u = sin(pi x) sin(pi y)
    sin(pi z) (lap u = -3 pi^2 u) over nodes at least 3 h inside the cube;
    the same for the d/dz weights; and the mixed-order batch (orders 2 / 4
    per node)."""
    x, y, z = nodes.jittered_cube(100, seed=6)
    X, Y, Z = (torch.as_tensor(a, device=dev) for a in (x, y, z))
    N = x.shape[0]
    u = torch.sin(math.pi * X) * torch.sin(math.pi * Y) * torch.sin(math.pi * Z)
    inner = ((X > 0.03) & (X < 0.97) & (Y > 0.03) & (Y < 0.97) & (Z > 0.03) & (Z < 0.97))
    dz_exact = math.pi * torch.sin(math.pi * X) * torch.sin(math.pi * Y) * torch.cos(math.pi * Z)
    res = {"n_nodes": N}
    for m, n in ((2, 20), (4, 70)):
        knn_ms = timed(torch, stream, lambda: rb.rbffd_knn3(X, Y, Z, n))
        nbr = rb.rbffd_knn3(X, Y, Z, n)
        ms = timed(torch, stream, lambda: rb.rbffd_weights3(X, Y, Z, nbr, m, n))
        w, st = rb.rbffd_weights3(X, Y, Z, nbr, m, n)
        lap = (w * u[nbr.long()]).sum(1)
        err = (lap - (-3.0 * math.pi ** 2) * u)[inner].abs().max().item()
        fl = weights3_flops(n, m)
        # d/dz: du/dz = pi sin(pi x) sin(pi y) cos(pi z)
        ms_dz = timed(torch, stream, lambda: rb.rbffd_weights3(X, Y, Z, nbr, m, n, op=rb.OP3_DZ))
        wz, stz = rb.rbffd_weights3(X, Y, Z, nbr, m, n, op=rb.OP3_DZ)
        err_dz = ((wz * u[nbr.long()]).sum(1) - dz_exact)[inner].abs().max().item()
        res[f"m{m}_n{n}"] = {
            "knn_ms": knn_ms, "weights_ms": ms, "stencils_per_s": N / (ms * 1e-3),
            "flops_per_stencil": fl, "frac_fp64_peak": fl * N / 1e12 / (ms * 1e-3) / FP64_PEAK_TFLOPS,
            "failed": int((st != 0).sum().item()), "max_abs_err_inner": err,
            "d_dz": {"ms": ms_dz, "failed": int((stz != 0).sum().item()),
                     "max_abs_err_inner": err_dz}}
        del w, wz, nbr, lap
    # per-node order uniform on {2, 4} (seeded): one call, bucketed on the
    # device, against the two single-order launches scaled to their shares
    nbr = rb.rbffd_knn3(X, Y, Z, 70)
    order = torch.as_tensor(np.random.default_rng(36).choice(np.array([2, 4], np.int8), N),
                            device=dev)
    ms = timed(torch, stream, lambda: rb.rbffd_weights3_batch(X, Y, Z, nbr, order))
    _, st = rb.rbffd_weights3_batch(X, Y, Z, nbr, order)
    n4 = int((order == 4).sum().item())
    single = (n4 * res["m4_n70"]["weights_ms"] + (N - n4) * res["m2_n20"]["weights_ms"]) / N
    fl = n4 * weights3_flops(70, 4) + (N - n4) * weights3_flops(20, 2)
    res["mixed_order_m2_m4"] = {
        "ms": ms, "stencils_per_s": N / (ms * 1e-3), "n_order4": n4,
        "speedup_vs_single_order_launches": single / ms,
        "frac_fp64_peak": fl / 1e12 / (ms * 1e-3) / FP64_PEAK_TFLOPS,
        "failed": int((st != 0).sum().item())}
    return res


def extras_adjoint(torch, rb, nodes, dev, stream):
    """Forward with saved factors, and the adjoint, on the 200k-node annulus
    (m = 4, n = 30), cotangent G ~ N(0, 1)."""
    ns = nodes.workload("annulus_200k_m4")
    X = torch.as_tensor(ns.x, device=dev)
    Y = torch.as_tensor(ns.y, device=dev)
    nbr = rb.rbffd_knn(X, Y, 30)
    G = torch.as_tensor(nodes.gaussian_cotangent(ns.n_nodes, 30, seed=55), device=dev)
    N = ns.n_nodes
    plain = timed(torch, stream, lambda: rb.rbffd_weights(X, Y, nbr, m=4, n=30))
    fwd = timed(torch, stream, lambda: rb.rbffd_weights(X, Y, nbr, m=4, n=30, save=True))
    _, st, sv = rb.rbffd_weights(X, Y, nbr, m=4, n=30, save=True)
    bwd = timed(torch, stream,
                lambda: rb.rbffd_weights_backward(X, Y, nbr, G, sv, status=st, m=4, n=30))
    return {"n_nodes": N, "forward_ms": plain, "forward_saving_factors_ms": fwd,
            "backward_ms": bwd, "backward_stencils_per_s": N / (bwd * 1e-3),
            "save_bytes": int(sv.numel())}


def extras_time_loop(torch, rb, nodes, dev, stream, steps=200, dt=1e-6):
    """The paper's explicit loop (eq. (3)) on unit disks: ms per step and the
    bandwidth of the paper's per-node data model, 8 (4 + n) + 4 (1 + n) bytes
    (weights, values, f and indices), at several N (cache regimes of the
    MI355X: 4 MB L2 per XCD, 256 MB Infinity Cache, 8 TB/s HBM)."""
    res = []
    for n_target, n_bnd, m, n in ((10_000, 300, 2, 12), (100_000, 1000, 2, 12),
                                  (100_000, 1000, 4, 30), (1_000_000, 3000, 2, 12)):
        ns = nodes.unit_disk(n_target, n_bnd, seed=2)
        X = torch.as_tensor(ns.x, device=dev)
        Y = torch.as_tensor(ns.y, device=dev)
        nbr = rb.rbffd_knn(X, Y, n)
        w, st, _ = rb.rbffd_weights(X, Y, nbr, m=m, n=n)
        u_exact, F = nodes.manufactured(ns.x, ns.y)
        f = torch.as_tensor(-F, device=dev)
        B = torch.as_tensor(ns.is_boundary, device=dev)
        u = torch.as_tensor(np.where(ns.is_boundary != 0, u_exact, 0.0), device=dev)
        work = torch.empty_like(u)
        ws = torch.empty(ns.n_nodes * n * 12 + 1024, dtype=torch.uint8, device=dev)
        ms = timed(torch, stream, lambda: rb.rbffd_time_steps(nbr, w, n, f, u, dt, steps,
                                                              is_boundary=B, u_work=work,
                                                              workspace=ws))
        per = ms / steps
        nbytes = ns.n_nodes * (8 * (4 + n) + 4 * (1 + n))
        row = {"n_nodes": ns.n_nodes, "m": m, "n": n, "steps": steps,
               "ms_per_step": per, "node_updates_per_s": ns.n_nodes / (per * 1e-3),
               "model_bytes_per_step": nbytes, "gb_per_s": nbytes / (per * 1e-3) / 1e9,
               "frac_hbm_8tbs": nbytes / (per * 1e-3) / 8e12}
        if n_target == 10_000:
            gms = graph_timed(torch, lambda: rb.rbffd_time_steps(nbr, w, n, f, u, dt, 100,
                                                                 is_boundary=B, u_work=work,
                                                                 workspace=ws))
            row["graph_100_steps_ms_per_step"] = gms / 100
        res.append(row)
    return res


def extras_time_loop_sweep(torch, rb, nodes, dev, stream, dt=1e-6):
    """The cache-regime study of the paper's Table 1, redone for the MI355X:
    microseconds per explicit step and GB/s on the paper's per-node data
    model 8 (4 + n) + 4 (1 + n) bytes, for unit disks of ~1e3 ... 4e6 nodes
    at n = 12, 15, 20, 30, 45, 60 (weights of order m = 2 on each support).
    The MI355X has 4 MB of L2 per XCD and 256 MB of Infinity Cache; the
    model puts those capacities at N = 4e6 / (8 (4 + n) + 4 (1 + n)) and
    256e6 / (...) nodes."""
    ns_list = (1000, 3000, 10_000, 30_000, 100_000, 300_000, 1_000_000, 4_000_000)
    res = []
    for n_target in ns_list:
        ns = nodes.unit_disk(n_target, max(100, int(3 * math.sqrt(n_target))), seed=2)
        X = torch.as_tensor(ns.x, device=dev)
        Y = torch.as_tensor(ns.y, device=dev)
        u_exact, F = nodes.manufactured(ns.x, ns.y)
        f = torch.as_tensor(-F, device=dev)
        B = torch.as_tensor(ns.is_boundary, device=dev)
        u = torch.as_tensor(np.where(ns.is_boundary != 0, u_exact, 0.0), device=dev)
        work = torch.empty_like(u)
        nbr60 = rb.rbffd_knn(X, Y, 60)
        steps = 200 if ns.n_nodes <= 100_000 else 50
        for n in (12, 15, 20, 30, 45, 60):
            nbr = nbr60[:, :n].contiguous()
            w, st, _ = rb.rbffd_weights(X, Y, nbr, m=2, n=n)
            ws = torch.empty(ns.n_nodes * n * 12 + 1024, dtype=torch.uint8, device=dev)
            run = (lambda: rb.rbffd_time_steps(nbr, w, n, f, u, dt, steps, is_boundary=B,
                                                u_work=work, workspace=ws))
            ms = timed(torch, stream, run)
            per = ms / steps
            nbytes = ns.n_nodes * (8 * (4 + n) + 4 * (1 + n))
            row = {"n_nodes": ns.n_nodes, "n": n, "steps": steps,
                   "us_per_step": per * 1e3, "model_bytes": nbytes,
                   "gb_per_s": nbytes / (per * 1e-3) / 1e9,
                   "node_updates_per_s": ns.n_nodes / (per * 1e-3)}
            if ns.n_nodes <= 300_000:
                # the same steps replayed from a captured graph: no host
                # launch between steps
                per_g = graph_timed(torch, run) / steps
                row["us_per_step_graph"] = per_g * 1e3
                row["gb_per_s_graph"] = nbytes / (per_g * 1e-3) / 1e9
            res.append(row)
            del w, ws
        del nbr60
    return res


def graph_timed(torch, fn, reps=3):
    """Median time of one replay of fn captured in a graph (fn allocates its
    outputs and workspace from the graph's private pool)."""
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        fn()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        fn()
    g.replay()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        g.replay()
        e1.record()
        e1.synchronize()
        ts.append(e0.elapsed_time(e1))
    return float(np.median(ts))


if __name__ == "__main__":
    main()
