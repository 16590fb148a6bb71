"""Benchmark: AU-NMF iterations per second on one MI355X.

Workload (default): dense float32 A = W0 H0 + |N(0, 0.01)| with m = n = 65536
(17.2 GB), W0 and H0 U(0,1) of rank 50, factorised at k = 50 by HALS. One
step is one full iteration of Algorithm 1: H H^T, A H^T, the W sweep, W^T W,
the normalisation, W^T A and the H sweep, all in the library's HIP kernels,
with A resident in HBM. Prints one JSON line.

  python bench.py [--steps K] [--warmup W] [--gpus 1] [--workload NAME]
                  [--no-cpu-baseline] [--sample-rows R]

roofline: the dominant kernels are the two large products (A H^T and W^T A,
2 m n k algorithmic flops per launch, k unpadded). Their average launch time
comes from the library's hipEvents on the stream the kernels run on;
achieved = 2 m n k / that time, against the FP32 matrix peak. traffic is the
HBM byte count per launch from the committed rocprofv3 counter summary,
reported only while the product kernel source is unchanged since the counters
were taken.

cpu_baseline: the FP64 oracle (tests only, never the product path) timed on
the host for three iterations of the same algorithm on the workload's own
matrix (copied to the host and upcast to float64 before timing); where the
host lacks the memory, or with --cpu-sample, on a square sample of the same
planted matrix family, scaled by (m n) / (sample rows)^2.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3
PEAK_FP64_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_dense_65536x65536_k50.json")
TRAFFIC_FILE_CSR = os.path.join(ROOT, "profiles", "traffic_csr_spmm_1048576_d1e-4_k50.json")
SPARSE_SOURCES = ("sparse.hip", "common.h", "grid.h")
LOWP_SOURCES = ("gemm_bf16.hip", "common.h")
TRAFFIC_FILE_FP8 = os.path.join(ROOT, "profiles", "traffic_fp8_131072x65536_k100.json")
TRAFFIC_FILE_BF16 = os.path.join(ROOT, "profiles", "traffic_bf16_131072x65536_k100.json")
COPY_CAL_BYTES = 3 << 30

WORKLOADS = {
    "dense-65536x65536-k50-hals-f32": dict(m=65536, n=65536, k=50, k_true=50, algo="hals",
                                           dtype="f32"),
    # the same matrix under the other two local updates (Section 6.3 compares
    # the time per iteration of MU, HALS and ABPP)
    "dense-65536x65536-k50-mu-f32": dict(m=65536, n=65536, k=50, k_true=50, algo="mu",
                                         dtype="f32"),
    "dense-65536x65536-k50-abpp-f32": dict(m=65536, n=65536, k=50, k_true=50, algo="abpp",
                                           dtype="f32"),
    "dense-2000x1000-k10-mu-f64": dict(m=2000, n=1000, k=10, k_true=10, algo="mu", dtype="f64"),
    "csr-1048576x1048576-d1e-4-k50-abpp-f32": dict(m=1 << 20, n=1 << 20, k=50, density=1e-4,
                                                   algo="abpp", dtype="f32", sparse=True),
    "dense-131072x65536-k100-hals-bf16": dict(m=131072, n=65536, k=100, k_true=100, algo="hals",
                                              dtype="bf16"),
    "dense-131072x65536-k100-hals-fp8": dict(m=131072, n=65536, k=100, k_true=100, algo="hals",
                                             dtype="fp8"),
    # Shapes of the paper's Table 1 data sets (synthetic stand-ins; the table
    # quotes 30 iterations at k = 50 on 1536 processors, algorithm not named).
    "dense-1013400x13824-k50-hals-f32": dict(m=1013400, n=13824, k=50, k_true=50, algo="hals",
                                             dtype="f32", table1_s=5.73,
                                             table1_set="Video (dense, 1 Million x 13,824)"),
    "csr-627047x11708841-nnz365M-k50-hals-f32": dict(
        m=627047, n=11708841, k=50, density=3.65e8 / (627047.0 * 11708841.0), algo="hals",
        dtype="f32", sparse=True, table1_s=67.0,
        table1_set="Stack Exchange (sparse, 627,047 x 12 Million)"),
    "csr-118142155x118142155-nnz1020M-powerlaw-k50-hals-f32": dict(
        m=118142155, n=118142155, k=50, nnz=1019903190, gen="powerlaw", algo="hals",
        dtype="f32", sparse=True, table1_s=1500.0,
        table1_set="Webbase-2001 (sparse, 118 Million x 118 Million, 1,019,903,190 entries)"),
    "csr-207360x138240-d1e-3-k50-mu-f32": dict(
        m=207360, n=138240, k=50, density=1e-3, algo="mu", dtype="f32", sparse=True,
        paper_iter_s=0.065,
        paper_set="Sparse synthetic (Erdos-Renyi 207,360 x 138,240, density 0.001), MU, "
                  "16 nodes (Section 6.1)"),
    "dense-8192x4096-k64-mu50-autograd-f32": dict(m=8192, n=4096, k=64, k_true=64, algo="mu",
                                                  dtype="f32", autograd=True, iters=50,
                                                  ckpt_every=10),
    "dense-8192x4096-k64-hals50-autograd-f32": dict(m=8192, n=4096, k=64, k_true=64,
                                                    algo="hals", dtype="f32", autograd=True,
                                                    iters=50, ckpt_every=10),
}


def kernel_source_hash(files=("gemm.hip", "common.h")):
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_1609_09154_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(src_hash, path=TRAFFIC_FILE, workload=None):
    """The committed counter record, if it was taken on the current kernel
    source and (when given) on this workload."""
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_hash") != src_hash:
        return None
    if workload is not None and t.get("workload", workload) != workload:
        return None
    return t


def cpu_baseline(wl, sample_rows, iters=6):
    """Time the FP64 oracle on the host: `iters` iterations of the same
    algorithm on a sample_rows x sample_rows planted matrix of rank k_true."""
    import numpy as np

    import oracle
    from synth import init_factors, planted_dense

    cores = len(os.sched_getaffinity(0))
    for var in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ.setdefault(var, str(cores))
    s = sample_rows
    A = planted_dense(s, s, wl["k_true"], sigma=0.01, seed=1609).astype(np.float32).astype(np.float64)
    W0, H0 = init_factors(s, s, wl["k"], seed=9154)
    oracle.run(A, wl["k"], wl["algo"], 1, W0, H0, track_error=False)  # warm-up
    t0 = time.perf_counter()
    oracle.run(A, wl["k"], wl["algo"], iters, W0, H0, track_error=False)
    dt = (time.perf_counter() - t0) / iters
    scale = (wl["m"] * wl["n"]) / float(s * s)
    try:
        from threadpoolctl import threadpool_info
        used = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        used = cores
    return {"value": 1.0 / (dt * scale), "unit": "iters/s", "cores": int(used), "kind": "oracle",
            "sample": "%d iterations of FP64 %s on a %dx%d planted matrix (k=%d), %.3f s/iter, "
                      "scaled by %.1f to %dx%d" % (iters, wl["algo"].upper(), s, s, wl["k"], dt,
                                                   scale, wl["m"], wl["n"])}


def cpu_baseline_full(A_dev, wl, W0n, H0n, iters=3):
    """Time the FP64 oracle on the workload itself: `iters` iterations of the
    same algorithm on the full matrix, after one untimed iteration, with A
    copied to the host and upcast to float64 once before timing (the
    oracle's products then read it in place)."""
    import oracle

    cores = len(os.sched_getaffinity(0))
    for var in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ.setdefault(var, str(cores))
    A64 = A_dev.cpu().double().numpy()
    k = wl["k"]
    oracle.run(A64, k, wl["algo"], 1, W0n, H0n, track_error=False)  # warm-up
    t0 = time.perf_counter()
    oracle.run(A64, k, wl["algo"], iters, W0n, H0n, track_error=False)
    dt = (time.perf_counter() - t0) / iters
    try:
        from threadpoolctl import threadpool_info
        used = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        used = cores
    return {"value": 1.0 / dt, "unit": "iters/s", "cores": int(used), "kind": "oracle",
            "sample": "%d iterations of FP64 %s on the full %dx%d matrix of this workload "
                      "(k=%d; A upcast to float64 on the host before timing, one untimed "
                      "iteration first), %.3f s/iter" % (iters, wl["algo"].upper(), wl["m"],
                                                         wl["n"], k, dt)}


def host_bytes_free():
    try:
        import psutil
        return psutil.virtual_memory().available
    except Exception:
        return 0


def bpp_report(st, steps, rhs_per_iter):
    """ABPP solver work per iteration from the library's tallies: the
    eliminations' algorithmic FP64 flops against the FP64 vector peak (the
    solver runs on the vector ALUs in double), and how much of each
    elimination's size is its own (size / largest size in its wavefront)."""
    ms = st["ms_luc"] / steps
    fl = st["bpp_flops"] / steps
    tf = fl / (ms * 1e-3) / 1e12 if ms > 0 else 0.0
    mx = st["bpp_size_max_mean"]
    return {"ms_per_iter": round(ms, 4), "rhs_per_iter": rhs_per_iter,
            "solves_per_rhs": round(st["bpp_solves"] / float(steps * rhs_per_iter), 3),
            "algorithmic_flops_per_iter": fl,
            "roofline": {"bound": "alu", "achieved": round(tf, 3), "peak": PEAK_FP64_TFLOPS,
                         "unit": "TFLOP/s", "frac": round(tf / PEAK_FP64_TFLOPS, 4)},
            "size_mean": round(st["bpp_size_mean"], 3), "size_wave_max_mean": round(mx, 3),
            "size_class_mean": round(st["bpp_size_class_mean"], 3),
            "size_mean_over_wave_max": round(st["bpp_size_mean"] / mx, 4) if mx > 0 else None}


def add_paper_context(out, wl):
    """For the Table 1 shapes and the paper's MU timing: the paper's time
    beside ours (other hardware, context only)."""
    if "paper_iter_s" in wl:
        out["paper_context"] = {
            "data_set_shape": wl["paper_set"],
            "paper_seconds_per_iteration": wl["paper_iter_s"],
            "this_seconds_per_iteration": round(out["ms_per_step"] / 1000.0, 5),
        }
        return
    if "table1_s" not in wl:
        return
    out["paper_context"] = {
        "data_set_shape": wl["table1_set"],
        "paper_seconds_30_iterations": wl["table1_s"],
        "paper_platform": "1536 processors (Table 1), algorithm not named",
        "this_seconds_30_iterations": round(30.0 * out["ms_per_step"] / 1000.0, 3),
    }


def copy_calibration(dev):
    """One device copy of COPY_CAL_BYTES: a dispatch of known traffic that
    scales the HBM counters of the other dispatches in a counter run."""
    import torch

    src = torch.ones(COPY_CAL_BYTES // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst


def run_sparse(args, wl):
    """Sparse workload: ER CSR A, ABPP. roofline: the SpMM on HBM, with its
    compulsory bytes (values and column ids once, row pointers, the dense
    operand once, the output once) per launch."""
    import numpy as np
    import torch

    import paper_1609_09154_amd as nmf
    from synth import erdos_renyi_csr, init_factors

    m, n, k = wl["m"], wl["n"], wl["k"]
    dev = torch.device("cuda:0")
    print("[bench] generating %s" % args.workload, file=sys.stderr, flush=True)
    if wl.get("gen") == "powerlaw":
        # drawn on the device: the host copies would be tens of GB; the
        # initial factors are U(0,1) from torch's seeded generator there
        from synth import powerlaw_csr_torch

        rp, ci, cv = powerlaw_csr_torch(m, n, wl["nnz"], seed=1609, device=dev)
        nnz = ci.numel()
        gen = torch.Generator(device=dev)

        def init():
            gen.manual_seed(9154)
            return (torch.rand((m, k), generator=gen, device=dev, dtype=torch.float32),
                    torch.rand((k, n), generator=gen, device=dev, dtype=torch.float32))

        W, H = init()
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
    else:
        csr = erdos_renyi_csr(m, n, wl["density"], seed=1609)
        nnz = csr.nnz
        rp = torch.from_numpy(csr.rowptr).to(dev)
        ci = torch.from_numpy(csr.colidx).to(dev)
        cv = torch.from_numpy(csr.vals.astype(np.float32)).to(dev)
        W0n, H0n = init_factors(m, n, k, seed=9154)
        W0 = torch.from_numpy(W0n.astype(np.float32)).to(dev)
        H0 = torch.from_numpy(H0n.astype(np.float32)).to(dev)
        del csr

        def init():
            return W0.clone(), H0.clone()

        W, H = init()
    torch.cuda.synchronize()
    print("[bench] warmup %d" % args.warmup, file=sys.stderr, flush=True)
    if args.warmup > 0:
        nmf.nmf_csr(rp, ci, cv, n, W, H, algo=wl["algo"], iters=args.warmup, objective=False)
        del W, H
        W, H = init()
    torch.cuda.synchronize()
    print("[bench] timing %d steps" % args.steps, file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    _, st = nmf.nmf_csr(rp, ci, cv, n, W, H, algo=wl["algo"], iters=args.steps, objective=False,
                        timers=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_step = 1000.0 * elapsed / args.steps
    comp_bytes = 8.0 * nnz + 8.0 * (m + 1) + 4.0 * n * k + 4.0 * m * k
    ms_spmm = 0.5 * (st["ms_mm_aht"] + st["ms_mm_wta"]) / args.steps
    achieved = comp_bytes / (ms_spmm * 1e-3) / 1e9
    tr = load_traffic(kernel_source_hash(SPARSE_SOURCES), TRAFFIC_FILE_CSR, args.workload)
    traffic = tr["hbm_bytes_per_launch"] if tr else None
    out = {
        "metric": "NMF iterations/s (sparse %s, %s CSR %dx%d, %d stored entries, k=%d)"
                  % (wl["algo"].upper(), "power-law" if wl.get("gen") == "powerlaw" else "ER",
                     m, n, nnz, k),
        "value": round(args.steps / elapsed, 3), "unit": "iters/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "m": m, "n": n, "k": k, "nnz": nnz,
                   "algorithm": wl["algo"], "parallelism": "single-gpu"},
        "phase_ms_per_step": {p: round(st[f] / args.steps, 4) for p, f in
                              (("mm", "ms_mm"), ("luc", "ms_luc"), ("gram", "ms_gram"))},
        "setup_ms": round(st["ms_setup"], 3),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": traffic,
                     "kernel": "csr_spmm (A H^T and A^T W)", "ms_per_launch": round(ms_spmm, 4),
                     "algorithmic_bytes_per_launch": comp_bytes,
                     "useful_gbs": round(achieved, 1),
                     "traffic_gbs": (round(traffic / (ms_spmm * 1e-3) / 1e9, 1) if traffic
                                     else None),
                     "traffic_frac": (round(traffic / (ms_spmm * 1e-3) / 1e9 / PEAK_HBM_GBS, 4)
                                      if traffic else None)},
    }
    if wl["algo"] == "abpp":
        out["bpp_pivots_per_rhs"] = round(st["bpp_pivots"] / float(args.steps * (m + n)), 3)
        out["nnls_solves_per_s"] = round(args.steps * (m + n) / (st["ms_luc"] * 1e-3), 1)
        out["bpp"] = bpp_report(st, args.steps, m + n)
    if args.copy_calibration:
        copy_calibration(dev)
    add_paper_context(out, wl)
    print(json.dumps(out), flush=True)


def run_lowp(args, wl):
    """Precision workloads: the same planted matrix stored in bfloat16 or
    FP8 E4M3 (the two large products on the BF16 / FP8 matrix cores,
    everything else float32) and in float32, factorised from the same
    initial factors. value is the reduced-precision rate; the FP32 rate and
    both final relative errors (direct residual against the float32 A,
    double accumulation) are reported beside it. roofline: the products
    stream A (2 or 1 bytes per entry) once per launch: HBM-bound at k or 2k
    flops per byte."""
    import torch

    import paper_1609_09154_amd as nmf
    from synth import init_factors, planted_dense_torch

    m, n, k = wl["m"], wl["n"], wl["k"]
    dev = torch.device("cuda:0")
    print("[bench] generating %s" % args.workload, file=sys.stderr, flush=True)
    A32 = planted_dense_torch(m, n, wl["k_true"], sigma=0.01, seed=1609, device=dev,
                              dtype=torch.float32)
    lp = wl["dtype"]
    esize = 2 if lp == "bf16" else 1
    Ab = A32.to(torch.bfloat16 if lp == "bf16" else torch.float8_e4m3fn)
    W0n, H0n = init_factors(m, n, k, seed=9154)
    W0 = torch.from_numpy(W0n).to(dev, torch.float32)
    H0 = torch.from_numpy(H0n).to(dev, torch.float32)
    torch.cuda.synchronize()
    res = {}
    for tag, A in ((lp, Ab), ("f32", A32)):
        print("[bench] %s: warmup %d" % (tag, args.warmup), file=sys.stderr, flush=True)
        W, H = W0.clone(), H0.clone()
        nmf.nmf_dense(A, W, H, algo=wl["algo"], iters=args.warmup, objective=False)
        W.copy_(W0)
        H.copy_(H0)
        torch.cuda.synchronize()
        print("[bench] %s: timing %d steps" % (tag, args.steps), file=sys.stderr, flush=True)
        t0 = time.perf_counter()
        _, st = nmf.nmf_dense(A, W, H, algo=wl["algo"], iters=args.steps, objective=False,
                              timers=True)
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        rel = nmf.nmf_dense_relerr(A32, W, H.t().contiguous())
        res[tag] = dict(elapsed=elapsed, stats=st, rel_err=rel)
    b = res[lp]
    ms_launch = 0.5 * (b["stats"]["ms_mm_aht"] + b["stats"]["ms_mm_wta"]) / args.steps
    bytes_launch = float(esize) * m * n
    tr = load_traffic(kernel_source_hash(LOWP_SOURCES),
                      TRAFFIC_FILE_FP8 if lp == "fp8" else TRAFFIC_FILE_BF16, args.workload)
    traffic = tr["hbm_bytes_per_launch"] if tr else None
    achieved = bytes_launch / (ms_launch * 1e-3) / 1e9
    f = res["f32"]
    ms_launch32 = 0.5 * (f["stats"]["ms_mm_aht"] + f["stats"]["ms_mm_wta"]) / args.steps
    out = {
        "metric": "NMF iterations/s (dense %s, A %dx%d %s, k=%d; %s products)"
                  % (wl["algo"].upper(), m, n, lp, k, lp.upper()),
        "value": round(args.steps / b["elapsed"], 3), "unit": "iters/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(1000.0 * b["elapsed"] / args.steps, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": lp, "data": "synthetic",
        "config": {"workload": args.workload, "m": m, "n": n, "k": k, "algorithm": wl["algo"],
                   "parallelism": "single-gpu"},
        "setup_ms": round(b["stats"]["ms_setup"], 3),
        "phase_ms_per_step": {p: round(b["stats"][q] / args.steps, 4) for p, q in
                              (("mm", "ms_mm"), ("luc", "ms_luc"), ("gram", "ms_gram"))},
        "rel_err_after_steps": {lp: b["rel_err"], "f32": f["rel_err"],
                                lp + "_minus_f32_relative": (b["rel_err"] - f["rel_err"])
                                / f["rel_err"]},
        "f32_same_problem": {"value": round(args.steps / f["elapsed"], 3), "unit": "iters/s",
                             "ms_per_step": round(1000.0 * f["elapsed"] / args.steps, 3),
                             "ms_per_product": round(ms_launch32, 4),
                             "tflops_products": round(2.0 * m * n * k / (ms_launch32 * 1e-3)
                                                      / 1e12, 2)},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4),
                     "traffic": traffic,
                     "kernel": ("gemm_lp_nt_kernel<uint16_t> (A H^T and A^T W, BF16 MFMA "
                                "16x16x32)" if lp == "bf16" else
                                "gemm_lp_nt_kernel<uint8_t> (A H^T and A^T W, FP8 MFMA "
                                "16x16x128)"),
                     "ms_per_launch": round(ms_launch, 4),
                     "algorithmic_bytes_per_launch": bytes_launch,
                     "tflops": round(2.0 * m * n * k / (ms_launch * 1e-3) / 1e12, 2)},
    }
    if args.copy_calibration:
        copy_calibration(dev)
    print(json.dumps(out), flush=True)


def run_autograd(args, wl):
    """Differentiation workloads: one step = 50 unrolled MU or HALS
    iterations forward (checkpoints every 10) plus the backward pass to
    dL/dA, dL/dW0, dL/dH0 for L = <GW, W_T> + <GH, H_T> (fixed random GW,
    GH), all in the library. value is steps/s; the forward alone and the
    backward alone are reported beside it. roofline: the large products of
    forward, recompute and adjoint (6 per iteration: 2 of each, 2 m n k flops
    each) plus the rank-2k dL/dA update (4 m n k flops per iteration),
    against the FP32 matrix peak."""
    import numpy as np
    import torch

    import paper_1609_09154_amd as nmf
    from synth import init_factors, planted_dense_torch, uniform

    m, n, k, T, every = wl["m"], wl["n"], wl["k"], wl["iters"], wl["ckpt_every"]
    dev = torch.device("cuda:0")
    print("[bench] generating %s" % args.workload, file=sys.stderr, flush=True)
    A = planted_dense_torch(m, n, wl["k_true"], sigma=0.01, seed=1609, device=dev,
                            dtype=torch.float32)
    W0n, H0n = init_factors(m, n, k, seed=9154)
    W0 = torch.from_numpy(W0n).to(dev, torch.float32)
    H0 = torch.from_numpy(H0n).to(dev, torch.float32)
    GW = torch.from_numpy(uniform((m, k), seed=11) - 0.5).to(dev, torch.float32)
    GH = torch.from_numpy(uniform((k, n), seed=12) - 0.5).to(dev, torch.float32)

    algo = wl["algo"]

    def fwd():
        if algo == "hals":
            return nmf.nmf_hals_unrolled_forward(A, W0, H0, T, ckpt_every=every)
        return nmf.nmf_mu_unrolled_forward(A, W0, H0, T, ckpt_every=every)

    def bwd(ck):
        if algo == "hals":
            return nmf.nmf_hals_unrolled_backward(A, ck, GW, GH, T, ckpt_every=every)
        return nmf.nmf_mu_unrolled_backward(A, ck, GW, GH, T, ckpt_every=every)

    print("[bench] warmup %d" % args.warmup, file=sys.stderr, flush=True)
    for _ in range(max(args.warmup, 1)):
        _, _, ck = fwd()
        bwd(ck)
    torch.cuda.synchronize()
    print("[bench] timing %d steps" % args.steps, file=sys.stderr, flush=True)
    tf = tb = 0.0
    t0 = time.perf_counter()
    for _ in range(args.steps):
        a = time.perf_counter()
        _, _, ck = fwd()
        torch.cuda.synchronize()
        b = time.perf_counter()
        bwd(ck)
        torch.cuda.synchronize()
        tf += b - a
        tb += time.perf_counter() - b
    elapsed = time.perf_counter() - t0
    flops = (6.0 * 2.0 * m * n * k + 4.0 * m * n * k) * T
    achieved = flops / (elapsed / args.steps) / 1e12
    out = {
        "metric": "unrolled-%s layer steps/s (forward %d %s iterations + backward to A, W0, "
                  "H0; A %dx%d fp32, k=%d)" % (algo.upper(), T, algo.upper(), m, n, k),
        "value": round(args.steps / elapsed, 3), "unit": "steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(1000.0 * elapsed / args.steps, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": args.workload, "m": m, "n": n, "k": k, "iters": T,
                   "ckpt_every": every, "parallelism": "single-gpu"},
        "ms_forward": round(1000.0 * tf / args.steps, 3),
        "ms_backward": round(1000.0 * tb / args.steps, 3),
        "forward_iters_per_s": round(T * args.steps / tf, 1),
        "roofline": {"bound": "mfma", "achieved": round(achieved, 2), "peak": PEAK_FP32_TFLOPS,
                     "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_TFLOPS, 4),
                     "traffic": None,
                     "kernel": "whole step (products, rank updates, row adjoints)",
                     "algorithmic_flops_per_step": flops},
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="dense-65536x65536-k50-hals-f32", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--sample-rows", type=int, default=16384)
    ap.add_argument("--cpu-sample", action="store_true",
                    help="time the CPU baseline on a square sample of the matrix family "
                         "instead of the workload's own matrix")
    ap.add_argument("--check", action="store_true", help="also report the final relative error")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after the run, copy a 3 GiB device buffer once (reference kernel "
                         "of known traffic for HBM counter runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1609_09154_amd as nmf
    from synth import init_factors, planted_dense_torch

    wl = WORKLOADS[args.workload]
    if wl.get("sparse"):
        return run_sparse(args, wl)
    if wl["dtype"] in ("bf16", "fp8"):
        return run_lowp(args, wl)
    if wl.get("autograd"):
        return run_autograd(args, wl)
    m, n, k = wl["m"], wl["n"], wl["k"]
    tdt = torch.float32 if wl["dtype"] == "f32" else torch.float64
    dev = torch.device("cuda:0")
    print("[bench] generating %s" % args.workload, file=sys.stderr, flush=True)
    A = planted_dense_torch(m, n, wl["k_true"], sigma=0.01, seed=1609, device=dev, dtype=tdt)
    W0n, H0n = init_factors(m, n, k, seed=9154)
    W0 = torch.from_numpy(W0n).to(dev, tdt)
    H0 = torch.from_numpy(H0n).to(dev, tdt)
    torch.cuda.synchronize()

    print("[bench] warmup %d" % args.warmup, file=sys.stderr, flush=True)
    W, H = W0.clone(), H0.clone()
    nmf.nmf_dense(A, W, H, algo=wl["algo"], iters=args.warmup, objective=False)
    W.copy_(W0)
    H.copy_(H0)
    torch.cuda.synchronize()

    print("[bench] timing %d steps" % args.steps, file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    _, stats = nmf.nmf_dense(A, W, H, algo=wl["algo"], iters=args.steps, objective=False,
                             timers=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    ms_per_step = 1000.0 * elapsed / args.steps
    value = args.steps / elapsed

    flops_per_launch = 2.0 * m * n * k
    ms_launch = 0.5 * (stats["ms_mm_aht"] + stats["ms_mm_wta"]) / args.steps
    peak = PEAK_FP32_TFLOPS if wl["dtype"] == "f32" else PEAK_FP64_TFLOPS
    achieved = flops_per_launch / (ms_launch * 1e-3) / 1e12
    src_hash = kernel_source_hash()
    tr = load_traffic(src_hash, TRAFFIC_FILE, args.workload)
    roofline = {"bound": "mfma", "achieved": round(achieved, 2), "peak": peak, "unit": "TFLOP/s",
                "frac": round(achieved / peak, 4),
                "traffic": (tr["hbm_bytes_per_launch"] if tr else None),
                "kernel": "dense products A H^T and W^T A (MFMA 16x16x4 %s)" % wl["dtype"],
                "ms_per_launch": round(ms_launch, 4),
                "ms_aht": round(stats["ms_mm_aht"] / args.steps, 4),
                "ms_wta": round(stats["ms_mm_wta"] / args.steps, 4),
                "algorithmic_flops_per_launch": flops_per_launch}
    iter_flops = 4.0 * m * n * k
    out = {
        "metric": "NMF iterations/s (dense %s, A %dx%d %s, k=%d)"
                  % (wl["algo"].upper(), m, n, "fp32" if wl["dtype"] == "f32" else "fp64", k),
        "value": round(value, 3), "unit": "iters/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": wl["dtype"], "data": "synthetic",
        "config": {"workload": args.workload, "m": m, "n": n, "k": k, "algorithm": wl["algo"],
                   "parallelism": "single-gpu"},
        "tflops_products": round(iter_flops / (ms_per_step * 1e-3) / 1e12, 2),
        "phase_ms_per_step": {p: round(stats[f] / args.steps, 4) for p, f in
                              (("mm", "ms_mm"), ("luc", "ms_luc"), ("gram", "ms_gram"))},
        "roofline": roofline,
    }
    if wl["algo"] == "abpp":
        out["bpp"] = bpp_report(stats, args.steps, m + n)
    if args.check:
        rel = nmf.nmf_dense_relerr(A, W, H.t().contiguous())
        out["final_rel_err"] = rel
    if args.copy_calibration:
        copy_calibration(dev)
    add_paper_context(out, wl)
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline", file=sys.stderr, flush=True)
        esize = 4 if wl["dtype"] == "f32" else 8
        if host_bytes_free() > (8 + esize) * m * n * 1.25 and not args.cpu_sample:
            # the oracle on the workload's own matrix (host copy in float64)
            out["cpu_baseline"] = cpu_baseline_full(A, wl, W0n, H0n)
        else:
            out["cpu_baseline"] = cpu_baseline(wl, min(args.sample_rows, m))
    del A
    torch.cuda.empty_cache()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
