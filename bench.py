#!/usr/bin/env python
"""LABFM hot path benchmark on one MI355X: prints one JSON line.

Workload (the headline): 512 x 512 cell-centred lattice on [0,1]^2 jittered
by U(-0.3 s, 0.3 s) per coordinate (seed 2), order 8 interior / order 4 in the
boundary band of width R0, R0 = 4.4 s with count-driven growth, HERMITE ABFs
(sigma = 1) on the Wendland C2 RBF.  One step = neighbour search (count and
fill) + weights {d/dx, d/dy, Laplacian} for every node + application of the
three operators to a field.  `value` = order-8 nodes whose weight set passes
the 1e-10 moment-residual gate, per second of step time.

Secondary (not `value`): RK4 advection-diffusion with composed hyperviscosity
on the 1024 x 1024 periodic order-6 workload, FP32 application.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_FP64 = 78.6e12      # MI355X FP64 vector / matrix, FLOP/s
PEAK_FP32_MFMA = 157.3e12
PEAK_BF16 = 2.5e15       # dense BF16 matrix
PEAK_HBM = 8.0e12        # bytes/s


def measured_traffic(kernel, sources):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, or None if the kernel's sources changed since it was taken."""
    import glob
    import hashlib

    h = hashlib.sha256()
    for src in sources:
        with open(os.path.join(ROOT, "paper_1912_06441_amd", "csrc", src), "rb") as fh:
            h.update(fh.read())
    digest = h.hexdigest()[:16]
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        with open(path) as fh:
            for line in fh:
                parts = line.split()
                if len(parts) == 4 and parts[0] == "TRAFFIC" and parts[1] == kernel:
                    if parts[2] == "src=" + digest:
                        return float(parts[3].split("=")[1])
    return None


def factor_flops(N, p, nd):
    """The factor kernel's share of weight_flops: basis evaluation 10Np, assembly
    2Np^2, LU 2p^3/3 and the first solve 2 nd p^2."""
    return 10.0 * N * p + 2.0 * N * p * p + 2.0 * p ** 3 / 3.0 + 2.0 * nd * p * p


def weight_flops(N, p, nd, iters):
    """Algorithmic FP64 flops of one weight set: basis evaluation 10Np (the
    monomials and ABFs of every neighbour), assembly 2Np^2, LU 2p^3/3,
    (1 + it) x [solve 2 nd p^2 + weights 2 N p nd + residual 2 N p nd]."""
    return (10.0 * N * p + 2.0 * N * p * p + 2.0 * p ** 3 / 3.0
            + (1.0 + iters) * (2.0 * nd * p * p + 4.0 * N * p * nd))


def cpu_model():
    """`lscpu`'s model name of the host (or /proc/cpuinfo's), and nproc."""
    import subprocess

    name = ""
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for ln in out.splitlines():
            if ln.startswith("Model name:"):
                name = ln.split(":", 1)[1].strip()
                break
    except (OSError, subprocess.SubprocessError):
        pass
    if not name:
        try:
            with open("/proc/cpuinfo") as fh:
                for ln in fh:
                    if ln.startswith("model name"):
                        name = ln.split(":", 1)[1].strip()
                        break
        except OSError:
            pass
    return name, os.cpu_count()


def run_cpu_baseline(nd, cfg, runs=5, sample1=8192):
    """The oracle (plain FP64 C, OpenMP over nodes) on the host cores, median of
    `runs`: all threads over the whole step of the full workload (neighbours +
    FP64 weights + 3 operators), and one thread over the weights of a seeded
    sample of `sample1` order-8 nodes (the other nodes' order set to 0, which
    the oracle rejects at once)."""
    import numpy as np

    import oracle as O
    from paper_1912_06441_amd import workloads as WL

    f = WL.trig_field(nd["x"], nd["y"], WL.trig_poly(0))[0]
    threads = O.num_threads()
    rates, good = [], 0
    stage = {"neighbours": [], "weights": [], "apply_3ops": []}
    for _ in range(runs):
        t0 = time.perf_counter()
        rp, col, R = O.neighbours(nd["x"], nd["y"], nd["domain"], nd["R"], nd["order"])
        t1 = time.perf_counter()
        w, st, res, _ = O.weights(nd["x"], nd["y"], nd["domain"], R, nd["order"], rp, col)
        t2 = time.perf_counter()
        for d in range(3):
            O.apply(rp, col, w[d], f)
        t3 = time.perf_counter()
        dt = t3 - t0
        stage["neighbours"].append(1e3 * (t1 - t0))
        stage["weights"].append(1e3 * (t2 - t1))
        stage["apply_3ops"].append(1e3 * (t3 - t2))
        good = int(((st == 0) & (nd["order"] == 8)).sum())
        rates.append(good / dt)
    # one thread: weights of a sample of order-8 nodes
    idx8 = np.nonzero(nd["order"] == 8)[0]
    pick = np.random.default_rng(12345).choice(idx8, min(sample1, idx8.size), replace=False)
    order_s = np.zeros_like(nd["order"])
    order_s[pick] = 8
    rates1, good1 = [], 0
    O.set_num_threads(1)
    try:
        for _ in range(runs):
            t0 = time.perf_counter()
            w, st, res, _ = O.weights(nd["x"], nd["y"], nd["domain"], R, order_s, rp, col)
            dt = time.perf_counter() - t0
            good1 = int((st[pick] == 0).sum())
            rates1.append(good1 / dt)
    finally:
        O.set_num_threads(threads)
    model, nproc = cpu_model()
    return {"value": float(np.median(rates)), "unit": "weight-sets/s (order 8)", "cores": threads,
            "kind": "oracle",
            "sample": "the full 512x512 workload, whole steps (neighbours + FP64 weights + 3 operators), "
                      "median of %d runs (%d order-8 nodes at the gate per run)" % (runs, good),
            "runs": [round(r, 1) for r in rates], "nproc": nproc, "cpu_model": model,
            "stage_ms_median": {k: float(np.median(v)) for k, v in stage.items()},
            "single_thread": {"value": float(np.median(rates1)), "unit": "weight-sets/s (order 8)", "cores": 1,
                              "sample": "FP64 weights of %d seeded order-8 nodes of the same workload, "
                                        "median of %d runs" % (good1, runs),
                              "runs": [round(r, 1) for r in rates1]}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--prec", choices=["fp64", "mixed"], default="fp64")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-rk4", action="store_true")
    ap.add_argument("--rk4-steps", type=int, default=200)
    ap.add_argument("--no-burgers", action="store_true", help="skip the Burgers step measurement")
    ap.add_argument("--no-poisson", action="store_true", help="skip the Poisson solve measurement")
    ap.add_argument("--no-ns", action="store_true", help="skip the Taylor-Green Navier-Stokes measurement")
    ap.add_argument("--no-3d", action="store_true", help="skip the three-dimensional weights measurement")
    ap.add_argument("--burgers-steps", type=int, default=200)
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-set batched weights measurement")
    ap.add_argument("--no-c4", action="store_true", help="skip the learned warm start measurement")
    ap.add_argument("--c4-train-sets", type=int, default=32, help="96x96 lattices of training stencils")
    ap.add_argument("--c4-epochs", type=int, default=4)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy 1 GiB device to device 4 times (counter calibration) and exit")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch

        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(4):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_per_launch": src.numel() * 8, "launches": 4}))
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only (the method's kernels run on one device); "
              "--gpus %d is not supported" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1912_06441_amd as L
    from paper_1912_06441_amd import workloads as WL

    dev = torch.device("cuda:0")
    cfg = WL.config("c2")
    nd = WL.make_nodes(cfg)
    n = nd["x"].size
    x = torch.from_numpy(nd["x"]).to(dev)
    y = torch.from_numpy(nd["y"]).to(dev)
    R0 = torch.from_numpy(nd["R"]).to(dev)
    order = torch.from_numpy(nd["order"]).to(dev)
    f = torch.from_numpy(WL.trig_field(nd["x"], nd["y"], WL.trig_poly(0))[0]).to(dev)
    prec = L.PREC_FP64 if args.prec == "fp64" else L.PREC_MIXED
    ctx = L.Context(0)
    R = R0.clone()

    # sizes and output buffers (nnz is deterministic for a node set)
    rp, col = ctx.build_neighbours(x, y, R, order, nd["domain"])
    nnz = col.numel()
    bufs = (torch.empty((3, nnz), dtype=torch.float64, device=dev), None,
            torch.empty(n, dtype=torch.int8, device=dev), torch.empty(n, dtype=torch.float32, device=dev),
            torch.empty(n, dtype=torch.int8, device=dev))
    out = torch.empty((3, n), dtype=torch.float64, device=dev)

    def step():
        R.copy_(R0)
        rp_, col_ = ctx.build_neighbours(x, y, R, order, nd["domain"])
        ctx.weights(x, y, R, order, rp_, col_, nd["domain"], prec=prec, out=bufs)
        ctx.apply_operator(rp_, col_, bufs[0], f, out=out)
        return rp_, col_

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ctx.timing(True)
    # per-step events on the stream the library launches on (torch's current stream)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record()
    for k in range(args.steps):
        rp, col = step()
        ev[k + 1].record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ctx.timing(False)
    ms = (t1 - t0) * 1e3 / args.steps
    step_ms = np.array([ev[k].elapsed_time(ev[k + 1]) for k in range(args.steps)])
    # read the order-8 kernels (factor, then weights and refinement) separately, then every weights kernel
    k8f = ctx.timing_read("weights64f_k8")
    k8r = ctx.timing_read("weights64r_k8")
    kw_rest = ctx.timing_read("weights")
    kw = (k8f[0] + k8r[0] + kw_rest[0], k8f[1] + k8r[1] + kw_rest[1])
    kn = ctx.timing_read("neigh")
    ka = ctx.timing_read("apply")
    ctx.timing_read(None)

    status = bufs[2].cpu().numpy()
    iters = bufs[4].cpu().numpy().astype(np.float64)
    resid = bufs[3].cpu().numpy()
    N = np.diff(rp.cpu().numpy())
    is8 = nd["order"] == 8
    good8 = int(((status == 0) & is8).sum())
    value = good8 / (ms / 1e3)

    # roofline of the dominant kernel (the order-8 factor kernel: basis, assembly, LU and the
    # first solve), algorithmic flops per launch; and of the order-8 weights as a whole
    N8 = N[is8].astype(np.float64)
    flops8 = float(weight_flops(N8, 44, 3, iters[is8]).sum())
    flops8f = float(factor_flops(N8, 44, 3).sum())
    k8f_ms = k8f[1] / max(k8f[0], 1)
    k8r_ms = k8r[1] / max(k8r[0], 1)
    launches8 = max(k8f[0], 1) / args.steps  # launches per step (chunks of the work list)
    achieved = flops8f / launches8 / (k8f_ms / 1e3)
    k8_ms = (k8f[1] + k8r[1]) / args.steps
    achieved8 = flops8 / (k8_ms / 1e3)
    # operator application: algorithmic bytes per launch (col 4 B + 3 FP64 weights per entry;
    # row_ptr, u_i and 3 FP64 outputs per node)
    apply_bytes = nnz * (4 + 3 * 8) + n * (8 + 8 + 3 * 8)
    ka_ms = ka[1] / max(ka[0], 1)

    rec = {
        "metric": "node weight-sets/sec (order 8) and operator apps (nodes/s) at 1e-10 rel err",
        "value": value,
        "unit": "weight-sets/s (order 8)",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.prec == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": "512x512 jittered lattice (eps 0.3 s, seed 2), order 8 interior / 4 boundary band, "
                               "R0 = 4.4 s + growth, Hermite x Wendland C2 ABFs; step = neighbours + weights "
                               "{dx, dy, lap} + 3-operator application",
                   "nodes": n, "nnz": nnz, "order8_nodes": int(is8.sum()), "prec": args.prec},
        "step_ms": {"median": float(np.median(step_ms)), "min": float(step_ms.min()), "max": float(step_ms.max()),
                    "steps": args.steps},
        "stages_ms": {"neighbours": kn[1] / args.steps, "weights": kw[1] / args.steps,
                      "weights_order8_kernels": k8_ms, "order8_factor_kernel": k8f_ms,
                      "order8_refine_kernel": k8r_ms, "apply_3ops": ka_ms},
        "accuracy": {"nodes_passing_1e-10": int((status == 0).sum()), "nodes": n,
                     "max_moment_residual": float(resid.max()), "mean_refinement_iters": float(iters.mean())},
        "operator_apps": {"value": n / (ka_ms / 1e3), "unit": "nodes/s (3 fused FP64 operators)",
                          "GB_per_s": apply_bytes / (ka_ms / 1e3) / 1e9},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP64 / 1e12, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP64,
                     "traffic": measured_traffic("weights64f_k8", ["weights_split.hip", "weights_common.hpp",
                                                                   "basis.hpp"]),
                     "kernel": "weights64f_k8", "flops_per_launch": flops8f / launches8},
        "roofline_weights_order8": {"bound": "alu", "achieved": achieved8 / 1e12, "peak": PEAK_FP64 / 1e12,
                                    "unit": "TFLOP/s", "frac": achieved8 / PEAK_FP64,
                                    "kernels": ["weights64f_k8", "weights64r_k8"], "flops_per_step": flops8},
        "roofline_apply": {"bound": "hbm", "achieved": apply_bytes / (ka_ms / 1e3) / 1e9, "peak": PEAK_HBM / 1e9,
                           "unit": "GB/s", "frac": apply_bytes / (ka_ms / 1e3) / PEAK_HBM,
                           "traffic": measured_traffic("apply_f64", ["apply.hip", "stencil_rows.hpp"]),
                           "kernel": "apply_f64",
                           "bytes_per_launch": apply_bytes},
    }

    # the other precision on the same workload, for comparison at the same accuracy gate
    other = L.PREC_MIXED if prec == L.PREC_FP64 else L.PREC_FP64
    rec["compare"] = compare_precision(ctx, torch, np, L, x, y, R0, order, nd, other, bufs, args.steps)

    if not args.no_rk4:
        rec["rk4_c5"] = run_rk4(ctx, torch, np, L, WL, args.rk4_steps)
        rec["apply_fp32_c5"] = run_apply_c5(ctx, torch, np, L, WL)
    if not args.no_burgers:
        rec["burgers_1024"] = run_burgers(ctx, torch, np, L, WL, args.burgers_steps)
    if not args.no_poisson:
        rec["poisson_1024"] = run_poisson(ctx, torch, np, L, WL)
    if not args.no_ns:
        rec["taylor_green_256"] = run_ns(ctx, torch, np, L, WL)
    if not args.no_3d:
        rec["weights3d_64"] = run_weights3d(ctx, torch, np, L, WL)
        rec["weights3d_32_k5"] = run_weights3d(ctx, torch, np, L, WL, side=32, k=5)
        rec["weights3d_32_k6"] = run_weights3d(ctx, torch, np, L, WL, side=32, k=6)
    if not args.no_batch:
        rec["batch_c3"] = run_batch(ctx, torch, np, L, WL, reps=3)
    rec["mlp_bf16"] = run_mlp(ctx, torch, L, WL)
    if not args.no_c4:
        rec["warm_start_c4"] = run_c4(ctx, torch, np, L, WL, args.c4_train_sets, args.c4_epochs)

    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = run_cpu_baseline(nd, cfg)
    ctx.close()
    print(json.dumps(rec), flush=True)


def compare_precision(ctx, torch, np, L, x, y, R0, order, nd, prec, bufs, reps):
    """Weights-only timing of the other precision mode on the same workload."""
    R = R0.clone()
    rp, col = ctx.build_neighbours(x, y, R, order, nd["domain"])
    ctx.weights(x, y, R, order, rp, col, nd["domain"], prec=prec, out=bufs)
    torch.cuda.synchronize()
    ctx.timing(True)
    for _ in range(reps):
        ctx.weights(x, y, R, order, rp, col, nd["domain"], prec=prec, out=bufs)
    torch.cuda.synchronize()
    ctx.timing(False)
    kw = ctx.timing_read("weights")
    ctx.timing_read(None)
    st = bufs[2].cpu().numpy()
    it = bufs[4].cpu().numpy()
    res = bufs[3].cpu().numpy()
    good8 = int(((st == 0) & (nd["order"] == 8)).sum())
    ms = kw[1] / reps
    rec = {"prec": "fp64" if prec == L.PREC_FP64 else "mixed", "weights_ms": ms,
           "weight_sets_per_s_order8": good8 / (ms / 1e3), "nodes_passing_1e-10": int((st == 0).sum()),
           "max_moment_residual": float(res.max()), "fp64_fallback_nodes": int((it >= 64).sum()),
           "mean_refinement_iters": float(it[it < 64].mean())}
    if prec == L.PREC_MIXED:
        # matrix-core work of the assembly as issued: neighbours in chunks of 16, p padded to 16-wide
        # tiles (2 x ceil16(N) x ceil16(p)^2 per system), over the time of all weight kernels
        N = np.diff(rp.cpu().numpy()).astype(np.float64)
        k = nd["order"].astype(np.int64)
        p = (k * k + 3 * k) // 2
        pp = 16.0 * np.ceil(p / 16.0)
        mf = float((2.0 * 16.0 * np.ceil(N / 16.0) * pp * pp).sum())
        rec["matrix_core_flops"] = mf
        rec["matrix_core_frac_of_fp32_peak"] = mf / (ms / 1e3) / PEAK_FP32_MFMA
    return rec


def run_rk4(ctx, torch, np, L, WL, nsteps):
    """1024x1024 periodic order-6 RK4 (FP32 application): ms per step and
    operator applications per second (3 stencil passes per stage)."""
    dev = torch.device("cuda:0")
    cfg = WL.config("c5")
    nd = WL.make_nodes(cfg)
    n = nd["x"].size
    x = torch.from_numpy(nd["x"]).to(dev)
    y = torch.from_numpy(nd["y"]).to(dev)
    R = torch.from_numpy(nd["R"]).to(dev)
    order = torch.from_numpy(nd["order"]).to(dev)
    rp, col = ctx.build_neighbours(x, y, R, order, nd["domain"])
    w64, _, st, res, _ = ctx.weights(x, y, R, order, rp, col, nd["domain"], ops=1 | 2 | 4 | 8)
    a, nu = cfg["a"], cfg["nu"]
    _, wlin = ctx.combine(w64[:3], [-a[0], -a[1], nu], want64=False, want32=True)
    wbh = w64[3].to(torch.float32)
    s = nd["s"]
    h = 0.5 * cfg["R_s"] * s
    dt = cfg["dt_s"] * s
    gamma = cfg["beta"] * h ** 8 / dt
    u = torch.from_numpy(WL.gaussian_pulse(nd["x"], nd["y"])).to(dev).to(torch.float32)
    scratch = torch.empty(5 * n, dtype=torch.float32, device=dev)
    ctx.step(rp, col, wlin, wbh, gamma, dt, u, 5, scratch=scratch)  # warm-up + graph capture
    torch.cuda.synchronize()
    ctx.timing(True)
    t0 = time.perf_counter()
    ctx.step(rp, col, wlin, wbh, gamma, dt, u, nsteps, scratch=scratch)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ctx.timing(False)
    kg = ctx.timing_read("step")
    ctx.timing_read(None)
    nnz = col.numel()
    ms_step = kg[1] / nsteps
    # per stage: pass A reads col + 2 weight streams (4 B each), pass B col + 1 weight stream;
    # per node per stage ~ 8 x 4 B of state reads/writes
    bytes_step = 4 * (nnz * (4 + 4 + 4) + nnz * (4 + 4) + n * 8 * 4)
    return {"nodes": n, "nnz": nnz, "steps": nsteps, "ms_per_rk4_step": ms_step,
            "wall_ms_per_rk4_step": (t1 - t0) * 1e3 / nsteps,
            "operator_apps_nodes_per_s": 12 * n / (ms_step / 1e3),
            "GB_per_s": bytes_step / (ms_step / 1e3) / 1e9, "hbm_frac": bytes_step / (ms_step / 1e3) / PEAK_HBM,
            "weights_all_ok": bool((st == 0).all().item()), "u_max": float(u.abs().max().item())}


def run_apply_c5(ctx, torch, np, L, WL, reps=20):
    """One FP32 operator (the Laplacian) applied on the 1024x1024 periodic
    order-6 set: algorithmic bytes per node N (4 B index + 4 B weight) + 8 B
    of row offset + 4 B u_i + 4 B result (408 B at the mean N)."""
    dev = torch.device("cuda:0")
    cfg = WL.config("c5")
    nd = WL.make_nodes(cfg)
    n = nd["x"].size
    x = torch.from_numpy(nd["x"]).to(dev)
    y = torch.from_numpy(nd["y"]).to(dev)
    R = torch.from_numpy(nd["R"]).to(dev)
    order = torch.from_numpy(nd["order"]).to(dev)
    rp, col = ctx.build_neighbours(x, y, R, order, nd["domain"])
    _, w32, st, _, _ = ctx.weights(x, y, R, order, rp, col, nd["domain"], ops=4, want64=False, want32=True)
    u = torch.from_numpy(WL.gaussian_pulse(nd["x"], nd["y"])).to(dev).to(torch.float32)
    w = w32[0].contiguous()
    out = torch.empty(n, dtype=torch.float32, device=dev)
    for _ in range(3):
        ctx.apply_operator(rp, col, w, u, out=out.view(1, -1))
    torch.cuda.synchronize()
    ctx.timing(True)
    for _ in range(reps):
        ctx.apply_operator(rp, col, w, u, out=out.view(1, -1))
    torch.cuda.synchronize()
    ctx.timing(False)
    nk, ms = ctx.timing_read("apply_f32")
    ctx.timing_read(None)
    ms /= max(nk, 1)
    nnz = col.numel()
    bytes_launch = nnz * (4 + 4) + n * (8 + 4 + 4)
    return {"nodes": n, "nnz": nnz, "ms_per_apply": ms, "nodes_per_s": n / (ms / 1e3),
            "bytes_per_node": bytes_launch / n, "GB_per_s": bytes_launch / (ms / 1e3) / 1e9,
            "hbm_frac": bytes_launch / (ms / 1e3) / PEAK_HBM,
            "traffic": measured_traffic("apply_f32", ["apply.hip", "stencil_rows.hpp"]),
            "weights_all_ok": bool((st == 0).all().item())}


def run_c4(ctx, torch, np, L, WL, train_sets, epochs, batch=512, reps=3):
    """Learned warm start end to end on the GPU: training stencils from jittered
    96x96 periodic lattices (GPU neighbours, moment matrices and coefficients
    from labfm_moment_systems, features), the network trained with the
    library's kernels (moment-residual loss, Adam), then the 1024x1024 order-8
    set through the FP64, mixed, warm-started and factorisation-free routes at
    the 1e-10 gate: ms per 1 M nodes, fallback rate, refinement sweeps."""
    dev = torch.device("cuda:0")
    cfg = WL.config("c4")
    k, ops, kmax = cfg["k"], cfg["ops"], cfg["kmax"]
    t0 = time.perf_counter()
    feats, Ms, psis = [], [], []
    for i in range(train_sets):
        seed = cfg["train_seed0"] + i
        eps = float(np.random.default_rng(seed).uniform(0.0, cfg["eps_max"]))
        xs, ys, s = WL.jittered_lattice(cfg["train_side"], eps=eps, seed=seed, periodic=True)
        dom = WL.unit_domain(True)
        x, y = torch.from_numpy(xs).to(dev), torch.from_numpy(ys).to(dev)
        R = torch.full((xs.size,), cfg["R_s"] * s, dtype=torch.float64, device=dev)
        order = torch.full((xs.size,), k, dtype=torch.int8, device=dev)
        rp, col = ctx.build_neighbours(x, y, R, order, dom)
        M, psi, st = ctx.moment_systems(x, y, R, k, rp, col, dom, ops=ops)
        keep = st == 0
        feats.append(ctx.mlp_features(x, y, R, rp, col, dom, kmax=kmax)[keep])
        Ms.append(M[keep])
        psis.append(psi[keep])
    X = torch.cat(feats)
    Mt = torch.cat(Ms)
    del feats, Ms
    # per-component median and 1.4826 x median absolute deviation of the training coefficients
    P = torch.cat(psis).cpu().numpy().astype(np.float64)
    mu = np.median(P, axis=0)
    sd = 1.4826 * np.median(np.abs(P - mu), axis=0)
    sd = np.where(sd > 0, sd, 1.0)
    net = L.MLP(ctx, dims=cfg["dims"], order=k, ops=ops, kmax=kmax, seed=0)
    net.set_output_scaling(mu, sd)
    ntrain = X.shape[0]
    g = torch.Generator(device="cuda").manual_seed(0)
    cache = net.cache_for(batch)
    steps = epochs * (ntrain // batch)
    t = 0
    for e in range(epochs):
        perm = torch.randperm(ntrain, device="cuda", generator=g)
        for b in range(ntrain // batch):
            idx = perm[b * batch:(b + 1) * batch]
            lr = cfg["lr"] * 0.5 * (1.0 + np.cos(np.pi * t / steps))
            net.train_step(X[idx].contiguous(), Mt[idx].contiguous(), lr, cache=cache)
            t += 1
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    # initial moment residual of the trained network on held-out stencils (first 65536 of the set)
    xs, ys, s = WL.jittered_lattice(cfg["eval_side"], eps=cfg["eval_eps"], seed=cfg["eval_seed"], periodic=True)
    dom = WL.unit_domain(True)
    n = xs.size
    x, y = torch.from_numpy(xs).to(dev), torch.from_numpy(ys).to(dev)
    R = torch.full((n,), cfg["R_s"] * s, dtype=torch.float64, device=dev)
    order = torch.full((n,), k, dtype=torch.int8, device=dev)
    rp, col = ctx.build_neighbours(x, y, R, order, dom)
    m = 65536
    rp_s = rp[:m + 1].contiguous()
    Me, _, st_e = ctx.moment_systems(x, y, R, k, rp_s, col, dom, ops=ops)
    fe = ctx.mlp_features(x, y, R, rp, col, dom, kmax=kmax)[:m].contiguous()
    r_tr = net.moment_loss(net.forward(fe), Me)[0].sqrt()
    del Me, fe, X, Mt
    torch.cuda.empty_cache()
    routes = {}
    for name, prec in (("fp64", L.PREC_FP64), ("mixed", L.PREC_MIXED), ("mlp", L.PREC_MLP),
                       ("mlp_nolu", L.PREC_MLP_NOLU)):
        out = ctx.weights(x, y, R, order, rp, col, dom, prec=prec, mlp=net)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2 * reps)]
        for r_ in range(reps):
            ev[2 * r_].record()
            ctx.weights(x, y, R, order, rp, col, dom, prec=prec, mlp=net, out=out)
            ev[2 * r_ + 1].record()
        torch.cuda.synchronize()
        ms = min(ev[2 * r_].elapsed_time(ev[2 * r_ + 1]) for r_ in range(reps))
        st = out[2].cpu().numpy()
        it = out[4].cpu().numpy().astype(np.int64)
        res = out[3].cpu().numpy()
        direct = it < 64
        routes[name] = {"ms_per_1M_nodes": ms * (1 << 20) / n, "ns_per_node": 1e6 * ms / n,
                        "nodes_ok": int((st == 0).sum()), "max_resid_ok": float(res[st == 0].max()),
                        "fallback_nodes": int((~direct).sum()), "fallback_frac": float((~direct).mean()),
                        "mean_sweeps": float(it[direct].mean()) if direct.any() else None}
        del out
    return {"train_stencils": int(ntrain), "train_sets": train_sets, "epochs": epochs, "train_s": t_train,
            "eval_nodes": n, "initial_resid_median_trained": float(r_tr.median().item()),
            "initial_resid_zero_start": 2.0, "routes": routes}


def run_burgers(ctx, torch, np, L, WL, nsteps):
    """Viscous Burgers' equation (FP32, Re = 100) on the 1024x1024 periodic
    order-6 node set: ms per RK4 step of the one-pass two-field stage kernel."""
    dev = torch.device("cuda:0")
    cfg = WL.config("c5")
    nd = WL.make_nodes(cfg)
    n = nd["x"].size
    x = torch.from_numpy(nd["x"]).to(dev)
    y = torch.from_numpy(nd["y"]).to(dev)
    R = torch.from_numpy(nd["R"]).to(dev)
    order = torch.from_numpy(nd["order"]).to(dev)
    rp, col = ctx.build_neighbours(x, y, R, order, nd["domain"])
    w64, _, st, _, _ = ctx.weights(x, y, R, order, rp, col, nd["domain"], ops=L.OP_DX | L.OP_DY | L.OP_LAP)
    w = [w64[d].to(torch.float32) for d in range(3)]  # one allocation each: 16-byte aligned streams
    h = 0.5 * cfg["R_s"] * nd["s"]
    Re = 100.0
    # half the step of eq. (tstep): at the full step a mode localised on this
    # noisy node set (eps 0.3 s) lifts max|u| from 1 to ~21 within 25 steps;
    # at half the step the field decays as the viscous solution does
    dt = 0.5 * WL.burgers_dt(h, 1.0, Re)
    xs, ys = nd["x"], nd["y"]
    u = torch.from_numpy(np.sin(2 * np.pi * xs) * np.sin(2 * np.pi * ys)).to(dev).to(torch.float32)
    v = torch.from_numpy(-np.cos(2 * np.pi * xs) * np.cos(2 * np.pi * ys)).to(dev).to(torch.float32)
    scratch = torch.empty(6 * n, dtype=torch.float32, device=dev)
    ctx.burgers_step(rp, col, w[0], w[1], w[2], 1.0 / Re, dt, u, v, 5, scratch=scratch)  # warm-up + capture
    torch.cuda.synchronize()
    ctx.timing(True)
    ctx.burgers_step(rp, col, w[0], w[1], w[2], 1.0 / Re, dt, u, v, nsteps, scratch=scratch)
    torch.cuda.synchronize()
    ctx.timing(False)
    kg = ctx.timing_read("burgers")
    ctx.timing_read(None)
    nnz = col.numel()
    ms_step = kg[1] / nsteps
    # per step: 4 stages x (col + 3 FP32 weight streams per entry); per node the row bounds
    # (4 x 8 B), the packing of (u, v) into pairs (16 B) and the stage states of both fields:
    # own pair 4 x 8, own u, v 4 x 8, accumulators 3 x 8 read + 3 x 8 written, pairs 3 x 8
    # written, new u, v 8 B (144 B)
    bytes_step = 4 * nnz * (4 + 3 * 4) + n * (4 * 8 + 16 + 144)
    return {"nodes": n, "nnz": nnz, "steps": nsteps, "Re": Re, "dt": dt, "ms_per_rk4_step": ms_step,
            "GB_per_s": bytes_step / (ms_step / 1e3) / 1e9, "hbm_frac": bytes_step / (ms_step / 1e3) / PEAK_HBM,
            "bytes_per_step": bytes_step, "weights_all_ok": bool((st == 0).all().item()),
            "finite": bool(torch.isfinite(u).all().item() and torch.isfinite(v).all().item()),
            "u_max": float(torch.maximum(u.abs().max(), v.abs().max()).item())}


def run_poisson(ctx, torch, np, L, WL, tol=1e-10):
    """Periodic Poisson solve (Jacobi-BiCGStab, FP64) with the order-6
    Laplacian of the 1024x1024 node set, node 0 pinned to the exact value."""
    dev = torch.device("cuda:0")
    cfg = WL.config("c5")
    nd = WL.make_nodes(cfg)
    n = nd["x"].size
    x = torch.from_numpy(nd["x"]).to(dev)
    y = torch.from_numpy(nd["y"]).to(dev)
    R = torch.from_numpy(nd["R"]).to(dev)
    order = torch.from_numpy(nd["order"]).to(dev)
    rp, col = ctx.build_neighbours(x, y, R, order, nd["domain"])
    w64, _, st, _, _ = ctx.weights(x, y, R, order, rp, col, nd["domain"], ops=L.OP_LAP)
    w = w64[0].contiguous()
    fixed_np = np.zeros(n, np.int8)
    fixed_np[0] = 1
    F_np, x0_np = WL.poisson_system(nd["x"], nd["y"], fixed_np)
    F = torch.from_numpy(F_np).to(dev)
    fixed = torch.from_numpy(fixed_np).to(dev)
    scratch = torch.empty(8 * n, dtype=torch.float64, device=dev)
    phi = torch.from_numpy(x0_np).to(dev)
    ctx.poisson_solve(rp, col, w, F, phi=phi, fixed=fixed, tol=tol, max_iters=20, scratch=scratch)  # warm-up
    phi = torch.from_numpy(x0_np).to(dev)
    torch.cuda.synchronize()
    ctx.timing(True)
    t0 = time.perf_counter()
    phi, it, res, ok = ctx.poisson_solve(rp, col, w, F, phi=phi, fixed=fixed, tol=tol, max_iters=20000,
                                         check_every=32, scratch=scratch)
    t1 = time.perf_counter()
    ctx.timing(False)
    ki = ctx.timing_read("poisson_iterations")
    ctx.timing_read(None)
    nnz = col.numel()
    ex = WL.poisson_solution(nd["x"], nd["y"])
    err = float(np.linalg.norm(phi.cpu().numpy() - ex) / np.linalg.norm(ex))
    ms_it = ki[1] / max(it, 1)
    # per iteration: two products (col 4 B + w 8 B per entry; row bounds, x_i, y_i and the
    # Dirichlet flag per row) and the vector updates and reductions (25 FP64 vectors of n:
    # p-update 6, (r0, v) 2, s-update 8, (t, s) and (t, t) 2, r-update with its two sums 7)
    bytes_it = 2 * (nnz * 12 + n * 25) + 25 * 8 * n
    return {"nodes": n, "nnz": nnz, "iterations": it, "converged": ok, "rel_resid": res, "L2_error": err,
            "solve_ms": (t1 - t0) * 1e3, "ms_per_iteration": ms_it,
            "GB_per_s": bytes_it / (ms_it / 1e3) / 1e9, "hbm_frac": bytes_it / (ms_it / 1e3) / PEAK_HBM,
            "weights_all_ok": bool((st == 0).all().item())}


def run_ns(ctx, torch, np, L, WL, side=256, k=6, nsteps=10):
    """Taylor-Green vortices (vorticity-streamfunction, FP64, Re = 100) on a
    256x256 periodic order-6 set: ms per RK4 step (four stream-function
    solves to 1e-10, warm-started) and the error against the exact decay."""
    dev = torch.device("cuda:0")
    cfg = WL.config("taylor_green")
    x_np, y_np, s = WL.jittered_lattice(side, eps=WL.paper_jitter(cfg["eps_paper"]), seed=cfg["seed"], periodic=True)
    n = x_np.size
    x = torch.from_numpy(x_np).to(dev)
    y = torch.from_numpy(y_np).to(dev)
    R = torch.full((n,), 2.0 * cfg["h_over_dr"] * s, dtype=torch.float64, device=dev)
    order = torch.full((n,), k, dtype=torch.int8, device=dev)
    dom = WL.unit_domain(True)
    rp, col = ctx.build_neighbours(x, y, R, order, dom)
    w, _, st, _, _ = ctx.weights(x, y, R, order, rp, col, dom, ops=7, abf=cfg["abf"], rbf=cfg["rbf"])
    wx, wy, wl = (w[d].contiguous() for d in range(3))
    fixed = torch.zeros(n, dtype=torch.int8, device=dev)
    fixed[0] = 1
    Re = cfg["Re"]
    h = cfg["h_over_dr"] * s
    dt = WL.burgers_dt(h, 1.0, Re)
    om = torch.from_numpy(WL.taylor_green_vorticity(x_np, y_np, 0.0, Re)).to(dev)
    psi = torch.zeros(n, dtype=torch.float64, device=dev)
    scratch = torch.empty(14 * n, dtype=torch.float64, device=dev)
    ctx.ns_step(rp, col, wx, wy, wl, 1.0 / Re, dt, om, 1, psi=psi, psi_fixed=fixed, tol=cfg["tol"], scratch=scratch)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    om, psi, it, ok = ctx.ns_step(rp, col, wx, wy, wl, 1.0 / Re, dt, om, nsteps, psi=psi, psi_fixed=fixed,
                                  tol=cfg["tol"], scratch=scratch)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ex = WL.taylor_green_vorticity(x_np, y_np, (nsteps + 1) * dt, Re)
    err = float(np.linalg.norm(om.cpu().numpy() - ex) / np.linalg.norm(ex))
    return {"nodes": n, "nnz": col.numel(), "order": k, "steps": nsteps, "ms_per_rk4_step": (t1 - t0) * 1e3 / nsteps,
            "bicgstab_iterations_per_solve": it / (4.0 * nsteps), "all_solves_converged": ok, "L2_error": err,
            "weights_all_ok": bool((st == 0).all().item())}


def run_weights3d(ctx, torch, np, L, WL, reps=3, side=None, k=None):
    """Three-dimensional FP64 weights {dx, dy, lap, dz} of order k (4: p = 34,
    the 64^3 default) on a periodic lattice: neighbours, then weight sets per
    second."""
    dev = torch.device("cuda:0")
    cfg = WL.config("c3d")
    side = cfg["bench_side"] if side is None else side
    k = cfg["bench_k"] if k is None else k
    x_np, y_np, z_np, s = WL.jittered_lattice3(side, eps=cfg["eps"], seed=cfg["seed"], periodic=True)
    n = x_np.size
    x, y, z = (torch.from_numpy(a).to(dev) for a in (x_np, y_np, z_np))
    R = torch.full((n,), cfg["R_s"][k] * s, dtype=torch.float64, device=dev)
    dom = WL.unit_domain3(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rp, col = ctx.build_neighbours3(x, y, z, R, dom)
    torch.cuda.synchronize()
    t_neigh = (time.perf_counter() - t0) * 1e3
    ctx.weights3(x, y, z, R, k, rp, col, dom, sigma=cfg["sigma"])  # warm-up
    torch.cuda.synchronize()
    ctx.timing(True)
    for _ in range(reps):
        w, st, res, it = ctx.weights3(x, y, z, R, k, rp, col, dom, sigma=cfg["sigma"])
    torch.cuda.synchronize()
    ctx.timing(False)
    kw = ctx.timing_read("weights3d")
    ctx.timing_read(None)
    ms = kw[1] / max(kw[0], 1)
    st_np = st.cpu().numpy()
    N = np.diff(rp.cpu().numpy()).astype(np.float64)
    its = it.cpu().numpy().astype(np.float64)
    p, nd = sum(m * (m + 1) // 2 for m in range(2, k + 2)), 4
    flops = float((2 * N * p * p + 2 * p ** 3 / 3 + (1 + its) * (2 * nd * p * p + 4 * N * p * nd)).sum())
    return {"nodes": n, "nnz": col.numel(), "order": k, "p": p, "mean_N": float(N.mean()), "ms": ms,
            "neighbours_ms": t_neigh, "weight_sets_per_s": int((st_np == 0).sum()) / (ms / 1e3),
            "nodes_passing_1e-10": int((st_np == 0).sum()), "max_moment_residual": float(res.max()),
            "fp64_tflops": flops / (ms / 1e3) / 1e12, "frac_of_fp64_peak": flops / (ms / 1e3) / PEAK_FP64}


def run_mlp(ctx, torch, L, WL, B=1 << 20, reps=5):
    """Warm-start network inference on the matrix cores (BF16 operands, FP32
    accumulation): 192 -> 256 -> 256 -> 256 -> 132 over 2^20 stencils."""
    cfg = WL.config("c4")
    net = L.MLP(ctx, dims=cfg["dims"], order=cfg["k"], ops=cfg["ops"], kmax=cfg["kmax"], seed=0)
    g = torch.Generator(device="cuda").manual_seed(0)
    X = torch.randn((B, cfg["dims"][0]), device="cuda", generator=g)
    out = net.forward(X)
    torch.cuda.synchronize()
    ctx.timing(True)
    for _ in range(reps):
        net.forward(X, out=out)
    torch.cuda.synchronize()
    ctx.timing(False)
    nk, ms = ctx.timing_read("mlp_forward")
    ctx.timing_read(None)
    ms /= max(nk, 1)
    d = cfg["dims"]
    flops = 2.0 * B * sum(d[l] * d[l + 1] for l in range(len(d) - 1))
    return {"rows": B, "dims": list(d), "ms_per_forward": ms, "tflops": flops / (ms / 1e3) / 1e12,
            "frac_of_bf16_dense_peak": flops / (ms / 1e3) / PEAK_BF16, "rows_per_s": B / (ms / 1e3)}


def run_batch(ctx, torch, np, L, WL, reps):
    """64 independent node sets (3.5M nodes, orders 2/4/6/8, log-uniform sizes):
    weights of all sets as one captured launch sequence, against one call per
    set.  Weight sets per second count nodes passing the 1e-10 moment gate."""
    dev = torch.device("cuda:0")
    cfg = WL.config("c3")
    sets = []
    for S in WL.batch_sets(cfg):
        x = torch.from_numpy(S["x"]).to(dev)
        y = torch.from_numpy(S["y"]).to(dev)
        R = torch.from_numpy(S["R"]).to(dev)
        order = torch.from_numpy(S["order"]).to(dev)
        rp, col = ctx.build_neighbours(x, y, R, order, S["domain"])
        sets.append(dict(x=x, y=y, R=R, order=order, row_ptr=rp, col=col, domain=S["domain"], k=S["k"]))
    n = sum(S["x"].numel() for S in sets)
    nnz = sum(S["col"].numel() for S in sets)
    res = {"sets": len(sets), "nodes": n, "nnz": nnz,
           "sets_per_order": {str(k): sum(1 for S in sets if S["k"] == k) for k in cfg["orders"]}}

    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / reps

    for name, prec in (("fp64", L.PREC_FP64), ("mixed_autotuned", L.PREC_MIXED)):
        outs = ctx.weights_batched(sets, prec=prec, use_graph=True)  # plan: tuning, capture, first run
        ms = timed(lambda: ctx.weights_batched(sets, prec=prec, use_graph=True, outs=outs))
        good = sum(int((o[2] == 0).sum().item()) for o in outs)
        worst = max(float(o[3][o[2] == 0].max().item()) if bool((o[2] == 0).any()) else 0.0 for o in outs)
        res["batched_" + name] = {"ms": ms, "weight_sets_per_s": good / (ms / 1e3), "nodes_passing_1e-10": good,
                                  "max_moment_residual": worst}
        del outs
    res["routes"] = {str(k): {1: "mixed", 2: "fp64"}.get(ctx.autotune_query(k)[0], "untuned")
                     for k in cfg["orders"]}
    # per order class: the same batch launched eagerly, each order's kernel timed on its own
    outs = ctx.weights_batched(sets, prec=L.PREC_FP64, use_graph=False)
    torch.cuda.synchronize()
    counts = np.zeros(9, dtype=np.int64)
    for S in sets:
        counts += np.bincount(S["order"].cpu().numpy().astype(np.int64), minlength=9)[:9]
    ctx.timing(True)
    for _ in range(reps):
        ctx.weights_batched(sets, prec=L.PREC_FP64, use_graph=False, outs=outs)
    torch.cuda.synchronize()
    ctx.timing(False)
    per = {}
    for k in range(1, 9):
        # the two FP64 kernels of order k: factor, then weights and refinement
        nf, ms_f = ctx.timing_read("weights64f_k%d" % k)
        nr, ms_r = ctx.timing_read("weights64r_k%d" % k)
        nk, ms_k = nf, ms_f + ms_r
        if counts[k] and nk:
            per[str(k)] = {"nodes": int(counts[k]), "ms": ms_k / reps,
                           "weight_sets_per_s": int(counts[k]) / (ms_k / reps / 1e3)}
    ctx.timing_read(None)
    res["per_order_fp64"] = per
    del outs
    single = [None] * len(sets)

    def per_set():
        for t, S in enumerate(sets):
            single[t] = ctx.weights(S["x"], S["y"], S["R"], S["order"], S["row_ptr"], S["col"], S["domain"],
                                    prec=L.PREC_FP64, out=single[t])
    per_set()
    ms = timed(per_set)
    good = sum(int((o[2] == 0).sum().item()) for o in single)
    res["per_set_calls_fp64"] = {"ms": ms, "weight_sets_per_s": good / (ms / 1e3), "nodes_passing_1e-10": good}
    return res


if __name__ == "__main__":
    main()
