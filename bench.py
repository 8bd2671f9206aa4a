#!/usr/bin/env python3
"""Benchmark of the block multi-shift solve (one GPU).

A step is one full bms_solve of the workload: all n_pf right-hand sides and
all shifts of the rational approximation to a true FP64 relative residual
<= tol. value = RHS columns solved (every shift passing) per second of wall
time, inputs resident in HBM, on the product path (iteration chunks replayed
from captured hipGraphs). Printed as one JSON line, with:
  roofline      the dominant kernel's algorithmic GB/s (HIP events around each
                launch on the library stream, summed over one further solve of
                the same problem with per-kernel timing on, whose chunks launch
                directly) against the 8 TB/s HBM peak; traffic = measured HBM bytes per
                launch from the committed rocprofv3 counter summary of that
                kernel (profiles/traffic_<workload>_<precision>.json), null when
                the kernel's source changed since the counters were taken
  per_vector    the same library at n = 1 in FP64 (multi-shift CG per column)
  other_precision  the same solve in the other precision (FP64 <-> mixed)
  autotuned     kernel variants bms_autotune picked on this problem (before warmup)
  batch         the workload's uneven batch of lattices through bms_solve_batch
                (all at once) and one after the other
  cpu_baseline  the FP64 CPU oracle's multi-shift CG on a bounded sample
The precision of the timed solves is the workload's (mixed at 32^4).
"""
import hashlib
import argparse
import json
import re
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "RHS-solves/sec at 1e-10 residual, block vs per-vector CG; Dslash HBM GB/s"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def set_omp_threads(k):
    """Thread count of the oracle's OpenMP regions from here on (None: unchanged)."""
    import ctypes
    try:
        ctypes.CDLL("libgomp.so.1").omp_set_num_threads(int(k))
        return True
    except OSError:
        return False


def cpu_oracle_sample(U, B, w, r, per_vector_iters, budget_s, threads=None):
    """Time the oracle's multi-shift CG (one column, all shifts) per iteration
    by differencing two bounded runs, then scale to a full solve."""
    import numpy as np

    from oracle import oracle as O
    if threads is not None and not set_omp_threads(threads):
        raise RuntimeError("cannot set the OpenMP thread count")
    dims, bc, m = w["dims"], (1, 1, 1, -1), w["mass"]
    sh = np.sort(r.beta)
    b = np.ascontiguousarray(B[..., 0])
    t0 = time.time()
    O.mscg(dims, bc, U, m, sh, b, 1e-30, 1)
    t1 = time.time() - t0
    # per-iteration estimate from the first run, then a longer run within budget
    n2 = max(3, min(40, int(budget_s / max(t1, 1e-3))))
    t0 = time.time()
    O.mscg(dims, bc, U, m, sh, b, 1e-30, n2)
    t2 = time.time() - t0
    per_it = max((t2 - t1) / (n2 - 1), 1e-9)
    solve_s = per_it * per_vector_iters
    if threads is None:
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return dict(value=1.0 / solve_s, unit="RHS-solves/s", cores=threads, kind="oracle",
                sample=("oracle C FP64 multi-shift CG, 1 column x %d shifts at %s: %d vs 1 "
                        "iterations timed (%.1f s), %.3f s/iteration, scaled to the %d "
                        "iterations a per-vector solve of this workload takes"
                        % (len(sh), "x".join(map(str, dims)), n2, t1 + t2, per_it,
                           per_vector_iters)))


# source file of each kernel class (for the staleness check of stored counters)
KERNEL_SOURCE = {"update": "paper_1808_01829_amd/csrc/update_mfma.hip",
                 "hop": "paper_1808_01829_amd/csrc/hop.hip",
                 "gram": "paper_1808_01829_amd/csrc/blas.hip",
                 "force": "paper_1808_01829_amd/csrc/force.hip"}


def source_sha(kernel):
    path = os.path.join(ROOT, KERNEL_SOURCE.get(kernel, ""))
    if not os.path.isfile(path):
        return None
    return hashlib.sha256(open(path, "rb").read()).hexdigest()


def stored_traffic(workload, prec, kernel):
    """Measured HBM bytes per launch of `kernel` from the committed counter
    summary, or None if there is none or the kernel source changed since."""
    path = os.path.join(ROOT, "profiles", "traffic_%s_%s.json" % (workload, prec))
    if not os.path.isfile(path):
        return None
    d = json.load(open(path))
    k = d.get("kernels", {}).get(kernel)
    if not k or k.get("source_sha256") != source_sha(kernel):
        return None
    return k.get("bytes_per_launch")


def run_batch(args, w, r, bms, opts, torch, np):
    """The workload's uneven batch (same mass, disorder, n_pf and poles on each
    lattice): one bms_solve_batch (all concurrently), then the same solves one
    after the other; RHS columns with every shift at tol, per second."""
    from paper_1808_01829_amd.inputs import gaussian_block, random_gauge
    ctxs, Bs = [], []
    for k, dims in enumerate(w["batch"]):
        U = random_gauge(dims, w["eps"], 1000 * w["id"] + 10 * (k + 1))
        B = gaussian_block(dims, w["n"], 1000 * w["id"] + 10 * (k + 1) + 1)
        c = bms.Context(dims, (1, 1, 1, -1))
        c.set_gauge(torch.from_numpy(U).to("cuda:0"))
        ctxs.append(c)
        Bs.append(torch.from_numpy(B).to("cuda:0"))
    k = len(ctxs)
    shifts = [r.beta] * k
    ops = [opts] * k
    bms.solve_batch(ctxs, [w["mass"]] * k, shifts, Bs, tol=w["tol"], max_iter=20000, opts=ops)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, stats = bms.solve_batch(ctxs, [w["mass"]] * k, shifts, Bs, tol=w["tol"], max_iter=20000,
                               opts=ops, raise_on_error=False)
    torch.cuda.synchronize()
    tb = time.perf_counter() - t0
    solved = sum(int(np.sum(np.all(np.asarray(st["true_residual"]) <= w["tol"], axis=0)))
                 for st in stats)
    t0 = time.perf_counter()
    for c, B in zip(ctxs, Bs):
        c.solve(w["mass"], r.beta, B, tol=w["tol"], max_iter=20000, opts=opts)
    torch.cuda.synchronize()
    ts = time.perf_counter() - t0
    return dict(lattices=["x".join(map(str, d)) for d in w["batch"]], n_pf=w["n"],
                value=round(solved / tb, 4), unit="RHS-solves/s", s_concurrent=round(tb, 3),
                s_sequential=round(ts, 3), iterations=[st["iterations"] for st in stats],
                max_true_residual=max(st["max_true_residual"] for st in stats))


def per_vector(ctx, bms, m, r, Bd, tol, cols, torch):
    """Same library, n = 1, FP64, one column at a time (multi-shift CG)."""
    iters = []
    opts = bms.bms_default_opts()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for j in range(cols):
        _, st = ctx.solve(m, r.beta, Bd[..., j:j + 1].contiguous(), tol=tol, max_iter=50000,
                          opts=opts)
        iters.append(st["iterations"])
    torch.cuda.synchronize()
    return iters, cols / (time.perf_counter() - t0)


FP64_VALU_PEAK_TFLOPS = 78.6
MFMA_F64_PEAK_TFLOPS = 78.6   # dense FP64 matrix cores
MFMA_F32_PEAK_TFLOPS = 157.3  # dense FP32 matrix cores


def action_measure(ctx, r, Bd, X, torch, reps=5):
    """The action S_i = Re phi_i^dag (a0 phi_i + sum_j alpha_j X_ij) of the
    timed solve's own solutions: wall time per bms_action call (the reduction
    kernel, its partial sums and the read-back of n values), against its
    algorithmic bytes (B and every X read once)."""
    alpha = list(r.alpha)
    ctx.action(r.a0, alpha, Bd, X)  # warm-up (scratch allocation)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(reps):
        S = ctx.action(r.a0, alpha, Bd, X)
    us = (time.perf_counter() - t) / reps * 1e6
    nbytes = (1 + X.shape[0]) * Bd.numel() * Bd.element_size()
    gbs = nbytes / (us * 1e-6) / 1e9
    return dict(call="bms_action", avg_us=round(us, 1), algorithmic_bytes=int(nbytes),
                gbs=round(gbs, 1), hbm_frac=round(gbs / HBM_PEAK_GBS, 4),
                columns=len(S), note="wall time per call, read-back included")


def force_measure(bms, torch, np, configs, reps=3):
    """The whole bms_force call at the force workload (K = n_pf x N_s
    columns), random solutions (its cost does not depend on their values):
    time, algorithmic GB/s (every solution, the FP64 links and the output
    once) and FP64 TFLOP/s (y = D_oe x and the outer products: 1152 flops per
    odd site and column) against both roofs; the hops + per-link path
    (variant 0) timed beside it."""
    from paper_1808_01829_amd.inputs import random_gauge
    wf = configs.WORKLOADS["c4"]
    rf = configs.workload_coefficients("c4")
    dims, n, ns = wf["dims"], wf["n"], rf.n_poles
    ctx = bms.Context(dims, (1, 1, 1, -1))
    ctx.set_gauge(torch.from_numpy(random_gauge(dims, wf["eps"], 7001)).cuda())
    vh = int(np.prod(dims)) // 2
    g = torch.Generator(device="cuda").manual_seed(7002)
    X = torch.randn((ns, vh, 3, n), dtype=torch.complex128, device="cuda", generator=g)
    alpha = list(rf.alpha)
    vol = int(np.prod(dims))
    flops = (vol // 2) * n * ns * 1152.0
    res = {}
    for v in (-1, 0):
        ctx.set_variant(bms.BMS_KERNEL_FORCE, v)
        ctx.force(alpha, X)  # warm-up (scratch allocation)
        torch.cuda.synchronize()
        ctx.timing(True)
        for _ in range(reps):
            ctx.force(alpha, X)
        torch.cuda.synchronize()
        ms, nl, by = ctx.timing_read()["force"]
        ctx.timing(False)
        us = 1e3 * ms / nl
        res[v] = (us, by / nl)
    ctx.set_variant(bms.BMS_KERNEL_FORCE, -1)
    us, nbytes = res[-1]
    gbs = nbytes / (us * 1e-6) / 1e9
    tf = flops / (us * 1e-6) / 1e12
    return dict(kernel="k_force_fused (whole bms_force call)",
                workload="c4: %s, n_pf=%d, %d shifts (K=%d), FP64" % (
                    "x".join(map(str, dims)), n, ns, n * ns), avg_us=round(us, 1),
                algorithmic_bytes=round(nbytes), flops=flops, gbs=round(gbs, 1),
                hbm_frac=round(gbs / HBM_PEAK_GBS, 4), tflops=round(tf, 2),
                fp64_valu_frac=round(tf / FP64_VALU_PEAK_TFLOPS, 4),
                bound="fp64 valu", frac_of_binding_roof=round(tf / FP64_VALU_PEAK_TFLOPS, 4),
                traffic=stored_traffic("c4", "f64", "force"),
                hops_then_per_link_us=round(res[0][0], 1))


def shard_local(bms, torch, dims, eps, n, reps=10):
    """One GPU's share of the lattice split over 8 GPUs along t (the local
    sub-lattice with its own periodic wrap standing in for the halo): the two
    half hops at n columns in FP64 and FP32, their time and algorithmic GB/s
    (two-row links when the field passes the check), and the bytes of one
    t-face of the other parity that a half hop would exchange per
    neighbour."""
    from paper_1808_01829_amd.inputs import gaussian_block, random_gauge
    L = list(dims)
    L[3] = dims[3] // 8
    vh = L[0] * L[1] * L[2] * L[3] // 2
    ctx = bms.Context(L, (1, 1, 1, -1))
    ctx.set_gauge(torch.from_numpy(random_gauge(L, eps, 7101)).cuda())
    epl = 6 if ctx.link_rows() == 2 else 9
    v = torch.from_numpy(gaussian_block(L, n, 7102)).cuda()
    out = dict(lattice=L, n=n, link_rows=ctx.link_rows())
    for prec, name, b in ((bms.BMS_PREC_F64, "f64", 8), (bms.BMS_PREC_F32, "f32", 4)):
        x = v if b == 8 else v.to(torch.complex64)
        for par in (1, 0):
            ctx.apply_hop(par, x, prec)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            y = ctx.apply_hop(1, x, prec)
            ctx.apply_hop(0, y, prec)
        e1.record()
        torch.cuda.synchronize()
        us = e0.elapsed_time(e1) * 1e3 / reps / 2
        algo = vh * 8 * epl * 2 * b + 2 * vh * 3 * n * 2 * b
        face = L[0] * L[1] * L[2] // 2 * 3 * n * 2 * b
        out[name] = dict(us_per_hop=round(us, 1), gbs=round(algo / (us * 1e-6) / 1e9, 1),
                         face_bytes=face)
    ctx.close()
    return out


def operator_block_gain(bms, torch, dims, Ud, reps=5):
    """Half hops on one GPU for the unimproved operator (8 links per site)
    and the improved one (one-hop plus three-hop links, 16 per site; V = 9/8 U,
    W = -1/24 U, the cost does not depend on the values): time per hop at
    n = 16 and n = 1 in FP64 and FP32, algorithmic GB/s at n = 16, and the
    block gain per column, 16 x t(n=1) / t(n=16)."""
    vh = Ud.shape[1] // 2
    out = {}
    for name in ("unimproved", "improved"):
        ctx = bms.Context(dims, (1, 1, 1, -1))
        if name == "improved":
            ctx.set_gauge_improved(Ud * (9.0 / 8.0), Ud * (-1.0 / 24.0))
        else:
            ctx.set_gauge(Ud)
        nl = 16 if name == "improved" else 8
        res = {}
        for prec, dt, b in ((bms.BMS_PREC_F64, torch.complex128, 8),
                            (bms.BMS_PREC_F32, torch.complex64, 4)):
            t = {}
            for n in (1, 16):
                x = torch.zeros((vh, 3, n), dtype=dt, device="cuda")
                y = ctx.apply_hop(1, x, prec)
                torch.cuda.synchronize()
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record()
                for _ in range(reps):
                    y = ctx.apply_hop(1, x, prec)
                e1.record()
                torch.cuda.synchronize()
                t[n] = e0.elapsed_time(e1) * 1e3 / reps
            epl = 6 if ctx.link_rows() == 2 else 9  # link entries read (two-row SU(3) links: 6)
            algo = vh * nl * epl * 2 * b + 2 * vh * 3 * 16 * 2 * b
            res["f64" if b == 8 else "f32"] = dict(
                us_n16=round(t[16], 1), us_n1=round(t[1], 1),
                gbs_n16=round(algo / (t[16] * 1e-6) / 1e9, 1),
                block_gain_per_column=round(16 * t[1] / t[16], 2))
        out[name] = res
        ctx.close()
    return out


# traversals of the half hop timed by --hop-traversal: (ty, tz, tt, cap, nt),
# ty = 0 the natural site order (tiles otherwise), cap the resident
# work-groups per compute unit (0: none), nt the non-temporal link hint; all
# with the default kernel, then the streamed kernel (hop variant 4, whose cap
# is its ring depth)
HOP_TRAVERSALS = {
    "f64": [(0, 0, 0, c, 1) for c in range(5)] + [(8, 8, 8, c, 1) for c in range(1, 5)] +
           [(8, 8, 8, 2, 0), (8, 8, 4, 2, 1), (4, 4, 8, 2, 1), (16, 16, 2, 2, 1), (32, 8, 1, 2, 1)],
    "f32": [(0, 0, 0, c, 1) for c in range(5)] +
           [(8, 8, 8, 1, 1), (8, 8, 8, 2, 1), (4, 4, 8, 2, 1), (16, 16, 2, 2, 1), (32, 8, 1, 2, 1)],
}
HOP_STREAMED = [(8, 8, 8, 2, 1), (8, 8, 4, 2, 0), (8, 8, 8, 4, 1), (0, 0, 0, 2, 1), (0, 0, 0, 4, 1)]


def hop_traversal(bms, torch, dims, eps, n, reps=5):
    """Each half hop (both parities, n columns, two-row links when the field
    passes the check) under every traversal of HOP_TRAVERSALS with the default
    kernel and of HOP_STREAMED with the streamed one: one untimed launch, then
    `reps` launches timed with HIP events. The launch order is fixed
    (precision, kernel and traversal, parity; 1 + reps launches each), so a
    counter run of the same command maps its hop dispatches onto these rows."""
    from paper_1808_01829_amd.inputs import gaussian_block, random_gauge
    ctx = bms.Context(dims, (1, 1, 1, -1))
    ctx.set_gauge(torch.from_numpy(random_gauge(dims, eps, 7201)).cuda())
    v = torch.from_numpy(gaussian_block(dims, n, 7202)).cuda()
    rows = []
    for prec, name in ((bms.BMS_PREC_F64, "f64"), (bms.BMS_PREC_F32, "f32")):
        x = v if name == "f64" else v.to(torch.complex64)
        for variant, cfg in [(-1, c) for c in HOP_TRAVERSALS[name]] + [(4, c) for c in HOP_STREAMED]:
            ctx.set_variant(bms.BMS_KERNEL_HOP, variant)
            ctx.set_hop_config(prec, cfg)
            for par in (1, 0):
                ctx.apply_hop(par, x, prec)
                torch.cuda.synchronize()
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record()
                for _ in range(reps):
                    ctx.apply_hop(par, x, prec)
                e1.record()
                torch.cuda.synchronize()
                rows.append(dict(prec=name, variant=variant, cfg=list(cfg), par=par,
                                 us=round(e0.elapsed_time(e1) * 1e3 / reps, 1)))
        ctx.set_variant(bms.BMS_KERNEL_HOP, -1)
        ctx.set_hop_config(prec, None)
    out = dict(lattice=list(dims), n=n, link_rows=ctx.link_rows(), reps=reps, rows=rows)
    ctx.close()
    return out


def write_hop_traversal(fetch_csv, pmc_json, time_json, cal_fetch_csv, command, out_path):
    """A text table of --hop-traversal: per traversal and parity the time (a
    run without the profiler), and the FETCH_SIZE of one rocprofv3 --pmc run of
    the same command (median over the timed launches, scaled by the 1 GiB copy
    calibration), as bytes and as multiples of the block vector read."""
    fetch_factor, _ = copy_factor(cal_fetch_csv)
    hop = [v for k, v in _counter_rows(fetch_csv) if "k_hop" in k]
    run = json.loads([l for l in open(pmc_json) if l.startswith("{")][-1])
    tim = json.loads([l for l in open(time_json) if l.startswith("{")][-1])
    per = 1 + run["reps"]
    if len(hop) != per * len(run["rows"]):
        raise SystemExit("hop dispatches %d, expected %d" % (len(hop), per * len(run["rows"])))
    dims, n = run["lattice"], run["n"]
    vh = dims[0] * dims[1] * dims[2] * dims[3] // 2
    epl = 6 if run["link_rows"] == 2 else 9
    lines = ["# Half hop by traversal, %s lattice, n = %d, %d-entry links" %
             ("x".join(map(str, dims)), n, epl), "",
             "commands:",
             "  python3 bench.py --hop-traversal        (times: HIP events, %d launches each)" %
             run["reps"],
             "  " + command,
             "  python3 bench.py --write-hop-traversal <fetch csv> <pmc run json> "
             "<time run json> <copy fetch csv>",
             "fetch: FETCH_SIZE per dispatch x %.4f (1 GiB copy calibration); "
             "S = one block vector, G = the links" % fetch_factor, "",
             "variant -1: the default kernel; 4: the streamed kernel (cap = its ring depth)", "",
             "prec  var traversal (ty,tz,tt,cap,nt)  par     us   fetch MB   (fetch - G) / S   "
             "fetch GB/s"]
    for i, (r, t) in enumerate(zip(run["rows"], tim["rows"])):
        b = 8 if r["prec"] == "f64" else 4
        S = vh * 3 * n * 2 * b
        G = vh * 8 * epl * 2 * b
        vals = sorted(hop[i * per + 1:(i + 1) * per])
        f = vals[len(vals) // 2] * 1024 * fetch_factor
        lines.append("%-5s %3d %-28s %3d %7.1f %10.1f %17.2f %12.0f" %
                     (r["prec"], r.get("variant", -1), tuple(r["cfg"]), r["par"], t["us"],
                      f / 1e6, (f - G) / S, f / (t["us"] * 1e-6) / 1e9))
    with open(out_path, "w") as fo:
        fo.write("\n".join(lines) + "\n")
    return out_path


def rhmc_measure(bms, torch, np, configs):
    """One RHMC trajectory at the paper's settings (force solves at 1e-7,
    heatbath and action at 1e-14, two-level Omelyan with lambda = 1/6, three
    gauge steps per fermion step, tau = 1) on the 8^4 workload (n_pf = 4,
    m = 0.05, beta = 5.12): wall time, dH and the solver work."""
    from paper_1808_01829_amd.inputs import gaussian_block, random_gauge
    w = configs.WORKLOADS["c2"]
    dims, n = w["dims"], w["n"]
    c = bms.Context(dims, (1, 1, 1, -1))
    U = torch.from_numpy(random_gauge(dims, 0.3, 9001)).cuda()
    P = torch.from_numpy(np.random.default_rng(9002).standard_normal(
        (4, int(np.prod(dims)), 8))).cuda()
    eta = torch.from_numpy(gaussian_block(dims, n, 9003)).cuda()
    kw = dict(r_hb=configs.heatbath_coefficients("c2"), r_acc=configs.accept_coefficients("c2"),
              r_md=configs.workload_coefficients("c2"), tau=1.0, n_steps=10, n_gauge=3)
    bms.rhmc_trajectory(c, U.clone(), P.clone(), eta, 5.12, w["mass"], **kw)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = bms.rhmc_trajectory(c, U, P, eta, 5.12, w["mass"], **kw)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return dict(workload="c2: 8x8x8x8, n_pf=4, m=0.05, beta=5.12, tau=1, 10 steps x 3 gauge "
                         "steps, OMF2 lambda=1/6", s_per_trajectory=round(dt, 3),
                dH=res["dH"], acceptance=round(min(1.0, float(np.exp(-res["dH"]))), 4),
                force_evals=res["force_evals"], block_iterations=res["iterations"],
                heatbath_action_residual=res["max_residual_hb"])


KERNEL_CLASS_PREFIX = {"update": ("k_update_mfma", "k_update_n", "k_update_fast", "k_update<"),
                       "hop": ("k_hop",), "gram": ("k_gram4",),
                       "force": ("k_force_fused",)}


def _counter_rows(path):
    """(kernel name, counter value) of every dispatch in a rocprofv3
    counter_collection CSV."""
    import csv
    out = []
    with open(path) as f:
        for row in csv.DictReader(f):
            out.append((row.get("Kernel_Name", ""), float(row.get("Counter_Value", 0))))
    return out


COPY_BYTES = 1 << 30


def copy_factor(cal_csv):
    """Bytes per counted KiB: the 1 GiB copy of --copy-calibration over the
    largest per-dispatch value the counter read in that run (the copy's; the
    fill before it writes as much and reads nothing)."""
    kib = max(v for _, v in _counter_rows(cal_csv))
    return COPY_BYTES / (kib * 1024.0), kib


def write_traffic(workload, prec, fetch_csv, write_csv, cal_fetch_csv, cal_write_csv, commands,
                  algorithmic, out_dir):
    """<out_dir>/traffic_<workload>_<prec>.json from one FETCH_SIZE and one
    WRITE_SIZE rocprofv3 run (KiB per dispatch), scaled by what the same
    counters read for a plain 1 GiB copy; algorithmic: {class: bytes per
    launch}."""
    fetch_factor, cal_f = copy_factor(cal_fetch_csv)
    write_factor, cal_w = copy_factor(cal_write_csv)
    fetch, write = _counter_rows(fetch_csv), _counter_rows(write_csv)
    kernels = {}
    for cls, prefixes in KERNEL_CLASS_PREFIX.items():
        pat = re.compile(r"(^|[\s:])(%s)" % "|".join(re.escape(p) for p in prefixes))
        f = [v for k, v in fetch if pat.search(k)]
        w = [v for k, v in write if pat.search(k)]
        if not f or not w or cls not in algorithmic:
            continue
        fk, wk = sum(f) / len(f), sum(w) / len(w)
        b = fk * 1024 * fetch_factor + wk * 1024 * write_factor
        kernels[cls] = dict(source=KERNEL_SOURCE.get(cls), source_sha256=source_sha(cls),
                            launches=len(f), fetch_kib=round(fk, 1), write_kib=round(wk, 1),
                            bytes_per_launch=round(b),
                            algorithmic_bytes_per_launch=round(algorithmic[cls]),
                            ratio=round(b / algorithmic[cls], 3))
    out = dict(workload=workload, commands=commands,
               calibration=dict(copy_bytes=COPY_BYTES, copy_fetch_kib=cal_f, copy_write_kib=cal_w,
                                fetch_factor=round(fetch_factor, 4),
                                write_factor=round(write_factor, 4),
                                command="rocprofv3 --pmc FETCH_SIZE|WRITE_SIZE -- python3 bench.py "
                                        "--copy-calibration"),
               kernels=kernels)
    path = os.path.join(out_dir, "traffic_%s_%s.json" % (workload, prec))
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    return path


def trace_gaps(path, split_ms=50.0):
    """Idle time of the GPU inside the first solve of a rocprofv3 kernel trace
    (--kernel-trace CSV): the dispatches are cut into bursts at host pauses
    longer than split_ms; the first burst with update kernels is the solve.
    Returns its span, the time some kernel ran (union of the intervals) and
    the distribution of the gaps between one kernel's end and the next one's
    start (launch latency, host checks between chunks, host work between
    phases): what a persistent kernel could at most remove."""
    import csv
    ev = []
    with open(path) as f:
        for row in csv.DictReader(f):
            ev.append((int(row["Start_Timestamp"]), int(row["End_Timestamp"]),
                       row.get("Kernel_Name", "")))
    ev.sort()
    bursts, cur, last_end = [], [], None
    for e in ev:
        if cur and e[0] - last_end > split_ms * 1e6:
            bursts.append(cur)
            cur = []
        cur.append(e)
        last_end = e[1] if last_end is None or not cur[:-1] else max(last_end, e[1])
    if cur:
        bursts.append(cur)
    solve = next(b for b in bursts if any("k_update" in e[2] for e in b))
    busy, gaps, end = 0, [], None
    for a, b, _ in solve:
        if end is None or a >= end:
            if end is not None:
                gaps.append(a - end)
            busy += b - a
            end = b
        elif b > end:
            busy += b - end
            end = b
    span = solve[-1][1] - solve[0][0]
    edges = [(0, 5e3), (5e3, 20e3), (20e3, 100e3), (100e3, 1e6), (1e6, 1e18)]
    hist = {("%g-%g us" % (lo / 1e3, hi / 1e3) if hi < 1e18 else ">%g us" % (lo / 1e3)):
            dict(count=sum(lo <= g < hi for g in gaps),
                 ms=round(sum(g for g in gaps if lo <= g < hi) / 1e6, 2)) for lo, hi in edges}
    return dict(kernels=len(solve), span_ms=round(span / 1e6, 2), busy_ms=round(busy / 1e6, 2),
                idle_ms=round((span - busy) / 1e6, 2), idle_frac=round((span - busy) / span, 4),
                mean_gap_us=round(sum(gaps) / max(1, len(gaps)) / 1e3, 2), gaps=hist)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c5")
    ap.add_argument("--precision", choices=["f64", "mixed"], default=None)
    ap.add_argument("--baseline-cols", type=int, default=2,
                    help="columns solved one at a time (n = 1, FP64) for the per-vector rate")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--other-precision", type=int, default=1,
                    help="also time this many solves in the other precision (reported aside)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-autotune", action="store_true",
                    help="skip bms_autotune (kernel variants picked on this problem before warmup)")
    ap.add_argument("--tune-cache", default=None,
                    help="JSON-lines file of bms_autotune results: a hit skips the sweep")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the workload's uneven batch of lattices (reported aside)")
    ap.add_argument("--seeds", type=int, default=3,
                    help="gauge/RHS seeds: the timed seed plus one solve on each further seed "
                         "(median, min, max reported aside)")
    ap.add_argument("--no-force", action="store_true",
                    help="skip the force-kernel measurement (reported aside)")
    ap.add_argument("--link-rows", type=int, default=2, choices=(2, 3),
                    help="rows of each SU(3) link the hop reads (2: third row rebuilt)")
    ap.add_argument("--no-rhmc", action="store_true",
                    help="skip the RHMC trajectory measurement (reported aside)")
    ap.add_argument("--no-operators", action="store_true",
                    help="skip the unimproved/improved operator comparison (reported aside)")
    ap.add_argument("--force-only", action="store_true",
                    help="only the force measurement (for profiling the force kernel)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only a 1 GiB device copy (calibrates the HBM traffic counters)")
    ap.add_argument("--write-traffic", nargs=6,
                    metavar=("PREC", "FETCH_CSV", "WRITE_CSV", "CAL_FETCH_CSV", "CAL_WRITE_CSV",
                             "RUN_JSON"),
                    help="write traffic_<workload>_<PREC>.json from two rocprofv3 counter CSVs "
                         "of this benchmark, scaled by the same counters on the 1 GiB copy of "
                         "--copy-calibration, with the algorithmic bytes from that run's JSON "
                         "line; then exit (no GPU)")
    ap.add_argument("--traffic-out", default=os.path.join(ROOT, "profiles"),
                    help="with --write-traffic: folder of the JSON file")
    ap.add_argument("--profile-command", default="",
                    help="with --write-traffic: the command the counter runs used ({} = counter)")
    ap.add_argument("--hop-traversal", action="store_true",
                    help="only the half hops of the workload under a fixed list of traversals "
                         "(times per launch, one JSON line)")
    ap.add_argument("--write-hop-traversal", nargs=4,
                    metavar=("FETCH_CSV", "PMC_RUN_JSON", "TIME_RUN_JSON", "CAL_FETCH_CSV"),
                    help="write profiles/hop_traversal_<workload>.txt from a FETCH_SIZE run and "
                         "a plain run of --hop-traversal; then exit (no GPU)")
    ap.add_argument("--trace-gaps", metavar="KERNEL_TRACE_CSV", default=None,
                    help="print the GPU idle time inside the first solve of a rocprofv3 "
                         "kernel trace of this benchmark; then exit (no GPU)")
    args = ap.parse_args()
    if args.trace_gaps:
        print(json.dumps(trace_gaps(args.trace_gaps)))
        return
    if args.write_hop_traversal:
        fcsv, prun, trun, cfcsv = args.write_hop_traversal
        cmd = ("rocprofv3 --pmc FETCH_SIZE --kernel-include-regex k_hop --output-format csv "
               "-d <dir> -o run -- python3 -u bench.py --hop-traversal")
        print(write_hop_traversal(fcsv, prun, trun, cfcsv, cmd,
                                  os.path.join(args.traffic_out,
                                               "hop_traversal_%s.txt" % args.workload)))
        return
    if args.write_traffic:
        prec, fcsv, wcsv, cfcsv, cwcsv, run = args.write_traffic
        line = [l for l in open(run) if l.startswith("{")][-1]
        d = json.loads(line)
        if "kernels" in d:  # a benchmark line: bytes and launches per kernel class
            algo = {k: v["bytes"] / v["launches"] for k, v in d["kernels"].items() if v["bytes"]}
        else:  # the force-only line
            algo = {"force": d["algorithmic_bytes"]}
        cmd = args.profile_command
        print(write_traffic(args.workload, prec, fcsv, wcsv, cfcsv, cwcsv,
                            [cmd.replace("{}", "FETCH_SIZE"), cmd.replace("{}", "WRITE_SIZE")],
                            algo, args.traffic_out))
        return
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1808_01829_amd import bms
    from paper_1808_01829_amd.inputs import configs, gaussian_block, random_gauge

    if args.copy_calibration:
        a = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        a.fill_(1)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps(dict(copied_bytes=1 << 30)), flush=True)
        return
    if args.force_only:
        print(json.dumps(force_measure(bms, torch, np, configs)), flush=True)
        return
    if args.hop_traversal:
        w = configs.WORKLOADS[args.workload]
        print(json.dumps(hop_traversal(bms, torch, w["dims"], w["eps"], w["n"])), flush=True)
        return

    w = configs.WORKLOADS[args.workload]
    r = configs.workload_coefficients(args.workload)
    prec = args.precision or w["precision"]
    dims, n, m, tol = w["dims"], w["n"], w["mass"], w["tol"]
    log("bench: workload %s dims %s n %d shifts %d precision %s" % (args.workload, dims, n,
                                                                     r.n_poles, prec))
    t = time.time()
    U = random_gauge(dims, w["eps"], 1000 * w["id"])
    B = gaussian_block(dims, n, 1000 * w["id"] + 1)
    log("bench: inputs generated in %.1f s" % (time.time() - t))
    dev = torch.device("cuda:0")
    Ud = torch.from_numpy(U).to(dev)
    Bd = torch.from_numpy(B).to(dev)
    ctx = bms.Context(dims, (1, 1, 1, -1))
    ctx.set_link_rows(args.link_rows)
    ctx.set_gauge(Ud)
    link_rows = ctx.link_rows()
    opts = bms.bms_default_opts()
    opts.precision = bms.BMS_PREC_F64 if prec == "f64" else bms.BMS_PREC_MIXED
    if w.get("reliable"):
        opts.reliable_interval = w["reliable"]

    tuned = None
    if args.tune_cache:
        ctx.set_tune_cache(args.tune_cache)
    if not args.no_autotune:
        t = time.time()
        tuned = ctx.autotune(m, r.beta, Bd, precision=opts.precision, iters=16)
        log("bench: autotune %.1f s: %s" % (time.time() - t, tuned))
    X = None
    for i in range(args.warmup):
        X, st = ctx.solve(m, r.beta, Bd, tol=tol, max_iter=20000, opts=opts)
        log("bench: warmup %d: %d iterations, max true residual %.2e" % (
            i, st["iterations"], st["max_true_residual"]))
    del X
    # The timed steps run the product path: every chunk of iterations replayed
    # from its captured hipGraph, no per-kernel events. Per-kernel durations
    # come from one further solve of the same problem with timing on (chunks
    # then launch directly, with HIP events on the library stream between the
    # kernels); the rocprofv3 kernel trace of the bench command agrees.
    torch.cuda.synchronize()
    solved = 0
    iters, phases = [], []
    maxres = 0.0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        X, st = ctx.solve(m, r.beta, Bd, tol=tol, max_iter=20000, opts=opts)
        res = np.asarray(st["true_residual"])
        solved += int(np.sum(np.all(res <= tol, axis=0)))
        iters.append(st["iterations"])
        phases.append({k: st[k] for k in ("multishift_iterations", "refine_iterations",
                                          "iterations_f64", "iterations_f32", "hop_calls",
                                          "reliable_updates")})
        maxres = max(maxres, st["max_true_residual"])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    log("bench: %d steps in %.3f s, iterations %s, max true residual %.2e" % (
        args.steps, elapsed, iters, maxres))
    value = solved / elapsed
    del X
    ctx.timing(True)
    t0 = time.perf_counter()
    X, st_timed = ctx.solve(m, r.beta, Bd, tol=tol, max_iter=20000, opts=opts)
    torch.cuda.synchronize()
    s_timed = time.perf_counter() - t0
    kt = ctx.timing_read()
    kf = ctx.timing_flops()
    # per-launch bound of each class: each launch against whichever roof binds it
    kfloor = {k: ctx.timing_floor(k, HBM_PEAK_GBS * 1e9, MFMA_F64_PEAK_TFLOPS * 1e12,
                                  MFMA_F32_PEAK_TFLOPS * 1e12) for k in kt}
    ctx.timing(False)
    log("bench: one instrumented solve (direct launches, events) %.3f s, %d iterations" % (
        s_timed, st_timed["iterations"]))

    kernels = {}
    for name, (ms, nl, by) in kt.items():
        if nl:
            kernels[name] = dict(ms_total=ms, launches=nl, avg_us=1e3 * ms / nl, bytes=by,
                                 gbs=(by / (ms * 1e-3) / 1e9) if ms > 0 and by > 0 else None)
    dom = max((k for k in kernels if kernels[k]["gbs"]), key=lambda k: kernels[k]["ms_total"])
    dk = kernels[dom]
    roofline = dict(bound="hbm", kernel=dom, achieved=round(dk["gbs"], 1), peak=HBM_PEAK_GBS,
                    unit="GB/s", frac=round(dk["gbs"] / HBM_PEAK_GBS, 4),
                    traffic=stored_traffic(args.workload, prec, dom),
                    algorithmic_bytes_per_launch=round(dk["bytes"] / dk["launches"]))
    # the same launches against the matrix cores: their time at the FP64 and
    # FP32 MFMA peaks next to their time at the HBM peak (the larger bounds)
    f64, f32 = kf.get(dom, (0.0, 0.0))
    if f64 + f32 > 0:
        t = dk["ms_total"] * 1e-3
        t_mfma = f64 / (MFMA_F64_PEAK_TFLOPS * 1e12) + f32 / (MFMA_F32_PEAK_TFLOPS * 1e12)
        t_hbm = dk["bytes"] / (HBM_PEAK_GBS * 1e9)
        roofline["mfma"] = dict(
            flops_f64_per_launch=round(f64 / dk["launches"]),
            flops_f32_per_launch=round(f32 / dk["launches"]),
            peaks_tflops=dict(f64=MFMA_F64_PEAK_TFLOPS, f32=MFMA_F32_PEAK_TFLOPS),
            frac=round(t_mfma / t, 4),
            note="time at the MFMA peaks / measured time; the HBM view above is %.4f" % (
                t_hbm / t))
        # each launch against whichever roof binds it (the window-closing
        # launches on the matrix cores, the others on HBM)
        t_floor = kfloor[dom]
        roofline["per_launch_bound"] = dict(
            frac=round(t_floor / t, 4), floor_ms_per_launch=round(t_floor / dk["launches"] * 1e3, 4),
            note="sum over launches of max(bytes / HBM peak, MFMA flops / MFMA peaks) / measured time")

    action = action_measure(ctx, r, Bd, X, torch)
    log("bench: action %s" % action)
    del X

    # per-vector baseline: same library, n = 1, FP64, one column at a time
    pv_iters = [0]
    pv_rate = float("nan")
    if args.baseline_cols > 0:
        pv_iters, pv_rate = per_vector(ctx, bms, m, r, Bd, tol, args.baseline_cols, torch)
        log("bench: per-vector FP64 %d columns, %.4f RHS-solves/s, iterations %s" % (
            args.baseline_cols, pv_rate, pv_iters))

    other = None
    if args.other_precision > 0:
        op = "mixed" if prec == "f64" else "f64"
        oo = bms.bms_default_opts()
        oo.precision = bms.BMS_PREC_F64 if op == "f64" else bms.BMS_PREC_MIXED
        if w.get("reliable"):
            oo.reliable_interval = w["reliable"]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        osolved, ost = 0, None
        for i in range(args.other_precision):
            _, ost = ctx.solve(m, r.beta, Bd, tol=tol, max_iter=20000, opts=oo, raise_on_error=False)
            res = np.asarray(ost["true_residual"])
            osolved += int(np.sum(np.all(res <= tol, axis=0)))
        torch.cuda.synchronize()
        ot = time.perf_counter() - t0
        other = dict(precision=op, value=round(osolved / ot, 4), unit="RHS-solves/s",
                     s_per_solve=round(ot / args.other_precision, 3),
                     iterations=ost["iterations"],
                     multishift_iterations=ost["multishift_iterations"],
                     refine_iterations=ost["refine_iterations"],
                     iterations_f64=ost["iterations_f64"], iterations_f32=ost["iterations_f32"],
                     reliable_updates=ost["reliable_updates"],
                     max_true_residual=ost["max_true_residual"])
        log("bench: %s: %s" % (op, other))

    seeds = None
    if args.seeds > 1:
        vals = [value]
        for k in range(1, args.seeds):
            Uk = random_gauge(dims, w["eps"], 1000 * w["id"] + 10 * k)
            Bk = gaussian_block(dims, n, 1000 * w["id"] + 10 * k + 1)
            ctx.set_gauge(torch.from_numpy(Uk).to(dev))
            Bkd = torch.from_numpy(Bk).to(dev)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, sk = ctx.solve(m, r.beta, Bkd, tol=tol, max_iter=20000, opts=opts,
                              raise_on_error=False)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            res = np.asarray(sk["true_residual"])
            vals.append(int(np.sum(np.all(res <= tol, axis=0))) / dt)
            del Bkd
        ctx.set_gauge(Ud)
        seeds = dict(values=[round(v, 4) for v in vals], median=round(float(np.median(vals)), 4),
                     min=round(min(vals), 4), max=round(max(vals), 4), unit="RHS-solves/s",
                     note="first: the timed seed (mean of the timed steps); others: one solve each")
        log("bench: seeds %s" % (seeds,))

    operators = None
    shard = None
    if not args.no_operators:
        operators = operator_block_gain(bms, torch, dims, Ud)
        log("bench: operators %s" % (operators,))
        if dims[3] % 16 == 0:
            shard = shard_local(bms, torch, dims, w["eps"], n)
            log("bench: one GPU's share of a t-split over 8 GPUs %s" % (shard,))

    rhmc = None
    if not args.no_rhmc:
        rhmc = rhmc_measure(bms, torch, np, configs)
        log("bench: rhmc %s" % (rhmc,))

    force = None
    if not args.no_force:
        force = force_measure(bms, torch, np, configs)
        log("bench: force %s" % (force,))

    batch = None
    if w.get("batch") and not args.no_batch:
        batch = run_batch(args, w, r, bms, opts, torch, np)
        log("bench: batch %s" % (batch,))

    cpu = None
    cpu1 = None
    if not args.no_cpu:
        try:
            cpu = cpu_oracle_sample(U, B, w, r, int(np.mean(pv_iters or iters)), args.cpu_seconds)
            cpu1 = cpu_oracle_sample(U, B, w, r, int(np.mean(pv_iters or iters)),
                                     args.cpu_seconds / 2, threads=1)
            set_omp_threads(cpu["cores"])
        except Exception as e:  # the oracle is optional for the measurement
            log("bench: cpu baseline failed: %r" % (e,))

    out = dict(
        metric=METRIC, value=round(value, 4), unit="RHS-solves/s", n_gpus=1, steps=args.steps,
        warmup=args.warmup, ms_per_step=round(1e3 * elapsed / args.steps, 3),
        higher_is_better=True, scaling="weak", vs_baseline=None,
        dtype="f64" if prec == "f64" else "f32+f64",
        data="synthetic",
        config=dict(workload="%s: %s lattice, SU(3) U=exp(i*%g*H), staggered m=%g, n_pf=%d, "
                             "%d poles of x^(-%g), tol %g, %s"
                             % (args.workload, "x".join(map(str, dims)), w["eps"], m, n,
                                r.n_poles, w["power"], tol, prec),
                    lattice=list(dims), n_pf=n, n_shifts=r.n_poles, tol=tol, precision=prec),
        roofline=roofline,
        cpu_baseline=cpu,
        cpu_baseline_1thread=cpu1,
        rhs_shift_solves_per_s=round(value * r.n_poles, 3),
        dslash=dict(kernel="hop (both half hops)", link_rows=link_rows,
                    gbs=round(kernels["hop"]["gbs"], 1) if "hop" in kernels else None,
                    hbm_frac=round(kernels["hop"]["gbs"] / HBM_PEAK_GBS, 4)
                    if "hop" in kernels else None),
        seeds=seeds,
        action=action,
        force=force,
        operators=operators,
        shard_local=shard,
        rhmc=rhmc,
        per_vector=dict(value=round(pv_rate, 4) if pv_rate == pv_rate else None,
                        unit="RHS-solves/s", columns=args.baseline_cols,
                        iterations=pv_iters, dtype="f64"),
        block_over_per_vector=round(value / pv_rate, 3) if pv_rate == pv_rate else None,
        other_precision=other,
        autotuned=tuned,
        batch=batch,
        iterations=iters, iteration_phases=phases[0] if phases else None,
        timed_path="hipGraph replay of every chunk of %d iterations (use_graph=%d, no "
                   "per-kernel events)" % (opts.check_interval, opts.use_graph),
        kernel_timing=dict(source="one further solve with per-kernel HIP events (direct "
                                  "launches)", s_per_solve=round(s_timed, 3),
                           iterations=st_timed["iterations"]),
        max_true_residual=maxres,
        dslash_gbs=kernels.get("hop", {}).get("gbs"),
        kernels=kernels,
    )
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
