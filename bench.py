"""Benchmark: gradient evaluations per second of exponential-free open GRAPE.

Workload (one "step"): forward RK4 sweep, cost, backward adjoint sweep with
segment recompute, and the per-slice gradient, for a batch of B independent
control arrays on the transmon(3) x resonator(80) model: d = 240, K = 4
controls (resonator and qubit I/Q), J = 3 collapse operators, N_t = 10000
slices of dt = 0.002/kappa, smooth Gaussian-filtered noise controls
(problem b uses seed 2 + b), checkpoints for the slices whose forward states
do not fit in HBM.  float32 is the headline; the same workload is timed in
float64 for the FP32-vs-FP64 comparison.  Inputs are generated on the host
and resident in HBM before the timed region starts.

Prints one JSON line (rank 0).  With no flags: N = 1 GPU, 1 warmup step, 2
timed steps per precision, the secondary lines (extras), the serving leg and
the CPU oracle baseline on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "gradient evals/s at d=240 FP32 vs FP64 (≤1e-5 err); served p50/p99 latency"
HBM_PEAK_GBS = 8000.0


def _parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--batch", type=int, default=128)
    ap.add_argument("--n-t", type=int, default=10000)
    ap.add_argument("--gmode", default="grape1", choices=["grape1", "exact"])
    ap.add_argument("--path", default="banded", choices=["banded", "dense", "auto"])
    ap.add_argument("--precisions", default="f32,f64")
    ap.add_argument("--resident", default="auto",
                    help="final slices whose forward states stay in HBM (no checkpoint recompute): "
                         "'auto' = as many as fit in the free device memory, or a count")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-slices", type=int, default=600, help="slices of the CPU oracle sample")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the secondary lines (exact gradient, small batches, dense path)")
    ap.add_argument("--profile-every", type=int, default=97)
    ap.add_argument("--fused", type=int, default=1, help="1: fused RK4 steps where the operators allow; 0: stage kernels")
    ap.add_argument("--serve-requests", type=int, default=4096,
                    help="requests of the serving leg's stream at the main offered load (0 = no serving leg)")
    ap.add_argument("--serve-saturation", type=int, default=512,
                    help="requests submitted at once to measure the saturation throughput")
    ap.add_argument("--serve-loads", default="0.5,0.8,0.95", help="offered loads as fractions of saturation")
    ap.add_argument("--serve-main-load", type=float, default=0.8,
                    help="the offered load that gets the full --serve-requests stream")
    ap.add_argument("--serve-side-requests", type=int, default=1024,
                    help="requests at the other offered loads")
    ap.add_argument("--serve-budget-gib", type=float, default=64.0)
    ap.add_argument("--serve-resident", type=int, default=1,
                    help="1: requests keep the packed halves of their forward states (no recompute)")
    ap.add_argument("--serve-slices", type=int, default=32, help="slices per request and server step")
    ap.add_argument("--serve-only", action="store_true")
    ap.add_argument("--workload", default="c3", choices=["c3", "c4"],
                    help="c3: the headline; c4: dense random d=512 precision comparison (own JSON line)")
    return ap.parse_args()


PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3, "bf16x3": 2500.0, "f16x3": 2500.0}
# Vector FMA issue rate of the chip without packed FP32 instructions (the
# library is built without them): 256 CUs x 4 SIMDs x 16 lanes x 2 flop x
# 2.4 GHz = 78.6 TFLOP/s in float32 and in float64 (the published 157.3
# TFLOP/s float32 vector peak counts packed FP32).
VALU_PEAK_TFLOPS = 78.6
# Algorithmic flops of one element of one stage of the banded right-hand
# side of the multi-level x oscillator model: 5 diagonals of A Y and 5 of
# Y A^dag with complex coefficients (8 flop each), 3 dissipator taps with real
# factors (real product 1 flop + real x complex multiply-add 4 flop each),
# and the stage update rho + c L (4 flop).
FLOP_PER_ELEM_STAGE = 10 * 8 + 3 * 5 + 4


def dense_leg(args, n_t=None, batch=None, precs=None):
    """Dense random d = 512 problem (K = 4, J = 4, N_t = 1000, dt = 0.005) on
    the dense matrix-core path in float64, float32 and the two 16-bit split
    precisions; error of problem 0 against the stored float64 oracle values.
    Roofline of the first GEMM of every stage (X = A Y and C_m Y for all m):
    B (1 + J) complex 512^3 products per launch, 8 d^3 real flops each; the
    split precisions execute three 16-bit products per real product."""
    import workloads as wl

    n_t = args.n_t if n_t is None else n_t
    B = args.batch if batch is None else batch
    w = wl.config_c4(n_t=n_t)
    if B > 1:
        w.u = np.stack([wl.controls_uniform(8 + b, n_t, 4) for b in range(B)])
    gpath = os.path.join(ROOT, "tests", "golden", "c4_dense_d512_nt1000.npz")
    golden = dict(np.load(gpath)) if os.path.exists(gpath) else None
    precs = precs or [p for p in args.precisions.split(",") if p]
    out = {"workload": "dense random d=512, K=4, J=4, N_t=%d, dt=0.005" % n_t, "batch": B,
           "path": "dense", "gradient": "grape1", "results": {}}
    flops = B * (1 + w.J) * 8.0 * w.d ** 3
    for prec in precs:
        r = run_gpu(args, prec, w, golden, batch=B, n_t=n_t, path="dense", gmode="grape1",
                    steps=1 if batch else None, warmup=1 if batch else None)
        tf = flops / (r["kern_us"] * 1e-6) / 1e12 if r["kern_us"] > 0 else None
        executed = tf * (3 if "x3" in prec else 1) if tf else None
        b = _brief(r)
        b["roofline"] = {"bound": "mfma", "kernel": "zgemm (first GEMM of each stage)", "achieved_useful": tf,
                         "achieved_executed": executed, "peak": PEAK_TFLOPS[prec], "unit": "TFLOP/s",
                         "frac": executed / PEAK_TFLOPS[prec] if executed else None}
        out["results"][prec] = b
        _log(f"[c4] {prec}: {b}")
    return out


def serving_leg(args):
    """Continuous batching of forward + gradient requests of mixed shape
    (transmon(n_q) x resonator(N), d in {20, 40, 90, 160, 240}) and length
    (N_t in [500, 5000]), float32, under an HBM budget.  The saturation
    throughput is measured with a first sample submitted at once; the next
    requests then arrive as a Poisson stream at each offered load (the main
    load gets the full stream of args.serve_requests, the others a shorter
    one)."""
    import workloads as wl
    from paper_1609_03170_amd.serve import ServingLoop

    n_sat, n_main, n_side = args.serve_saturation, args.serve_requests, args.serve_side_requests
    reqs = wl.serving_requests(n_sat + max(n_main, n_side), seed=10, arrival_seed=9, rate=1.0)
    models = {s: wl.serving_model(s) for s in wl.SERVING_SHAPES}
    loop = ServingLoop(models, prec="f32", budget_bytes=int(args.serve_budget_gib * 2**30),
                       max_slices=args.serve_slices, resident=bool(args.serve_resident))
    _log(f"[serve] saturation run: {n_sat} requests at t=0")
    sat = loop.run([dict(r, arrival=0.0) for r in reqs[:n_sat]], wl.serving_controls, log=_log)
    thr = sat.throughput()
    out = {"saturation_req_per_s": thr, "saturation_requests": n_sat, "budget_gib": args.serve_budget_gib,
           "fused": bool(loop.problems[next(iter(models))].fused), "resident_states": bool(args.serve_resident),
           "workload": "Poisson stream, d in {20,40,90,160,240}, N_t ~ U[500,5000], dt=0.002, float32, "
                       "first-order gradient", "loads": []}
    tail = reqs[n_sat:]
    t_first = tail[0]["arrival"]
    for load in [float(x) for x in args.serve_loads.split(",") if x]:
        n = n_main if abs(load - args.serve_main_load) < 1e-9 else n_side
        rate = load * thr
        _log(f"[serve] offered load {load:.2f} x saturation = {rate:.2f} req/s, {n} requests")
        stream = [dict(r, arrival=r["arrival"] - t_first) for r in tail[:n]]
        res = loop.run(stream, wl.serving_controls, time_scale=1.0 / rate, log=_log)
        # algorithmic HBM bytes of the banded stage model (18 d^2 float32
        # complex elements per slice) over the wall time of the run
        work = sum(18.0 * (r["shape"][0] * r["shape"][1]) ** 2 * 8 * r["n_t"] for r in stream)
        out["loads"].append({"offered_load": load, "offered_req_per_s": rate, "requests": n,
                             "throughput_req_per_s": res.throughput(), "p50_ms": 1000 * res.percentile(50),
                             "p99_ms": 1000 * res.percentile(99), "peak_hbm_gib": res.peak_bytes / 2**30,
                             "hbm_frac": work / res.wall / (HBM_PEAK_GBS * 1e9)})
    loop.close()
    return out


def _brief(r, golden_err=True):
    keys = ("prec", "batch", "path", "gradient", "fused", "steps", "value", "ms_per_step", "kern_us",
            "resident_slices", "workspace_gib")
    out = {k: r[k] for k in keys if k in r}
    out["ms_per_grad_eval"] = r["ms_per_step"] / r["batch"]
    if golden_err and "err_phi" in r:
        out["err_vs_oracle"] = {"phi": r["err_phi"], "grad": r["err_grad"], "problem": 0}
    return out


def fused_roofline(r, d):
    """Roofline of the fused RK4 step kernel from a run's event-sampled mean
    launch time: ALU (its binding resource) against the FMA issue rate, and
    its HBM bytes (the state read once with its halo, written once, the
    float32 compensation term read on one triangle and written on both)."""
    B, us = r["batch"], r["kern_us"]
    if not us or us <= 0:
        return None
    herm = d * (d + 1) // 2
    flops = B * 4.0 * herm * FLOP_PER_ELEM_STAGE
    s = 8 if r["prec"] == "f32" else 16
    hbm_bytes = B * d * d * (2 * s + ((2 + 4) if r["prec"] == "f32" else 0))
    # the forward steps of the resident slices also write the packed
    # Hermitian half of their state (first-order gradient): averaged over the
    # evaluation's launches (forward N_t, recompute N_t - resident, adjoint N_t)
    n_t, res = r.get("n_t"), r.get("resident_slices", 0)
    if n_t and res and r.get("gradient") == "grape1":
        hbm_bytes += B * herm * s * res / (3.0 * n_t - res)
    stage_model = B * 4 * 2.0 * d * d * s  # four stage kernels, each reading and writing the state once
    t = us * 1e-6
    return {"bound": "alu", "kernel": "rk4_fused_kernel", "achieved": flops / t / 1e12, "peak": VALU_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": flops / t / 1e12 / VALU_PEAK_TFLOPS,
            "algorithmic_flops_per_launch": flops, "kernel_avg_us": us, "kernel_samples": r["kern_n"],
            "hbm": {"algorithmic_bytes_per_launch": hbm_bytes, "achieved": hbm_bytes / t / 1e9,
                    "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": hbm_bytes / t / 1e9 / HBM_PEAK_GBS},
            "four_stage_model": {"bytes_per_launch": stage_model, "equivalent_GBs": stage_model / t / 1e9,
                                 "frac_of_hbm_peak": stage_model / t / 1e9 / HBM_PEAK_GBS}}


def extras_leg(args, w, golden):
    """Secondary lines, one timed evaluation each (after one untimed):
    the batch beyond the Infinity Cache (B = 256) and the pure checkpointed
    memory mode (no resident states) with the fused kernel's roofline; the
    four stage kernels instead of the fused step; the exact gradient through
    the autograd Function (OpenGrapeCost, its backward being the adjoint
    sweep); single-problem latency and the batch sweep; adaptive
    Dormand-Prince 5(4) steps; the dense matrix-core path at B = 16 in both
    precisions; the dense d = 512 precision comparison."""
    import workloads as wl

    out = {}
    w256 = wl.config_c3(batch=256, n_t=args.n_t)
    r = run_gpu(args, "f32", w256, golden, batch=256, steps=1, warmup=1)
    b = _brief(r)
    b["roofline"] = fused_roofline(r, w.d)
    out["b256_f32"] = b
    r = run_gpu(args, "f32", w, golden, steps=1, warmup=1, resident=0)
    b = _brief(r)
    b["roofline"] = fused_roofline(r, w.d)
    b["memory"] = "sqrt(N_t) checkpoints only: O(sqrt(N_t) d^2) per problem"
    out["checkpoints_only_f32"] = b
    r = run_gpu(args, "f32", w, golden, steps=1, warmup=1, fused=0)
    out["stage_kernels_f32"] = _brief(r)
    r = run_gpu(args, "f32", w, golden, steps=1, warmup=1, gmode="exact", autograd=True)
    out["exact_autograd_f32"] = _brief(r)
    for prec, B in (("f32", 1), ("f64", 1), ("f32", 16), ("f32", 64)):
        r = run_gpu(args, prec, w, golden, batch=B, steps=1, warmup=1)
        out[f"b{B}_{prec}"] = _brief(r)
    r = run_gpu(args, "f32", w, golden, batch=32, steps=1, warmup=0, adaptive=(1e-5, 1e-8))
    b = _brief(r)
    b["steps_per_slice"], b["tolerances"] = r["steps_per_slice"], r["tolerances"]
    out["adaptive_f32"] = b
    for prec in ("f32", "f64"):
        B = 16
        r = run_gpu(args, prec, w, golden, batch=B, steps=1, warmup=1, path="dense")
        b = _brief(r)
        flops = B * (1 + w.J) * 8.0 * w.d ** 3
        tf = flops / (r["kern_us"] * 1e-6) / 1e12 if r["kern_us"] > 0 else None
        b["roofline"] = {"bound": "mfma", "kernel": "zgemm_kernel (first GEMM of each stage)", "achieved": tf,
                         "peak": PEAK_TFLOPS[prec], "unit": "TFLOP/s",
                         "frac": tf / PEAK_TFLOPS[prec] if tf else None}
        out[f"dense_{prec}"] = b
    out["dense_d512"] = dense_leg(args, n_t=1000, batch=1, precs=["f64", "f32", "bf16x3", "f16x3"])
    return out


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


def run_gpu(args, prec, w, golden, batch=None, steps=None, warmup=None, path=None, gmode=None, adaptive=None,
            n_t=None, resident=None, fused=None, autograd=False):
    """Time `steps` gradient evaluations of the first `batch` problems of w
    (after `warmup` untimed ones); defaults from the command line.  With
    autograd, every evaluation is phi = OpenGrapeCost(u); phi.sum().backward()."""
    import torch

    from paper_1609_03170_amd import Problem, open_grape_cost

    dev = torch.device("cuda", 0)
    B = args.batch if batch is None else batch
    n_t = args.n_t if n_t is None else n_t
    steps = args.steps if steps is None else steps
    warmup = args.warmup if warmup is None else warmup
    path = args.path if path is None else path
    gmode = args.gmode if gmode is None else gmode
    fused = args.fused if fused is None else fused
    p = Problem.from_workload(w, prec=prec, path=path, gmode=gmode)
    p.set_fused(bool(fused))
    if adaptive:
        p.set_adaptive(*adaptive)
    u_all = w.u.reshape(-1, w.u.shape[-2], w.K)[:, :n_t]
    u = torch.tensor(np.ascontiguousarray(u_all[:B]), device=dev)
    rho0 = torch.tensor(np.broadcast_to(w.rho0, (B, w.d, w.d)).copy(), device=dev)
    sigma = torch.tensor(w.sigma, device=dev)
    res = 0
    if not adaptive:
        res_arg = args.resident if resident is None else resident
        if res_arg == "auto":
            torch.cuda.empty_cache()
            free, total = torch.cuda.mem_get_info(dev)
            budget = free - max(4 << 30, int(0.03 * total))  # headroom for the rest of the process
            res = p.resident_for_budget(B, n_t, budget)
        else:
            res = min(int(res_arg), n_t)
        p.set_resident(res)
    ws_gib = p.workspace_bytes(B, n_t) / 2**30
    ws = None if autograd else torch.empty(p.workspace_bytes(B, n_t), dtype=torch.uint8, device=dev)
    _log(f"[bench] {prec} B={B} N_t={n_t} path={p.path} fused={p.fused} gmode={gmode} autograd={autograd} "
         f"resident={res} workspace={ws_gib:.2f} GiB")

    def step():
        if autograd:
            uu = u.clone().requires_grad_(True)
            phi = open_grape_cost(uu, p, rho0, sigma, w.dt)
            phi.sum().backward()
            return phi.detach(), uu.grad
        return p.cost_and_grad(u, rho0, sigma, w.dt, workspace=ws)

    for i in range(warmup):
        step()
        torch.cuda.synchronize()
        _log(f"[bench] {prec} warmup {i + 1}/{warmup} done")
    torch.cuda.synchronize()
    p.profile(args.profile_every)
    t0 = time.perf_counter()
    for i in range(steps):
        phi, g = step()
        torch.cuda.synchronize()
        _log(f"[bench] {prec} B={B} {path} {gmode} step {i + 1}/{steps} done ({time.perf_counter() - t0:.2f} s)")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    kern_us, kern_n = p.profile_read()
    p.profile(0)
    stats = p.adaptive_stats(B) if adaptive else None
    phi = phi.cpu().numpy()
    g = g.cpu().numpy()
    out = dict(prec=prec, batch=B, steps=steps, elapsed=elapsed, ms_per_step=1000 * elapsed / steps,
               value=B * steps / elapsed, kern_us=kern_us, kern_n=kern_n, path=p.path, gradient=gmode,
               fused=p.fused, resident_slices=res, workspace_gib=ws_gib, n_t=n_t)
    if autograd:
        out["interface"] = "OpenGrapeCost (torch.autograd.Function)"
    if stats is not None:
        out["steps_per_slice"] = {"forward_accepted": float(stats[:, 0].mean()) / n_t,
                                  "forward_rejected": float(stats[:, 1].mean()) / n_t,
                                  "adjoint_accepted": float(stats[:, 2].mean()) / n_t,
                                  "adjoint_rejected": float(stats[:, 3].mean()) / n_t}
        out["tolerances"] = {"rtol": adaptive[0], "atol": adaptive[1]}
        golden = None  # the stored values are those of fixed RK4 steps
    gkey = "g_grape1" if gmode == "grape1" else "g_exact"
    if golden is not None and golden[gkey].shape[0] == n_t and golden[gkey].shape[1] == w.K:
        out["err_phi"] = float(abs(phi[0] - golden["phi"]) / abs(golden["phi"]))
        out["err_grad"] = float(np.linalg.norm(g[0] - golden[gkey]) / np.linalg.norm(golden[gkey]))
    p.close()
    del ws
    torch.cuda.empty_cache()
    return out


PROFILE = os.path.join("profiles", "rk4_fused_kernel_transmon240_b128_f32.md")
LIB = os.path.join("paper_1609_03170_amd", "libopengrape.so")


def lib_hash(root=None):
    """First 16 hex digits of the SHA-256 of the built library (the code
    object the counters were taken on)."""
    import hashlib

    path = os.path.join(root or ROOT, LIB)
    if not os.path.exists(path):
        return None
    return hashlib.sha256(open(path, "rb").read()).hexdigest()[:16]


def measured_traffic(prec, batch, path, fused=True):
    """HBM bytes per launch of the fused step kernel from the committed
    rocprofv3 counter summary (L2 misses x 128 B + WRITE_SIZE), or None when
    there is none for this configuration or the library was rebuilt since the
    counters were taken (its hash differs)."""
    if prec != "f32" or batch != 128 or path != "banded" or not fused:
        return None
    summary = os.path.join(ROOT, PROFILE)
    if not os.path.exists(summary):
        return None
    fields = {}
    for line in open(summary):
        if ":" in line and not line.startswith((" ", "|", "#")):
            k, v = line.split(":", 1)
            fields[k.strip()] = v.strip()
    if fields.get("lib-sha256-16") is None or fields.get("lib-sha256-16") != lib_hash():
        return None
    try:
        return float(fields["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def _oracle_sample(w, u, n_t):
    import resource

    from oracle import rk

    m = rk.Model.from_workload(w, sparse=True)
    r0 = resource.getrusage(resource.RUSAGE_SELF)
    t0 = time.perf_counter()
    rhos = rk.forward(m, u, w.rho0, w.dt)
    lams = rk.backward(m, u, w.sigma, w.dt)
    rk.gradient_grape1(m, u, rhos, lams, w.dt)
    wall = time.perf_counter() - t0
    r1 = resource.getrusage(resource.RUSAGE_SELF)
    cpu = (r1.ru_utime - r0.ru_utime) + (r1.ru_stime - r0.ru_stime)
    return wall, cpu


def _host():
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "cpu_model": model, "numpy": np.__version__}


def cpu_baseline(args, w):
    """The float64 oracle on the host cores, on a bounded sample: the first
    args.cpu_slices slices of problem 0 (forward + backward + first-order
    gradient), scaled to one full gradient evaluation; then a shorter sample
    with every thread pool limited to one thread."""
    n = args.cpu_slices
    u = w.u.reshape(-1, args.n_t, w.K)[0]
    wall, cpu = _oracle_sample(w, u[:n], args.n_t)
    per_eval = wall * args.n_t / n
    out = {"value": 1.0 / per_eval, "unit": "grad-evals/s", "cores": max(1, int(round(cpu / wall))),
           "kind": "oracle",
           "sample": f"float64 NumPy/SciPy-sparse oracle, problem 0, first {n} of {args.n_t} slices "
                     f"(forward + backward + Eq. (13) gradient) in {wall:.1f} s, scaled x{args.n_t / n:.0f}",
           "host": _host()}
    try:
        from threadpoolctl import threadpool_limits

        n1 = max(1, n // 3)
        with threadpool_limits(limits=1):
            wall1, _ = _oracle_sample(w, u[:n1], args.n_t)
        out["one_thread_value"] = n1 / (wall1 * args.n_t)
        out["one_thread_sample"] = f"first {n1} slices in {wall1:.1f} s"
    except ImportError:
        pass
    out["other_configs"] = cpu_other_configs()
    return out


def cpu_other_configs():
    """The oracle's time per gradient evaluation at the other configurations
    (dense operators): C1 in full, C2 and the dense d = 512 case on their
    first slices, scaled to the full N_t."""
    import workloads as wl

    res = {}
    for name, w, n in (("C1 d=10 N_t=200", wl.config_c1(), 200), ("C2 d=90 N_t=2000", wl.config_c2(), 100),
                       ("C4 d=512 N_t=1000", wl.config_c4(), 3)):
        from oracle import rk

        u = w.u.reshape(-1, w.u.shape[-2], w.K)[0]
        n_t = u.shape[0]
        m = rk.Model.from_workload(w, sparse=False)
        t0 = time.perf_counter()
        rhos = rk.forward(m, u[:n], w.rho0, w.dt)
        lams = rk.backward(m, u[:n], w.sigma, w.dt)
        rk.gradient_grape1(m, u[:n], rhos, lams, w.dt)
        wall = time.perf_counter() - t0
        res[name] = {"s_per_grad_eval": wall * n_t / n, "sample_slices": n}
    return res


def main():
    args = _parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (the path has no multi-GPU component here); got --gpus {args.gpus}",
              file=sys.stderr)
        sys.exit(2)
    if args.serve_only:
        print(json.dumps({"serving": serving_leg(args)}), flush=True)
        return
    if args.workload == "c4":
        print(json.dumps(dense_leg(args)), flush=True)
        return
    import workloads as wl

    _log(f"[bench] generating inputs B={args.batch} N_t={args.n_t}")
    w = wl.config_c3(batch=args.batch, n_t=args.n_t)
    gpath = os.path.join(ROOT, "tests", "golden", "c3_cqed_d240.npz")
    golden = dict(np.load(gpath)) if os.path.exists(gpath) else None
    results = {}
    for prec in [p for p in args.precisions.split(",") if p]:
        results[prec] = run_gpu(args, prec, w, golden)
        _log(f"[bench] {prec}: {results[prec]}")
    head = results.get("f32") or next(iter(results.values()))
    d = w.d
    elem = 8 if head["prec"] == "f32" else 16
    line = {
        "metric": METRIC,
        "value": head["value"],
        "unit": "grad-evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": head["prec"],
        "data": "synthetic",
        "config": {
            "workload": "transmon(3)xresonator(80) d=240, K=4, J=3, N_t=10000, dt=0.002/kappa, smooth-noise controls",
            "batch": args.batch, "n_t": args.n_t, "path": head["path"], "gradient": args.gmode,
            "fused_rk4_step": head["fused"], "resident_slices": head["resident_slices"],
            "ckpt_stride": int(math.ceil(math.sqrt(max(args.n_t - head["resident_slices"], 1)))),
            "workspace_gib": round(head["workspace_gib"], 2), "parallelism": "none (1 GPU)",
        },
        "rk_steps_per_s": head["value"] * args.n_t * 2,
    }
    if head["fused"]:
        roof = fused_roofline(head, d)
        roof["traffic"] = measured_traffic(head["prec"], args.batch, head["path"], head["fused"])
        roof["traffic_unit"] = "HBM bytes per launch (rocprofv3: TCC_MISS_sum x 128 B + WRITE_SIZE)"
    else:
        per_launch = args.batch * 2 * d * d * elem
        ach = per_launch / (head["kern_us"] * 1e-6) / 1e9 if head["kern_us"] > 0 else None
        roof = {"bound": "hbm", "kernel": "band_stage_kernel", "achieved": ach, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": ach / HBM_PEAK_GBS if ach else None, "traffic": None,
                "kernel_avg_us": head["kern_us"], "kernel_samples": head["kern_n"],
                "algorithmic_bytes_per_launch": per_launch}
    line["roofline"] = roof
    # whole path against the HBM model of the stage kernels: per slice the
    # forward and adjoint sweeps run 4 stages that read and write one state,
    # and the gradient reads rho and lambda (18 d^2 elements per slice; the
    # checkpoint recompute is not counted)
    path_bytes = 18.0 * d * d * elem * args.n_t
    line["path_roofline"] = {"algorithmic_bytes_per_grad_eval": path_bytes,
                             "achieved": head["value"] * path_bytes / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                             "frac": head["value"] * path_bytes / 1e9 / HBM_PEAK_GBS}
    if "err_phi" in head:
        line["err_vs_oracle"] = {"phi": head["err_phi"], "grad": head["err_grad"], "problem": 0}
    if "f64" in results and "f32" in results:
        f64 = results["f64"]
        line["fp64"] = {"value": f64["value"], "ms_per_step": f64["ms_per_step"],
                        "resident_slices": f64["resident_slices"], "kernel_avg_us": f64["kern_us"],
                        "roofline": fused_roofline(f64, d) if f64["fused"] else None,
                        "err_vs_oracle": {"phi": f64.get("err_phi"), "grad": f64.get("err_grad")}}
        line["speedup_fp32_over_fp64"] = head["value"] / f64["value"]
    if not args.no_extras:
        line["extras"] = extras_leg(args, w, golden)
    if args.serve_requests > 0:
        line["serving"] = serving_leg(args)
    if not args.no_cpu_baseline:
        _log("[bench] cpu baseline (oracle sample)")
        line["cpu_baseline"] = cpu_baseline(args, w)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
