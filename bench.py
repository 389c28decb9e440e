#!/usr/bin/env python
"""Benchmark of the fermion-determinant-ratio path on one MI355X.

Workload (one "step" = one complete estimate of log det(D'^+D')/det(D^+D)
for one proposal U -> U', through the domain-decomposition factorisation
det D = prod_b det D_b * det Dhat of the paper's Sec. 3):
  8^4 lattice, kappa = 0.135, links exp(i 0.5 H), 16 blocks of 4^4, U'
  redraws the active links of every block; the 16 block ratios (BLOCKS) and
  the Schur-complement ratio (SCHUR), each over a path of N = 8 factors with
  one complex Gaussian noise vector per factor; FGCR(16)+SAP(4 cycles, 5 MR)
  to 1e-10 with FP32 preconditioner and block solves refined in FP64.

Prints one JSON line: estimates/s of the mixed-precision form, the plain
FP64 form on the same GPU, the stencil's HBM roofline fraction at 32^4, and
the FP64 CPU oracle on a bounded sample.
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
# compulsory bytes per site of one stencil application: 24 reals in, 24 out,
# four 18-real links (each neighbour spinor and link counted once)
BYTES_PER_SITE = {"f64": 120 * 8, "f32": 120 * 4}

WORKLOAD = dict(name="wilson8_dd16", L=(8, 8, 8, 8), B=(4, 4, 4, 4), kappa=0.135, scale=0.5, n_steps=8,
                n_noise=1, seed=1112124301)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_inputs(wl):
    from paper_1112_1243_amd import synth
    U = synth.gauge_field(wl["L"], wl["scale"], wl["seed"])
    return U


def estimate(ctx, wdr, gU, gUp, wl, params, seed):
    """One complete estimate: block ratios + Schur ratio."""
    sb, lb, ib = ctx.logdet_ratio(gU, gUp, wl["kappa"], wdr.OP_BLOCKS, wl["n_steps"], wl["n_noise"],
                                  wdr.NOISE_GAUSS, seed, params)
    ss, ls, is_ = ctx.logdet_ratio(gU, gUp, wl["kappa"], wdr.OP_SCHUR, wl["n_steps"], wl["n_noise"],
                                   wdr.NOISE_GAUSS, seed, params)
    ok = bool(ib.converged and is_.converged)
    return lb + ls, ok, ib.total_iters + is_.total_iters


def dslash_roofline(wdr, torch, L=(32, 32, 32, 32), prec_name="f32", reps=30):
    """Average duration of one stencil launch on internal fields, by HIP
    events on the stream the kernel is launched on."""
    from paper_1112_1243_amd import synth
    prec = wdr.F32 if prec_name == "f32" else wdr.F64
    ctx = wdr.Context(L, (4, 4, 4, 4))
    V = ctx.V
    U = synth.gauge_field(L, 0.2, 1112124303)
    gU = ctx.gauge(torch.from_numpy(U).cuda())
    del U
    psi = torch.from_numpy(synth.spinor(L, 5)).cuda()
    a = ctx.pack(psi, prec)
    b = ctx.internal_field(prec)
    for _ in range(3):
        ctx.apply_D_internal(gU, 0.155, a, b, prec)
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for i in range(reps):
        if i % 2 == 0:
            ctx.apply_D_internal(gU, 0.155, a, b, prec)
        else:
            ctx.apply_D_internal(gU, 0.155, b, a, prec)
    e1.record(st)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    alg = BYTES_PER_SITE[prec_name] * V
    gbs = alg / (ms * 1e-3) / 1e9
    del gU, a, b, psi
    ctx.close()
    return {"kernel": "k_dslash<%s, all hops>" % ("float" if prec_name == "f32" else "double"),
            "lattice": "x".join(map(str, L)), "bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": None,
            "avg_launch_us": round(ms * 1e3, 2), "bytes_per_launch": alg}


def cpu_baseline(wl, U, Up, budget_s=20.0):
    """FP64 CPU oracle on a bounded sample: one BLOCKS and one SCHUR sample
    (one factor, one noise vector) of the same workload, scaled to a full
    estimate (2 ops x n_steps x n_noise samples)."""
    import oracle
    lat = oracle.Lattice(wl["L"], wl["B"])
    Ui1 = oracle.interpolate(U, Up, 1, wl["n_steps"])
    t0 = time.perf_counter()
    for op in (oracle.OP_BLOCKS, oracle.OP_SCHUR):
        eta = oracle.noise(lat, oracle.NOISE_GAUSS, 7, 0, 0, support=oracle.noise_support(lat, op))
        oracle.sample(lat, U, Ui1, wl["kappa"], op, eta, tol=1e-10, block_tol=1e-13)
    dt = time.perf_counter() - t0
    per_estimate = dt / 2 * 2 * wl["n_steps"] * wl["n_noise"]
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": round(1.0 / per_estimate, 6), "unit": "estimates/s", "cores": threads, "kind": "oracle",
            "sample": "1 BLOCKS + 1 SCHUR sample (one path factor, one noise vector) at 8^4, FP64 CGNE to 1e-10, "
                      "%.1f s, scaled x%d to one estimate" % (dt, wl["n_steps"] * wl["n_noise"])}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-dslash", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU: this build has no multi-GPU path (every proposal, path factor and "
              "noise vector is independent; see the sharding notes in the design document)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1112_1243_amd import synth, wdr
    import oracle  # noqa: F401  (CPU baseline only)

    wl = WORKLOAD
    from oracle import Lattice, active_links
    lat = Lattice(wl["L"], wl["B"])
    U = make_inputs(wl)
    Up = synth.redraw(U, active_links(lat), wl["scale"], wl["seed"])

    ctx = wdr.Context(wl["L"], wl["B"])
    gU = ctx.gauge(torch.from_numpy(U).cuda())
    gUp = ctx.gauge(torch.from_numpy(Up).cuda())
    mixed = wdr.default_params(inner=wdr.F32)
    fp64 = wdr.default_params(inner=wdr.F64)

    for w in range(args.warmup):
        estimate(ctx, wdr, gU, gUp, wl, mixed, 1000 + w)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    all_ok = True
    iters = 0
    lrs = []
    for k in range(args.steps):
        lr, ok, it = estimate(ctx, wdr, gU, gUp, wl, mixed, 2000 + k)
        all_ok &= ok
        iters += it
        lrs.append(lr)
        log("step %d: log R = %.10f converged=%s iters=%d" % (k, lr, ok, it))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    value = args.steps / dt

    fp64_rate = None
    if not args.no_fp64:
        t1 = time.perf_counter()
        n64 = max(1, min(2, args.steps))
        for k in range(n64):
            estimate(ctx, wdr, gU, gUp, wl, fp64, 2000 + k)
        torch.cuda.synchronize()
        fp64_rate = n64 / (time.perf_counter() - t1)
        log("plain fp64 form: %.3f estimates/s" % fp64_rate)
    del gU, gUp
    ctx.close()

    roof = None
    if not args.no_dslash:
        roof = dslash_roofline(wdr, torch, prec_name="f32")
        r64 = dslash_roofline(wdr, torch, prec_name="f64")
        log("dslash f32:", roof)
        log("dslash f64:", r64)
        roof["f64"] = {k: r64[k] for k in ("achieved", "frac", "avg_launch_us", "bytes_per_launch")}

    cpu = None if args.no_cpu else cpu_baseline(wl, U, Up)
    if cpu:
        log("cpu baseline:", cpu)

    out = {
        "metric": "det-ratio estimates/sec at 1e-10 residual (+ Dslash HBM GB/s, % peak)",
        "value": round(value, 4),
        "unit": "estimates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": "%s: 8^4 lattice, 16 blocks of 4^4, kappa 0.135, links exp(i 0.5 H), active links "
                               "redrawn, BLOCKS + SCHUR ratios, N=8 factors x 1 Gaussian noise, FGCR(16)+SAP(4,5) "
                               "to 1e-10" % wl["name"],
                   "converged": all_ok, "total_outer_iters": iters, "mean_log_ratio": float(np.mean(lrs))},
        "fp64_estimates_per_s": None if fp64_rate is None else round(fp64_rate, 4),
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
