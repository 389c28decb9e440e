#!/usr/bin/env python
"""Benchmark of the fermion-determinant-ratio path on one MI355X.

Headline workload (one "step" = one complete estimate of the Schur-complement
ratio log det(Dhat'^+ Dhat') / det(Dhat^+ Dhat) of the paper's Sec. 3 eq.
ddfactor for one proposal U -> U', Sec. 4):
  32^4 lattice, 4096 blocks of 4^4, kappa = 0.155, links exp(i 0.2 H), U'
  redraws the active links of every block; N = 32 factors of eq. param with
  one complex Gaussian noise vector each, all 32 samples solved as one batch;
  CG on the normal equations with FP16 inner iterations, an FP32 middle level
  and FP64 outer reliable updates (true residual 1e-10), FP16 block solves
  with FP64 defect correction to 1e-13; block-solve depth and launch forms
  chosen by wdr_autotune beforehand.

Prints one JSON line: estimates/s of that form, the plain FP64
single-proposal form on the same GPU, the dominant kernel's HBM roofline
fraction, the whole estimate's compulsory bytes against its time, and the
FP64 CPU oracle on a bounded sample.  Other workloads follow as extra keys.
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
# four links (each neighbour spinor and link counted once).  SU(3) fields are
# read as two rows per link (12 reals), other fields as 18 reals.
BYTES_PER_SITE = {("f64", True): 96 * 8, ("f32", True): 96 * 4, ("f64", False): 120 * 8, ("f32", False): 120 * 4}
KERNEL = {"f64": "k_dslash_blk<double, B=4, all hops> (SU(3) links, two rows)",
          "f32": "k_dslash_blk<float, B=4, all hops> (SU(3) links, two rows)"}
# the clover term adds its two hermitian 6 x 6 blocks per site (72 reals)
CLOVER_BYTES_PER_SITE = {"f64": 72 * 8, "f32": 72 * 4}
CSW = 1.7
# HBM traffic per launch from rocprofv3 counter runs on the committed kernel
# sources (FETCH_SIZE x 2.0, WRITE_SIZE x 1.0: a plain 1 GiB elementwise copy
# reads 1 GiB as FETCH_SIZE 0.5 GiB because every read request on gfx950 is
# 128 B while FETCH_SIZE counts 64 B per request; WRITE_SIZE reads exactly).
# Reported only while the stencil sources hash to the value recorded there.
COUNTERS = os.path.join(ROOT, "profiles", "dslash_blk_32x32x32x32_counters.md")
STENCIL_SOURCES = ["paper_1112_1243_amd/csrc/dslash.hip", "paper_1112_1243_amd/csrc/half.hip",
                   "paper_1112_1243_amd/csrc/stencil.h", "paper_1112_1243_amd/csrc/blk_stencil.h",
                   "paper_1112_1243_amd/csrc/wdr_internal.h"]

WORKLOAD = dict(name="wilson8_dd16", L=(8, 8, 8, 8), B=(4, 4, 4, 4), kappa=0.135, scale=0.5, n_steps=8,
                n_noise=1, seed=1112124301)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_inputs(wl):
    from paper_1112_1243_amd import synth
    U = synth.gauge_field(wl["L"], wl["scale"], wl["seed"])
    return U


def proposal_mask(ctx, rule):
    """[site, mu] mask of the links a proposal redraws, from the library's
    geometry maps: 'active' = the active links of every block (both ends in
    the block, at most one on its boundary); 'core6' = the same for the core
    of every block without its outer layer (6^4 in 8^4 blocks); 'black_blocks'
    = every link with both ends in the same black block."""
    if rule == "active":
        return ctx.active_links(0, ctx.B[0] - 1).cpu().numpy().astype(bool)
    if rule == "core6":
        return ctx.active_links(1, ctx.B[0] - 2).cpu().numpy().astype(bool)
    assert rule == "black_blocks"
    bid, col, _, _ = [t.cpu().numpy() for t in ctx.site_maps()]
    L = ctx.L
    site = np.arange(ctx.V)
    x = [site % L[0], (site // L[0]) % L[1], (site // (L[0] * L[1])) % L[2], site // (L[0] * L[1] * L[2])]
    mask = np.zeros((ctx.V, 4), bool)
    for mu in range(4):
        y = [c.copy() for c in x]
        y[mu] = (y[mu] + 1) % L[mu]
        nb = y[0] + L[0] * (y[1] + L[1] * (y[2] + L[2] * y[3]))
        mask[:, mu] = (bid == bid[nb]) & (col == 0)
    return mask


def clover_workload(wdr, torch, L=(16, 16, 16, 16), N=8, kappa=0.135, scale=0.5, seed=1112124310):
    """FULL and SCHUR estimates with and without the clover term (c_sw 1.7)
    on the same 16^4 proposal: N factors x 1 Gaussian noise, all batched,
    CGNE with FP32 iterations and FP64 reliable updates to 1e-10; block
    solves to 1e-13 (FP32 block MR rounds without the term, FP32 even-odd
    CGNE rounds on the blocks with it).  The *_f16 entries: the clover
    estimates with FP16 CG steps and an FP32 middle level."""
    from paper_1112_1243_amd import synth
    ctx = wdr.Context(L, (4, 4, 4, 4))
    U = synth.gauge_field(L, scale, seed)
    Up = synth.redraw(U, proposal_mask(ctx, "active"), scale, seed)
    p = wdr.default_params(solver=wdr.SOLVER_CGNE, inner=wdr.F32, max_iter=20000)
    out = {"workload": "%s lattice, 4^4 blocks, kappa %.3f, links exp(i %.1f H), active links redrawn, FULL and "
                       "SCHUR ratios, N=%d factors x 1 Gaussian noise (batched), CGNE FP32 iterations + FP64 reliable "
                       "updates to 1e-10, block solves to 1e-13" % ("x".join(map(str, L)), kappa, scale, N),
           "unit": "estimates/s"}
    p16 = wdr.default_params(solver=wdr.SOLVER_CGNE, inner=wdr.F16, middle=wdr.F32, max_iter=20000)
    for op, suffix, csws, prm in ((wdr.OP_FULL, "", (CSW, 0.0), p), (wdr.OP_SCHUR, "_schur", (CSW, 0.0), p),
                                  (wdr.OP_FULL, "_f16", (CSW,), p16), (wdr.OP_SCHUR, "_schur_f16", (CSW,), p16)):
        for csw in csws:
            gU = ctx.gauge(torch.from_numpy(U).cuda(), csw, kappa)
            gUp = ctx.gauge(torch.from_numpy(Up).cuda(), csw, kappa)
            ctx.logdet_ratio(gU, gUp, kappa, op, 1, 1, wdr.NOISE_GAUSS, 1, prm)  # warm-up
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s, lr, info = ctx.logdet_ratio(gU, gUp, kappa, op, N, 1, wdr.NOISE_GAUSS, seed, prm)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            key = ("clover" if csw else "wilson") + suffix
            out[key] = {"value": round(1.0 / dt, 3), "iterations_total": int(info.total_iters),
                        "converged": bool(info.converged), "log_ratio": round(float(lr), 4)}
            if csw:
                out[key]["csw"] = csw
            log("%s 16^4: %.3f s, iterations %d, log R %.4f" % (key, dt, info.total_iters, lr))
            del gU, gUp
    ctx.close()
    return out


def slab_halo(wdr, torch, kappa=0.155, scale=0.2, seed=1112124330, reps=50):
    """One GPU's share of a 32^4 lattice cut along t over 8 GPUs: the slab
    32^3 x 4 (one block in t) with an open t boundary.  Times (HIP events,
    FP32 internal fields) the slab's own D, the face pack and the unpack of
    the hops across both faces, next to the plain D of the same slab with a
    periodic t boundary (the one-GPU stand-in for the exchange); the faces
    are what one peer copy per direction would move over xGMI."""
    from paper_1112_1243_amd import synth
    L, B = (32, 32, 32, 4), (4, 4, 4, 4)
    U = synth.gauge_field(L, scale, seed)
    psi = synth.spinor(L, seed + 1)
    Ud, pd = torch.from_numpy(U).cuda(), torch.from_numpy(psi).cuda()
    ctx, per = wdr.Context(L, B, (1, 1, 1, 0)), wdr.Context(L, B, (1, 1, 1, 1))
    gU, gP = ctx.gauge(Ud), per.gauge(Ud)
    prec = wdr.F32
    fin, fout, fref = ctx.pack(pd, prec), ctx.internal_field(prec), per.internal_field(prec)
    lo, hi = ctx.halo_field(prec), ctx.halo_field(prec)

    def timed(fn):
        for _ in range(3):
            fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps * 1e3

    t_int = timed(lambda: ctx.apply_D_internal(gU, kappa, fin, fout, prec))
    t_pack = timed(lambda: ctx.halo_pack(Ud, fin, lo, hi, prec))
    t_unp = timed(lambda: ctx.halo_unpack(Ud, kappa, hi, lo, 1, 1, fout, prec))
    t_per = timed(lambda: per.apply_D_internal(gP, kappa, fin, fref, prec))
    # the sharded pieces give the periodic D (ring of one slab)
    ctx.apply_D_internal(gU, kappa, fin, fout, prec)
    ctx.halo_pack(Ud, fin, lo, hi, prec)
    ctx.halo_unpack(Ud, kappa, hi, lo, 1, 1, fout, prec)
    a, b = ctx.unpack(fout, prec), per.unpack(fref, prec)
    diff = float((a - b).abs().max() / b.abs().max())
    face = int(lo.numel())
    out = {"workload": "32x32x32x4 slab of a 32^4 lattice cut along t over 8 GPUs, 4^4 blocks, kappa %.3f, links "
                       "exp(i %.1f H), FP32 fields" % (kappa, scale),
           "unit": "us", "slab_D_open_t_us": round(t_int, 2), "halo_pack_us": round(t_pack, 2),
           "halo_unpack_us": round(t_unp, 2), "periodic_D_us": round(t_per, 2),
           "face_bytes_per_direction": face,
           "xgmi_us_per_direction_at_153GBs": round(face / 153e9 * 1e6, 2),
           "sharded_vs_periodic_max_rel_diff": diff}
    log("slab halo:", out)
    del gU, gP
    ctx.close()
    per.close()
    return out


def cg_forms(wdr, torch, N=16, kappa=0.135, scale=0.5, seed=1112124320):
    """FULL estimates (N factors x 1 Gaussian noise, all batched; CGNE with
    FP32 steps and FP64 reliable updates to 1e-10) at 8^4, 16^4 and 32^4 with
    the CG steps as separate launches (the default form) and as one
    cooperative launch per period of update_every steps (grid-wide barriers
    between the phases); the faster of three timed runs of each."""
    from paper_1112_1243_amd import synth
    out = {"workload": "FULL ratio, 4^4 blocks, kappa %.3f, links exp(i %.1f H), active links redrawn, N=%d factors "
                       "x 1 Gaussian noise (batched), CGNE FP32 steps + FP64 reliable updates to 1e-10"
                       % (kappa, scale, N), "unit": "ms per estimate"}
    p = wdr.default_params(solver=wdr.SOLVER_CGNE, inner=wdr.F32, max_iter=20000)
    for L in ((8, 8, 8, 8), (16, 16, 16, 16), (32, 32, 32, 32)):
        ctx = wdr.Context(L, (4, 4, 4, 4))
        U = synth.gauge_field(L, scale, seed)
        Up = synth.redraw(U, proposal_mask(ctx, "active"), scale, seed + 1)
        gU, gUp = ctx.gauge(torch.from_numpy(U).cuda()), ctx.gauge(torch.from_numpy(Up).cuda())
        del U, Up
        row = {}
        for name, form in (("launches", wdr.CG_LAUNCHES), ("persistent", wdr.CG_PERSISTENT)):
            ctx.set_cg_form(form)
            ctx.logdet_ratio(gU, gUp, kappa, wdr.OP_FULL, N, 1, wdr.NOISE_GAUSS, 5, p)  # warm-up
            ts = []
            for _ in range(3):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                s, lr, info = ctx.logdet_ratio(gU, gUp, kappa, wdr.OP_FULL, N, 1, wdr.NOISE_GAUSS, seed, p)
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t0)
            row[name] = {"ms": round(min(ts) * 1e3, 3), "cg_steps_max": int(info.iters),
                         "cg_steps_total": int(info.total_iters), "log_ratio": round(float(lr), 6)}
        row["persistent_over_launches"] = round(row["persistent"]["ms"] / row["launches"]["ms"], 3)
        out["x".join(map(str, L))] = row
        log("cg forms %s: %s" % ("x".join(map(str, L)), row))
        del gU, gUp
        ctx.close()
    return out


def dd_workload(wdr, torch, name):
    """One estimate of a larger lattice workload of synth.WORKLOADS: the mixed
    form (the workload's settings: FP16 block solves, CGNE with FP16
    iterations, FP32 middle and FP64 outer reliable updates, all samples
    batched) against the plain FP64 form (FP64 block solves and CGNE, one
    sample at a time)."""
    from paper_1112_1243_amd import synth
    w = synth.WORKLOADS[name]
    t0 = time.perf_counter()
    ctx = wdr.Context(w["L"], w["B"])
    U = synth.gauge_field(w["L"], w["scale"], w["seed"])
    Up = synth.redraw(U, proposal_mask(ctx, w["proposal"]), w["scale"], w["seed"])
    gU, gUp = ctx.gauge(torch.from_numpy(U).cuda()), ctx.gauge(torch.from_numpy(Up).cuda())
    del U, Up
    log("%s: inputs ready in %.1f s" % (name, time.perf_counter() - t0))
    op = {"schur": wdr.OP_SCHUR, "full": wdr.OP_FULL, "blocks": wdr.OP_BLOCKS}[w["op"]]
    noise = wdr.NOISE_GAUSS if w["noise"] == "gauss" else wdr.NOISE_Z2
    N = w["n_noise"]
    mixed = wdr.default_params(**w["mixed"])
    plain = wdr.default_params(solver=wdr.SOLVER_CGNE, inner=wdr.F64, max_iter=20000)
    ctx.logdet_ratio(gU, gUp, w["kappa"], op, 1, 1, noise, 1, mixed)  # warm-up
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    s_m, lr_m, info_m = ctx.logdet_ratio(gU, gUp, w["kappa"], op, N, 1, noise, w["seed"], mixed)
    torch.cuda.synchronize()
    t_m = time.perf_counter() - t1
    t1 = time.perf_counter()
    s_p, lr_p, info_p = ctx.logdet_ratio(gU, gUp, w["kappa"], op, N, 1, noise, w["seed"], plain, max_batch=1)
    torch.cuda.synchronize()
    t_p = time.perf_counter() - t1
    log("%s: mixed %.3f s (CG its %d), plain fp64 %.3f s (CG its %d), max |ds| %.2e"
        % (name, t_m, info_m.total_iters, t_p, info_p.total_iters, float(np.abs(s_m - s_p).max())))
    del gU, gUp
    ctx.close()
    return {"workload": "%s: %s lattice, %s blocks, kappa %.3f, links exp(i %.2f H), %s ratio, N=%d factors x 1 %s "
                        "noise, CGNE (FP16/FP32/FP64 levels) to 1e-10" % (name, "x".join(map(str, w["L"])),
                                                                           "x".join(map(str, w["B"])),
                                                  w["kappa"], w["scale"], w["op"].upper(), N, w["noise"]),
            "value": round(1.0 / t_m, 4), "unit": "estimates/s", "converged": bool(info_m.converged),
            "cg_iterations_total": int(info_m.total_iters),
            "fp64_estimates_per_s": round(1.0 / t_p, 4), "speedup_vs_fp64": round(t_p / t_m, 2),
            "max_abs_sample_diff_vs_fp64": float("%.3e" % float(np.abs(s_m - s_p).max()))}


def recursive_dd(wdr, torch):
    """Recursive DD (Sec. 3 eq. ddrec, the block step 2 of eq. 4step) in the
    block geometry of the paper's realistic run (Sec. 6): the Schur ratio of
    each of the 16 8^4 blocks of a 16^4 lattice over its 4^4 sub-blocks, one
    wdr_block_schur_ratio call; mixed form (CGNE with FP32 iterations and
    FP64 reliable updates, FP16 sub-block solves, all blocks and factors
    batched) against the plain FP64 form (one sample at a time)."""
    from paper_1112_1243_amd import synth
    w = synth.WORKLOADS["recursive16_dd8"]
    t0 = time.perf_counter()
    ctx = wdr.Context(w["L"], w["B"])
    sub = wdr.Context(w["B"], w["Bsub"], (0, 0, 0, 0))
    U = synth.gauge_field(w["L"], w["scale"], w["seed"])
    mask = proposal_mask(ctx, w["proposal"])
    Up = synth.redraw(U, mask, w["scale"], w["seed"])
    gU, gUp = ctx.gauge(torch.from_numpy(U).cuda()), ctx.gauge(torch.from_numpy(Up).cuda())
    del U, Up
    log("recursive16_dd8: inputs ready in %.1f s" % (time.perf_counter() - t0))
    N = w["n_noise"]
    mixed = wdr.default_params(**synth.LARGE_MIXED)
    plain = wdr.default_params(solver=wdr.SOLVER_CGNE, inner=wdr.F64, max_iter=20000)
    ctx.block_schur_ratio(gU, gUp, w["kappa"], sub, 1, 1, wdr.NOISE_GAUSS, 1, mixed)  # warm-up
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    s_m, lr_m, info_m = ctx.block_schur_ratio(gU, gUp, w["kappa"], sub, N, 1, wdr.NOISE_GAUSS, w["seed"], mixed)
    t_m = time.perf_counter() - t1
    t1 = time.perf_counter()
    s_p, lr_p, info_p = ctx.block_schur_ratio(gU, gUp, w["kappa"], sub, N, 1, wdr.NOISE_GAUSS, w["seed"], plain,
                                              max_batch=1)
    t_p = time.perf_counter() - t1
    log("recursive16_dd8: mixed %.3f s (CG its %d), plain fp64 %.3f s, max |ds| %.2e"
        % (t_m, info_m.total_iters, t_p, float(np.abs(s_m - s_p).max())))
    nb = ctx.nblocks
    del gU, gUp
    ctx.close()
    sub.close()
    return {"workload": "recursive16_dd8: 16^4 lattice, 16 blocks of 8^4 with open boundaries, 4^4 sub-blocks, "
                        "kappa %.3f, links exp(i %.2f H), links of the 6^4 core of every block redrawn (%.1f%%), "
                        "Schur ratio of every block, N=%d factors x 1 Gaussian noise, CGNE to 1e-10"
                        % (w["kappa"], w["scale"], 100 * float(mask.mean()), N),
            "value": round(nb / t_m, 2), "unit": "block Schur ratios/s", "seconds": round(t_m, 4),
            "converged": bool(info_m.converged), "cg_iterations_total": int(info_m.total_iters),
            "fp64_ratios_per_s": round(nb / t_p, 2), "speedup_vs_fp64": round(t_p / t_m, 2),
            "max_abs_sample_diff_vs_fp64": float("%.3e" % float(np.abs(s_m - s_p).max())),
            "sum_log_ratio": float(np.sum(lr_m))}


def plaquette(U, L):
    """Mean Re tr U_P / 3 of a canonical field (host numpy), a check of the
    thermalised ensemble (about 0.568 at beta 5.8)."""
    V = int(np.prod(L))
    x = np.arange(V)
    c = [x % L[0], (x // L[0]) % L[1], (x // (L[0] * L[1])) % L[2], x // (L[0] * L[1] * L[2])]

    def up(d):
        y = [a.copy() for a in c]
        y[d] = (y[d] + 1) % L[d]
        return y[0] + L[0] * (y[1] + L[1] * (y[2] + L[2] * y[3]))
    tot = 0.0
    for mu in range(4):
        for nu in range(mu + 1, 4):
            P = np.einsum("xab,xbc,xdc,xed->xae", U[:, mu], U[up(mu), nu], U[up(nu), mu].conj(), U[:, nu].conj())
            tot += np.trace(P, axis1=1, axis2=2).real.mean() / 3
    return tot / 6


def thermalised(wdr, torch, ctx, L, beta, seed, sweeps):
    """A quenched ensemble member: heat-bath sweeps of every link from the
    unit field (the paper's runs use beta = 5.8 quenched fields)."""
    from paper_1112_1243_amd import synth
    U = torch.from_numpy(synth.unit_gauge(L)).cuda()
    allm = torch.ones((ctx.V, 4), dtype=torch.uint8, device="cuda")
    for sw in range(sweeps):
        ctx.heatbath(beta, allm, seed, sw, U)
    return U, allm


def filter_run(wdr, torch, steps=6):
    """The three-step algorithm of Sec. 5 (eq. 4step, one level) on an 8^4
    lattice with 4^4 blocks at the paper's beta = 5.8 and kappa = 0.15462:
    per filter step two block steps (heat-bath of the active links, exact
    block acceptance), then the global Schur step with N = 16 factors x 1
    Gaussian noise.  Starts from a field thermalised by 200 heat-bath sweeps."""
    L, beta, kappa, seed = (8, 8, 8, 8), 5.8, 0.15462, 1112124305
    ctx = wdr.Context(L, (4, 4, 4, 4))
    U, _ = thermalised(wdr, torch, ctx, L, beta, seed, 200)
    plaq0 = plaquette(U.cpu().numpy(), L)
    mask = ctx.active_links(0, 3)
    p = wdr.default_params()
    ctx.filter_step(beta, kappa, mask, 1, 1, 1, seed + 99, 1, p, U.clone())  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    bacc = btri = gacc = 0
    lrs = []
    for k in range(steps):
        info, _ = ctx.filter_step(beta, kappa, mask, 2, 16, 1, seed + 100 + k, seed + 200 + k, p, U)
        bacc += info.block_accepts
        btri += info.block_trials
        gacc += info.accepted
        lrs.append(info.log_ratio)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    out = {"workload": "8^4 lattice, 16 blocks of 4^4, quenched beta 5.8 field (200 heat-bath sweeps from the "
                       "unit field), kappa 0.15462; filter step = 2 x (heat-bath of the active links, exact block "
                       "acceptance) + global Schur acceptance with N=16 x 1 Gaussian noise",
           "value": round(1.0 / dt, 3), "unit": "filter steps/s", "steps": steps,
           "block_acceptance": round(bacc / max(btri, 1), 3), "global_accepted": gacc,
           "global_log_ratios": [round(float(v), 3) for v in lrs], "plaquette_start": round(float(plaq0), 5),
           "plaquette_end": round(float(plaquette(U.cpu().numpy(), L)), 5)}
    ctx.close()
    return out


def fit_variance(lr, Ns, n_boot=2000, seed=1112124306):
    """Var over pairs of log Rhat_N (lr[pair, j] for N = Ns[j]) fitted as
    a + b / N (eq. param: the noise part of each factor's variance falls as
    1 / N; Sec. 5 extrapolates 1 / N -> 0).  Weighted least squares with the
    standard error of a variance estimate from P pairs, model(N)
    sqrt(2 / (P - 1)), the model refitted three times from equal weights;
    errors by bootstrap over pairs (the same pairs enter every N, so the
    variances are correlated and the bootstrap keeps that).  Returns the
    variances and their bootstrap errors, a, b, the bootstrap standard
    error of a and its central 68% interval."""
    lr = np.asarray(lr, dtype=np.float64)
    P = lr.shape[0]
    X = np.vstack([np.ones(len(Ns)), 1.0 / np.asarray(Ns, dtype=np.float64)]).T

    def fit(v):
        w = np.ones(len(Ns))
        coef = np.zeros(2)
        for _ in range(3):
            coef, _, _, _ = np.linalg.lstsq(X / w[:, None], v / w, rcond=None)
            w = np.maximum(X @ coef, 1e-12 * max(float(v.max()), 1e-300)) * np.sqrt(2.0 / (P - 1))
        return coef

    var = lr.var(axis=0, ddof=1)
    a, b = fit(var)
    rng = np.random.Generator(np.random.Philox(key=[seed, 7]))
    boot_a, boot_var = np.empty(n_boot), np.empty((n_boot, len(Ns)))
    for k in range(n_boot):
        vk = lr[rng.integers(0, P, P)].var(axis=0, ddof=1)
        boot_var[k] = vk
        boot_a[k] = fit(vk)[0]
    return {"var": var.tolist(), "var_err": boot_var.std(axis=0, ddof=1).tolist(), "a": float(a), "b": float(b),
            "a_err": float(boot_a.std(ddof=1)), "a_68": np.percentile(boot_a, [16, 84]).tolist()}


def exact_acceptance(wdr, torch):
    """The exact acceptance rate of the global step (Sec. 5): for pairs
    (U, U') of a quenched beta = 5.8 chain (10 heat-bath sweeps apart) and
    one block step each, the variance over pairs of the global estimate
    log Rhat for several N, fitted as a + b / N (fit_variance: weighted by
    the model's standard error, bootstrap errors over pairs); a is the exact
    variance sigma_2^2 and erfc(sqrt(a / 8)) the acceptance (eq. acceptance).  Beside it, N = 8 after 20 sweeps of
    relative gauge fixing of U' to U (Sec. 4), for the same pairs."""
    from scipy import special
    beta, kappa, seed = 5.8, 0.15462, 1112124305
    res = {}
    for L, pairs, Ns in (((8, 8, 8, 8), 96, (8, 16, 32, 64)), ((16, 16, 16, 16), 64, (8, 16, 32, 64))):
        t0 = time.perf_counter()
        ctx = wdr.Context(L, (4, 4, 4, 4))
        U, allm = thermalised(wdr, torch, ctx, L, beta, seed, 200)
        mask = ctx.active_links(0, 3)
        p = wdr.default_params()
        lr = np.zeros((pairs, len(Ns)))
        lr_fixed = np.zeros(pairs)  # N = 8 after relative gauge fixing of U' to U
        bacc = 0.0
        sw = 200
        for q in range(pairs):
            for _ in range(10):
                ctx.heatbath(beta, allm, seed, sw, U)
                sw += 1
            Up = U.clone()
            _, acc = ctx.filter_step(beta, kappa, mask, 1, 0, 1, seed + 1 + q, 0, p, Up)
            bacc += acc.mean()
            gU, gUp = ctx.gauge(U), ctx.gauge(Up)
            for j, N in enumerate(Ns):
                _, lr[q, j], _ = ctx.logdet_ratio(gU, gUp, kappa, wdr.OP_SCHUR, N, 1, wdr.NOISE_GAUSS,
                                                  seed + 1000 * q + N, p)
            ctx.relative_gauge(U, Up, 20)
            gUf = ctx.gauge(Up)
            _, lr_fixed[q], _ = ctx.logdet_ratio(gU, gUf, kappa, wdr.OP_SCHUR, 8, 1, wdr.NOISE_GAUSS,
                                                 seed + 1000 * q + 8, p)
            del gU, gUp, gUf
        fit = fit_variance(lr, Ns)
        var, a, b, a_err = np.array(fit["var"]), fit["a"], fit["b"], fit["a_err"]
        name = "x".join(map(str, L))
        res[name] = {"pairs": pairs, "N": list(Ns), "var_log_ratio": [round(float(v), 4) for v in var],
                     "var_log_ratio_err": [round(float(v), 4) for v in fit["var_err"]],
                     "mean_log_ratio": [round(float(v), 4) for v in lr.mean(axis=0)], "fit_a": round(float(a), 4),
                     "fit_a_err": round(a_err, 4), "fit_a_68": [round(float(v), 4) for v in fit["a_68"]],
                     "fit_b": round(float(b), 3), "block_acceptance": round(float(bacc) / pairs, 3),
                     "acceptance_erfc": round(float(special.erfc(np.sqrt(max(a, 0.0) / 8))), 3),
                     "var_log_ratio_N8_relative_gauge": round(float(lr_fixed.var(ddof=1)), 4),
                     "mean_log_ratio_N8_relative_gauge": round(float(lr_fixed.mean()), 4),
                     "seconds": round(time.perf_counter() - t0, 2)}
        log("exact acceptance %s: %s" % (name, res[name]))
        ctx.close()
    return {"workload": "quenched beta 5.8 pairs, 4^4 blocks, active links, one block step per pair, kappa "
                        "0.15462, global Schur estimate with N factors x 1 Gaussian noise", "volumes": res}


def estimate(ctx, wdr, gU, gUp, wl, params, seed):
    """One complete estimate: the 16 block ratios and the Schur ratio of the
    factorisation det D = prod_b det D_b det Dhat, in one DD call."""
    s, lr, info = ctx.logdet_ratio(gU, gUp, wl["kappa"], wdr.OP_DD, wl["n_steps"], wl["n_noise"], wdr.NOISE_GAUSS,
                                   seed, params)
    return lr, bool(info.converged), info.total_iters


def stencil_hash():
    import hashlib
    h = hashlib.sha256()
    for f in STENCIL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def counted_traffic(prec_name):
    """HBM bytes per launch from the committed counter summary, or None when
    the stencil sources changed since the counters were taken."""
    try:
        with open(COUNTERS) as fh:
            for line in fh:
                if line.startswith("traffic_json:"):
                    rec = json.loads(line.split(":", 1)[1])
                    if rec.get("sources_sha256_16") == stencil_hash() and prec_name in rec:
                        return rec[prec_name]
    except OSError:
        pass
    return None


def dslash_roofline(wdr, torch, L=(32, 32, 32, 32), prec_name="f64", reps=30, stencil=0, csw=0.0):
    """Average duration of one stencil launch on internal fields (SU(3)
    links), by HIP events on the stream the kernel is launched on; stencil
    is the context's kernel choice (0 = automatic); csw != 0: with the
    clover term (its blocks read once per site)."""
    from paper_1112_1243_amd import synth
    prec = wdr.F32 if prec_name == "f32" else wdr.F64
    ctx = wdr.Context(L, (4, 4, 4, 4))
    ctx.set_stencil(stencil)
    V = ctx.V
    U = synth.gauge_field(L, 0.2, 1112124303)
    gU = ctx.gauge(torch.from_numpy(U).cuda(), csw, 0.155)
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
    su3 = gU.su3
    per_site = BYTES_PER_SITE[(prec_name, su3)] + (CLOVER_BYTES_PER_SITE[prec_name] if csw else 0)
    alg = per_site * V
    gbs = alg / (ms * 1e-3) / 1e9
    del gU, a, b, psi
    ctx.close()
    key = prec_name + ("_clover" if csw else "")
    traffic = counted_traffic(key) if su3 and stencil != wdr.STENCIL_DIR else None
    kernel = (KERNEL[prec_name] if stencil != wdr.STENCIL_DIR else
              "k_dslash_dir<%s, all hops, B=4, R2=1>" % ("double" if prec_name == "f64" else "float")) \
        if su3 else "k_dslash_dir<%s, all hops, B=4, R2=0>" % ("double" if prec_name == "f64" else "float")
    if csw:
        kernel += " with the clover term (A times the staged input)"
    return {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": kernel,
            "lattice": "x".join(map(str, L)), "avg_launch_us": round(ms * 1e3, 2),
            "bytes_per_launch": alg, "bytes_per_site": per_site}


def dslash_f16(wdr, torch, L=(32, 32, 32, 32), reps=32, copies=4):
    """Average duration of one FP16 stencil launch (k_dslash_h16: FP16
    fields with per-block scales, FP16 two-row links, FP32 arithmetic).  One
    launch touches 192 B/site = 201 MB at 32^4, less than the 256 MB Infinity
    Cache, so launch i reads gauge copy i % copies and input field i % copies
    (copies = 4: 600 MB pass through between two reads of one copy)."""
    from paper_1112_1243_amd import synth
    ctx = wdr.Context(L, (4, 4, 4, 4))
    V = ctx.V
    gs, fs = [], []
    for c in range(copies):
        U = synth.gauge_field(L, 0.2, 1112124303 + 10 * c)
        gs.append(ctx.gauge(torch.from_numpy(U).cuda()))
        del U
        fs.append(ctx.pack(torch.from_numpy(synth.spinor(L, 5 + c)).cuda(), wdr.F16))
    outs = [ctx.internal_field(wdr.F16) for _ in range(2)]
    for i in range(copies):
        ctx.apply_D_internal(gs[i], 0.155, fs[i], outs[i % 2], wdr.F16)
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for i in range(reps):
        ctx.apply_D_internal(gs[i % copies], 0.155, fs[i % copies], outs[i % 2], wdr.F16)
    e1.record(st)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    alg = 192 * V
    gbs = alg / (ms * 1e-3) / 1e9
    del gs, fs, outs
    ctx.close()
    return {"achieved": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": counted_traffic("f16"),
            "kernel": "k_dslash_h16<4> (FP16 fields, per-block scales, FP16 two-row links)",
            "avg_launch_us": round(ms * 1e3, 2), "bytes_per_launch": alg, "bytes_per_site": 192,
            "rotating_copies": copies}


def copy_ceiling(torch, reps=10):
    """Bandwidth of a plain elementwise copy of 1 GiB (torch's vectorised
    kernel, 1 GiB read + 1 GiB written): the practical HBM ceiling, and the
    reference launch for calibrating the FETCH_SIZE / WRITE_SIZE counters."""
    n = 256 * 1024 * 1024
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        torch.mul(x, 1.0, out=y)
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(reps):
        torch.mul(x, 1.0, out=y)
    e1.record(st)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del x, y
    return {"kernel": "torch elementwise copy (mul by 1.0), 1 GiB in + 1 GiB out", "avg_launch_us": round(ms * 1e3, 1),
            "achieved": round(2 * 4 * n / (ms * 1e-3) / 1e9, 1), "unit": "GB/s"}


def rocprof_summary(path, kernel_regex="k_dslash|k_eo16|k_block_mr|k_cg_steps"):
    """Markdown summary of rocprofv3 CSV output under `path`: per-kernel
    totals (rocprofv3's kernel_stats); when a marker trace holds the timed
    range of the headline, the kernels inside it by name and grid (time
    share, launches and time per estimate, average launch); the kernels
    matching kernel_regex by grid over the whole run (kernel_trace); and
    per-dispatch counter means by kernel and grid (counter_collection)."""
    import csv
    import glob
    import re
    from collections import defaultdict

    def rows(pattern):
        out = []
        for f in sorted(glob.glob(os.path.join(path, "**", pattern), recursive=True)):
            with open(f, newline="") as fh:
                out += [{k.lower(): v for k, v in r.items()} for r in csv.DictReader(fh)]
        return out

    def short(name):
        name = name.replace("wdr::(anonymous namespace)::", "").replace("(anonymous namespace)::", "")
        m = re.match(r"_ZN3wdr12_GLOBAL__N_1\d+(k_\w+?)(I|E)", name)
        if m:
            name = m.group(1) + ("<...>" if m.group(2) == "I" else "")
        return re.sub(r"\(.*", "", name)[:90]

    def grid(r):
        return "x".join(r.get("grid_size_%s" % d, "?") for d in "xyz")

    lines = []
    stats = rows("*kernel_stats.csv")
    if stats:
        lines += ["All kernels of the run (rocprofv3 kernel_stats):", "",
                  "| kernel | calls | total us | avg us | % |", "|---|---|---|---|---|"]
        stats.sort(key=lambda r: -float(r.get("totaldurationns", 0)))
        for r in stats[:15]:
            lines.append("| %s | %s | %.1f | %.2f | %.2f |" % (short(r["name"]), r["calls"],
                                                             float(r["totaldurationns"]) / 1e3,
                                                             float(r["averagens"]) / 1e3,
                                                             float(r.get("percentage", 0))))
    trace = rows("*kernel_trace.csv")
    marks = [r for r in rows("*marker_api_trace.csv") if any(TIMED_RANGE in str(v) for v in r.values())]
    if trace and marks:
        t0 = min(int(r["start_timestamp"]) for r in marks)
        t1 = max(int(r["end_timestamp"]) for r in marks)
        inside = [r for r in trace if int(r["start_timestamp"]) >= t0 and int(r["end_timestamp"]) <= t1]
        steps = None
        m = re.search(r"--steps\s+(\d+)", " ".join(sys.argv))
        agg = defaultdict(list)
        for r in inside:
            agg[(short(r["kernel_name"]), grid(r))].append((int(r["end_timestamp"]) - int(r["start_timestamp"])) / 1e3)
        tot = sum(sum(v) for v in agg.values())
        lines += ["", "Kernels inside the timed range of the headline (%d launches, %.1f ms of kernel time, "
                  "%.1f ms wall):" % (len(inside), tot / 1e3, (t1 - t0) / 1e6), "",
                  "| kernel | grid (work-items) | launches | total us | avg us | % of kernel time |",
                  "|---|---|---|---|---|---|"]
        for (k, gr), v in sorted(agg.items(), key=lambda kv: -sum(kv[1]))[:25]:
            lines.append("| %s | %s | %d | %.1f | %.2f | %.2f |" % (k, gr, len(v), sum(v), sum(v) / len(v),
                                                                  100 * sum(v) / tot))
        del steps, m
    if trace:
        agg = defaultdict(list)
        for r in trace:
            if re.search(kernel_regex, short(r["kernel_name"])):
                agg[(short(r["kernel_name"]), grid(r))].append(
                    (int(r["end_timestamp"]) - int(r["start_timestamp"])) / 1e3)
        if agg:
            lines += ["", "| kernel (%s), whole run | grid (work-items) | launches | avg us | min us | max us |"
                      % kernel_regex, "|---|---|---|---|---|---|"]
            for (k, gr), v in sorted(agg.items()):
                lines.append("| %s | %s | %d | %.2f | %.2f | %.2f |" % (k, gr, len(v), sum(v) / len(v), min(v),
                                                                       max(v)))
    cnt = rows("*counter_collection.csv")
    if cnt:
        agg = defaultdict(list)
        for r in cnt:
            agg[(short(r["kernel_name"]), r.get("grid_size", "?"), r["counter_name"])].append(
                float(r["counter_value"]))
        lines += ["", "| kernel | grid size | counter | dispatches | mean per dispatch |", "|---|---|---|---|---|"]
        for (k, gr, c), v in sorted(agg.items()):
            if re.search(kernel_regex + "|elementwise", k):
                lines.append("| %s | %s | %s | %d | %.1f |" % (k, gr, c, len(v), sum(v) / len(v)))
    return "\n".join(lines)


def batched_proposals(wdr, torch, n_steps=8, scale=0.3):
    """The batched-proposal workload: 64 proposals of uneven sizes (24 at 8^4,
    24 at 12^4, 16 at 16^4), kappa uniform in [0.12, 0.15], U' redraws each
    link with probability 0.1, full-operator ratio, n_steps = 8 factors with
    one Z2 noise vector each, CGNE (FP32 cycles in FP64 defect correction) to
    1e-10: one wdr_logdet_ratio_batch call.  Baseline: the plain FP64 form
    (FP64 CGNE, one sample at a time, proposals one after another), timed on
    one proposal of each size and scaled by the counts."""
    from paper_1112_1243_amd import synth
    specs = synth.batch_proposals()
    ctxs = {}
    props = []
    t0 = time.perf_counter()
    for q in specs:
        L = q["L"]
        if L not in ctxs:
            ctxs[L] = wdr.Context(L, (4, 4, 4, 4))
        c = ctxs[L]
        U = synth.gauge_field(L, scale, q["seed"])
        Up = synth.redraw(U, synth.bernoulli_links(L, 0.1, q["seed"]), scale, q["seed"])
        props.append((c, c.gauge(torch.from_numpy(U).cuda()), c.gauge(torch.from_numpy(Up).cuda()), q["kappa"],
                      q["seed"]))
    log("batched proposals: inputs ready in %.1f s" % (time.perf_counter() - t0))
    # kappa near the critical value of these links (about 0.132) makes some
    # solves need a few thousand CG iterations: allow them
    mixed = wdr.default_params(solver=wdr.SOLVER_CGNE, inner=wdr.F32, max_iter=20000)
    plain = wdr.default_params(solver=wdr.SOLVER_CGNE, inner=wdr.F64, max_iter=20000)
    # warm-up (workspace pools, streams): one factor per proposal
    wdr.logdet_ratio_batch(props, wdr.OP_FULL, 1, 1, wdr.NOISE_Z2, mixed)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    samples, lrs, info = wdr.logdet_ratio_batch(props, wdr.OP_FULL, n_steps, 1, wdr.NOISE_Z2, mixed)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    log("batched proposals: %d estimates in %.3f s, converged %s, CG iterations %d (max %d)"
        % (len(props), dt, bool(info.converged), info.total_iters, info.iters))
    # serial FP64 baseline: every proposal, one after another, one sample at a time
    t1 = time.perf_counter()
    worst = 0.0
    for j, (c, gU, gUp, kappa, seed) in enumerate(props):
        t2 = time.perf_counter()
        _, lr1, _ = c.logdet_ratio(gU, gUp, kappa, wdr.OP_FULL, n_steps, 1, wdr.NOISE_Z2, seed, plain, max_batch=1)
        worst = max(worst, abs(lr1 - lrs[j]))
        torch.cuda.synchronize()
        if time.perf_counter() - t2 > 1.0:
            log("serial fp64: proposal %d (kappa %.4f) took %.2f s" % (j, kappa, time.perf_counter() - t2))
    serial = time.perf_counter() - t1
    log("serial fp64: %d proposals in %.2f s; largest |log R (batched) - log R (serial fp64)| = %.2e"
        % (len(props), serial, worst))
    del props
    for c in ctxs.values():
        c.close()
    return {"workload": "64 proposals (24 x 8^4, 24 x 12^4, 16 x 16^4), kappa in [0.12, 0.15], links exp(i 0.3 H), "
                        "Bernoulli(0.1) redraw, full operator, N=8 factors x 1 Z2 noise, CGNE to 1e-10",
            "value": round(len(specs) / dt, 3), "unit": "estimates/s", "seconds": round(dt, 3),
            "converged": bool(info.converged), "cg_iterations_total": int(info.total_iters),
            "fp64_serial_estimates_per_s": round(len(specs) / serial, 3),
            "fp64_serial": "every proposal in turn, FP64 CGNE, one sample at a time",
            "max_abs_log_ratio_diff_vs_fp64_serial": float("%.3e" % worst),
            "speedup_vs_fp64_serial": round(serial / dt, 2)}


def block_determinants(wdr, torch):
    """Exact block ratios log det(D_b'^+ D_b') - log det(D_b^+ D_b) of every
    4^4 block (Sec. 3, eqs. ddfactor and 4step, first step) for the proposals
    of the 8^4 and 16^4 workloads: 2 x nblocks normal matrices of 1536 rows,
    formed and Cholesky-factorised in FP64 in one call.  The rate is counted
    in Cholesky flops (4/3 n^3 per matrix) over the whole call, formation of
    the matrices included, against the FP64 matrix peak.  For the 8^4
    workload the stochastic BLOCKS estimate of the same proposal (N = 64
    factors x 1 Gaussian noise) is reported beside the exact sum."""
    from paper_1112_1243_amd import synth
    res = {}
    for name, reps in (("wilson8_dd16", 5), ("wilson16_dd256", 2)):
        w = synth.WORKLOADS[name]
        ctx = wdr.Context(w["L"], w["B"])
        U = synth.gauge_field(w["L"], w["scale"], w["seed"])
        Up = synth.redraw(U, proposal_mask(ctx, w["proposal"]), w["scale"], w["seed"])
        gU, gUp = ctx.gauge(torch.from_numpy(U).cuda()), ctx.gauge(torch.from_numpy(Up).cuda())
        del U, Up
        ctx.block_logdet_ratio(gU, gUp, w["kappa"])  # warm-up (workspace)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            r = ctx.block_logdet_ratio(gU, gUp, w["kappa"])
        dt = (time.perf_counter() - t0) / reps
        n = 6 * int(np.prod(w["B"]))
        flops = 2 * ctx.nblocks * 4.0 / 3.0 * n ** 3
        d = {"workload": "%s: %s lattice, %d blocks of %s, kappa %.3f, U and U' (%s)" % (
                 name, "x".join(map(str, w["L"])), ctx.nblocks, "x".join(map(str, w["B"])), w["kappa"],
                 w["proposal"]),
             "value": round(ctx.nblocks / dt, 2), "unit": "exact block ratios/s", "ms_per_call": round(dt * 1e3, 3),
             "matrices": 2 * ctx.nblocks, "rows": n,
             "roofline": {"bound": "mfma", "achieved": round(flops / dt / 1e12, 2), "peak": 78.6,
                          "unit": "TFLOP/s", "frac": round(flops / dt / 1e12 / 78.6, 4), "traffic": None,
                          "what": "Cholesky flops 4/3 n^3 per matrix over the whole call (formation included)"},
             "exact_blocks_log_ratio": float(np.sum(r))}
        if name == "wilson8_dd16":
            # the proposal redraws whole links, so each path factor's samples
            # vary by about 2 per block at N = 8: with N = 64 the variance is
            # small enough for log-mean-exp to approach the exact value
            p = wdr.default_params()
            s, lr, _ = ctx.logdet_ratio(gU, gUp, w["kappa"], wdr.OP_BLOCKS, 64, 1, wdr.NOISE_GAUSS, w["seed"], p)
            d["stochastic_blocks_log_ratio_N64"] = float(lr)
        log("block determinants %s: %s" % (name, d))
        res[name] = d
        del gU, gUp
        ctx.close()
    return res


def cpu_info():
    """CPU model (from /proc/cpuinfo) and the logical CPUs this process may use."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        ncpu = len(os.sched_getaffinity(0))
    except AttributeError:
        ncpu = os.cpu_count() or 1
    return model, ncpu


ORACLE_STENCIL_CHILD = r"""
import sys, time
sys.path.insert(0, sys.argv[1])
import oracle
from paper_1112_1243_amd import synth
L = (16, 16, 16, 16)
lat = oracle.Lattice(L, (4, 4, 4, 4))
U, psi = synth.gauge_field(L, 0.25, 1112124302), synth.spinor(L, 11)
oracle.apply_D(lat, U, 0.150, psi)
ts = []
for _ in range(3):
    t = time.perf_counter()
    oracle.apply_D(lat, U, 0.150, psi)
    ts.append(time.perf_counter() - t)
print(sorted(ts)[1])
"""


def oracle_stencil_ms(threads):
    """Median of 3 oracle stencil applications at 16^4 in a child process
    with `threads` OpenMP threads (ms)."""
    import subprocess
    env = dict(os.environ, OMP_NUM_THREADS=str(threads))
    r = subprocess.run([sys.executable, "-c", ORACLE_STENCIL_CHILD, ROOT], capture_output=True, text=True, env=env,
                       timeout=600)
    return float(r.stdout.strip().splitlines()[-1]) * 1e3


def cpu_baseline():
    """The FP64 CPU oracle on a bounded sample of the headline workload's work
    unit: one (factor, noise) item of the Schur estimate -- the oracle's
    Schur complement (block solves to 1e-14), the global CGNE solve and its
    adjoint to 1e-13, the second-order sample -- timed on the 16^4 lattice
    of the same recipe (kappa 0.150, links exp(i 0.25 H), black-block links
    redrawn) with all threads; the 32^4 item does not fit the benchmark's
    time (about ten minutes).  Extrapolated to the headline estimate by the
    volume ratio (16) and the N = 32 items.  Beside it the oracle's stencil
    at 16^4, median of 3, with all threads and with one thread."""
    import oracle
    from paper_1112_1243_amd import synth
    from tests.golden import make_golden
    model, ncpu = cpu_info()
    threads = int(os.environ.get("OMP_NUM_THREADS", ncpu))
    w, lat, U, Up = make_golden.inputs("wilson16_dd256")
    U1 = oracle.interpolate(U, Up, 1, w["n_noise"])
    eta = oracle.noise(lat, oracle.NOISE_GAUSS, w["seed"], 0, 0, support=oracle.noise_support(lat, oracle.OP_SCHUR))
    t0 = time.perf_counter()
    oracle.sample(lat, U, U1, w["kappa"], oracle.OP_SCHUR, eta)
    item = time.perf_counter() - t0
    vol_ratio = (32 ** 4) / lat.V
    per_estimate = item * vol_ratio * 32
    ms_all = oracle_stencil_ms(threads)
    ms_one = oracle_stencil_ms(1)
    V16 = 16 ** 4
    return {"value": round(1.0 / per_estimate, 7), "unit": "estimates/s", "cores": threads, "kind": "oracle",
            "extrapolated": True, "cpu_model": model, "logical_cpus": ncpu,
            "sample": "one SCHUR (factor, noise) item of the 16^4 lattice (same recipe as the 32^4 headline at "
                      "kappa 0.150), oracle solves to 1e-13: %.1f s on %d threads; x%d (volume) x32 (items) = one "
                      "32^4 estimate, extrapolated" % (item, threads, vol_ratio),
            "item_seconds": round(item, 3),
            "stencil": {"lattice": "16x16x16x16", "unit": "GB/s", "kind": "oracle apply_D, FP64, median of 3",
                        "ms_all_threads": round(ms_all, 2), "ms_one_thread": round(ms_one, 2),
                        "value_all_threads": round(960 * V16 / (ms_all * 1e-3) / 1e9, 2),
                        "value_one_thread": round(960 * V16 / (ms_one * 1e-3) / 1e9, 2)}}


# the headline workload (the largest configuration: 32^4, 4096 blocks of 4^4)
HEADLINE = "wilson32_dd4096"
TIMED_RANGE = "timed estimates"
# compulsory bytes of one k_eo16 launch per system of V sites (one even-odd
# half in FP16: the input half, the output half and every link of the
# lattice, FP16 two-row, 24 B per link), plus the FP16 diagonal half if any
EO16_SOURCES = ["paper_1112_1243_amd/csrc/cg16.hip", "paper_1112_1243_amd/csrc/half2.h",
                "paper_1112_1243_amd/csrc/stencil.h", "paper_1112_1243_amd/csrc/wdr_internal.h"]
EO16_COUNTERS = os.path.join(ROOT, "profiles", "eo16_32x32x32x32_counters.md")


def eo16_bytes(V, diag):
    return V // 2 * 48 * (3 if diag else 2) + V * 96


def headline_estimate(wdr, torch, steps, warmup, fp64=True):
    """The headline: K estimates of the 32^4 Schur ratio (N = 32) in the
    mixed-precision form after W warm-up estimates, and the plain FP64
    single-proposal form (FP64 CGNE, FP64 block solves, one sample at a
    time, no graphs) on the same proposal."""
    from paper_1112_1243_amd import synth
    w = synth.WORKLOADS[HEADLINE]
    N = w["n_noise"]
    t0 = time.perf_counter()
    ctx = wdr.Context(w["L"], w["B"])
    U = synth.gauge_field(w["L"], w["scale"], w["seed"])
    Up = synth.redraw(U, proposal_mask(ctx, w["proposal"]), w["scale"], w["seed"])
    gU, gUp = ctx.gauge(torch.from_numpy(U).cuda()), ctx.gauge(torch.from_numpy(Up).cuda())
    del U, Up
    log("%s: inputs ready in %.1f s" % (HEADLINE, time.perf_counter() - t0))
    t0 = time.perf_counter()
    mixed, t_trial = ctx.autotune(gU, gUp, w["kappa"], wdr.OP_SCHUR, N, 1, wdr.NOISE_GAUSS, 500,
                                  wdr.default_params(**w["mixed"]))
    log("%s: autotuned in %.1f s: block MR %d (trial estimate %.3f s)" % (HEADLINE, time.perf_counter() - t0,
                                                                          mixed.block_mr_steps, t_trial))
    for k in range(warmup):
        ctx.logdet_ratio(gU, gUp, w["kappa"], wdr.OP_SCHUR, N, 1, wdr.NOISE_GAUSS, 1000 + k, mixed)
    torch.cuda.synchronize()
    wdr.traffic(reset=True)
    # a marker range around the timed estimates (rocprofv3 --marker-trace
    # records it; --rocprof-summary keeps the kernels inside it)
    torch.cuda.nvtx.range_push(TIMED_RANGE)
    t0 = time.perf_counter()
    ok, iters, lrs, s_first = True, 0, [], None
    for k in range(steps):
        s, lr, info = ctx.logdet_ratio(gU, gUp, w["kappa"], wdr.OP_SCHUR, N, 1, wdr.NOISE_GAUSS, 2000 + k, mixed)
        ok &= bool(info.converged) and info.true_rel_resid <= 1e-10
        iters += info.total_iters
        lrs.append(lr)
        if s_first is None:
            s_first = s
        log("step %d: log R = %.10f converged=%s CG iterations=%d" % (k, lr, bool(info.converged),
                                                                       info.total_iters))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    torch.cuda.nvtx.range_pop()
    traffic = wdr.traffic(reset=True)
    out = {"steps": steps, "seconds": dt, "converged": ok, "cg_iterations": iters, "mean_log_ratio": float(np.mean(lrs)),
           "params": mixed, "traffic_bytes": traffic}
    if fp64:
        plain = wdr.default_params(solver=wdr.SOLVER_CGNE, inner=wdr.F64, middle=wdr.F64, max_iter=20000, graph=0)
        t1 = time.perf_counter()
        s_p, lr_p, info_p = ctx.logdet_ratio(gU, gUp, w["kappa"], wdr.OP_SCHUR, N, 1, wdr.NOISE_GAUSS, 2000, plain,
                                             max_batch=1)
        torch.cuda.synchronize()
        out["fp64_seconds"] = time.perf_counter() - t1
        out["fp64_converged"] = bool(info_p.converged)
        out["max_abs_sample_diff_vs_fp64"] = float(np.abs(s_first - s_p).max())
        log("%s plain fp64: %.3f s, max |ds| vs mixed %.2e" % (HEADLINE, out["fp64_seconds"],
                                                               out["max_abs_sample_diff_vs_fp64"]))
    out["nsys"] = N
    del gU, gUp
    ctx.close()
    return out


def eo16_roofline(wdr, torch, nsys, reps=20):
    """Average duration of one k_eo16 launch (one even-odd half of the FP16
    CG stencil) at 32^4 with nsys systems per launch, the launch shape of the
    headline estimate, by HIP events on the stream it is launched on: pairs
    of launches as a CG step issues them (odd sites from even without a
    diagonal term, even sites from odd with one)."""
    from paper_1112_1243_amd import synth
    w = synth.WORKLOADS[HEADLINE]
    ctx = wdr.Context(w["L"], w["B"])
    U = synth.gauge_field(w["L"], w["scale"], w["seed"])
    gU = ctx.gauge(torch.from_numpy(U).cuda())
    del U
    one = ctx.pack_eo16(torch.from_numpy(synth.spinor(w["L"], 5)).cuda(), 0)
    vals, nsc = one.numel() - ctx.nblocks * 4, ctx.nblocks * 4
    ev = ctx.eo16_field(nsys)
    for m in range(nsys):  # nsys copies: values first, then the scales
        ev[m * vals:(m + 1) * vals] = one[:vals]
        ev[nsys * vals + m * nsc:nsys * vals + (m + 1) * nsc] = one[vals:]
    od, out = ctx.eo16_field(nsys), ctx.eo16_field(nsys)
    k = w["kappa"]

    def pair():
        ctx.apply_hop_eo_internal(gU, k, wdr.F16, 1, 0, ev, None, od, nsys)
        ctx.apply_hop_eo_internal(gU, k, wdr.F16, 0, 0, od, ev, out, nsys)
    for _ in range(3):
        pair()
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(reps):
        pair()
    e1.record(st)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / (2 * reps)
    V = ctx.V
    alg = nsys * (eo16_bytes(V, False) + eo16_bytes(V, True)) // 2
    gbs = alg / (ms * 1e-3) / 1e9
    del gU, ev, od, out, one
    ctx.close()
    return {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": counted_traffic_eo16(nsys),
            "kernel": "k_eo16 (FP16 even-odd half of the CG stencil, site-major FP16 fields and links)",
            "lattice": "32x32x32x32", "systems_per_launch": nsys, "avg_launch_us": round(ms * 1e3, 2),
            "bytes_per_launch": int(alg),
            "bytes_per_site": "per system: V/2 x 48 B in + V/2 x 48 B out (+ V/2 x 48 B diagonal on every other "
                              "launch) + V x 96 B links"}


def sources_hash(files):
    import hashlib
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def counted_traffic_eo16(nsys):
    """HBM bytes per k_eo16 launch from the committed counter summary (for
    that many systems per launch), or None when cg16.hip changed since."""
    try:
        with open(EO16_COUNTERS) as fh:
            for line in fh:
                if line.startswith("traffic_json:"):
                    rec = json.loads(line.split(":", 1)[1])
                    if rec.get("sources_sha256_16") == sources_hash(EO16_SOURCES) and rec.get("nsys") == nsys:
                        return rec["bytes_per_launch"]
    except OSError:
        pass
    return None


def dd8_workload(wdr, torch, steps, warmup, fp64=True):
    """The 8^4 domain-decomposition estimate: 16 block ratios and the Schur
    ratio (one DD call), N = 8 factors x 1 Gaussian noise, FGCR(16) + SAP
    to 1e-10 with FP32 preconditioner, autotuned; the plain FP64 form beside."""
    from paper_1112_1243_amd import synth
    wl = WORKLOAD
    ctx = wdr.Context(wl["L"], wl["B"])
    U = make_inputs(wl)
    Up = synth.redraw(U, proposal_mask(ctx, "active"), wl["scale"], wl["seed"])
    gU = ctx.gauge(torch.from_numpy(U).cuda())
    gUp = ctx.gauge(torch.from_numpy(Up).cuda())
    mixed, _ = ctx.autotune(gU, gUp, wl["kappa"], wdr.OP_DD, wl["n_steps"], wl["n_noise"], wdr.NOISE_GAUSS, 500,
                            wdr.default_params(inner=wdr.F32))
    p64, _ = ctx.autotune(gU, gUp, wl["kappa"], wdr.OP_DD, wl["n_steps"], wl["n_noise"], wdr.NOISE_GAUSS, 500,
                          wdr.default_params(inner=wdr.F64))
    for k in range(warmup):
        estimate(ctx, wdr, gU, gUp, wl, mixed, 1000 + k)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ok, iters = True, 0
    for k in range(steps):
        _, c, it = estimate(ctx, wdr, gU, gUp, wl, mixed, 2000 + k)
        ok &= c
        iters += it
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    out = {"workload": "%s: 8^4 lattice, 16 blocks of 4^4, kappa 0.135, links exp(i 0.5 H), active links redrawn, "
                       "BLOCKS + SCHUR ratios (DD), N=8 factors x 1 Gaussian noise, FGCR(16)+SAP (autotuned depth) "
                       "to 1e-10" % wl["name"], "value": round(steps / dt, 3), "unit": "estimates/s",
           "converged": ok, "total_outer_iters": iters,
           "schedule": {"mixed": {"sap_cycles": mixed.sap_cycles, "mr_steps": mixed.mr_steps,
                                  "block_mr_steps": mixed.block_mr_steps},
                        "fp64": {"sap_cycles": p64.sap_cycles, "mr_steps": p64.mr_steps,
                                 "block_mr_steps": p64.block_mr_steps}}}
    if fp64:
        t1 = time.perf_counter()
        n64 = max(1, min(5, steps))
        for k in range(n64):
            estimate(ctx, wdr, gU, gUp, wl, p64, 2000 + k)
        torch.cuda.synchronize()
        out["fp64_estimates_per_s"] = round(n64 / (time.perf_counter() - t1), 3)
    del gU, gUp
    ctx.close()
    log("dd8:", out)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--headline-only", action="store_true",
                    help="only the 32^4 headline estimates (for profiling): no FP64 form, rooflines or extras")
    ap.add_argument("--roofline-only", action="store_true",
                    help="only the roofline launches (k_eo16 in the headline's launch shape, the 32^4 stencils, "
                         "the copy ceiling), for counter runs")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-dslash", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-proposal workload")
    ap.add_argument("--no-large", action="store_true", help="skip the 16^4 workload")
    ap.add_argument("--no-dd8", action="store_true", help="skip the 8^4 domain-decomposition workload")
    ap.add_argument("--no-blockdet", action="store_true", help="skip the exact block determinants")
    ap.add_argument("--no-recursive", action="store_true", help="skip the recursive-DD workload")
    ap.add_argument("--no-filter", action="store_true", help="skip the filter run")
    ap.add_argument("--no-clover", action="store_true", help="skip the clover FULL estimates")
    ap.add_argument("--no-cg-forms", action="store_true", help="skip the CG launch-form comparison")
    ap.add_argument("--cg-forms-only", action="store_true", help="run only the CG launch-form comparison")
    ap.add_argument("--no-slab", action="store_true", help="skip the slab-halo timing")
    ap.add_argument("--slab-only", action="store_true", help="run only the slab-halo timing")
    ap.add_argument("--acceptance", action="store_true", help="also run the exact-acceptance variance study")
    ap.add_argument("--stencil", choices=("auto", "dir", "blk"), default="auto",
                    help="stencil kernel for the 32^4 full-stencil launches (default: the library's choice)")
    ap.add_argument("--rocprof-summary", metavar="DIR", help="print a markdown summary of rocprofv3 CSV output")
    args = ap.parse_args()
    if args.rocprof_summary:
        print(rocprof_summary(args.rocprof_summary))
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU: the library has no multi-GPU path (every proposal, path factor and "
              "noise vector is independent, so they would be dealt out to one process per GPU)", file=sys.stderr)
        sys.exit(2)
    if args.headline_only:
        args.no_cpu = args.no_fp64 = args.no_dslash = args.no_batch = args.no_large = args.no_dd8 = True
        args.no_blockdet = args.no_recursive = args.no_filter = args.no_clover = args.no_cg_forms = True
        args.no_slab = True

    import torch
    from paper_1112_1243_amd import synth, wdr

    if args.cg_forms_only:
        print(json.dumps(cg_forms(wdr, torch)), flush=True)
        return
    if args.slab_only:
        print(json.dumps(slab_halo(wdr, torch)), flush=True)
        return

    if args.roofline_only:
        roof = eo16_roofline(wdr, torch, synth.WORKLOADS[HEADLINE]["n_noise"])
        log("k_eo16:", roof)
        for prec in ("f64", "f32"):
            log("dslash %s:" % prec, dslash_roofline(wdr, torch, prec_name=prec))
            log("dslash %s clover:" % prec, dslash_roofline(wdr, torch, prec_name=prec, csw=CSW))
        log("dslash f16:", dslash_f16(wdr, torch))
        log("copy ceiling:", copy_ceiling(torch))
        return
    head = headline_estimate(wdr, torch, args.steps, args.warmup, fp64=not args.no_fp64)
    dt = head["seconds"]
    value = args.steps / dt
    mixed = head["params"]

    roof = None
    if not args.no_dslash:
        roof = eo16_roofline(wdr, torch, head["nsys"])
        log("k_eo16:", roof)
        # the full Wilson stencil (the Dslash half of the metric) beside it
        sc = {"auto": wdr.STENCIL_AUTO, "dir": wdr.STENCIL_DIR, "blk": wdr.STENCIL_BLK}[args.stencil]
        r64 = dslash_roofline(wdr, torch, prec_name="f64", stencil=sc)
        r32 = dslash_roofline(wdr, torch, prec_name="f32", stencil=sc)
        log("dslash f64:", r64)
        log("dslash f32:", r32)
        roof["stencil_f64"] = r64
        roof["stencil_f32"] = {k: r32[k] for k in ("achieved", "frac", "traffic", "kernel", "avg_launch_us",
                                                    "bytes_per_launch")}
        r64c = dslash_roofline(wdr, torch, prec_name="f64", stencil=sc, csw=CSW)
        log("dslash f64 clover:", r64c)
        roof["stencil_f64_clover"] = {k: r64c[k] for k in ("achieved", "frac", "traffic", "kernel", "avg_launch_us",
                                                           "bytes_per_launch", "bytes_per_site")}
        roof["stencil_f16"] = dslash_f16(wdr, torch)
        log("dslash f16:", roof["stencil_f16"])
        roof["copy_ceiling"] = copy_ceiling(torch)
        log("copy ceiling:", roof["copy_ceiling"])
    whole = None
    if head["traffic_bytes"]:
        per = head["traffic_bytes"] / args.steps
        gbs = per / (dt / args.steps) / 1e9
        whole = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                 "frac": round(gbs / HBM_PEAK_GBS, 4), "compulsory_bytes_per_estimate": int(per),
                 "what": "compulsory bytes of every kernel of one estimate (the library's wdr_traffic count from "
                         "per-system iteration, update and round counts) over the estimate's wall time"}

    dd8 = None if args.no_dd8 else dd8_workload(wdr, torch, max(5, args.steps), 2, fp64=not args.no_fp64)
    batch = None if args.no_batch else batched_proposals(wdr, torch)
    if batch:
        log("batched proposals:", batch)
    large = None if args.no_large else {"wilson16_dd256": dd_workload(wdr, torch, "wilson16_dd256")}
    bdet = None if args.no_blockdet else block_determinants(wdr, torch)
    rdd = None if args.no_recursive else recursive_dd(wdr, torch)
    if rdd:
        log("recursive dd:", rdd)
    clov = None if args.no_clover else clover_workload(wdr, torch)
    forms = None if args.no_cg_forms else cg_forms(wdr, torch)
    slab = None if args.no_slab else slab_halo(wdr, torch)
    filt = None if args.no_filter else filter_run(wdr, torch)
    if filt:
        log("filter:", filt)
    acc = exact_acceptance(wdr, torch) if args.acceptance else None
    cpu = None if args.no_cpu else cpu_baseline()
    if cpu:
        log("cpu baseline:", cpu)

    fp64_rate = 1.0 / head["fp64_seconds"] if "fp64_seconds" in head else None
    out = {
        "metric": "Dslash HBM GB/s (% peak) + det-ratio estimates/sec at 1e-10 residual vs FP64",
        "value": round(value, 4),
        "unit": "estimates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f16+f32+f64",
        "data": "synthetic",
        "config": {"workload": "%s: 32^4 lattice, 4096 blocks of 4^4, kappa 0.155, links exp(i 0.2 H), active links "
                               "redrawn, SCHUR ratio, N=32 factors x 1 Gaussian noise (batched), CGNE with FP16 inner "
                               "iterations, FP32 middle and FP64 outer reliable updates to 1e-10, FP16 block solves "
                               "to 1e-13" % HEADLINE,
                   "converged": head["converged"], "cg_iterations": head["cg_iterations"],
                   "mean_log_ratio": head["mean_log_ratio"],
                   "schedule": {"block_mr_steps": mixed.block_mr_steps, "inner": mixed.inner,
                                "middle": mixed.middle}},
        "fp64_estimates_per_s": None if fp64_rate is None else round(fp64_rate, 4),
        "speedup_vs_fp64": None if fp64_rate is None else round(value / fp64_rate, 3),
        "max_abs_sample_diff_vs_fp64": head.get("max_abs_sample_diff_vs_fp64"),
        "roofline": roof,
        "whole_estimate_roofline": whole,
        "wilson8_dd16": dd8,
        "batched_proposals": batch,
        "large_lattices": large,
        "block_determinants": bdet,
        "recursive_dd": rdd,
        "filter": filt,
        "clover_16": clov,
        "cg_forms": forms,
        "slab_halo": slab,
        "exact_acceptance": acc,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
