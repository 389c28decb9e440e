"""GPU parity of the global solvers and of the stochastic log-det-ratio
samples against the FP64 oracle (paper Sec. 4); C-ABI error paths."""
import numpy as np
import pytest

import oracle
from paper_1112_1243_amd import synth
from tests.gpu_util import dev, host, rel, say, torch_cuda

pytestmark = pytest.mark.gpu


def _setup(L, B, scale, seed, bc=(1, 1, 1, 1)):
    torch_cuda()
    from paper_1112_1243_amd import wdr
    say("setup", L, B, scale, seed)
    lat = oracle.Lattice(L, B, bc)
    ctx = wdr.Context(L, B, bc)
    U = synth.gauge_field(L, scale, seed)
    return wdr, lat, ctx, U


@pytest.mark.parametrize("solver,kappa,scale,inner,middle,bc", [
    (0, 0.135, 0.5, 1, 0, (1, 1, 1, 1)), (1, 0.135, 0.5, 1, 0, (1, 1, 1, 1)), (1, 0.150, 0.25, 1, 0, (1, 1, 1, 1)),
    (1, 0.150, 0.25, 0, 0, (1, 1, 1, 1)), (0, 0.135, 0.5, 0, 0, (1, 1, 1, 1)), (0, 0.135, 0.5, 2, 0, (1, 1, 1, 1)),
    # FP16 even-odd CG: two levels and three levels, periodic and antiperiodic time
    (1, 0.150, 0.25, 2, 0, (1, 1, 1, 1)), (1, 0.150, 0.25, 2, 1, (1, 1, 1, 1)),
    (1, 0.155, 0.2, 2, 1, (1, 1, 1, -1)), (1, 0.135, 0.5, 2, 1, (1, -1, 1, -1)),
])
def test_solve_true_residual(solver, kappa, scale, inner, middle, bc):
    """The oracle's own stencil checks the GPU solution: ||b - D x|| <= 1e-10 ||b||
    (CGNE with inner FP32: FP32 CG steps under FP64 reliable updates; inner
    FP16: FP16 CG steps, with an FP32 middle level when middle = F32)."""
    wdr, lat, ctx, U = _setup((8, 8, 8, 8), (4, 4, 4, 4), scale, 201, bc)
    b = synth.spinor(lat.L, 202)
    gU = ctx.gauge(dev(U))
    x, info = ctx.solve(gU, kappa, dev(b), wdr.default_params(solver=solver, inner=inner, middle=middle,
                                                              max_iter=20000))
    x = host(x)
    r = np.linalg.norm(b - oracle.apply_D(lat, U, kappa, x)) / np.linalg.norm(b)
    say("solve", solver, kappa, info.as_dict(), "oracle residual", r)
    assert info.converged and r <= 1.05e-10
    want, _, _, _ = oracle.solve(lat, U, kappa, b, tol=1e-13)
    assert rel(x, want) < 1e-8
    del gU
    ctx.close()


def _pair(lat, U, scale, seed, rule):
    if rule == "bernoulli":
        mask = synth.bernoulli_links(lat.L, 0.1, seed)
    elif rule == "active":
        mask = oracle.active_links(lat)
    else:
        mask = np.zeros((lat.V, 4), bool)
    return synth.redraw(U, mask, scale, seed)


# solver settings of the parity cases: (solver, inner, middle)
SOLVERS = {
    "fgcr_f32": (0, 1, 0),   # FGCR(16) + FP32 Schwarz, FP32 block MR
    "fgcr_f16": (0, 2, 0),   # FGCR(16) + FP16 Schwarz, FP16 block MR
    "cgne_f64": (1, 0, 0),   # FP64 everywhere
    "cgne_f32": (1, 1, 0),   # FP32 CG iterations, FP64 reliable updates, FP32 block MR
    "cgne_f16": (1, 2, 0),   # FP16 CG iterations and block MR under FP64 reliable updates
    "cgne_f16_3": (1, 2, 1),  # three levels: FP16 CG steps, FP32 middle updates, FP64 outer updates
}


def _params(wdr, name, **kw):
    solver, inner, middle = SOLVERS[name]
    return wdr.default_params(solver=solver, inner=inner, middle=middle, max_iter=20000, **kw)


@pytest.mark.parametrize("op,kind,L,B,kappa,scale,rule,N,K,solver", [
    # 4^4 lattice, kappa 0.12, Z2 noise, Bernoulli(0.1) proposal (the small workload)
    (oracle.OP_FULL, oracle.NOISE_Z2, (4, 4, 4, 4), (2, 2, 2, 2), 0.12, 0.3, "bernoulli", 3, 2, "cgne_f32"),
    (oracle.OP_FULL, oracle.NOISE_GAUSS, (4, 4, 4, 4), (2, 2, 2, 2), 0.12, 0.3, "bernoulli", 2, 2, "fgcr_f32"),
    # 8^4 lattice with 16 blocks of 4^4, active links redrawn, Gaussian noise
    (oracle.OP_SCHUR, oracle.NOISE_GAUSS, (8, 8, 8, 8), (4, 4, 4, 4), 0.135, 0.5, "active", 2, 1, "fgcr_f32"),
    (oracle.OP_BLOCKS, oracle.NOISE_GAUSS, (8, 8, 8, 8), (4, 4, 4, 4), 0.135, 0.5, "active", 2, 1, "fgcr_f32"),
    (oracle.OP_SCHUR, oracle.NOISE_GAUSS, (8, 8, 8, 8), (4, 4, 4, 4), 0.150, 0.25, "active", 1, 1, "cgne_f32"),
    # FP16 Schwarz preconditioner and FP16 block solves inside the FP64 outer solves
    (oracle.OP_SCHUR, oracle.NOISE_GAUSS, (8, 8, 8, 8), (4, 4, 4, 4), 0.135, 0.5, "active", 2, 1, "fgcr_f16"),
    (oracle.OP_BLOCKS, oracle.NOISE_GAUSS, (8, 8, 8, 8), (4, 4, 4, 4), 0.135, 0.5, "active", 1, 1, "fgcr_f16"),
    # the solver form of the 16^4 and 32^4 workloads (CGNE with FP16 inner
    # precision) on the subcritical and the supercritical kappa
    (oracle.OP_SCHUR, oracle.NOISE_GAUSS, (8, 8, 8, 8), (4, 4, 4, 4), 0.135, 0.5, "active", 2, 1, "cgne_f16"),
    (oracle.OP_SCHUR, oracle.NOISE_GAUSS, (8, 8, 8, 8), (4, 4, 4, 4), 0.155, 0.2, "active", 2, 1, "cgne_f16"),
    (oracle.OP_BLOCKS, oracle.NOISE_GAUSS, (8, 8, 8, 8), (4, 4, 4, 4), 0.155, 0.2, "active", 2, 1, "cgne_f16"),
    (oracle.OP_FULL, oracle.NOISE_GAUSS, (8, 8, 8, 8), (4, 4, 4, 4), 0.150, 0.25, "active", 2, 1, "cgne_f16"),
    (oracle.OP_SCHUR, oracle.NOISE_GAUSS, (8, 8, 8, 8), (4, 4, 4, 4), 0.155, 0.2, "active", 2, 2, "cgne_f16_3"),
    (oracle.OP_FULL, oracle.NOISE_Z2, (8, 8, 8, 8), (4, 4, 4, 4), 0.135, 0.5, "bernoulli", 3, 1, "cgne_f16_3"),
])
def test_samples_match_oracle(op, kind, L, B, kappa, scale, rule, N, K, solver):
    """s_{i,k} within 1e-8 absolute of the oracle at solver residual 1e-10."""
    wdr, lat, ctx, U = _setup(L, B, scale, 1112124300 + len(L) * L[0])
    Up = _pair(lat, U, scale, 303, rule)
    gU, gUp = ctx.gauge(dev(U)), ctx.gauge(dev(Up))
    seed = 99
    p = _params(wdr, solver)
    s, lr, info = ctx.logdet_ratio(gU, gUp, kappa, op, N, K, kind, seed, p)
    want, lr_want = oracle.logdet_ratio(lat, U, Up, kappa, op, N, K, kind, seed)
    err = np.abs(s - want).max()
    say("samples op", op, solver, "max |ds|", err, "log R", lr, lr_want, info.as_dict())
    assert s.shape == want.shape
    assert info.converged
    assert err < 1e-8
    # the library sums the per-block log ratios of BLOCKS
    assert abs(lr - float(np.sum(lr_want))) < 1e-8 * max(1, s.size)
    del gU, gUp
    ctx.close()


@pytest.mark.parametrize("solver,form,kappa,scale", [("cgne_f16", 2, 0.155, 0.2), ("cgne_f32", 2, 0.155, 0.2),
                                                     ("fgcr_f16", 2, 0.135, 0.5), ("cgne_f16", 1, 0.155, 0.2)])
def test_dd_samples_match_oracle(solver, form, kappa, scale):
    """The DD estimate (every block ratio and the Schur ratio of one
    proposal in one call) against the oracle's BLOCKS and SCHUR samples,
    with the block-MR launch form forced: two blocks per CU (the form the
    block solves of the 16^4 and 32^4 estimates take by their size) or one.
    FGCR + Schwarz runs at the subcritical kappa (it stalls above 1/8)."""
    wdr, lat, ctx, U = _setup((8, 8, 8, 8), (4, 4, 4, 4), scale, 1112124334)
    ctx.set_mr_form(form)
    Up = _pair(lat, U, scale, 311, "active")
    gU, gUp = ctx.gauge(dev(U)), ctx.gauge(dev(Up))
    N = 2
    s, lr, info = ctx.logdet_ratio(gU, gUp, kappa, wdr.OP_DD, N, 1, wdr.NOISE_GAUSS, 43, _params(wdr, solver))
    wb, lb = oracle.logdet_ratio(lat, U, Up, kappa, oracle.OP_BLOCKS, N, 1, oracle.NOISE_GAUSS, 43)
    ws, ls = oracle.logdet_ratio(lat, U, Up, kappa, oracle.OP_SCHUR, N, 1, oracle.NOISE_GAUSS, 43)
    eb, es = np.abs(s[..., :-1] - wb).max(), np.abs(s[..., -1] - ws).max()
    say("dd", solver, "form", form, "max |ds| blocks", eb, "schur", es, info.as_dict())
    assert info.converged and eb < 1e-8 and es < 1e-8
    assert abs(lr - (float(np.sum(lb)) + float(ls))) < 1e-8 * s.size
    del gU, gUp
    ctx.close()


def test_block_staged_stencil_in_estimates():
    """SCHUR and BLOCKS samples at 8^4 with the block-staged stencils forced
    (D, the Dirichlet blocks and, in the even-odd CGNE, both halves with and
    without gamma_5; batched systems, compaction lists) match the oracle as
    with the default choice."""
    wdr, lat, ctx, U = _setup((8, 8, 8, 8), (4, 4, 4, 4), 0.5, 1112124332)
    ctx.set_stencil(wdr.STENCIL_BLK)
    Up = _pair(lat, U, 0.5, 307, "active")
    gU, gUp = ctx.gauge(dev(U)), ctx.gauge(dev(Up))
    for op, solver in ((wdr.OP_SCHUR, wdr.SOLVER_FGCR_SAP), (wdr.OP_BLOCKS, wdr.SOLVER_FGCR_SAP),
                       (wdr.OP_SCHUR, wdr.SOLVER_CGNE)):
        s, lr, info = ctx.logdet_ratio(gU, gUp, 0.135, op, 2, 1, wdr.NOISE_GAUSS, 41,
                                       wdr.default_params(solver=solver))
        want, _ = oracle.logdet_ratio(lat, U, Up, 0.135, op, 2, 1, oracle.NOISE_GAUSS, 41)
        say("blk stencil op", op, "solver", solver, "max |ds|", np.abs(s - want).max())
        assert info.converged and np.abs(s - want).max() < 1e-8
    del gU, gUp
    ctx.close()


def test_estimates_are_bit_reproducible():
    """Two DD estimates with the same key give the same samples bit for bit:
    the reductions run in a fixed order, and the host's scheduling decisions
    (lagged flag reads, convergence forecasts, compaction) only decide which
    no-op steps are queued."""
    wdr, lat, ctx, U = _setup((8, 8, 8, 8), (4, 4, 4, 4), 0.5, 1112124333)
    Up = _pair(lat, U, 0.5, 309, "active")
    gU, gUp = ctx.gauge(dev(U)), ctx.gauge(dev(Up))
    p = wdr.default_params()
    a, la, ia = ctx.logdet_ratio(gU, gUp, 0.135, wdr.OP_DD, 4, 1, wdr.NOISE_GAUSS, 23, p)
    b, lb, ib = ctx.logdet_ratio(gU, gUp, 0.135, wdr.OP_DD, 4, 1, wdr.NOISE_GAUSS, 23, p)
    assert ia.converged and ib.converged
    assert np.array_equal(a, b) and la == lb
    del gU, gUp
    ctx.close()


def test_dd_equals_blocks_and_schur():
    """The DD estimate (block ratios and Schur ratio of one proposal in one
    call, run concurrently on one path) gives the samples of the separate
    BLOCKS and SCHUR calls with the same key, and their summed log ratio."""
    wdr, lat, ctx, U = _setup((8, 8, 8, 8), (4, 4, 4, 4), 0.5, 305)
    Up = _pair(lat, U, 0.5, 306, "active")
    gU, gUp = ctx.gauge(dev(U)), ctx.gauge(dev(Up))
    for inner in (wdr.F32, wdr.F16):
        p = wdr.default_params(inner=inner)
        sd, lrd, info = ctx.logdet_ratio(gU, gUp, 0.135, wdr.OP_DD, 3, 1, wdr.NOISE_GAUSS, 17, p)
        sb, lrb, _ = ctx.logdet_ratio(gU, gUp, 0.135, wdr.OP_BLOCKS, 3, 1, wdr.NOISE_GAUSS, 17, p)
        ss, lrs, _ = ctx.logdet_ratio(gU, gUp, 0.135, wdr.OP_SCHUR, 3, 1, wdr.NOISE_GAUSS, 17, p)
        say("dd", inner, np.abs(sd[..., :-1] - sb).max(), np.abs(sd[..., -1] - ss).max(), lrd, lrb + lrs)
        assert sd.shape == (3, 1, ctx.nblocks + 1) and info.converged
        assert np.abs(sd[..., :-1] - sb).max() < 1e-12 and np.abs(sd[..., -1] - ss).max() < 1e-12
        assert abs(lrd - (lrb + lrs)) < 1e-10
    del gU, gUp
    ctx.close()


def test_autotune_keeps_results():
    """The tuned schedule (Schwarz depth, block-solve rounds) changes time
    only: samples stay within solver accuracy of the default schedule; the
    second call returns the cached choice."""
    wdr, lat, ctx, U = _setup((8, 8, 8, 8), (4, 4, 4, 4), 0.5, 307)
    Up = _pair(lat, U, 0.5, 308, "active")
    gU, gUp = ctx.gauge(dev(U)), ctx.gauge(dev(Up))
    p0 = wdr.default_params()
    tuned, secs = ctx.autotune(gU, gUp, 0.135, wdr.OP_DD, 4, 1, wdr.NOISE_GAUSS, 21, p0)
    say("tuned", tuned.sap_cycles, tuned.mr_steps, tuned.block_mr_steps, secs)
    assert secs > 0 and tuned.sap_cycles >= 1 and tuned.mr_steps >= 1 and tuned.block_mr_steps >= 1
    again, _ = ctx.autotune(gU, gUp, 0.135, wdr.OP_DD, 4, 1, wdr.NOISE_GAUSS, 21, p0)
    assert (again.sap_cycles, again.mr_steps, again.block_mr_steps) == \
        (tuned.sap_cycles, tuned.mr_steps, tuned.block_mr_steps)
    s0, l0, _ = ctx.logdet_ratio(gU, gUp, 0.135, wdr.OP_DD, 4, 1, wdr.NOISE_GAUSS, 22, p0)
    s1, l1, info = ctx.logdet_ratio(gU, gUp, 0.135, wdr.OP_DD, 4, 1, wdr.NOISE_GAUSS, 22, tuned)
    assert info.converged and np.abs(s1 - s0).max() < 1e-8
    del gU, gUp
    ctx.close()


def test_unchanged_field_gives_zero():
    wdr, lat, ctx, U = _setup((8, 8, 8, 8), (4, 4, 4, 4), 0.5, 304)
    gU = ctx.gauge(dev(U))
    s, lr, info = ctx.logdet_ratio(gU, gU, 0.135, wdr.OP_SCHUR, 1, 2, wdr.NOISE_GAUSS, 5, wdr.default_params())
    assert np.abs(s).max() < 1e-8
    del gU
    ctx.close()


def test_abi_errors():
    torch_cuda()
    from paper_1112_1243_amd import wdr
    with pytest.raises(wdr.WdrError) as e:
        wdr.Context((8, 8, 8, 8), (3, 4, 4, 4))
    assert e.value.status == wdr.EINVAL
    with pytest.raises(wdr.WdrError):
        wdr.Context((8, 8, 8, 8), (4, 4, 4, 4), bc=(1, 1, 1, 2))
    ctx = wdr.Context((8, 8, 8, 8), (4, 4, 4, 4))
    other = wdr.Context((8, 8, 8, 8), (4, 4, 4, 4))
    U = synth.gauge_field((8, 8, 8, 8), 0.5, 1)
    gU = other.gauge(dev(U))
    psi = dev(synth.spinor((8, 8, 8, 8), 2))
    with pytest.raises(wdr.WdrError) as e:
        ctx.apply_D(gU, 0.13, psi)
    assert e.value.status == wdr.ESTATE
    gU2 = ctx.gauge(dev(U))
    with pytest.raises(wdr.WdrError) as e:
        ctx.apply_D(gU2, -0.1, psi)
    assert e.value.status == wdr.EINVAL
    # one iteration cannot reach 1e-10: ENOCONV with the info filled in
    x, info = ctx.solve(gU2, 0.135, psi, wdr.default_params(max_iter=1), allow_noconv=True)
    assert info.converged == 0 and info.iters == 1 and 0 < info.true_rel_resid < 1
    with pytest.raises(wdr.WdrError) as e:
        ctx.solve(gU2, 0.135, psi, wdr.default_params(max_iter=1))
    assert e.value.status == wdr.ENOCONV
    for bad in (dict(update_every=0), dict(update_every=65), dict(graph=2), dict(middle=2),
                dict(middle=wdr.F32, inner=wdr.F32), dict(middle=wdr.F32, inner=wdr.F16, solver=wdr.SOLVER_FGCR_SAP)):
        kw = dict(solver=wdr.SOLVER_CGNE)
        kw.update(bad)
        with pytest.raises(wdr.WdrError) as e:
            ctx.solve(gU2, 0.135, psi, wdr.default_params(**kw))
        assert e.value.status == wdr.EINVAL
    # blocks of 8^4 are too large for the block solver
    big = wdr.Context((16, 16, 16, 16), (8, 8, 8, 8))
    gB = big.gauge(dev(synth.unit_gauge((16, 16, 16, 16))))
    with pytest.raises(wdr.WdrError) as e:
        big.sap(gB, 0.1, dev(np.zeros((big.V, 4, 3), complex)), wdr.default_params())
    assert e.value.status == wdr.EINVAL
    del gU, gU2, gB
    for c in (ctx, other, big):
        c.close()


def test_non_finite_inputs_end_solves():
    """A NaN in the right-hand side ends CGNE, FGCR and the block solver at
    once with ENOCONV (no run to the iteration cap, and a NaN block is never
    counted as converged)."""
    import time
    wdr, lat, ctx, U = _setup((8, 8, 8, 8), (4, 4, 4, 4), 0.5, 1112124340)
    gU = ctx.gauge(dev(U))
    b = synth.spinor(lat.L, 341)
    b[37, 1, 2] = np.nan
    for params in (wdr.default_params(solver=wdr.SOLVER_CGNE, inner=wdr.F32, max_iter=20000),
                   wdr.default_params(solver=wdr.SOLVER_FGCR_SAP, max_iter=20000)):
        t0 = time.perf_counter()
        x, info = ctx.solve(gU, 0.135, dev(b), params, allow_noconv=True)
        dt = time.perf_counter() - t0
        say("NaN rhs solver", params.solver, info.as_dict(), "%.3f s" % dt)
        assert info.converged == 0 and info.iters <= 1 and dt < 5
    with pytest.raises(wdr.WdrError) as e:
        ctx.block_solve(gU, 0.135, 2, dev(b), wdr.default_params(inner=wdr.F32))
    assert e.value.status == wdr.ENOCONV
    del gU
    ctx.close()
