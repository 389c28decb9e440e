"""GPU parity of the persistent form of the CG steps (one cooperative launch
per period of update_every steps, phases separated by grid-wide barriers)
against the FP64 oracle, and against the launch-per-phase form (paper
Sec. 4: the inversions, one for each factor of eq. param)."""
import numpy as np
import pytest

import oracle
from paper_1112_1243_amd import synth
from tests.gpu_util import dev, host, rel, say, torch_cuda

pytestmark = pytest.mark.gpu


def _setup(L, B, scale, seed, bc=(1, 1, 1, 1)):
    torch_cuda()
    from paper_1112_1243_amd import wdr
    say("setup", L, B, scale, seed, bc)
    lat = oracle.Lattice(L, B, bc)
    ctx = wdr.Context(L, B, bc)
    U = synth.gauge_field(L, scale, seed)
    return wdr, lat, ctx, U


@pytest.mark.parametrize("inner,kappa,scale,bc", [(1, 0.135, 0.5, (1, 1, 1, 1)), (0, 0.150, 0.25, (1, 1, 1, -1)),
                                                  (1, 0.155, 0.2, (1, -1, 1, -1))])
def test_persistent_solve_true_residual(inner, kappa, scale, bc):
    """The oracle's stencil checks the persistent-form solution
    (||b - D x|| <= 1.05e-10 ||b||); it is within 1e-8 of the oracle's
    solution and of the launch form's, with about the same iterations."""
    wdr, lat, ctx, U = _setup((8, 8, 8, 8), (4, 4, 4, 4), scale, 601, bc)
    b = synth.spinor(lat.L, 602)
    gU = ctx.gauge(dev(U))
    p = wdr.default_params(solver=1, inner=inner, max_iter=20000)
    xl, il = ctx.solve(gU, kappa, dev(b), p)
    ctx.set_cg_form(wdr.CG_PERSISTENT)
    x, info = ctx.solve(gU, kappa, dev(b), p)
    x, xl = host(x), host(xl)
    r = np.linalg.norm(b - oracle.apply_D(lat, U, kappa, x)) / np.linalg.norm(b)
    say("persistent solve", inner, kappa, info.as_dict(), "launches", il.as_dict(), "oracle residual", r)
    assert info.converged and r <= 1.05e-10
    want, _, _, _ = oracle.solve(lat, U, kappa, b, tol=1e-13)
    assert rel(x, want) < 1e-8 and rel(x, xl) < 1e-8
    assert abs(info.iters - il.iters) <= max(8, il.iters // 10)
    del gU
    ctx.close()


@pytest.mark.parametrize("op,N,K", [("FULL", 4, 2), ("SCHUR", 2, 1)])
def test_persistent_samples_match_oracle(op, N, K):
    """Batched samples (systems that converge at different steps, so the
    launches shrink to the live systems on the way) with the persistent CG
    steps, within 1e-8 of the oracle's."""
    wdr, lat, ctx, U = _setup((8, 8, 8, 8), (4, 4, 4, 4), 0.5, 603)
    Up = synth.redraw(U, oracle.active_links(lat), 0.5, 604)
    gU, gUp = ctx.gauge(dev(U)), ctx.gauge(dev(Up))
    ctx.set_cg_form(wdr.CG_PERSISTENT)
    kappa = 0.135
    p = wdr.default_params(solver=1, inner=1, max_iter=20000)
    wop, oop = getattr(wdr, "OP_" + op), getattr(oracle, "OP_" + op)
    s, lr, info = ctx.logdet_ratio(gU, gUp, kappa, wop, N, K, wdr.NOISE_GAUSS, 81, p)
    want, lr_want = oracle.logdet_ratio(lat, U, Up, kappa, oop, N, K, oracle.NOISE_GAUSS, 81)
    err = np.abs(s - want).max()
    say("persistent", op, "max |ds|", err, "log R", lr, float(np.sum(lr_want)), info.as_dict())
    assert info.converged and err < 1e-8
    assert abs(lr - float(np.sum(lr_want))) < 1e-8 * s.size
    del gU, gUp
    ctx.close()


def test_persistent_16x16x16x16_full_samples():
    """16^4 FULL samples (two systems, 256 blocks each) with the persistent
    CG steps within 1e-8 of the oracle's."""
    wdr, lat, ctx, U = _setup((16, 16, 16, 16), (4, 4, 4, 4), 0.5, 605)
    Up = synth.redraw(U, oracle.active_links(lat), 0.5, 606)
    gU, gUp = ctx.gauge(dev(U)), ctx.gauge(dev(Up))
    ctx.set_cg_form(wdr.CG_PERSISTENT)
    kappa = 0.13
    p = wdr.default_params(solver=1, inner=1, max_iter=20000)
    s, lr, info = ctx.logdet_ratio(gU, gUp, kappa, wdr.OP_FULL, 1, 2, wdr.NOISE_GAUSS, 83, p)
    want, _ = oracle.logdet_ratio(lat, U, Up, kappa, oracle.OP_FULL, 1, 2, oracle.NOISE_GAUSS, 83)
    err = np.abs(s - want).max()
    say("persistent 16^4 FULL max |ds|", err, info.as_dict())
    assert info.converged and err < 1e-8
    del gU, gUp
    ctx.close()


def test_persistent_batch_and_fallbacks():
    """A batch over two contexts with the persistent form (run one context
    after the other) equals the launch form's batch to 1e-9; the form does
    not apply to a clover operator (its solves keep the launches, checked
    by the oracle); an unknown form is refused."""
    torch_cuda()
    from paper_1112_1243_amd import wdr
    ctxs, gauges, props = [], [], []
    for L, seed in (((8, 8, 8, 8), 607), ((8, 8, 8, 12), 608)):
        ctx = wdr.Context(L, (4, 4, 4, 4))
        lat = oracle.Lattice(L, (4, 4, 4, 4))
        U = synth.gauge_field(L, 0.5, seed)
        Up = synth.redraw(U, oracle.active_links(lat), 0.5, seed + 100)
        g0, g1 = ctx.gauge(dev(U)), ctx.gauge(dev(Up))
        ctxs.append(ctx)
        gauges += [g0, g1]
        props.append((ctx, g0, g1, 0.135, seed))
    p = wdr.default_params(solver=1, inner=1, max_iter=20000)
    s0, l0, _ = wdr.logdet_ratio_batch(props, wdr.OP_FULL, 2, 1, wdr.NOISE_GAUSS, p)
    for c in ctxs:
        c.set_cg_form(wdr.CG_PERSISTENT)
    s1, l1, info = wdr.logdet_ratio_batch(props, wdr.OP_FULL, 2, 1, wdr.NOISE_GAUSS, p)
    d = max(float(np.abs(np.asarray(a) - np.asarray(b)).max()) for a, b in zip(s0, s1))
    say("persistent batch max |ds| vs launches", d, info.as_dict())
    assert info.converged and d < 1e-9
    # clover: the launches carry it
    wdr2, lat, ctx, U = _setup((8, 8, 8, 8), (4, 4, 4, 4), 0.5, 609)
    ctx.set_cg_form(wdr.CG_PERSISTENT)
    kappa, csw = 0.135, 1.7
    gC = ctx.gauge(dev(U), csw, kappa)
    b = synth.spinor(lat.L, 610)
    x, info = ctx.solve(gC, kappa, dev(b), p)
    T = oracle.clover_term(lat, U, csw, kappa)
    r = np.linalg.norm(b - oracle.apply_D(lat, U, kappa, host(x), T)) / np.linalg.norm(b)
    say("persistent form, clover solve", info.as_dict(), r)
    assert info.converged and r <= 1.05e-10
    with pytest.raises(wdr.WdrError) as e:
        ctx.set_cg_form(7)
    assert e.value.status == wdr.EINVAL
    del gauges, gC
    for c in ctxs:
        c.close()
    ctx.close()
