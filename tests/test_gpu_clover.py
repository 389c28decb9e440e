"""GPU parity of the clover (Sheikholeslami-Wohlert) term against the FP64
oracle: the term itself and its inverse, D / D_b / D_ee with the term on
both stencil forms and on a general block shape, CGNE solves with FP64 and
FP32 inner levels, Dirichlet block solves and the Schur complement, FULL,
BLOCKS, SCHUR and DD samples; the C-ABI error paths of the calls that do
not take the term (Sec. 3: active links for Wilson fermions with clover
term, eqs. domdec and ddfactor; Sec. 7: the clover action)."""
import numpy as np
import pytest

import oracle
from paper_1112_1243_amd import synth
from tests.gpu_util import dev, host, rel, say, torch_cuda

pytestmark = pytest.mark.gpu

CSW = 1.7


def _setup(L, B, scale, seed, bc=(1, 1, 1, -1)):
    torch_cuda()
    from paper_1112_1243_amd import wdr
    say("setup", L, B, scale, seed, bc)
    lat = oracle.Lattice(L, B, bc)
    ctx = wdr.Context(L, B, bc)
    U = synth.gauge_field(L, scale, seed)
    return wdr, lat, ctx, U


GEOMS = [((8, 8, 8, 8), (4, 4, 4, 4)), ((4, 4, 8, 8), (2, 2, 4, 4))]


@pytest.mark.parametrize("L,B", GEOMS)
def test_clover_term_and_inverse(L, B):
    """A = 1 + T site by site within 1e-13 of the oracle's definition, and
    A^-1 within 1e-12 of numpy's inverse of the oracle's A."""
    wdr, lat, ctx, U = _setup(L, B, 0.7, 501)
    kappa = 0.13
    gU = ctx.gauge(dev(U), CSW, kappa)
    A = host(ctx.clover_field(gU))
    Ainv = host(ctx.clover_field(gU, inverse=True))
    want = np.eye(12)[None] + oracle.clover_term(lat, U, CSW, kappa)
    ea, ei = rel(A, want), rel(Ainv, np.linalg.inv(want))
    say("clover A", ea, "A^-1", ei)
    assert ea < 1e-13 and ei < 1e-12
    assert np.abs(want - np.eye(12)[None]).max() > 0.05
    del gU
    ctx.close()


@pytest.mark.parametrize("L,B", GEOMS)
@pytest.mark.parametrize("stencil", [1, 2])
def test_clover_operators(L, B, stencil):
    """D, D_b (both colours) and the block hops with the clover term in FP64
    (1e-13) and FP32 (2e-6) against the oracle, with the direction-parallel
    (1) and the block-staged (2) stencil forced (the general block shape has
    one form)."""
    wdr, lat, ctx, U = _setup(L, B, 0.6, 502)
    ctx.set_stencil(stencil)
    kappa = 0.14
    T = oracle.clover_term(lat, U, CSW, kappa)
    gU = ctx.gauge(dev(U), CSW, kappa)
    psi = synth.spinor(lat.L, 503)
    for prec, tol in ((wdr.F64, 1e-13), (wdr.F32, 2e-6)):
        e = rel(host(ctx.apply_D(gU, kappa, dev(psi), prec)), oracle.apply_D(lat, U, kappa, psi, T))
        say("D", prec, e)
        assert e < tol
        for colour in (0, 1, 2):
            e = rel(host(ctx.apply_Dblock(gU, kappa, dev(psi), colour, prec)),
                    oracle.apply_Dblock(lat, U, kappa, psi, colour, T))
            say("D_b", colour, prec, e)
            assert e < tol
        e = rel(host(ctx.apply_Dhop(gU, kappa, dev(psi), 1, prec)), oracle.apply_Dhop(lat, U, kappa, psi, 1))
        assert e < tol
    # the term matters
    assert rel(oracle.apply_D(lat, U, kappa, psi), oracle.apply_D(lat, U, kappa, psi, T)) > 1e-2
    del gU
    ctx.close()


def _dee_oracle(lat, U, kappa, T, psi, blocked):
    """A_ee psi_e - kappa^2 H_eo A_oo^-1 H_oe psi_e from the oracle's D (or
    D_b) with the clover term on fields supported on one parity, and numpy's
    inverse of the oracle's A on the odd sites."""
    _, _, par = lat.maps()
    ev = par == 0
    op = (lambda v: oracle.apply_Dblock(lat, U, kappa, v, 2, T)) if blocked else \
        (lambda v: oracle.apply_D(lat, U, kappa, v, T))
    pe = psi.copy()
    pe[~ev] = 0
    t = op(pe)                       # [A_ee psi_e ; -kappa H_oe psi_e]
    odd = t.copy()
    odd[ev] = 0
    Ainv = np.linalg.inv(np.eye(12)[None] + T)
    odd = np.einsum("xij,xj->xi", Ainv, odd.reshape(lat.V, 12)).reshape(lat.V, 4, 3)
    odd[ev] = 0
    u = op(odd)                      # even sites: -kappa H_eo A_oo^-1 (-kappa H_oe psi_e)
    out = t - u
    out[~ev] = 0
    return out


@pytest.mark.parametrize("blocked", [False, True])
def test_clover_even_odd_operator(blocked):
    wdr, lat, ctx, U = _setup((8, 8, 8, 8), (4, 4, 4, 4), 0.6, 504)
    kappa = 0.14
    T = oracle.clover_term(lat, U, CSW, kappa)
    gU = ctx.gauge(dev(U), CSW, kappa)
    psi = synth.spinor(lat.L, 505)
    e = rel(host(ctx.apply_Dee(gU, kappa, dev(psi), blocked)), _dee_oracle(lat, U, kappa, T, psi, blocked))
    say("D_ee clover blocked", blocked, e)
    assert e < 1e-12
    del gU
    ctx.close()


@pytest.mark.parametrize("inner,kappa,scale", [(0, 0.135, 0.5), (1, 0.135, 0.5), (1, 0.125, 0.3)])
def test_clover_solve(inner, kappa, scale):
    """Even-odd CGNE with the clover term: the oracle's clover operator
    checks the true residual (<= 1.05e-10) and the solution is within 1e-8
    of the oracle's own CGNE solution."""
    wdr, lat, ctx, U = _setup((8, 8, 8, 8), (4, 4, 4, 4), scale, 506)
    T = oracle.clover_term(lat, U, CSW, kappa)
    gU = ctx.gauge(dev(U), CSW, kappa)
    b = synth.spinor(lat.L, 507)
    x, info = ctx.solve(gU, kappa, dev(b), wdr.default_params(solver=1, inner=inner, max_iter=20000))
    x = host(x)
    r = np.linalg.norm(b - oracle.apply_D(lat, U, kappa, x, T)) / np.linalg.norm(b)
    say("clover solve inner", inner, kappa, info.as_dict(), "oracle residual", r)
    assert info.converged and r <= 1.05e-10
    want, _, _, _ = oracle.solve(lat, U, kappa, b, tol=1e-13, clov=T)
    assert rel(x, want) < 1e-8
    del gU
    ctx.close()


@pytest.mark.parametrize("inner,kind,N,K", [(1, 1, 2, 2), (0, 0, 3, 1)])
def test_clover_full_samples(inner, kind, N, K):
    """FULL samples of the clover operator (CGNE, FP32 / FP64 inner level)
    within 1e-8 of the oracle's, over a path whose interior points carry
    clover terms the library builds itself."""
    wdr, lat, ctx, U = _setup((8, 8, 8, 8), (4, 4, 4, 4), 0.5, 508)
    kappa = 0.135
    Up = synth.redraw(U, oracle.active_links(lat), 0.5, 509)
    gU, gUp = ctx.gauge(dev(U), CSW, kappa), ctx.gauge(dev(Up), CSW, kappa)
    p = wdr.default_params(solver=1, inner=inner, max_iter=20000)
    s, lr, info = ctx.logdet_ratio(gU, gUp, kappa, wdr.OP_FULL, N, K, kind, 77, p)
    want, lr_want = oracle.logdet_ratio(lat, U, Up, kappa, oracle.OP_FULL, N, K, kind, 77, csw=CSW)
    err = np.abs(s - want).max()
    say("clover FULL samples", inner, "max |ds|", err, "log R", lr, lr_want, info.as_dict())
    assert info.converged and err < 1e-8 and abs(lr - lr_want) < 1e-8 * s.size
    # without the term the samples differ
    plain, _ = oracle.logdet_ratio(lat, U, Up, kappa, oracle.OP_FULL, 1, 1, kind, 77)
    assert abs(plain[0, 0] - want[0, 0]) > 1e-3
    del gU, gUp
    ctx.close()


@pytest.mark.parametrize("L,B", GEOMS)
@pytest.mark.parametrize("inner", [0, 1])
def test_clover_block_solve(L, B, inner):
    """Dirichlet block solves with the clover term (black, white, all
    blocks; FP64 / FP32 CG iterations inside FP64 defect correction): every
    block's residual, taken with the oracle's block operator, within 1e-13 of
    its right-hand side, and the solution within 1e-11 of the oracle's."""
    wdr, lat, ctx, U = _setup(L, B, 0.6, 514)
    kappa = 0.14
    T = oracle.clover_term(lat, U, CSW, kappa)
    gU = ctx.gauge(dev(U), CSW, kappa)
    b = synth.spinor(lat.L, 515)
    bid, col, _ = lat.maps()
    p = wdr.default_params(inner=inner)
    for colour in (0, 1, 2):
        x, info = ctx.block_solve(gU, kappa, colour, dev(b), p)
        x = host(x)
        sel = np.ones(lat.V, bool) if colour == 2 else col == colour
        bb = b.copy()
        bb[~sel] = 0
        assert np.all(x[~sel] == 0)
        r = bb - oracle.apply_Dblock(lat, U, kappa, x, colour, T)
        worst = max(np.linalg.norm(r[bid == k]) / np.linalg.norm(bb[bid == k]) for k in np.unique(bid[sel]))
        want, _, _, _ = oracle.solve(lat, U, kappa, bb, "block", colour, tol=1e-14, clov=T)
        say("clover block solve", inner, colour, info.as_dict(), "worst block", worst, "vs oracle", rel(x, want))
        assert info.converged and info.true_rel_resid <= 1e-13 and worst <= 1.05e-13
        assert rel(x, want) < 1e-11
    # the term matters: the plain block solution differs
    plain, _, _, _ = oracle.solve(lat, U, kappa, b, "block", 2, tol=1e-14)
    assert rel(x, plain) > 1e-2
    del gU
    ctx.close()


@pytest.mark.parametrize("form", ["one", "two"])
def test_clover_f16_block_solve(form):
    """Dirichlet block solves with the clover term and an FP16 inner level:
    the FP16 block MR with A_ee - 1 and A_oo^-1 in LDS inside FP64 defect
    correction, in both launch forms (one or two blocks per CU).  Every
    block's residual, taken with the oracle's block operator, within 1e-13 of
    its right-hand side; the solution within 1e-11 of the oracle's."""
    wdr, lat, ctx, U = _setup((8, 8, 8, 8), (4, 4, 4, 4), 0.6, 536)
    ctx.set_mr_form(wdr.MR_ONE_PER_CU if form == "one" else wdr.MR_TWO_PER_CU)
    kappa = 0.14
    T = oracle.clover_term(lat, U, CSW, kappa)
    gU = ctx.gauge(dev(U), CSW, kappa)
    b = synth.spinor(lat.L, 537)
    bid, col, _ = lat.maps()
    p = wdr.default_params(inner=2)
    for colour in (0, 1, 2):
        x, info = ctx.block_solve(gU, kappa, colour, dev(b), p)
        x = host(x)
        sel = np.ones(lat.V, bool) if colour == 2 else col == colour
        bb = b.copy()
        bb[~sel] = 0
        assert np.all(x[~sel] == 0)
        r = bb - oracle.apply_Dblock(lat, U, kappa, x, colour, T)
        worst = max(np.linalg.norm(r[bid == k]) / np.linalg.norm(bb[bid == k]) for k in np.unique(bid[sel]))
        want, _, _, _ = oracle.solve(lat, U, kappa, bb, "block", colour, tol=1e-14, clov=T)
        say("clover F16 block solve", form, colour, info.as_dict(), "worst block", worst, "vs oracle", rel(x, want))
        assert info.converged and info.true_rel_resid <= 1e-13 and worst <= 1.05e-13
        assert rel(x, want) < 1e-11
    del gU
    ctx.close()


@pytest.mark.parametrize("inner", [0, 1, 2])
def test_clover_schur(inner):
    """The Schur complement 1 - D_bb^-1 D_bw D_ww^-1 D_wb with the clover
    term in every block operator, within 1e-11 of the oracle's; white sites
    exactly zero."""
    wdr, lat, ctx, U = _setup((8, 8, 8, 8), (4, 4, 4, 4), 0.6, 516)
    kappa = 0.14
    T = oracle.clover_term(lat, U, CSW, kappa)
    gU = ctx.gauge(dev(U), CSW, kappa)
    eta = synth.spinor(lat.L, 517)
    got = host(ctx.schur(gU, kappa, dev(eta), wdr.default_params(inner=inner)))
    want = oracle.schur_apply(lat, U, kappa, eta, clov=T)
    e = rel(got, want)
    say("clover schur", inner, e)
    assert e < 1e-11
    assert np.all(got[~oracle.colour_mask(lat, 0)] == 0)
    assert rel(want, oracle.schur_apply(lat, U, kappa, eta)) > 1e-2
    del gU
    ctx.close()


@pytest.mark.parametrize("op,inner,N,K", [("BLOCKS", 1, 2, 1), ("BLOCKS", 0, 1, 2), ("SCHUR", 1, 2, 1),
                                          ("SCHUR", 0, 1, 1), ("BLOCKS", 2, 2, 1), ("SCHUR", 2, 1, 2)])
def test_clover_block_and_schur_samples(op, inner, N, K):
    """BLOCKS (one sample per block) and SCHUR samples of the clover
    operator (CGNE for D; FP64, FP32 or FP16 inner level, the last with the
    FP16 block MR) within 1e-8 of the oracle's, over a path whose interior
    points carry clover terms the library builds itself."""
    wdr, lat, ctx, U = _setup((8, 8, 8, 8), (4, 4, 4, 4), 0.5, 518)
    kappa = 0.135
    Up = synth.redraw(U, oracle.active_links(lat), 0.5, 519)
    gU, gUp = ctx.gauge(dev(U), CSW, kappa), ctx.gauge(dev(Up), CSW, kappa)
    p = wdr.default_params(solver=1, inner=inner, max_iter=20000)
    wop, oop = getattr(wdr, "OP_" + op), getattr(oracle, "OP_" + op)
    s, lr, info = ctx.logdet_ratio(gU, gUp, kappa, wop, N, K, wdr.NOISE_GAUSS, 79, p)
    want, lr_want = oracle.logdet_ratio(lat, U, Up, kappa, oop, N, K, oracle.NOISE_GAUSS, 79, csw=CSW)
    err = np.abs(s - want).max()
    say("clover", op, "samples inner", inner, "max |ds|", err, "log R", lr, float(np.sum(lr_want)), info.as_dict())
    assert s.shape == want.shape
    assert info.converged and err < 1e-8
    assert abs(lr - float(np.sum(lr_want))) < 1e-8 * max(1, s.size)
    plain, _ = oracle.logdet_ratio(lat, U, Up, kappa, oop, 1, 1, oracle.NOISE_GAUSS, 79)
    assert np.abs(plain[0, 0] - want[0, 0]).max() > 1e-3
    del gU, gUp
    ctx.close()


def test_clover_dd_samples():
    """The DD estimate with the clover term (every block ratio and the Schur
    ratio of one proposal in one call, the two parts on concurrent
    contexts) against the oracle's BLOCKS and SCHUR samples."""
    wdr, lat, ctx, U = _setup((8, 8, 8, 8), (4, 4, 4, 4), 0.5, 520)
    kappa = 0.135
    Up = synth.redraw(U, oracle.active_links(lat), 0.5, 521)
    gU, gUp = ctx.gauge(dev(U), CSW, kappa), ctx.gauge(dev(Up), CSW, kappa)
    N = 1
    p = wdr.default_params(solver=1, inner=1, max_iter=20000)
    s, lr, info = ctx.logdet_ratio(gU, gUp, kappa, wdr.OP_DD, N, 1, wdr.NOISE_GAUSS, 45, p)
    wb, lb = oracle.logdet_ratio(lat, U, Up, kappa, oracle.OP_BLOCKS, N, 1, oracle.NOISE_GAUSS, 45, csw=CSW)
    ws, ls = oracle.logdet_ratio(lat, U, Up, kappa, oracle.OP_SCHUR, N, 1, oracle.NOISE_GAUSS, 45, csw=CSW)
    eb, es = np.abs(s[..., :-1] - wb).max(), np.abs(s[..., -1] - ws).max()
    say("clover dd max |ds| blocks", eb, "schur", es, info.as_dict())
    assert info.converged and eb < 1e-8 and es < 1e-8
    assert abs(lr - (float(np.sum(lb)) + float(ls))) < 1e-8 * s.size
    del gU, gUp
    ctx.close()


@pytest.mark.parametrize("L,B,blocks", [((4, 4, 8, 8), (2, 2, 4, 4), None), ((8, 8, 8, 8), (4, 4, 4, 4), [0, 9])])
def test_clover_block_logdet(L, B, blocks):
    """Exact block determinants with the clover term (det D_b = det A_oo
    det Dhat_b, Dhat_b = A_ee - kappa^2 H_eo A_oo^-1 H_oe) within 1e-8 of the
    oracle's dense LU of each block, and the ratios between two clover
    fields; on the 8^4 lattice of 4^4 blocks two blocks are checked."""
    wdr, lat, ctx, U = _setup(L, B, 0.6, 522)
    kappa = 0.14
    Up = synth.redraw(U, synth.bernoulli_links(lat.L, 0.1, 523), 0.6, 523)
    T, Tp = oracle.clover_term(lat, U, CSW, kappa), oracle.clover_term(lat, Up, CSW, kappa)
    gU, gUp = ctx.gauge(dev(U), CSW, kappa), ctx.gauge(dev(Up), CSW, kappa)
    idx = np.arange(lat.nblocks) if blocks is None else np.asarray(blocks)
    got = ctx.block_logdet(gU, kappa)
    want = oracle.block_log_dets(lat, U, kappa, blocks=idx, clov=T)
    e = np.abs(got[idx] - want[idx]).max()
    ratio = ctx.block_logdet_ratio(gU, gUp, kappa)
    want_r = oracle.block_log_dets(lat, Up, kappa, blocks=idx, clov=Tp) - want
    er = np.abs(ratio[idx] - want_r[idx]).max()
    say("clover block logdet", L, B, "max |d|", e, "ratio", er, "range", want[idx].min(), want[idx].max())
    assert e < 1e-8 and er < 1e-8 and np.abs(want_r[idx]).max() > 1e-3
    plain = ctx.gauge(dev(U))
    assert np.abs(ctx.block_logdet(plain, kappa)[idx] - got[idx]).max() > 1e-2
    del gU, gUp, plain
    ctx.close()


@pytest.mark.parametrize("L,B", GEOMS)
def test_clover_sap_matches_oracle(L, B):
    """The Schwarz procedure with the clover term (one lane per site in the
    block MR, A and A^-1 applied where the reduced block system needs them)
    against the oracle's, cycle for cycle: FP64 1e-12, FP32 2e-5."""
    wdr, lat, ctx, U = _setup(L, B, 0.5, 524)
    kappa = 0.135
    T = oracle.clover_term(lat, U, CSW, kappa)
    gU = ctx.gauge(dev(U), CSW, kappa)
    eta = synth.spinor(lat.L, 525)
    for ncy, nmr in ((1, 1), (2, 5)):
        want = oracle.sap(lat, U, kappa, eta, ncy, nmr, clov=T)
        for prec, tol in ((wdr.F64, 1e-12), (wdr.F32, 2e-5)):
            p = wdr.default_params(sap_cycles=ncy, mr_steps=nmr, inner=prec)
            e = rel(host(ctx.sap(gU, kappa, dev(eta), p)), want)
            say("clover sap", L, ncy, nmr, prec, e)
            assert e < tol
    assert rel(want, oracle.sap(lat, U, kappa, eta, 2, 5)) > 1e-2
    del gU
    ctx.close()


@pytest.mark.parametrize("inner", [0, 1])
def test_clover_fgcr_solve(inner):
    """FGCR with Schwarz preconditioning on the clover operator: the
    oracle's clover stencil checks the true residual (<= 1.05e-10) and the
    solution is within 1e-8 of the oracle's CGNE solution."""
    wdr, lat, ctx, U = _setup((8, 8, 8, 8), (4, 4, 4, 4), 0.5, 526)
    kappa = 0.125
    T = oracle.clover_term(lat, U, CSW, kappa)
    gU = ctx.gauge(dev(U), CSW, kappa)
    b = synth.spinor(lat.L, 527)
    x, info = ctx.solve(gU, kappa, dev(b), wdr.default_params(solver=0, inner=inner, max_iter=2000))
    x = host(x)
    r = np.linalg.norm(b - oracle.apply_D(lat, U, kappa, x, T)) / np.linalg.norm(b)
    say("clover fgcr inner", inner, info.as_dict(), "oracle residual", r)
    assert info.converged and r <= 1.05e-10
    want, _, _, _ = oracle.solve(lat, U, kappa, b, tol=1e-13, clov=T)
    assert rel(x, want) < 1e-8
    del gU
    ctx.close()


@pytest.mark.parametrize("op", ["FULL", "SCHUR", "DD"])
def test_clover_fgcr_samples(op):
    """FULL, SCHUR and DD samples of the clover operator with FGCR + Schwarz
    (FP32 inner level) within 1e-8 of the oracle's."""
    wdr, lat, ctx, U = _setup((8, 8, 8, 8), (4, 4, 4, 4), 0.5, 528)
    kappa = 0.125
    Up = synth.redraw(U, oracle.active_links(lat), 0.5, 529)
    gU, gUp = ctx.gauge(dev(U), CSW, kappa), ctx.gauge(dev(Up), CSW, kappa)
    p = wdr.default_params(solver=0, inner=1, max_iter=2000)
    s, lr, info = ctx.logdet_ratio(gU, gUp, kappa, getattr(wdr, "OP_" + op), 1, 1, wdr.NOISE_GAUSS, 85, p)
    if op == "DD":
        wb, _ = oracle.logdet_ratio(lat, U, Up, kappa, oracle.OP_BLOCKS, 1, 1, oracle.NOISE_GAUSS, 85, csw=CSW)
        ws, _ = oracle.logdet_ratio(lat, U, Up, kappa, oracle.OP_SCHUR, 1, 1, oracle.NOISE_GAUSS, 85, csw=CSW)
        err = max(np.abs(s[..., :-1] - wb).max(), np.abs(s[..., -1] - ws).max())
    else:
        want, _ = oracle.logdet_ratio(lat, U, Up, kappa, getattr(oracle, "OP_" + op), 1, 1, oracle.NOISE_GAUSS, 85,
                                      csw=CSW)
        err = np.abs(s - want).max()
    say("clover fgcr", op, "max |ds|", err, info.as_dict())
    assert info.converged and err < 1e-8
    del gU, gUp
    ctx.close()


def test_clover_f16_schwarz_sweeps_in_f32():
    """With the clover term an F16 inner level runs the Schwarz procedure in
    FP32 (the FP16 sweep keeps no blocks of A): the same result as F32 bit
    for bit, and the oracle's within 2e-5."""
    wdr, lat, ctx, U = _setup((8, 8, 8, 8), (4, 4, 4, 4), 0.5, 531)
    kappa = 0.135
    T = oracle.clover_term(lat, U, CSW, kappa)
    gU = ctx.gauge(dev(U), CSW, kappa)
    eta = synth.spinor(lat.L, 532)
    p16 = wdr.default_params(sap_cycles=2, mr_steps=5, inner=2)
    p32 = wdr.default_params(sap_cycles=2, mr_steps=5, inner=1)
    got = host(ctx.sap(gU, kappa, dev(eta), p16))
    want = oracle.sap(lat, U, kappa, eta, 2, 5, clov=T)
    say("clover F16 sap vs oracle", rel(got, want))
    assert np.array_equal(got, host(ctx.sap(gU, kappa, dev(eta), p32))) and rel(got, want) < 2e-5
    del gU
    ctx.close()


@pytest.mark.parametrize("op", ["solve", "SCHUR", "DD"])
def test_clover_fgcr_f16(op):
    """FGCR with an F16 inner level on the clover operator: the oracle's
    clover stencil checks the solve's true residual (<= 1.05e-10) and its
    solution (1e-8); SCHUR and DD samples within 1e-8 of the oracle's."""
    wdr, lat, ctx, U = _setup((8, 8, 8, 8), (4, 4, 4, 4), 0.5, 533)
    kappa = 0.125
    p = wdr.default_params(solver=0, inner=2, max_iter=2000)
    gU = ctx.gauge(dev(U), CSW, kappa)
    if op == "solve":
        T = oracle.clover_term(lat, U, CSW, kappa)
        b = synth.spinor(lat.L, 534)
        x, info = ctx.solve(gU, kappa, dev(b), p)
        x = host(x)
        r = np.linalg.norm(b - oracle.apply_D(lat, U, kappa, x, T)) / np.linalg.norm(b)
        want, _, _, _ = oracle.solve(lat, U, kappa, b, tol=1e-13, clov=T)
        say("clover fgcr F16 solve", info.as_dict(), "oracle residual", r, "vs oracle", rel(x, want))
        assert info.converged and r <= 1.05e-10 and rel(x, want) < 1e-8
        del gU
        ctx.close()
        return
    Up = synth.redraw(U, oracle.active_links(lat), 0.5, 535)
    gUp = ctx.gauge(dev(Up), CSW, kappa)
    s, lr, info = ctx.logdet_ratio(gU, gUp, kappa, getattr(wdr, "OP_" + op), 1, 1, wdr.NOISE_GAUSS, 86, p)
    if op == "DD":
        wb, _ = oracle.logdet_ratio(lat, U, Up, kappa, oracle.OP_BLOCKS, 1, 1, oracle.NOISE_GAUSS, 86, csw=CSW)
        ws, _ = oracle.logdet_ratio(lat, U, Up, kappa, oracle.OP_SCHUR, 1, 1, oracle.NOISE_GAUSS, 86, csw=CSW)
        err = max(np.abs(s[..., :-1] - wb).max(), np.abs(s[..., -1] - ws).max())
    else:
        want, _ = oracle.logdet_ratio(lat, U, Up, kappa, oracle.OP_SCHUR, 1, 1, oracle.NOISE_GAUSS, 86, csw=CSW)
        err = np.abs(s - want).max()
    say("clover fgcr F16", op, "max |ds|", err, info.as_dict())
    assert info.converged and err < 1e-8
    del gU, gUp
    ctx.close()


@pytest.mark.parametrize("middle,bc", [(1, (1, 1, 1, -1)), (0, (1, 1, 1, -1)), (1, (1, -1, 1, -1))])
def test_clover_f16_cg_solve(middle, bc):
    """CGNE with FP16 steps on the clover operator (A_oo^-1 and A_ee in FP32
    in the FP16 stencil halves), with an FP32 middle level or FP64 updates
    only: the oracle's clover stencil checks the true residual (<= 1.05e-10)
    and the solution is within 1e-8 of the oracle's."""
    wdr, lat, ctx, U = _setup((8, 8, 8, 8), (4, 4, 4, 4), 0.5, 530, bc)
    kappa = 0.135
    T = oracle.clover_term(lat, U, CSW, kappa)
    gU = ctx.gauge(dev(U), CSW, kappa)
    b = synth.spinor(lat.L, 531)
    x, info = ctx.solve(gU, kappa, dev(b), wdr.default_params(solver=1, inner=2, middle=middle, max_iter=20000))
    x = host(x)
    r = np.linalg.norm(b - oracle.apply_D(lat, U, kappa, x, T)) / np.linalg.norm(b)
    say("clover f16 cg middle", middle, bc, info.as_dict(), "oracle residual", r)
    assert info.converged and r <= 1.05e-10
    want, _, _, _ = oracle.solve(lat, U, kappa, b, tol=1e-13, clov=T)
    assert rel(x, want) < 1e-8
    del gU
    ctx.close()


@pytest.mark.parametrize("op", ["FULL", "SCHUR", "BLOCKS"])
def test_clover_f16_samples(op):
    """Samples of the clover operator with the FP16 inner level (FP16 CG
    steps, FP32 middle level; block solves by FP32 CG rounds) within 1e-8 of
    the oracle's."""
    wdr, lat, ctx, U = _setup((8, 8, 8, 8), (4, 4, 4, 4), 0.5, 532)
    kappa = 0.135
    Up = synth.redraw(U, oracle.active_links(lat), 0.5, 533)
    gU, gUp = ctx.gauge(dev(U), CSW, kappa), ctx.gauge(dev(Up), CSW, kappa)
    p = wdr.default_params(solver=1, inner=2, middle=1, max_iter=20000)
    N = 2
    s, lr, info = ctx.logdet_ratio(gU, gUp, kappa, getattr(wdr, "OP_" + op), N, 1, wdr.NOISE_GAUSS, 87, p)
    want, lr_want = oracle.logdet_ratio(lat, U, Up, kappa, getattr(oracle, "OP_" + op), N, 1, oracle.NOISE_GAUSS,
                                        87, csw=CSW)
    err = np.abs(s - want).max()
    say("clover f16", op, "max |ds|", err, info.as_dict())
    assert info.converged and err < 1e-8
    assert abs(lr - float(np.sum(lr_want))) < 1e-8 * s.size
    del gU, gUp
    ctx.close()


def test_clover_16x16x16x16_schur_f16_sample():
    """A 16^4 SCHUR sample of the clover operator with the settings of the
    large-lattice workloads (FP16 CG steps, FP32 middle level, FP64 reliable
    updates; block solves by FP32 CG rounds) within 1e-8 of the oracle's."""
    wdr, lat, ctx, U = _setup((16, 16, 16, 16), (4, 4, 4, 4), 0.25, 534)
    kappa = 0.135
    Up = synth.redraw(U, oracle.active_links(lat), 0.25, 535)
    gU, gUp = ctx.gauge(dev(U), CSW, kappa), ctx.gauge(dev(Up), CSW, kappa)
    p = wdr.default_params(solver=1, inner=2, middle=1, max_iter=20000)
    s, lr, info = ctx.logdet_ratio(gU, gUp, kappa, wdr.OP_SCHUR, 1, 1, wdr.NOISE_GAUSS, 89, p)
    want, _ = oracle.logdet_ratio(lat, U, Up, kappa, oracle.OP_SCHUR, 1, 1, oracle.NOISE_GAUSS, 89, csw=CSW)
    err = np.abs(s - want).max()
    say("clover 16^4 SCHUR f16 max |ds|", err, "sample", float(want.ravel()[0]), info.as_dict())
    assert info.converged and err < 1e-8
    del gU, gUp
    ctx.close()


def test_clover_16x16x16x16_operator_and_solve():
    """16^4 (256 blocks of 4^4): D with the clover term against the oracle on
    both stencil forms, and a CGNE solve whose true residual the oracle's
    clover operator checks."""
    wdr, lat, ctx, U = _setup((16, 16, 16, 16), (4, 4, 4, 4), 0.5, 510)
    kappa = 0.13
    T = oracle.clover_term(lat, U, CSW, kappa)
    gU = ctx.gauge(dev(U), CSW, kappa)
    psi = synth.spinor(lat.L, 511)
    want = oracle.apply_D(lat, U, kappa, psi, T)
    for stencil in (1, 2):
        ctx.set_stencil(stencil)
        e = rel(host(ctx.apply_D(gU, kappa, dev(psi))), want)
        say("16^4 clover D stencil", stencil, e)
        assert e < 1e-13
    ctx.set_stencil(0)
    x, info = ctx.solve(gU, kappa, dev(psi), wdr.default_params(solver=1, inner=1, max_iter=20000))
    r = np.linalg.norm(psi - oracle.apply_D(lat, U, kappa, host(x), T)) / np.linalg.norm(psi)
    say("16^4 clover solve", info.as_dict(), r)
    assert info.converged and r <= 1.05e-10
    del gU
    ctx.close()


def test_clover_error_paths():
    wdr, lat, ctx, U = _setup((8, 8, 8, 8), (4, 4, 4, 4), 0.5, 512)
    kappa = 0.135
    gU = ctx.gauge(dev(U), CSW, kappa)
    gP = ctx.gauge(dev(U))
    psi = dev(synth.spinor(lat.L, 513))

    def refused(fn):
        with pytest.raises(wdr.WdrError) as e:
            fn()
        assert e.value.status == wdr.EINVAL
        say("refused:", str(e.value)[:120])

    refused(lambda: ctx.apply_D(gU, 0.13, psi))                       # another kappa
    refused(lambda: ctx.apply_D(gU, kappa, psi, wdr.F16))             # FP16 stencil
    sub = wdr.Context((4, 4, 4, 4), (2, 2, 2, 2), (0, 0, 0, 0))
    # the clover term of a block needs links outside it: no recursive DD
    refused(lambda: ctx.block_schur_ratio(gU, gU, kappa, sub, 1, 1, 1, 1, wdr.default_params()))
    sub.close()
    refused(lambda: ctx.logdet_ratio(gU, gP, kappa, wdr.OP_FULL, 1, 1, 1, 1, wdr.default_params(solver=1)))
    refused(lambda: ctx.block_logdet(gU, 0.13))                           # another kappa
    refused(lambda: ctx.block_logdet_ratio(gU, gP, kappa))                 # csw differs
    refused(lambda: ctx.clover_field(gP))
    # removing the term gives back the plain operator
    ctx.set_clover(gU, 0.0, 0.0)
    assert rel(host(ctx.apply_D(gU, 0.13, psi)), host(ctx.apply_D(gP, 0.13, psi))) == 0
    del gU, gP
    ctx.close()
    # open boundaries cannot carry the term
    wdr, lat, ctx, U = _setup((8, 8, 8, 8), (4, 4, 4, 4), 0.5, 512, bc=(1, 1, 1, 0))
    g = ctx.gauge(dev(U))
    refused(lambda: ctx.set_clover(g, CSW, kappa))
    del g
    ctx.close()
