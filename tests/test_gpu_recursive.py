"""GPU parity of recursive domain decomposition (paper Sec. 3, eq. ddrec;
the block step 2 of eq. 4step): block fields, open boundaries, and the Schur
ratio of every block over its sub-blocks, against the FP64 oracle through
the C ABI."""
import numpy as np
import pytest

import oracle
from paper_1112_1243_amd import synth
from tests.gpu_util import dev, host, rel, say, torch_cuda
from tests.test_oracle_blockdet import extract_block

pytestmark = pytest.mark.gpu

OPEN = (0, 0, 0, 0)


def _wdr():
    torch_cuda()
    from paper_1112_1243_amd import wdr
    return wdr


def test_block_fields_bit_exact():
    """Gathering the links of every block undoes the boundary phase folded
    into the stored links; the result equals index arithmetic on the
    canonical field bit for bit."""
    wdr = _wdr()
    L, B, bc = (8, 8, 8, 8), (4, 4, 4, 4), (1, 1, 1, -1)
    ctx, lat = wdr.Context(L, B, bc), oracle.Lattice(L, B, bc)
    U = synth.gauge_field(L, 0.5, 601)
    gU = ctx.gauge(dev(U))
    f = host(ctx.block_fields(gU))
    for b in range(ctx.nblocks):
        want, _ = extract_block(lat, U, b)
        assert np.array_equal(f[b], want)
    del gU
    ctx.close()


def test_open_boundary_operator_and_schur_samples():
    """A lattice with open boundaries: D against the oracle, and SCHUR samples
    (one factor x two noise vectors) within 1e-8."""
    wdr = _wdr()
    L, B = (4, 4, 4, 4), (2, 2, 2, 2)
    ctx, lat = wdr.Context(L, B, OPEN), oracle.Lattice(L, B, OPEN)
    U = synth.gauge_field(L, 0.5, 603)
    Up = synth.redraw(U, synth.bernoulli_links(L, 0.1, 604), 0.5, 604)
    psi = synth.spinor(L, 605)
    gU, gUp = ctx.gauge(dev(U)), ctx.gauge(dev(Up))
    got = host(ctx.apply_D(gU, 0.13, dev(psi)))
    assert rel(got, oracle.apply_D(lat, U, 0.13, psi)) < 1e-14
    s, lr, info = ctx.logdet_ratio(gU, gUp, 0.13, wdr.OP_SCHUR, 1, 2, wdr.NOISE_GAUSS, 606, wdr.default_params())
    want, _ = oracle.logdet_ratio(lat, U, Up, 0.13, oracle.OP_SCHUR, 1, 2, oracle.NOISE_GAUSS, 606)
    say("open SCHUR samples", s.ravel(), "max |ds|", np.abs(s - want).max())
    assert info.converged and np.abs(s - want).max() < 1e-8 and np.abs(want).min() > 1e-3
    del gU, gUp
    ctx.close()


def test_block_schur_ratio_matches_oracle():
    """Every 4^4 block of an 8^4 lattice, its Schur complement over 2^4
    sub-blocks, all blocks in one call: three blocks against the oracle on the
    extracted open block with the same noise key (seed + block id)."""
    wdr = _wdr()
    L, B, kappa, seed = (8, 8, 8, 8), (4, 4, 4, 4), 0.13, 700
    ctx, lat = wdr.Context(L, B), oracle.Lattice(L, B)
    sub, slat = wdr.Context(B, (2, 2, 2, 2), OPEN), oracle.Lattice(B, (2, 2, 2, 2), OPEN)
    U = synth.gauge_field(L, 0.5, 607)
    Up = synth.redraw(U, oracle.active_links(lat), 0.5, 608)
    gU, gUp = ctx.gauge(dev(U)), ctx.gauge(dev(Up))
    N, K = 2, 1
    s, lrs, info = ctx.block_schur_ratio(gU, gUp, kappa, sub, N, K, wdr.NOISE_GAUSS, seed, wdr.default_params())
    assert info.converged and s.shape == (ctx.nblocks, N, K)
    for b in (0, 7, 15):
        Ub, _ = extract_block(lat, U, b)
        Upb, _ = extract_block(lat, Up, b)
        want, lr_want = oracle.logdet_ratio(slat, Ub, Upb, kappa, oracle.OP_SCHUR, N, K, oracle.NOISE_GAUSS,
                                            seed + b)
        say("block", b, s[b].ravel(), want.ravel())
        assert np.abs(s[b] - want).max() < 1e-8
        assert abs(lrs[b] - float(np.sum(lr_want))) < 1e-8
    del gU, gUp
    ctx.close()
    sub.close()


def test_block_schur_ratio_paper_geometry_matches_oracle():
    """The benchmark's recursive workload (the block geometry of the paper's
    Sec. 6): 8^4 blocks of a 16^4 lattice, 4^4 sub-blocks, links of every
    block's 6^4 core redrawn, solved with the large-lattice settings (FP16
    even-odd CG with FP32 and FP64 reliable updates, FP16 sub-block solves):
    sampled blocks against the oracle on the extracted open block."""
    wdr = _wdr()
    L, B, kappa, seed = (16, 16, 16, 16), (8, 8, 8, 8), 0.150, 710
    ctx, lat = wdr.Context(L, B), oracle.Lattice(L, B)
    sub, slat = wdr.Context(B, (4, 4, 4, 4), OPEN), oracle.Lattice(B, (4, 4, 4, 4), OPEN)
    U = synth.gauge_field(L, 0.25, 711)
    Up = synth.redraw(U, oracle.active_links(lat, 1, 6), 0.25, 712)
    gU, gUp = ctx.gauge(dev(U)), ctx.gauge(dev(Up))
    N, K = 2, 1
    p = wdr.default_params(**synth.LARGE_MIXED)
    s, lrs, info = ctx.block_schur_ratio(gU, gUp, kappa, sub, N, K, wdr.NOISE_GAUSS, seed, p)
    assert info.converged and s.shape == (ctx.nblocks, N, K)
    for b in (0, 9):
        Ub, _ = extract_block(lat, U, b)
        Upb, _ = extract_block(lat, Up, b)
        want, lr_want = oracle.logdet_ratio(slat, Ub, Upb, kappa, oracle.OP_SCHUR, N, K, oracle.NOISE_GAUSS,
                                            seed + b)
        say("paper geometry block", b, s[b].ravel(), want.ravel())
        assert np.abs(s[b] - want).max() < 1e-8
        assert abs(lrs[b] - float(np.sum(lr_want))) < 1e-8
    del gU, gUp
    ctx.close()
    sub.close()


def test_recursive_exact_agrees_with_stochastic():
    """eq. ddrec gives the block Schur ratio exactly from block determinants
    on two levels: log det(Dhat_b'^+ Dhat_b') - log det(Dhat_b^+ Dhat_b) =
    (ratio of block b of the lattice) - (sum of the ratios of its sub-blocks
    on the open block).  The stochastic estimate of the same ratio (N = 8
    factors x K = 32 noise vectors, a small rotation of the active links)
    agrees within 6 standard errors per block."""
    wdr = _wdr()
    L, B, kappa = (8, 8, 8, 8), (4, 4, 4, 4), 0.13
    ctx, lat = wdr.Context(L, B), oracle.Lattice(L, B)
    sub = wdr.Context(B, (2, 2, 2, 2), OPEN)
    U = synth.gauge_field(L, 0.5, 609)
    rot = synth.redraw(np.broadcast_to(np.eye(3, dtype=np.complex128), U.shape).copy(), oracle.active_links(lat),
                       0.1, 610)
    Up = np.ascontiguousarray(np.einsum("xmab,xmbc->xmac", rot, U))
    gU, gUp = ctx.gauge(dev(U)), ctx.gauge(dev(Up))
    whole = ctx.block_logdet_ratio(gU, gUp, kappa)
    f0, f1 = ctx.block_fields(gU), ctx.block_fields(gUp)
    exact = np.empty(ctx.nblocks)
    for b in range(ctx.nblocks):
        h0, h1 = sub.gauge(f0[b]), sub.gauge(f1[b])
        exact[b] = whole[b] - sub.block_logdet_ratio(h0, h1, kappa).sum()
        del h0, h1
    N, K = 8, 32
    s, _, info = ctx.block_schur_ratio(gU, gUp, kappa, sub, N, K, wdr.NOISE_GAUSS, 611, wdr.default_params())
    assert info.converged
    top = s.max(axis=2, keepdims=True)
    lme = (np.log(np.mean(np.exp(s - top), axis=2)) + top[:, :, 0]).sum(axis=1)
    se = np.sqrt((s.var(axis=2, ddof=1) / K).sum(axis=1))
    say("exact", exact[:4], "stochastic", lme[:4], "max |diff| / se", np.max(np.abs(lme - exact) / se))
    assert np.all(np.abs(lme - exact) < 6 * se + 1e-3)
    del gU, gUp
    ctx.close()
    sub.close()


def test_errors():
    wdr = _wdr()
    ctx = wdr.Context((8, 8, 8, 8), (4, 4, 4, 4))
    gU = ctx.gauge(dev(synth.unit_gauge((8, 8, 8, 8))))
    periodic = wdr.Context((4, 4, 4, 4), (2, 2, 2, 2))
    wrong = wdr.Context((4, 4, 4, 8), (2, 2, 2, 2), OPEN)
    for sub in (periodic, wrong):
        with pytest.raises(wdr.WdrError) as e:
            ctx.block_schur_ratio(gU, gU, 0.13, sub, 1, 1, wdr.NOISE_GAUSS, 1, wdr.default_params())
        assert e.value.status == wdr.EINVAL
    with pytest.raises(wdr.WdrError) as e:
        wdr.Context((4, 4, 4, 4), (2, 2, 2, 2), (1, 1, 1, 2))
    assert e.value.status == wdr.EINVAL
    del gU
    for c in (ctx, periodic, wrong):
        c.close()
