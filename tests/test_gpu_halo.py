"""GPU parity of the halo of a lattice cut along t into slabs of whole
blocks (the sharding of one large lattice, eq. domdec of Sec. 3: the slab's
own D with an open t boundary plus the block-interaction hops across the
cut): a ring of one slab, and two slabs of an 8^4 lattice exchanging faces,
reproduce the oracle's D of the whole lattice."""
import numpy as np
import pytest

import oracle
from paper_1112_1243_amd import synth
from tests.gpu_util import dev, host, rel, say, torch_cuda

pytestmark = pytest.mark.gpu

TOL = {0: 1e-13, 1: 2e-6}  # F64, F32


def _slab_D(wdr, ctx, U, psi, kappa, prec):
    """The slab's own D (open t boundary) in the internal layout, and its faces."""
    gU = ctx.gauge(dev(U))
    fin = ctx.pack(dev(psi), prec)
    fout = ctx.internal_field(prec)
    ctx.apply_D_internal(gU, kappa, fin, fout, prec)
    lo, hi = ctx.halo_field(prec), ctx.halo_field(prec)
    ctx.halo_pack(dev(U), fin, lo, hi, prec)
    del gU
    return fout, lo, hi


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("bct", [1, -1])
def test_halo_ring_of_one(prec, bct):
    """One slab (8^3 x 4, one block in t) whose faces go to itself equals
    the oracle's D with periodic / antiperiodic time."""
    torch_cuda()
    from paper_1112_1243_amd import wdr
    L, B = (8, 8, 8, 4), (4, 4, 4, 4)
    say("halo ring of one", prec, bct)
    ctx = wdr.Context(L, B, (1, 1, 1, 0))
    U = synth.gauge_field(L, 0.5, 701)
    psi = synth.spinor(L, 702)
    kappa = 0.14
    fout, lo, hi = _slab_D(wdr, ctx, U, psi, kappa, prec)
    ctx.halo_unpack(dev(U), kappa, hi, lo, bct, bct, fout, prec)
    got = host(ctx.unpack(fout, prec))
    want = oracle.apply_D(oracle.Lattice(L, B, (1, 1, 1, bct)), U, kappa, psi)
    e = rel(got, want)
    say("ring of one", prec, bct, e)
    assert e < TOL[prec]
    # without the faces the open slab differs on the two t slices only
    open_only = host(ctx.unpack(_slab_D(wdr, ctx, U, psi, kappa, prec)[0], prec))
    t = np.arange(oracle.Lattice(L, B).V) // (L[0] * L[1] * L[2])
    inner = (t > 0) & (t < L[3] - 1)
    assert rel(open_only[inner], want[inner]) < TOL[prec]
    assert rel(open_only, want) > 1e-2
    ctx.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_halo_two_slabs(prec):
    """An 8^4 lattice (antiperiodic time) cut into two 8^3 x 4 slabs: each
    slab's D plus the hops from the other slab's faces equals the oracle's
    D of the whole lattice."""
    torch_cuda()
    from paper_1112_1243_amd import wdr
    Lg, Ls, B, bct = (8, 8, 8, 8), (8, 8, 8, 4), (4, 4, 4, 4), -1
    kappa = 0.14
    U = synth.gauge_field(Lg, 0.5, 703)
    psi = synth.spinor(Lg, 704)
    F = 8 * 8 * 8
    Us = [U.reshape(8, F, 4, 3, 3)[4 * k:4 * k + 4].reshape(-1, 4, 3, 3) for k in (0, 1)]
    ps = [psi.reshape(8, F, 4, 3)[4 * k:4 * k + 4].reshape(-1, 4, 3) for k in (0, 1)]
    ctxs = [wdr.Context(Ls, B, (1, 1, 1, 0)) for _ in (0, 1)]
    slabs = [_slab_D(wdr, ctxs[k], Us[k], ps[k], kappa, prec) for k in (0, 1)]
    # slab 0 holds t = 0..3 (its bottom is the lattice's), slab 1 t = 4..7
    (f0, lo0, hi0), (f1, lo1, hi1) = slabs
    ctxs[0].halo_unpack(dev(Us[0]), kappa, hi1, lo1, bct, 1, f0, prec)
    ctxs[1].halo_unpack(dev(Us[1]), kappa, hi0, lo0, 1, bct, f1, prec)
    got = np.concatenate([host(ctxs[k].unpack(slabs[k][0], prec)).reshape(4, F, 4, 3) for k in (0, 1)])
    want = oracle.apply_D(oracle.Lattice(Lg, B, (1, 1, 1, bct)), U, kappa, psi)
    e = rel(got.reshape(-1, 4, 3), want)
    say("two slabs", prec, e)
    assert e < TOL[prec]
    for c in ctxs:
        c.close()


def test_halo_error_paths():
    torch_cuda()
    from paper_1112_1243_amd import wdr
    L, B = (8, 8, 8, 4), (4, 4, 4, 4)
    U = synth.gauge_field(L, 0.5, 705)
    ctx = wdr.Context(L, B, (1, 1, 1, 1))
    f = ctx.internal_field(0)
    lo, hi = ctx.halo_field(0), ctx.halo_field(0)
    assert lo.numel() == 6 * 8 * 8 * 8 * 16

    def refused(fn):
        with pytest.raises(wdr.WdrError) as e:
            fn()
        assert e.value.status == wdr.EINVAL
        say("refused:", str(e.value)[:100])

    refused(lambda: ctx.halo_pack(dev(U), f, lo, hi, 0))                     # t boundary not open
    ctx.close()
    ctx = wdr.Context(L, B, (1, 1, 1, 0))
    f = ctx.internal_field(0)
    refused(lambda: ctx.halo_pack(dev(U), f, lo, hi, 2))                     # FP16
    refused(lambda: ctx.halo_unpack(dev(U), 0.14, lo, hi, 2, 1, f, 0))       # sign
    ctx.close()
