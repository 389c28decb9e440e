"""GPU check of wdr_apply_D_noalloc (the variant of wdr_apply_D whose staging
fields live in the library's static device array instead of allocated
workspace), through the C ABI: two calls in a row, the second on a smaller
lattice, each bit-identical to wdr_apply_D and within FP64 / FP32 rounding of
the oracle's Wilson-Dirac operator (paper Sec. 5); sizes beyond the array
are rejected."""
import numpy as np
import pytest

import oracle
from paper_1112_1243_amd import synth
from tests.gpu_util import dev, host, rel, say, torch_cuda

pytestmark = pytest.mark.gpu


def _case(wdr, L, seed):
    B = (4, 4, 4, 4)
    ctx, lat = wdr.Context(L, B, (1, 1, 1, -1)), oracle.Lattice(L, B, (1, 1, 1, -1))
    U = synth.gauge_field(L, 0.5, seed)
    psi = synth.spinor(L, seed + 1)
    return ctx, lat, U, ctx.gauge(dev(U)), psi


def test_noalloc_apply_D_matches_pooled_form():
    torch = torch_cuda()
    from paper_1112_1243_amd import wdr
    k = 0.141
    for L, seed in (((16, 16, 16, 16), 1701), ((8, 8, 8, 8), 1703)):
        ctx, lat, U, gU, psi = _case(wdr, L, seed)
        want = oracle.apply_D(lat, U, k, psi)
        x = dev(psi)
        for prec, tol in ((wdr.F64, 1e-14), (wdr.F32, 2e-6)):
            out = torch.full((ctx.V, 4, 3), complex("nan"), dtype=torch.complex128, device="cuda")
            got = host(ctx.apply_D_noalloc(gU, k, x, out, prec))
            pooled = host(ctx.apply_D(gU, k, x, prec))
            say("noalloc", L, "prec", prec, "rel vs oracle", rel(got, want))
            assert np.array_equal(got, pooled)
            assert rel(got, want) < tol
        del gU
        ctx.close()


def test_noalloc_rejects_oversized_fields():
    torch_cuda()
    from paper_1112_1243_amd import wdr
    L = (24, 24, 24, 24)  # 331776 sites: two F64 fields exceed the 64 MiB array
    ctx = wdr.Context(L, (4, 4, 4, 4))
    gU = ctx.gauge(dev(synth.unit_gauge(L)))
    psi = dev(np.zeros((ctx.V, 4, 3), complex))
    out = ctx.spinor_like()
    with pytest.raises(wdr.WdrError) as e:
        ctx.apply_D_noalloc(gU, 0.13, psi, out, wdr.F64)
    assert e.value.status == wdr.EINVAL
    # two F32 fields of this lattice fit
    ctx.apply_D_noalloc(gU, 0.13, psi, out, wdr.F32)
    assert not host(out).any()
    del gU
    ctx.close()
