"""GPU parity of the FP16 storage format and the FP16 stencil (the inner
precision of the 32^4 workload: FP16 values with one power-of-two scale per
block of Sec. 3, arithmetic in FP32; the operator is the Wilson-Dirac
operator of Sec. 5) through the C ABI.

The storage rule is emulated here from its definition: per block,
s = 2^ceil(log2 m) with m the largest |component| (as FP32), values
fp16(fp32(v) / s) rounded to nearest even, read back exactly as fp16 * s.
Packing is then bit-exact.  The stencil is compared with the FP64 oracle
applied to the same rounded input and rounded links (first two rows in FP16,
third row rebuilt as the conjugated cross product): what remains is FP32
arithmetic and the rounding of the output, at most half an FP16 ulp of the
top binade, 2^-12 s_out <= 2^-11 max |out| per block."""
import numpy as np
import pytest

import oracle
from paper_1112_1243_amd import synth
from tests.gpu_util import dev, host, rel, say, torch_cuda

pytestmark = pytest.mark.gpu


def _wdr():
    torch_cuda()
    from paper_1112_1243_amd import wdr
    return wdr


def _pow2_at_least(m):
    """2^ceil(log2 m) per entry (1 where m == 0), from frexp as on the device."""
    f, e = np.frexp(m.astype(np.float32))
    p = np.ldexp(np.float32(1.0), np.where(f == 0.5, e - 1, e)).astype(np.float32)
    return np.where(m > 0, p, np.float32(1.0))


def _round16(v32, inv):
    return (v32 * inv).astype(np.float16)


def f16_spinor(lat, psi):
    """(rounded field as complex128, block scales in block-slot order)."""
    perm = oracle.block_order(lat)
    Vb = int(np.prod(lat.B))
    nb = lat.V // Vb
    blk = psi[perm].reshape(nb, Vb * 12)
    re, im = blk.real.astype(np.float32), blk.imag.astype(np.float32)
    m = np.maximum(np.abs(re).max(axis=1), np.abs(im).max(axis=1))
    s = _pow2_at_least(m)
    inv = (np.float32(1.0) / s)[:, None]
    hr, hi = _round16(re, inv), _round16(im, inv)
    q = (hr.astype(np.float32) * s[:, None]).astype(np.float64) + 1j * (hi.astype(np.float32) * s[:, None]).astype(
        np.float64)
    out = np.empty_like(psi)
    out[perm] = q.reshape(nb * Vb, 4, 3)
    return out, s


def f16_links(U):
    """Links as the FP16 stencil uses them: rows 0 and 1 rounded to FP16 (via
    FP32), row 2 rebuilt as conj(row0 x row1)."""
    r = (U.real.astype(np.float32).astype(np.float16).astype(np.float64) +
         1j * U.imag.astype(np.float32).astype(np.float16).astype(np.float64))
    out = r.copy()
    out[..., 2, :] = np.conj(np.cross(r[..., 0, :], r[..., 1, :]))
    return out


def _block_max(lat, f):
    perm = oracle.block_order(lat)
    Vb = int(np.prod(lat.B))
    return np.abs(np.concatenate([f.real, f.imag], axis=-1))[perm].reshape(lat.V // Vb, -1).max(axis=1)


CASES = [((8, 8, 8, 8), (1, 1, 1, -1)), ((8, 8, 8, 16), (1, 1, 1, 1)), ((16, 8, 8, 8), (1, -1, 1, 1)),
         ((8, 8, 8, 8), (0, 0, 0, 0))]


@pytest.mark.parametrize("L,bc", CASES)
def test_pack_bit_exact(L, bc):
    """Packing rounds to FP16 with the block scales of the storage rule, bit for
    bit; an all-zero block gets scale 1 and stays zero."""
    wdr = _wdr()
    B = (4, 4, 4, 4)
    ctx, lat = wdr.Context(L, B, bc), oracle.Lattice(L, B, bc)
    psi = synth.spinor(L, 1601) * 3.7
    bid, _, _ = lat.maps()
    psi[bid == 1] = 0
    want, s_want = f16_spinor(lat, psi)
    f = ctx.pack(dev(psi), wdr.F16)
    assert f.numel() == ctx.V * 12 * 4 + ctx.nblocks * 4
    torch = torch_cuda()
    s_got = host(f[ctx.V * 12 * 4:].view(torch.float32))
    got = host(ctx.unpack(f, wdr.F16))
    say("f16 pack max |q - psi| / max", rel(got, psi))
    assert np.array_equal(s_got, s_want)
    assert np.array_equal(got, want)
    assert not np.any(got[bid == 1])
    ctx.close()


@pytest.mark.parametrize("L,bc", CASES)
def test_apply_D_f16(L, bc):
    """FP16 stencil against the FP64 oracle on the rounded input and links
    (bound in the module docstring), and against the exact operator."""
    wdr = _wdr()
    B = (4, 4, 4, 4)
    ctx, lat = wdr.Context(L, B, bc), oracle.Lattice(L, B, bc)
    U = synth.gauge_field(L, 0.6, 1602)
    psi = synth.spinor(L, 1603)
    gU = ctx.gauge(dev(U))
    k = 0.155
    q, _ = f16_spinor(lat, psi)
    want = oracle.apply_D(lat, f16_links(U), k, q)
    got = host(ctx.unpack(ctx.apply_D_internal(gU, k, ctx.pack(dev(psi), wdr.F16), ctx.internal_field(wdr.F16),
                                               wdr.F16), wdr.F16))
    perm = oracle.block_order(lat)
    Vb = 256
    err = np.abs(np.concatenate([(got - want).real, (got - want).imag], axis=-1))[perm].reshape(lat.V // Vb, -1)
    bound = 2.0 ** -11 * _block_max(lat, want) * (1 + 1e-5) + 4e-6 * np.abs(want).max()
    exact = oracle.apply_D(lat, U, k, psi)
    say("f16 D: max err / bound", float((err.max(axis=1) / bound).max()), "rel vs exact", rel(got, exact))
    assert np.all(err.max(axis=1) <= bound)
    assert rel(got, exact) < 4e-3
    # the canonical entry point gives the same numbers
    assert np.array_equal(host(ctx.apply_D(gU, k, dev(psi), wdr.F16)), got)
    del gU
    ctx.close()


def test_apply_D_f16_full_size():
    """32^4, the lattice of the FP16 workload, every site against the exact
    FP64 operator and sampled blocks against the rounded-input bound."""
    wdr = _wdr()
    L, B = (32, 32, 32, 32), (4, 4, 4, 4)
    ctx, lat = wdr.Context(L, B), oracle.Lattice(L, B)
    U = synth.gauge_field(L, 0.2, 1604)
    psi = synth.spinor(L, 1605)
    gU = ctx.gauge(dev(U))
    k = 0.155
    got = host(ctx.apply_D(gU, k, dev(psi), wdr.F16))
    exact = oracle.apply_D(lat, U, k, psi)
    say("f16 D 32^4 rel vs exact", rel(got, exact))
    assert rel(got, exact) < 4e-3
    q, _ = f16_spinor(lat, psi)
    want = oracle.apply_D(lat, f16_links(U), k, q)
    d = got - want
    bm = _block_max(lat, want)
    perm = oracle.block_order(lat)
    err = np.abs(np.concatenate([d.real, d.imag], axis=-1))[perm].reshape(lat.V // 256, -1).max(axis=1)
    assert np.all(err <= 2.0 ** -11 * bm * (1 + 1e-5) + 4e-6 * np.abs(want).max())
    del gU
    ctx.close()


def test_f16_errors():
    wdr = _wdr()
    L = (8, 8, 8, 8)
    psi = dev(synth.spinor(L, 1606))
    small = wdr.Context(L, (2, 2, 2, 2))
    gs = small.gauge(dev(synth.gauge_field(L, 0.5, 1607)))
    with pytest.raises(wdr.WdrError) as e:
        small.apply_D(gs, 0.13, psi, wdr.F16)
    assert e.value.status == wdr.EINVAL
    ctx = wdr.Context(L, (4, 4, 4, 4))
    gN = ctx.gauge(dev(1.01 * synth.gauge_field(L, 0.5, 1608)))
    assert not gN.su3
    with pytest.raises(wdr.WdrError) as e:
        ctx.apply_D(gN, 0.13, psi, wdr.F16)
    assert e.value.status == wdr.EINVAL
    gU = ctx.gauge(dev(synth.gauge_field(L, 0.5, 1609)))
    with pytest.raises(wdr.WdrError) as e:
        ctx.apply_Dblock(gU, 0.13, psi, 0, wdr.F16)
    assert e.value.status == wdr.EINVAL
    del gs, gN, gU
    small.close()
    ctx.close()


def f16_half(lat, psi, parity):
    """The FP16 half-field rule of the even-odd CG: per block, the sites of
    one parity, s = 2^ceil(log2 m) over their components; returns the
    rounded field (other parity zero) as complex128."""
    perm = oracle.block_order(lat)
    Vb = int(np.prod(lat.B))
    nb, Vh = lat.V // Vb, Vb // 2
    sites = perm.reshape(nb, Vb)[:, parity * Vh:(parity + 1) * Vh]
    blk = psi[sites].reshape(nb, Vh * 12)
    re, im = blk.real.astype(np.float32), blk.imag.astype(np.float32)
    m = np.maximum(np.abs(re).max(axis=1), np.abs(im).max(axis=1))
    s = _pow2_at_least(m)
    inv = (np.float32(1.0) / s)[:, None]
    hr, hi = _round16(re, inv), _round16(im, inv)
    q = (hr.astype(np.float32) * s[:, None]).astype(np.float64) + 1j * (hi.astype(np.float32) * s[:, None]).astype(
        np.float64)
    out = np.zeros_like(psi)
    out[sites.ravel()] = q.reshape(nb * Vh, 4, 3)
    return out


def _half_block_max(lat, f, parity):
    perm = oracle.block_order(lat)
    Vb = int(np.prod(lat.B))
    sites = perm.reshape(lat.V // Vb, Vb)[:, parity * (Vb // 2):(parity + 1) * (Vb // 2)]
    return np.abs(np.concatenate([f.real, f.imag], axis=-1))[sites].reshape(sites.shape[0], -1).max(axis=1), sites


EO_CASES = [((8, 8, 8, 8), (1, 1, 1, -1)), ((8, 16, 8, 8), (1, -1, 1, 1)), ((8, 8, 8, 8), (0, 0, 0, 0))]


@pytest.mark.parametrize("L,bc", EO_CASES)
def test_eo16_pack_bit_exact(L, bc):
    """FP16 half fields of the even-odd CG: packing each parity follows the
    per-block rule bit for bit, the other parity unpacks to zero."""
    wdr = _wdr()
    B = (4, 4, 4, 4)
    ctx, lat = wdr.Context(L, B, bc), oracle.Lattice(L, B, bc)
    psi = synth.spinor(L, 1611) * 2.3
    _, _, par = lat.maps()
    for p in (0, 1):
        got = host(ctx.unpack_eo16(ctx.pack_eo16(dev(psi), p), p))
        want = f16_half(lat, psi, p)
        say("eo16 pack parity", p, "rel", rel(got, psi * (par == p)[:, None, None]))
        assert np.array_equal(got, want)
        assert not np.any(got[par != p])
    ctx.close()


@pytest.mark.parametrize("L,bc", EO_CASES)
@pytest.mark.parametrize("parity,dag,with_diag", [(0, 0, True), (1, 0, False), (0, 1, False), (1, 1, True)])
def test_eo16_stencil(L, bc, parity, dag, with_diag):
    """One even-odd half in FP16 (the kernel of the FP16 CG): out = diag -
    kappa H_{p,1-p} in (gamma_5-conjugated for dag) against the FP64 oracle
    on the rounded input, diagonal and links: the difference stays within the
    rounding of the output (2^-11 of each block half's maximum) plus the
    packed FP16 arithmetic of the hops (on stored values of magnitude <= 1:
    per hop at most 60 roundings of 2^-11 relative on terms up to 6, times
    kappa and the largest input scale, over 8 hops: 480 kappa 2^-11 s_max);
    and within 4e-3 of the exact operator, the error that matters to the
    solver (observed 5e-4 to 9e-4)."""
    wdr = _wdr()
    B = (4, 4, 4, 4)
    ctx, lat = wdr.Context(L, B, bc), oracle.Lattice(L, B, bc)
    U = synth.gauge_field(L, 0.5, 1612)
    gU = ctx.gauge(dev(U))
    k = 0.152
    psi, dg = synth.spinor(L, 1613), synth.spinor(L, 1614)
    _, _, par = lat.maps()
    fin = ctx.pack_eo16(dev(psi), 1 - parity)
    fdg = ctx.pack_eo16(dev(dg), parity) if with_diag else None
    out = ctx.apply_hop_eo_internal(gU, k, wdr.F16, parity, dag, fin, fdg, ctx.eo16_field())
    got = host(ctx.unpack_eo16(out, parity))

    def expected(links, src, diag):
        # with src on parity 1-p only, (D src) on parity p is -kappa H_{p,1-p} src
        s = oracle.g5(src) if dag else src
        h = oracle.apply_D(lat, links, k, s)
        if dag:
            h = oracle.g5(h)
        h[par != parity] = 0
        return h + (diag if diag is not None else 0)

    q = f16_half(lat, psi, 1 - parity)
    qd = f16_half(lat, dg, parity) if with_diag else None
    want = expected(f16_links(U), q, qd)
    bm, sites = _half_block_max(lat, want, parity)
    d = got - want
    err = np.abs(np.concatenate([d.real, d.imag], axis=-1))[sites].reshape(sites.shape[0], -1).max(axis=1)
    s_max = 2 * np.abs(q).max()  # the block scales stay below twice the largest component
    bound = 2.0 ** -11 * bm * (1 + 1e-5) + 480 * k * 2.0 ** -11 * s_max
    exact = expected(U, psi * (par == 1 - parity)[:, None, None], dg * (par == parity)[:, None, None]
                     if with_diag else None)
    say("eo16 p", parity, "dag", dag, "diag", with_diag, "max err / bound", float((err / bound).max()),
        "rel vs exact", rel(got, exact))
    assert not np.any(got[par != parity])
    assert np.all(err <= bound)
    assert rel(got, exact) < 4e-3
    # several systems in one launch give each system's result
    # two systems: all values first, then all block scales
    vals, nsc = fin.numel() - ctx.nblocks * 4, ctx.nblocks * 4

    def twice(f):
        f2 = ctx.eo16_field(2)
        f2[:vals] = f[:vals]
        f2[vals:2 * vals] = f[:vals]
        f2[2 * vals:2 * vals + nsc] = f[vals:]
        f2[2 * vals + nsc:] = f[vals:]
        return f2
    f2 = twice(fin)
    d2 = twice(fdg) if with_diag else None
    o2 = ctx.apply_hop_eo_internal(gU, k, wdr.F16, parity, dag, f2, d2, ctx.eo16_field(2), nsys=2)
    torch = torch_cuda()
    assert torch.equal(o2[:vals], out[:vals]) and torch.equal(o2[vals:2 * vals], out[:vals])
    assert torch.equal(o2[2 * vals:2 * vals + ctx.nblocks * 4], out[vals:])
    assert torch.equal(o2[2 * vals + ctx.nblocks * 4:], out[vals:])
    del gU
    ctx.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_eo_halves_internal(prec):
    """The FP64 and FP32 even-odd halves on internal fields (one launch each)
    against the oracle, with and without the diagonal term and gamma_5."""
    wdr = _wdr()
    L, B = (8, 8, 8, 8), (4, 4, 4, 4)
    ctx, lat = wdr.Context(L, B, (1, 1, 1, -1)), oracle.Lattice(L, B, (1, 1, 1, -1))
    U = synth.gauge_field(L, 0.5, 1615)
    gU = ctx.gauge(dev(U))
    k = 0.147
    psi, dg = synth.spinor(L, 1616), synth.spinor(L, 1617)
    _, _, par = lat.maps()
    for parity in (0, 1):
        for dag in (0, 1):
            src = psi * (par == 1 - parity)[:, None, None]
            h = oracle.apply_D(lat, U, k, oracle.g5(src) if dag else src)
            if dag:
                h = oracle.g5(h)
            h[par != parity] = 0
            want = h + dg * (par == parity)[:, None, None]
            out = ctx.internal_field(prec)
            ctx.apply_hop_eo_internal(gU, k, prec, parity, dag, ctx.pack(dev(psi), prec), ctx.pack(dev(dg), prec),
                                      out)
            got = host(ctx.unpack(out, prec))
            got[par != parity] = 0
            say("eo halves prec", prec, "p", parity, "dag", dag, "rel", rel(got, want))
            assert rel(got, want) < (1e-14 if prec == 0 else 2e-6)
    del gU
    ctx.close()
