"""GPU parity of batched estimates over several proposals (per-system links,
hopping parameter and noise key in one set of launches; groups of different
lattice sizes on their own streams) against the FP64 oracle and against
single-proposal calls; mixed-precision CGNE."""
import numpy as np
import pytest

import oracle
from paper_1112_1243_amd import synth
from tests.gpu_util import dev, say, torch_cuda

pytestmark = pytest.mark.gpu


def _proposal(wdr, ctx, lat, scale, seed, kappa, noise_seed):
    U = synth.gauge_field(lat.L, scale, seed)
    Up = synth.redraw(U, synth.bernoulli_links(lat.L, 0.1, seed + 1), scale, seed + 1)
    return dict(U=U, Up=Up, gU=ctx.gauge(dev(U)), gUp=ctx.gauge(dev(Up)), kappa=kappa, seed=noise_seed, ctx=ctx,
                lat=lat)


def test_batch_of_uneven_lattices_matches_oracle():
    """Two 4^4 proposals, one 8^4 and one 12^4 proposal (FULL ratio, Z2
    noise, CGNE with FP32 iterations) in one call: every sample within 1e-8
    of the oracle and equal to the single-proposal call.  The 12^4 lattice is
    the middle size of the batched workload: 81 blocks of 4^4, three per
    direction (no 2-colouring; the full operator needs none), a block count
    that is not a multiple of the 8 XCDs."""
    torch_cuda()
    from paper_1112_1243_amd import wdr
    L4, L8, L12 = (4, 4, 4, 4), (8, 8, 8, 8), (12, 12, 12, 12)
    c4, c8, c12 = wdr.Context(L4, (2, 2, 2, 2)), wdr.Context(L8, (4, 4, 4, 4)), wdr.Context(L12, (4, 4, 4, 4))
    l4, l8 = oracle.Lattice(L4, (2, 2, 2, 2)), oracle.Lattice(L8, (4, 4, 4, 4))
    l12 = oracle.Lattice(L12, (4, 4, 4, 4))
    assert c12.nblocks == 81
    props = [_proposal(wdr, c4, l4, 0.3, 401, 0.12, 1112124400),
             _proposal(wdr, c8, l8, 0.3, 403, 0.13, 1112124401),
             _proposal(wdr, c12, l12, 0.3, 407, 0.125, 1112124403),
             _proposal(wdr, c4, l4, 0.3, 405, 0.14, 1112124402)]
    N, K = 2, 1
    p = wdr.default_params(solver=wdr.SOLVER_CGNE)
    samples, lrs, info = wdr.logdet_ratio_batch([(q["ctx"], q["gU"], q["gUp"], q["kappa"], q["seed"]) for q in props],
                                                wdr.OP_FULL, N, K, wdr.NOISE_Z2, p)
    say("batch info", info.as_dict())
    assert info.converged
    for q, s, lr in zip(props, samples, lrs):
        want, lr_want = oracle.logdet_ratio(q["lat"], q["U"], q["Up"], q["kappa"], oracle.OP_FULL, N, K,
                                            oracle.NOISE_Z2, q["seed"])
        say("proposal", q["lat"].L, q["kappa"], "max |ds|", np.abs(s - want).max())
        assert s.shape == want.shape and np.abs(s - want).max() < 1e-8
        assert abs(lr - float(np.sum(lr_want))) < 1e-8 * s.size
        s1, lr1, _ = q["ctx"].logdet_ratio(q["gU"], q["gUp"], q["kappa"], wdr.OP_FULL, N, K, wdr.NOISE_Z2, q["seed"], p)
        assert np.abs(s1 - s).max() < 1e-12 and abs(lr1 - lr) < 1e-12
    for q in props:
        del q["gU"], q["gUp"]
    c4.close()
    c8.close()
    c12.close()


@pytest.mark.parametrize("op", [oracle.OP_SCHUR, oracle.OP_BLOCKS])
def test_batch_one_context_per_system_kappa(op):
    """Proposals with different kappa on one 8^4 context (FGCR + SAP, block
    solves): the batch equals the single-proposal calls, also when solved
    one sample at a time (max_batch = 1)."""
    torch_cuda()
    from paper_1112_1243_amd import wdr
    L, B = (8, 8, 8, 8), (4, 4, 4, 4)
    ctx, lat = wdr.Context(L, B), oracle.Lattice(L, B)
    props = []
    for j, kappa in enumerate((0.125, 0.135)):
        U = synth.gauge_field(L, 0.5, 410 + j)
        Up = synth.redraw(U, oracle.active_links(lat), 0.5, 420 + j)
        props.append((ctx, ctx.gauge(dev(U)), ctx.gauge(dev(Up)), kappa, 7 + j))
    p = wdr.default_params()
    N, K = 2, 1
    samples, lrs, info = wdr.logdet_ratio_batch(props, op, N, K, wdr.NOISE_GAUSS, p)
    one, lr_one, _ = wdr.logdet_ratio_batch(props, op, N, K, wdr.NOISE_GAUSS, p, max_batch=1)
    assert info.converged
    for (c, gU, gUp, kappa, seed), s, lr, s_1, l_1 in zip(props, samples, lrs, one, lr_one):
        s1, lr1, _ = ctx.logdet_ratio(gU, gUp, kappa, op, N, K, wdr.NOISE_GAUSS, seed, p)
        say("kappa", kappa, "batch vs single", np.abs(s1 - s).max(), "max_batch 1", np.abs(s_1 - s).max())
        assert np.abs(s1 - s).max() < 1e-12 and abs(lr1 - lr) < 1e-10
        assert np.abs(s_1 - s).max() < 1e-12
    del props
    ctx.close()


def test_cgne_graph_replays_match_eager():
    """Mixed CGNE with each update period replayed as a HIP graph equals the
    same solve launched kernel by kernel, on three calls in a row with eager
    work in between (proposals of different kappa retire at different
    periods, so the launch list shrinks and the graph is re-captured); other
    update periods stay within 1e-8 of the oracle."""
    import torch
    torch_cuda()
    from paper_1112_1243_amd import wdr
    L, B = (8, 8, 8, 8), (4, 4, 4, 4)
    ctx, lat = wdr.Context(L, B), oracle.Lattice(L, B)
    qs = [_proposal(wdr, ctx, lat, 0.3, 430 + 2 * j, kappa, 1112124410 + j)
          for j, kappa in enumerate((0.12, 0.125, 0.13, 0.14))]
    props = [(ctx, q["gU"], q["gUp"], q["kappa"], q["seed"]) for q in qs]
    N, K = 2, 2
    eager = wdr.default_params(solver=wdr.SOLVER_CGNE, graph=0)
    graph = wdr.default_params(solver=wdr.SOLVER_CGNE, graph=1)
    s0, lr0, i0 = wdr.logdet_ratio_batch(props, wdr.OP_FULL, N, K, wdr.NOISE_Z2, eager)
    assert i0.converged
    for rep in range(3):
        s1, lr1, i1 = wdr.logdet_ratio_batch(props, wdr.OP_FULL, N, K, wdr.NOISE_Z2, graph)
        d = max(np.abs(a - b).max() for a, b in zip(s1, s0))
        say("graph replay", rep, "max |ds| vs eager", d, i1.as_dict())
        assert i1.converged and d < 1e-12 and np.allclose(lr1, lr0, rtol=0, atol=1e-10)
        x = torch.randn(1 << 20, device="cuda")
        assert torch.isfinite(x.sum()).item()
        s0b, _, _ = wdr.logdet_ratio_batch(props, wdr.OP_FULL, N, K, wdr.NOISE_Z2, eager)
        assert max(np.abs(a - b).max() for a, b in zip(s0b, s0)) < 1e-12
    for ue in (1, 3, 9):
        p = wdr.default_params(solver=wdr.SOLVER_CGNE, update_every=ue)
        s2, _, i2 = wdr.logdet_ratio_batch(props[:2], wdr.OP_FULL, N, K, wdr.NOISE_Z2, p)
        assert i2.converged
        for q, s in zip(qs[:2], s2):
            want, _ = oracle.logdet_ratio(lat, q["U"], q["Up"], q["kappa"], oracle.OP_FULL, N, K,
                                          oracle.NOISE_Z2, q["seed"])
            say("update_every", ue, "kappa", q["kappa"], "max |ds|", np.abs(s - want).max())
            assert np.abs(s - want).max() < 1e-8
    del props, qs
    ctx.close()
