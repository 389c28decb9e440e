"""GPU parity at the full sizes of the 16^4 and 32^4 workloads, in the
launch configuration the benchmark times (every path factor a system of one
batched estimate, the mixed-precision solver settings of the workload).

Samples are checked element by element against stored oracle values
(tests/golden/schur_samples_*.txt, written by tests/golden/make_golden.py,
which calls only the oracle); the solutions of one Schur sample at 32^4 are
checked with the oracle's own stencil.  Paper Sec. 4 (eq. param: one
inversion per factor), Sec. 3 (eq. ddfactor)."""
import os

import numpy as np
import pytest

import oracle
from tests.golden import make_golden
from tests.gpu_util import dev, host, say, torch_cuda

pytestmark = pytest.mark.gpu


def _golden(name):
    vals = {}
    with open(make_golden.path_file(name)) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            i, k, s = line.split()
            vals[(int(i), int(k))] = float(s)
    return vals


@pytest.fixture(scope="module", params=["wilson16_dd256", "wilson32_dd4096"])
def workload(request):
    torch_cuda()
    from paper_1112_1243_amd import wdr
    name = request.param
    if not os.path.exists(make_golden.path_file(name)):
        pytest.skip("stored oracle samples for %s not written" % name)
    say("inputs", name)
    w, lat, U, Up = make_golden.inputs(name)
    ctx = wdr.Context(w["L"], w["B"])
    gU, gUp = ctx.gauge(dev(U)), ctx.gauge(dev(Up))
    say("uploaded", name)
    yield name, w, lat, ctx, U, Up, gU, gUp
    del gU, gUp
    ctx.close()


def test_schur_samples_match_stored_oracle(workload):
    """The workload's estimate (SCHUR ratio, N factors x 1 Gaussian noise,
    all factors batched) with its mixed-precision solver settings: the stored
    oracle samples of the first and last factor within 1e-8."""
    from paper_1112_1243_amd import wdr
    name, w, lat, ctx, U, Up, gU, gUp = workload
    N, steps = make_golden.CASES[name]
    assert N == w["n_noise"]
    p = wdr.default_params(**w["mixed"])
    s, lr, info = ctx.logdet_ratio(gU, gUp, w["kappa"], wdr.OP_SCHUR, N, 1, wdr.NOISE_GAUSS, w["seed"], p)
    want = _golden(name)
    assert set(want) == {(i, 0) for i in steps}
    for (i, k), v in sorted(want.items()):
        say(name, "factor", i, "gpu %.12f oracle %.12f diff %.2e" % (s[i, k], v, abs(s[i, k] - v)))
    assert info.converged and info.true_rel_resid <= 1e-10
    err = max(abs(s[i, k] - v) for (i, k), v in want.items())
    assert err < 1e-8
    assert np.all(np.isfinite(s))


def test_solutions_of_one_sample_pass_the_oracle_stencil(workload):
    """For the Schur sample of factor 0: the right-hand side y = A' Dhat eta
    built from the library's calls, the global solve D' z = y and the
    adjoint solve D' v = g5 P z with the workload's mixed settings; the
    oracle's stencil gives ||y - D' z|| <= 1.05e-10 ||y|| and the adjoint
    residual <= 1.05 adj_tol (the second-order sample needs no more)."""
    from paper_1112_1243_amd import wdr
    name, w, lat, ctx, U, Up, gU, gUp = workload
    if name != "wilson32_dd4096":
        pytest.skip("checked at the largest size")
    N = w["n_noise"]
    U1 = oracle.interpolate(U, Up, 1, N)
    g1 = ctx.gauge(dev(U1))
    p = wdr.default_params(**w["mixed"])
    kappa = w["kappa"]
    eta = ctx.noise(wdr.NOISE_GAUSS, w["seed"], 0, 0, black_only=True)
    phi = ctx.schur(gU, kappa, eta, p)
    y = ctx.apply_Dblock(g1, kappa, phi, 0)
    z, info = ctx.solve(g1, kappa, y, p)
    yh, zh = host(y), host(z)
    r = np.linalg.norm(yh - oracle.apply_D(lat, U1, kappa, zh)) / np.linalg.norm(yh)
    say("32^4 global solve", info.as_dict(), "oracle residual %.3e" % r)
    assert info.converged and r <= 1.05e-10
    black = oracle.colour_mask(lat, 0)
    pz = zh.copy()
    pz[~black] = 0
    rhs = oracle.g5(pz)
    pa = wdr.default_params(**w["mixed"])
    pa.tol = p.adj_tol
    v, ainfo = ctx.solve(g1, kappa, dev(rhs), pa)
    ra = np.linalg.norm(rhs - oracle.apply_D(lat, U1, kappa, host(v))) / np.linalg.norm(rhs)
    say("32^4 adjoint solve", ainfo.as_dict(), "oracle residual %.3e" % ra)
    assert ainfo.converged and ra <= 1.05 * p.adj_tol
    del g1
