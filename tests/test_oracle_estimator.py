"""Pins of the oracle's path (paper Sec. 4, eq. param), its stochastic
samples (Sec. 4) and the combination into log Rhat."""
import numpy as np
import pytest
import scipy.linalg

import oracle
from paper_1112_1243_amd import synth


# ---------------------------------------------------------------- path

def _pair(L, scale, p, seed):
    U = synth.gauge_field(L, scale, seed)
    Up = synth.redraw(U, synth.bernoulli_links(L, p, seed), scale, seed)
    return U, Up


def test_path_endpoints_and_su3():
    U, Up = _pair((4, 4, 4, 4), 0.6, 0.3, 41)
    N = 5
    assert np.array_equal(oracle.interpolate(U, Up, 0, N), U)
    assert np.array_equal(oracle.interpolate(U, Up, N, N), Up)
    same = np.all((U == Up).reshape(-1, 4, 9), axis=2)
    for i in range(1, N):
        Ui = oracle.interpolate(U, Up, i, N)
        assert np.array_equal(Ui[same], U[same])
        eye = np.eye(3)
        assert np.abs(Ui @ np.conj(np.swapaxes(Ui, -1, -2)) - eye).max() < 1e-13
        assert np.abs(np.linalg.det(Ui) - 1).max() < 1e-13


def test_path_is_geodesic():
    """Every step U_{i+1} U_i^+ = exp(log(W)/N): equal steps of length
    ||log W|| / N."""
    U, Up = _pair((2, 2, 2, 2), 1.0, 1.0, 42)
    N = 4
    W = Up @ np.conj(np.swapaxes(U, -1, -2))
    th = np.angle(np.linalg.eigvals(W))
    steps = []
    for i in range(N):
        a = oracle.interpolate(U, Up, i, N)
        b = oracle.interpolate(U, Up, i + 1, N)
        S = b @ np.conj(np.swapaxes(a, -1, -2))
        steps.append(np.angle(np.linalg.eigvals(S)))
    norms = [np.sort(np.abs(s), axis=-1) for s in steps]
    for n in norms[1:]:
        assert np.abs(n - norms[0]).max() < 1e-10
    # lengths: |theta_j| / N for links whose principal angles sum to zero
    ok = np.abs(th.sum(-1)) < 1e-9
    assert np.abs(np.sort(np.abs(th[ok]), -1) / N - norms[0][ok]).max() < 1e-10


def test_path_matches_scipy_fractional_power():
    """Where the principal log is already traceless, U_i = W^(i/N) U with
    scipy's principal fractional matrix power."""
    U, Up = _pair((2, 2, 2, 2), 0.8, 1.0, 43)
    N = 3
    U1 = oracle.interpolate(U, Up, 1, N)
    W = Up @ np.conj(np.swapaxes(U, -1, -2))
    checked = 0
    for s in range(U.shape[0]):
        for mu in range(4):
            th = np.angle(np.linalg.eigvals(W[s, mu]))
            if abs(th.sum()) > 1e-9:
                continue
            want = scipy.linalg.fractional_matrix_power(W[s, mu], 1.0 / N) @ U[s, mu]
            assert np.abs(U1[s, mu] - want).max() < 1e-10
            checked += 1
    assert checked > 20


# ---------------------------------------------------------------- samples

def _dense_ops(lat, U, k):
    D = oracle.dense(lambda v: oracle.apply_D(lat, U, k, v), lat.V)
    return D


def _schur_dense(lat, D):
    _, col, _ = lat.maps()
    bl = oracle.site_dofs(col == 0)
    wh = oracle.site_dofs(col == 1)
    A = D[np.ix_(bl, bl)]
    Bm = D[np.ix_(bl, wh)]
    C = D[np.ix_(wh, bl)]
    E = D[np.ix_(wh, wh)]
    return np.eye(len(bl)) - np.linalg.solve(A, Bm @ np.linalg.solve(E, C)), bl


def _quad(M, e):
    Me = M @ e
    return float(np.vdot(e, e).real - np.vdot(Me, Me).real)


@pytest.fixture(scope="module")
def small_case():
    lat = oracle.Lattice((4, 4, 4, 4), B=(2, 2, 2, 2))
    U, Up = _pair(lat.L, 0.5, 0.15, 44)
    k = 0.12
    return lat, U, Up, k, _dense_ops(lat, U, k), _dense_ops(lat, Up, k)


def test_sample_full_dense(small_case):
    lat, U, Up, k, D0, D1 = small_case
    eta = oracle.noise(lat, oracle.NOISE_GAUSS, 9, 0, 0)
    s = oracle.sample(lat, U, Up, k, oracle.OP_FULL, eta)
    M = np.linalg.solve(D1, D0)
    assert abs(s - _quad(M, eta.reshape(-1))) < 1e-9


def test_sample_blocks_dense(small_case):
    lat, U, Up, k, D0, D1 = small_case
    eta = oracle.noise(lat, oracle.NOISE_GAUSS, 9, 0, 1)
    s = oracle.sample(lat, U, Up, k, oracle.OP_BLOCKS, eta)
    bid, _, _ = lat.maps()
    assert s.shape == (lat.nblocks,)
    for b in range(lat.nblocks):
        idx = oracle.site_dofs(bid == b)
        M = np.linalg.solve(D1[np.ix_(idx, idx)], D0[np.ix_(idx, idx)])
        assert abs(s[b] - _quad(M, eta.reshape(-1)[idx])) < 1e-10


def test_sample_schur_dense(small_case):
    lat, U, Up, k, D0, D1 = small_case
    black = oracle.colour_mask(lat, 0)
    eta = oracle.noise(lat, oracle.NOISE_GAUSS, 9, 0, 2, support=black)
    s = oracle.sample(lat, U, Up, k, oracle.OP_SCHUR, eta)
    S0, bl = _schur_dense(lat, D0)
    S1, _ = _schur_dense(lat, D1)
    M = np.linalg.solve(S1, S0)
    assert abs(s - _quad(M, eta.reshape(-1)[bl])) < 1e-9


def test_sample_unchanged_field_is_zero(small_case):
    lat, U, _, k, _, _ = small_case
    for op in (oracle.OP_FULL, oracle.OP_SCHUR):
        eta = oracle.noise(lat, oracle.NOISE_GAUSS, 1, 0, 0, support=oracle.noise_support(lat, op))
        assert abs(oracle.sample(lat, U, U, k, op, eta)) < 1e-9


@pytest.mark.parametrize("kind", [oracle.NOISE_GAUSS, oracle.NOISE_Z2])
def test_sample_mean_is_minus_trace(kind):
    """E[s] = -tr(M^+ M - 1) for any noise with E[eta eta^+] = 1 (Sec. 4);
    the samples here use the dense M so only the noise is under test."""
    lat = oracle.Lattice((4, 4, 2, 2))
    U, Up = _pair(lat.L, 0.5, 0.2, 45)
    k = 0.12
    M = np.linalg.solve(_dense_ops(lat, Up, k), _dense_ops(lat, U, k))
    A = M.conj().T @ M - np.eye(M.shape[0])
    s = np.array([-np.vdot(e, A @ e).real for e in
                  (oracle.noise(lat, kind, 100 + j, 0, 0).reshape(-1) for j in range(3000))])
    assert abs(s.mean() + np.trace(A).real) < 4 * s.std() / np.sqrt(len(s))
    if kind == oracle.NOISE_GAUSS:
        var = np.trace(A @ A).real
        assert abs(s.var() / var - 1) < 0.15


def test_exp_sample_estimates_det_ratio():
    """E[exp(s)] = det(M^+ M)^-1 = det(D'^+D')/det(D^+D) for complex
    Gaussian noise when lambda_min(M^+ M) > 1/2 (Sec. 4)."""
    lat = oracle.Lattice((4, 4, 2, 2))
    U, Up = _pair(lat.L, 0.3, 0.05, 46)
    k = 0.1
    D0, D1 = _dense_ops(lat, U, k), _dense_ops(lat, Up, k)
    M = np.linalg.solve(D1, D0)
    MM = M.conj().T @ M
    assert np.linalg.eigvalsh(MM).min() > 0.5
    A = MM - np.eye(M.shape[0])
    es = np.array([np.exp(-np.vdot(e, A @ e).real) for e in
                   (oracle.noise(lat, oracle.NOISE_GAUSS, 500 + j, 0, 0).reshape(-1) for j in range(4000))])
    want = np.exp(2 * (oracle.log_abs_det(D1) - oracle.log_abs_det(D0)))
    assert abs(es.mean() - want) < 4 * es.std() / np.sqrt(len(es))


# ---------------------------------------------------------------- log ratio

def test_param_factorisation_and_bias():
    """eq. param: prod_i det(M_i^+ M_i) = det(M^+ M); the expectation of
    sum_i s_i, -sum_i tr(M_i^+ M_i - 1), approaches log R like 1/N."""
    lat = oracle.Lattice((4, 4, 2, 2))
    U, Up = _pair(lat.L, 0.5, 0.2, 47)
    k = 0.12
    exact = oracle.exact_log_ratio(lat, U, Up, k)
    gaps = []
    for N in (2, 4, 8):
        Ds = [_dense_ops(lat, oracle.interpolate(U, Up, i, N), k) for i in range(N + 1)]
        logdets = [oracle.log_abs_det(D) for D in Ds]
        assert abs(2 * (logdets[-1] - logdets[0]) - exact) < 1e-9
        tr = 0.0
        for i in range(N):
            M = np.linalg.solve(Ds[i + 1], Ds[i])
            tr += -np.trace(M.conj().T @ M - np.eye(M.shape[0])).real
        gaps.append(tr - exact)
    assert gaps[0] < 0 and gaps[1] < 0 and gaps[2] < 0    # log(1+x) <= x
    assert 1.6 < gaps[0] / gaps[1] < 2.6 and 1.6 < gaps[1] / gaps[2] < 2.6


def test_logdet_ratio_mean_over_seeds():
    """Mean of log Rhat (N steps, K = 1) over seeds equals
    -sum_i tr(M_i^+ M_i - 1) within statistics."""
    lat = oracle.Lattice((4, 4, 2, 2))
    U, Up = _pair(lat.L, 0.5, 0.2, 48)
    k = 0.12
    N = 3
    Ds = [_dense_ops(lat, oracle.interpolate(U, Up, i, N), k) for i in range(N + 1)]
    want = 0.0
    for i in range(N):
        M = np.linalg.solve(Ds[i + 1], Ds[i])
        want += -np.trace(M.conj().T @ M - np.eye(M.shape[0])).real
    vals = []
    for seed in range(40):
        samples, lr = oracle.logdet_ratio(lat, U, Up, k, oracle.OP_FULL, N, 1, oracle.NOISE_GAUSS, 1000 + seed)
        assert samples.shape == (N, 1)
        assert abs(lr - samples.sum()) < 1e-12
        vals.append(lr)
    vals = np.array(vals)
    assert abs(vals.mean() - want) < 4 * vals.std() / np.sqrt(len(vals))


def test_combine_log_mean_exp():
    """The combination of eq. param (the product over factors of the noise
    average of exp(sample), Sec. 4), pinned by facts that do not retype it:
    hand-computed cases, invariances, overflow-safe values and the law of
    large numbers for log-normal samples."""
    # hand-computed: log((1 + 3) / 2) = log 2, and a constant factor is itself
    assert abs(oracle.combine(np.array([[0.0, np.log(3.0)]])) - np.log(2.0)) < 1e-15
    assert abs(oracle.combine(np.array([[0.7, 0.7, 0.7], [-1.2, -1.2, -1.2]])) - (0.7 - 1.2)) < 1e-15
    # factors add, noise vectors average: reordering the noise vectors of a
    # factor changes nothing, shifting a factor's samples by c shifts log R by c
    rng = np.random.Generator(np.random.Philox(key=[3, 5]))
    s = rng.normal(0.0, 1.0, (4, 6))
    base = oracle.combine(s)
    assert abs(oracle.combine(s[:, ::-1]) - base) < 1e-13
    assert abs(oracle.combine(s + np.array([[0.5], [0.0], [-2.0], [1.0]])) - (base - 0.5)) < 1e-13
    assert abs(oracle.combine(s[:2]) + oracle.combine(s[2:]) - base) < 1e-13
    # Jensen: the log of the mean exceeds the mean of the logs (unbiased in R,
    # not in log R), equal only for constant samples
    assert base > s.mean(axis=1).sum()
    # samples near 800 overflow exp in FP64: the value must still be exact
    assert abs(oracle.combine(np.array([[800.0, 801.0]])) - (800.0 + np.log((1.0 + np.e) / 2.0))) < 1e-12
    # log-normal samples: E exp(s) = exp(mu + sigma^2 / 2) for s ~ N(mu, sigma^2)
    mu, sig = -0.4, 0.6
    big = rng.normal(mu, sig, (1, 400000))
    assert abs(oracle.combine(big) - (mu + sig * sig / 2)) < 5e-3
    # the blocks axis of a DD estimate is carried through factor by factor
    s3 = rng.normal(0.0, 1.0, (3, 5, 2))
    got = oracle.combine(s3)
    assert got.shape == (2,)
    for b in range(2):
        assert abs(got[b] - oracle.combine(s3[:, :, b])) < 1e-13
