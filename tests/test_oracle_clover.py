"""Pins of the oracle's clover term (Sheikholeslami-Wohlert; the action Sec. 3
defines the active links for and Sec. 7 names as the next one): closed forms
on constant abelian fields, the unit field, hermiticity and chirality,
gauge covariance, the exact set of sites a link reaches, and the samples of
the clover operator against dense linear algebra."""
import itertools

import numpy as np
import pytest

import oracle
from paper_1112_1243_amd import synth


def _flux_field(L, a, b, n):
    """U(1) links times the colour identity with the same plaquette
    exp(i phi), phi = 2 pi n / (L_a L_b), on every (a, b) plaquette (run a-side
    first) and 1 on every other plaquette: U_b(x) = exp(i phi x_a), and
    U_a(x) = exp(-i phi L_a x_b) on the last slice x_a = L_a - 1 (the twist
    that closes the flux on the torus)."""
    V = int(np.prod(L))
    lat = oracle.Lattice(L)
    x = lat.coords()
    phi = 2 * np.pi * n / (L[a] * L[b])
    th = np.zeros((V, 4))
    th[:, b] = phi * x[:, a]
    last = x[:, a] == L[a] - 1
    th[last, a] = -phi * L[a] * x[last, b]
    U = np.exp(1j * th)[:, :, None, None] * np.eye(3)[None, None]
    return lat, np.ascontiguousarray(U), phi


def _plaquette(lat, U, s, a, b):
    sh = lambda s, mu: oracle.core._shift(lat, s, mu, 1)
    return U[s, a] @ U[sh(s, a), b] @ np.conj(U[sh(s, b), a]).T @ np.conj(U[s, b]).T


def test_flux_field_has_the_stated_plaquettes():
    lat, U, phi = _flux_field((4, 6, 4, 4), 0, 1, 1)
    for s in range(0, lat.V, 7):
        for a, b in itertools.permutations(range(4), 2):
            want = np.exp(1j * phi) if (a, b) == (0, 1) else np.exp(-1j * phi) if (a, b) == (1, 0) else 1.0
            assert np.abs(_plaquette(lat, U, s, a, b) - want * np.eye(3)).max() < 1e-12


@pytest.mark.parametrize("plane", [(0, 1), (0, 3)])
def test_abelian_closed_forms(plane):
    """On the flux field of plane (a, b) each of the four leaves is exp(i phi),
    Fhat_ab = i sin(phi) and T = -c_sw kappa sin(phi) sigma_ab.  Worked out by
    hand in the chiral basis (gamma_k = [[0, -i s_k], [i s_k, 0]], gamma_4 =
    [[0, 1], [1, 0]]):
        sigma_01 = i gamma_1 gamma_2 = -diag(s_3, s_3)  =>  T = c k sin(phi) diag(1, -1, 1, -1)
        sigma_03 = i gamma_1 gamma_4 = diag(s_1, -s_1)  =>  T = -c k sin(phi) [[s_1, 0], [0, -s_1]]
    (times the colour identity; the same at every site)."""
    a, b = plane
    L = (4, 6, 4, 6)
    lat, U, phi = _flux_field(L, a, b, 1)
    csw, kappa = 1.7, 0.13
    T = oracle.clover_term(lat, U, csw, kappa).reshape(lat.V, 4, 3, 4, 3)
    c = csw * kappa * np.sin(phi)
    if plane == (0, 1):
        spin = c * np.diag([1.0, -1.0, 1.0, -1.0])
    else:
        s1 = np.array([[0.0, 1.0], [1.0, 0.0]])
        spin = -c * np.block([[s1, np.zeros((2, 2))], [np.zeros((2, 2)), -s1]])
    want = np.einsum("st,ab->satb", spin, np.eye(3))
    assert np.abs(T - want[None]).max() < 1e-13
    assert abs(c) > 0.05  # the field is not trivially small


def test_unit_field_has_no_clover_term():
    """Fhat = 0 on the unit field, so D keeps its free-field closed forms."""
    lat = oracle.Lattice((4, 4, 4, 6), bc=(1, 1, 1, -1))
    U = synth.unit_gauge(lat.L)
    T = oracle.clover_term(lat, U, 1.9, 0.13)
    assert np.all(T == 0)
    psi = synth.spinor(lat.L, 3)
    assert np.array_equal(oracle.apply_D(lat, U, 0.13, psi, T), oracle.apply_D(lat, U, 0.13, psi))


def test_hermitian_chiral_traceless():
    """T(x) is hermitian, commutes with gamma_5 (no entries between the two
    chiralities) and has zero trace over spin for every colour pair."""
    lat = oracle.Lattice((4, 4, 4, 4))
    U = synth.gauge_field(lat.L, 0.8, 21)
    T = oracle.clover_term(lat, U, 1.5, 0.14)
    assert np.abs(T - np.conj(np.swapaxes(T, 1, 2))).max() < 1e-14
    T5 = T.reshape(lat.V, 4, 3, 4, 3)
    assert np.abs(T5[:, :2, :, 2:, :]).max() == 0 and np.abs(T5[:, 2:, :, :2, :]).max() == 0
    assert np.abs(np.einsum("xsasb->xab", T5)).max() < 1e-14
    assert np.abs(T).max() > 0.05


def test_gauge_covariance():
    """T[U^g](x) = g(x) T[U](x) g(x)^+ (acting on colour), U^g_mu(x) =
    g(x) U_mu(x) g(x+mu)^+: every leaf is a closed loop at x."""
    lat = oracle.Lattice((4, 4, 4, 4))
    U = synth.gauge_field(lat.L, 0.8, 22)
    g = synth.gauge_field(lat.L, 2.0, 23)[:, 0]
    x = lat.coords()
    Ug = np.empty_like(U)
    for mu in range(4):
        y = x.copy()
        y[:, mu] = (y[:, mu] + 1) % lat.L[mu]
        t = y[:, 0] + lat.L[0] * (y[:, 1] + lat.L[1] * (y[:, 2] + lat.L[2] * y[:, 3]))
        Ug[:, mu] = g @ U[:, mu] @ np.conj(np.swapaxes(g[t], -1, -2))
    T = oracle.clover_term(lat, U, 1.3, 0.12).reshape(lat.V, 4, 3, 4, 3)
    Tg = oracle.clover_term(lat, Ug, 1.3, 0.12).reshape(lat.V, 4, 3, 4, 3)
    want = np.einsum("xab,xsbtc,xdc->xsatd", g, T, np.conj(g))
    assert np.abs(Tg - want).max() < 1e-13


def test_one_link_reaches_exactly_its_plaquette_corners():
    """Changing the link U_mu(y) changes T at the corners of the plaquettes
    that contain it and nowhere else: y, y + mu, and y + nu, y + mu + nu,
    y - nu, y + mu - nu for every nu != mu (14 sites)."""
    lat = oracle.Lattice((4, 4, 4, 4))
    U = synth.gauge_field(lat.L, 0.7, 24)
    T0 = oracle.clover_term(lat, U, 1.0, 0.125)
    y, mu = 77, 2
    U2 = U.copy()
    U2[y, mu] = synth.gauge_field((1, 1, 1, 1), 1.0, 25)[0, 0] @ U[y, mu]
    T1 = oracle.clover_term(lat, U2, 1.0, 0.125)
    changed = set(np.nonzero(np.abs(T1 - T0).max(axis=(1, 2)) > 1e-12)[0].tolist())
    sh = lambda s, nu, d: oracle.core._shift(lat, s, nu, d)
    ym = sh(y, mu, 1)
    want = {y, ym}
    for nu in range(4):
        if nu != mu:
            want |= {sh(y, nu, 1), sh(ym, nu, 1), sh(y, nu, -1), sh(ym, nu, -1)}
    assert len(want) == 14
    assert changed == want


def test_clover_operator_gamma5_hermitian():
    lat = oracle.Lattice((4, 4, 4, 6), bc=(1, 1, 1, -1))
    U = synth.gauge_field(lat.L, 0.7, 26)
    kappa = 0.13
    T = oracle.clover_term(lat, U, 1.8, kappa)
    psi = synth.spinor(lat.L, 1)
    chi = synth.spinor(lat.L, 2)
    lhs = np.vdot(chi, oracle.g5(oracle.apply_D(lat, U, kappa, oracle.g5(psi), T)))
    rhs = np.vdot(oracle.apply_D(lat, U, kappa, chi, T), psi)
    assert abs(lhs - rhs) < 1e-11 * abs(rhs)
    # the clover term changes D
    assert np.abs(oracle.apply_D(lat, U, kappa, psi, T) - oracle.apply_D(lat, U, kappa, psi)).max() > 1e-2


def test_block_operator_keeps_the_clover_diagonal():
    """D_b with the clover term = the masked D with the clover term on a lattice
    where the block is the whole lattice; and the Dirichlet blocks differ from D
    by the cross-boundary hops only."""
    lat = oracle.Lattice((4, 4, 4, 4), B=(2, 2, 2, 2))
    U = synth.gauge_field(lat.L, 0.6, 27)
    kappa = 0.12
    T = oracle.clover_term(lat, U, 1.4, kappa)
    psi = synth.spinor(lat.L, 4)
    lhs = oracle.apply_D(lat, U, kappa, psi, T)
    rhs = oracle.apply_Dblock(lat, U, kappa, psi, 2, T) + oracle.apply_Dhop(lat, U, kappa, psi, 0) + \
        oracle.apply_Dhop(lat, U, kappa, psi, 1)
    assert np.abs(lhs - rhs).max() < 1e-13


@pytest.fixture(scope="module")
def clover_case():
    lat = oracle.Lattice((4, 4, 4, 4), B=(2, 2, 2, 2))
    U = synth.gauge_field(lat.L, 0.5, 44)
    Up = synth.redraw(U, synth.bernoulli_links(lat.L, 0.15, 44), 0.5, 44)
    k, csw = 0.12, 1.6
    T0, T1 = oracle.clover_term(lat, U, csw, k), oracle.clover_term(lat, Up, csw, k)
    D0 = oracle.dense(lambda v: oracle.apply_D(lat, U, k, v, T0), lat.V)
    D1 = oracle.dense(lambda v: oracle.apply_D(lat, Up, k, v, T1), lat.V)
    return lat, U, Up, k, csw, D0, D1


def _quad(M, e):
    Me = M @ e
    return float(np.vdot(e, e).real - np.vdot(Me, Me).real)


def test_clover_solve_against_dense(clover_case):
    lat, U, Up, k, csw, D0, D1 = clover_case
    b = synth.spinor(lat.L, 9)
    x, _, it, res = oracle.solve(lat, Up, k, b, tol=1e-12, clov=oracle.clover_term(lat, Up, csw, k))
    assert res <= 1e-12 and it > 0
    xd = np.linalg.solve(D1, b.reshape(-1))
    assert np.abs(x.reshape(-1) - xd).max() < 1e-9 * np.abs(xd).max()


def test_clover_samples_against_dense(clover_case):
    """FULL, BLOCKS and SCHUR samples of the clover operator equal the dense
    quadratic forms eta^+ eta - |M eta|^2 of M = X'^-1 X."""
    lat, U, Up, k, csw, D0, D1 = clover_case
    eta = oracle.noise(lat, oracle.NOISE_GAUSS, 9, 0, 0)
    s = oracle.sample(lat, U, Up, k, oracle.OP_FULL, eta, csw=csw)
    assert abs(s - _quad(np.linalg.solve(D1, D0), eta.reshape(-1))) < 1e-9
    # the clover term matters for this sample
    assert abs(s - oracle.sample(lat, U, Up, k, oracle.OP_FULL, eta)) > 1e-3

    bid, col, _ = lat.maps()
    s = oracle.sample(lat, U, Up, k, oracle.OP_BLOCKS, eta, csw=csw)
    for blk in range(lat.nblocks):
        idx = oracle.site_dofs(bid == blk)
        M = np.linalg.solve(D1[np.ix_(idx, idx)], D0[np.ix_(idx, idx)])
        assert abs(s[blk] - _quad(M, eta.reshape(-1)[idx])) < 1e-10

    black = oracle.colour_mask(lat, 0)
    eta = oracle.noise(lat, oracle.NOISE_GAUSS, 9, 0, 2, support=black)
    s = oracle.sample(lat, U, Up, k, oracle.OP_SCHUR, eta, csw=csw)
    bl, wh = oracle.site_dofs(col == 0), oracle.site_dofs(col == 1)

    def schur(D):
        return np.eye(len(bl)) - np.linalg.solve(D[np.ix_(bl, bl)], D[np.ix_(bl, wh)] @
                                                 np.linalg.solve(D[np.ix_(wh, wh)], D[np.ix_(wh, bl)]))
    M = np.linalg.solve(schur(D1), schur(D0))
    assert abs(s - _quad(M, eta.reshape(-1)[bl])) < 1e-9


def test_clover_exact_log_ratio(clover_case):
    lat, U, Up, k, csw, D0, D1 = clover_case
    want = 2 * (oracle.log_abs_det(D1) - oracle.log_abs_det(D0))
    assert abs(oracle.exact_log_ratio(lat, U, Up, k, csw) - want) < 1e-9


def test_clover_block_dets_are_diagonal_blocks_of_D():
    """With the clover term each block entry is 2 log|det| of the block's
    diagonal slice of the full clover D (assembled by apply_D: its clover
    diagonal and in-block hops, not the block code), and the entries add up
    to log det of D_bb + D_ww, the block-diagonal part of eq. domdec."""
    lat = oracle.Lattice((4, 4, 4, 4), B=(2, 2, 2, 2))
    U = synth.gauge_field(lat.L, 0.5, 47)
    k, csw = 0.13, 1.7
    T = oracle.clover_term(lat, U, csw, k)
    bid, _, _ = lat.maps()
    got = oracle.block_log_dets(lat, U, k, clov=T)
    D = oracle.dense(lambda v: oracle.apply_D(lat, U, k, v, T), lat.V)
    Dblk = np.zeros_like(D)
    for b in range(lat.nblocks):
        idx = oracle.site_dofs(bid == b)
        Dblk[np.ix_(idx, idx)] = D[np.ix_(idx, idx)]
        assert abs(got[b] - 2 * oracle.log_abs_det(D[np.ix_(idx, idx)])) < 1e-11
    assert abs(got.sum() - 2 * oracle.log_abs_det(Dblk)) < 1e-9
    # the term matters
    assert np.abs(got - oracle.block_log_dets(lat, U, k)).max() > 1e-2


def _schwarz_clover(lat, U, k, T, eta, ncy):
    """Multiplicative Schwarz with exact block solves of the clover D: per
    colour c, x <- x + K_c (eta - D x), K_c = sum_{b in c} P_b D_b^-1 P_b."""
    bid, col, _ = lat.maps()
    D = oracle.dense(lambda v: oracle.apply_D(lat, U, k, v, T), lat.V)
    n = 12 * lat.V
    K = [np.zeros((n, n), complex), np.zeros((n, n), complex)]
    for b in range(lat.nblocks):
        idx = oracle.site_dofs(bid == b)
        c = col[idx[0] // 12]
        K[c][np.ix_(idx, idx)] = np.linalg.inv(D[np.ix_(idx, idx)])
    x = np.zeros(n, complex)
    e = eta.reshape(-1)
    for _ in range(ncy):
        for c in (0, 1):
            x = x + K[c] @ (e - D @ x)
    return x.reshape(eta.shape)


def test_clover_sap_exact_block_limit():
    """With the clover term, many MR steps solve every block exactly: SAP
    equals multiplicative Schwarz with dense inverses of the clover D's
    diagonal blocks."""
    lat = oracle.Lattice((4, 4, 4, 4), B=(2, 2, 2, 2))
    U = synth.gauge_field(lat.L, 0.5, 49)
    k = 0.11
    T = oracle.clover_term(lat, U, 1.7, k)
    eta = synth.spinor(lat.L, 50)
    x = oracle.sap(lat, U, k, eta, ncy=3, nmr=80, clov=T)
    want = _schwarz_clover(lat, U, k, T, eta, 3)
    assert np.abs(x - want).max() < 1e-10 * np.abs(want).max()
    assert np.abs(x - oracle.sap(lat, U, k, eta, ncy=3, nmr=80)).max() > 1e-3 * np.abs(want).max()


def test_clover_sap_odd_equations_exact():
    """The even-odd block solve with the clover term reconstructs the odd
    sites exactly (d_o = A_oo^-1 (r_o + kappa H_oe d_e)): after the last
    (white) half-cycle the clover residual vanishes on the odd white sites."""
    lat = oracle.Lattice((8, 8, 4, 4), B=(4, 4, 2, 2))
    U = synth.gauge_field(lat.L, 0.5, 51)
    k = 0.13
    T = oracle.clover_term(lat, U, 1.7, k)
    eta = synth.spinor(lat.L, 52)
    x = oracle.sap(lat, U, k, eta, ncy=2, nmr=3, clov=T)
    r = eta - oracle.apply_D(lat, U, k, x, T)
    _, col, par = lat.maps()
    odd_white = (col == 1) & (par == 1)
    assert np.abs(r[odd_white]).max() < 1e-13
    assert np.abs(r[~odd_white]).max() > 1e-3
