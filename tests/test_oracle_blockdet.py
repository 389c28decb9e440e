"""Pins of the oracle's exact block determinants: log det(D_b^+ D_b) of the
Dirichlet block operators (paper Sec. 3, eq. ddfactor; their ratios are the
first acceptance step of eq. 4step)."""
import numpy as np
import pytest

import oracle
from paper_1112_1243_amd import synth


def _dense(lat, apply):
    return oracle.dense(apply, lat.V)


def test_matches_slices_of_the_dense_block_operator():
    """Each entry is 2 log|det| of the block's slice of the dense D_bb + D_ww
    assembled on the whole lattice (a different assembly of the same matrix)."""
    lat = oracle.Lattice((4, 4, 4, 4), B=(2, 2, 2, 2))
    U = synth.gauge_field(lat.L, 0.6, 31)
    k = 0.125
    bid, _, _ = lat.maps()
    Dblk = _dense(lat, lambda v: oracle.apply_Dblock(lat, U, k, v, 2))
    got = oracle.block_log_dets(lat, U, k)
    for b in range(lat.nblocks):
        idx = oracle.site_dofs(bid == b)
        sign, ld = np.linalg.slogdet(Dblk[np.ix_(idx, idx)])
        assert abs(got[b] - 2 * ld) < 1e-11
        # gamma5-hermiticity makes det D_b real
        assert abs(sign.imag) < 1e-10


def test_ddfactor():
    """sum_b log det(D_b^+ D_b) + log det(Dhat^+ Dhat) = log det(D^+ D)."""
    lat = oracle.Lattice((4, 4, 4, 4), B=(2, 2, 2, 2))
    U = synth.gauge_field(lat.L, 0.5, 37)
    k = 0.13
    _, col, _ = lat.maps()
    D = _dense(lat, lambda v: oracle.apply_D(lat, U, k, v))
    black = oracle.site_dofs(col == 0)
    Dhat = oracle.dense(lambda v: oracle.schur_apply(lat, U, k, v), lat.V, cols=black)[black]
    total = oracle.block_log_dets(lat, U, k).sum() + 2 * oracle.log_abs_det(Dhat)
    assert abs(total - 2 * oracle.log_abs_det(D)) < 1e-8


def _plaquettes(B):
    """Elementary squares inside a B[0] x .. x B[3] box."""
    n = 0
    for mu in range(4):
        for nu in range(mu + 1, 4):
            n += (B[mu] - 1) * (B[nu] - 1) * int(np.prod([B[r] for r in range(4) if r not in (mu, nu)]))
    return n


@pytest.mark.parametrize("L,B", [((4, 4, 4, 4), (2, 2, 2, 2)), ((8, 4, 4, 4), (4, 2, 2, 2))])
def test_small_kappa_plaquette_expansion(L, B):
    """Unit links: log det D_b = tr log(1 - k H_b) = -sum_n k^n tr(H_b^n)/n.
    Odd n vanish (bipartite), and so does n = 2 ((1 - g_mu)(1 + g_mu) = 0
    kills every backtracking path).  At n = 4 only the elementary squares
    remain: 4 starting corners x 2 orientations, each with spin trace
    tr[(1 - g_mu)(1 - g_nu)(1 + g_mu)(1 + g_nu)] = -8 and colour trace 3, so
    log det(D_b^+ D_b) = 96 N_plaq k^4 + O(k^6)."""
    lat = oracle.Lattice(L, B=B)
    U = synth.unit_gauge(L)
    dev = []
    for k in (0.003, 0.006):
        ld = oracle.block_log_dets(lat, U, k, blocks=[0, lat.nblocks - 1])
        want = 96 * _plaquettes(B) * k ** 4
        assert abs(ld[-1] - ld[0]) < 1e-13
        dev.append(ld[0] / want - 1)
    # the relative correction is O(k^2): small, and four times larger at 2k
    assert abs(dev[0]) < 5e-4
    assert 3.0 < dev[1] / dev[0] < 5.0


def test_gauge_invariance():
    """det D_b is unchanged by U_mu(x) -> g(x) U_mu(x) g(x + mu)^+."""
    lat = oracle.Lattice((4, 4, 4, 4), B=(2, 2, 2, 2))
    U = synth.gauge_field(lat.L, 0.7, 41)
    g = synth.gauge_field(lat.L, 2.0, 42)[:, 0]
    x = lat.coords()
    Ug = np.empty_like(U)
    for mu in range(4):
        y = x.copy()
        y[:, mu] = (y[:, mu] + 1) % lat.L[mu]
        t = y[:, 0] + lat.L[0] * (y[:, 1] + lat.L[1] * (y[:, 2] + lat.L[2] * y[:, 3]))
        Ug[:, mu] = g @ U[:, mu] @ np.conj(np.swapaxes(g[t], -1, -2))
    a = oracle.block_log_dets(lat, U, 0.13)
    b = oracle.block_log_dets(lat, Ug, 0.13)
    assert np.abs(a - b).max() < 1e-10
    assert np.ptp(a) > 1e-3  # the blocks differ, so the comparison is not trivial


def test_locality():
    """Redrawing the links inside one block changes only that block's entry;
    redrawing links that cross block boundaries changes none."""
    lat = oracle.Lattice((4, 4, 4, 4), B=(2, 2, 2, 2))
    U = synth.gauge_field(lat.L, 0.5, 43)
    k = 0.13
    base = oracle.block_log_dets(lat, U, k)
    bid, _, _ = lat.maps()
    x = lat.coords()
    inside = np.zeros((lat.V, 4), bool)
    cross = np.zeros((lat.V, 4), bool)
    for mu in range(4):
        y = x.copy()
        y[:, mu] = (y[:, mu] + 1) % lat.L[mu]
        t = y[:, 0] + lat.L[0] * (y[:, 1] + lat.L[1] * (y[:, 2] + lat.L[2] * y[:, 3]))
        inside[:, mu] = (bid == 5) & (bid[t] == 5)
        cross[:, mu] = bid != bid[t]
    a = oracle.block_log_dets(lat, synth.redraw(U, inside, 0.5, 44), k)
    changed = np.abs(a - base) > 1e-9
    assert changed[5] and changed.sum() == 1
    c = oracle.block_log_dets(lat, synth.redraw(U, cross, 0.5, 45), k)
    assert np.abs(c - base).max() < 1e-12


def extract_block(lat, U, b):
    """Links of block b of lat as a canonical field of the block's extents
    (in-block lexicographic order), by index arithmetic."""
    bid, _, _ = lat.maps()
    x = lat.coords()
    sites = np.nonzero(bid == b)[0]
    loc = x[sites] % np.array(lat.B)
    B = lat.B
    order = np.argsort(loc[:, 0] + B[0] * (loc[:, 1] + B[1] * (loc[:, 2] + B[2] * loc[:, 3])))
    return np.ascontiguousarray(U[sites[order]]), sites[order]


@pytest.mark.parametrize("L,B", [((4, 4, 4, 4), (2, 2, 2, 2)), ((8, 4, 8, 4), (4, 2, 4, 2))])
def test_open_boundary_is_the_dirichlet_block(L, B):
    """Open boundaries (bc = 0 drops the hops that wrap): the lattice operator
    of an extracted block equals that block's Dirichlet operator D_b (Sec. 3,
    eq. domdec), which is what makes a block a lattice of its own for eq.
    ddrec."""
    lat = oracle.Lattice(L, B=B, bc=(1, 1, 1, -1))
    U = synth.gauge_field(L, 0.6, 61)
    psi = synth.spinor(L, 62)
    whole = oracle.apply_Dblock(lat, U, 0.13, psi, 2)
    small = oracle.Lattice(B, bc=(0, 0, 0, 0))
    for b in (0, lat.nblocks - 1):
        Ub, sites = extract_block(lat, U, b)
        got = oracle.apply_D(small, Ub, 0.13, np.ascontiguousarray(psi[sites]))
        assert np.abs(got - whole[sites]).max() < 1e-14


def test_ddrec_on_an_open_block():
    """eq. ddrec: det D_b = prod_b' det D_b' det Dhat_b, i.e. eq. ddfactor on a
    4^4 block of an 8^4 lattice, extracted with open boundaries, with 2^4
    sub-blocks (the open lattice operator is D_b by the test above)."""
    big = oracle.Lattice((8, 8, 8, 8), B=(4, 4, 4, 4))
    U = synth.gauge_field(big.L, 0.5, 63)
    k = 0.13
    Ub, _ = extract_block(big, U, 9)
    lat = oracle.Lattice((4, 4, 4, 4), B=(2, 2, 2, 2), bc=(0, 0, 0, 0))
    _, col, _ = lat.maps()
    D = _dense(lat, lambda v: oracle.apply_D(lat, Ub, k, v))
    ld_block = 2 * oracle.log_abs_det(D)
    black = oracle.site_dofs(col == 0)
    Dhat = oracle.dense(lambda v: oracle.schur_apply(lat, Ub, k, v), lat.V, cols=black)[black]
    total = oracle.block_log_dets(lat, Ub, k).sum() + 2 * oracle.log_abs_det(Dhat)
    assert abs(total - ld_block) < 1e-8
