"""Pins of the oracle's inversions (paper Sec. 4, "one inversion for each
factor") and of its Schwarz preconditioner (domain decomposition of Luscher
hep-lat/0310048, cited in Secs. 1 and 3)."""
import numpy as np
import pytest

import oracle
from paper_1112_1243_amd import synth


def test_cgne_full_matches_dense_solve():
    lat = oracle.Lattice((4, 4, 4, 4), bc=(1, 1, 1, -1))
    U = synth.gauge_field(lat.L, 0.5, 31)
    k = 0.13
    b = synth.spinor(lat.L, 4)
    x, y, it, res = oracle.solve(lat, U, k, b, tol=1e-12)
    assert res <= 1e-12 and it > 0
    D = oracle.dense(lambda v: oracle.apply_D(lat, U, k, v), lat.V)
    xd = np.linalg.solve(D, b.reshape(-1)).reshape(b.shape)
    assert np.abs(x - xd).max() < 1e-10 * np.abs(xd).max()
    # y solves the normal equations D D^+ y = b and x = D^+ y
    assert np.abs(oracle.g5(oracle.apply_D(lat, U, k, oracle.g5(y))) - x).max() < 1e-13


@pytest.mark.parametrize("colour", [0, 1, 2])
def test_cgne_blocks_matches_dense_solve(colour):
    lat = oracle.Lattice((4, 4, 4, 4), B=(2, 2, 2, 2))
    U = synth.gauge_field(lat.L, 0.5, 32)
    k = 0.14
    _, col, _ = lat.maps()
    b = synth.spinor(lat.L, 5)
    if colour < 2:
        b[col != colour] = 0
    x, _, _, res = oracle.solve(lat, U, k, b, "block", colour, tol=1e-13)
    assert res <= 1e-13
    Db = oracle.dense(lambda v: oracle.apply_Dblock(lat, U, k, v, 2), lat.V)
    sel = np.ones(lat.V, bool) if colour == 2 else col == colour
    idx = oracle.site_dofs(sel)
    xd = np.zeros(12 * lat.V, complex)
    xd[idx] = np.linalg.solve(Db[np.ix_(idx, idx)], b.reshape(-1)[idx])
    assert np.abs(x.reshape(-1) - xd).max() < 1e-11


def _schwarz_closed_form(lat, U, k, eta, ncy):
    """Multiplicative Schwarz with exact block solves: per colour c,
    x <- x + K_c (eta - D x), K_c = sum_{b in c} P_b D_b^-1 P_b."""
    bid, col, _ = lat.maps()
    D = oracle.dense(lambda v: oracle.apply_D(lat, U, k, v), lat.V)
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


def test_sap_exact_block_limit():
    """Many MR steps solve every block exactly: SAP then equals the
    multiplicative Schwarz iteration with dense block inverses."""
    lat = oracle.Lattice((4, 4, 4, 4), B=(2, 2, 2, 2))
    U = synth.gauge_field(lat.L, 0.5, 33)
    k = 0.11
    eta = synth.spinor(lat.L, 6)
    x = oracle.sap(lat, U, k, eta, ncy=3, nmr=80)
    want = _schwarz_closed_form(lat, U, k, eta, 3)
    assert np.abs(x - want).max() < 1e-10 * np.abs(want).max()


def test_sap_odd_equations_exact():
    """The even-odd block solve reconstructs the odd sites exactly: after the
    last (white) half-cycle the residual vanishes on odd white sites."""
    lat = oracle.Lattice((8, 8, 4, 4), B=(4, 4, 2, 2))
    U = synth.gauge_field(lat.L, 0.5, 34)
    k = 0.13
    eta = synth.spinor(lat.L, 7)
    x = oracle.sap(lat, U, k, eta, ncy=2, nmr=3)
    r = eta - oracle.apply_D(lat, U, k, x)
    _, col, par = lat.maps()
    odd_white = (col == 1) & (par == 1)
    assert np.abs(r[odd_white]).max() < 1e-13
    assert np.abs(r[~odd_white]).max() > 1e-3      # an approximation elsewhere


def test_sap_reduces_residual():
    lat = oracle.Lattice((8, 8, 8, 8), B=(4, 4, 4, 4))
    U = synth.gauge_field(lat.L, 0.5, 35)
    k = 0.135
    eta = synth.spinor(lat.L, 8)
    r0 = np.linalg.norm(eta)
    prev = r0
    for ncy in (1, 2, 4):
        x = oracle.sap(lat, U, k, eta, ncy=ncy, nmr=5)
        r = np.linalg.norm(eta - oracle.apply_D(lat, U, k, x))
        assert r < prev
        prev = r
