"""Pins of the oracle's domain decomposition (paper Sec. 3, eqs. domdec and
ddfactor) and of the geometry it rests on."""
import numpy as np

import oracle
from paper_1112_1243_amd import synth


def _site_index(L, x):
    return x[..., 0] + L[0] * (x[..., 1] + L[1] * (x[..., 2] + L[2] * x[..., 3]))


def test_site_maps_brute_force():
    lat = oracle.Lattice((8, 4, 4, 8), B=(4, 2, 2, 4))
    bid, col, par = lat.maps()
    for s in range(0, lat.V, 7):
        x = [(s // int(np.prod(lat.L[:mu]))) % lat.L[mu] for mu in range(4)]
        nb = [x[mu] // lat.B[mu] for mu in range(4)]
        NB = lat.NB
        assert bid[s] == nb[0] + NB[0] * (nb[1] + NB[1] * (nb[2] + NB[2] * nb[3]))
        assert col[s] == sum(nb) % 2
        assert par[s] == sum(x) % 2


def test_block_order_black_first():
    """Sec. 3: the sites of black blocks come first, block by block."""
    lat = oracle.Lattice((8, 8, 4, 4), B=(4, 4, 2, 2))
    perm = oracle.block_order(lat)
    assert sorted(perm.tolist()) == list(range(lat.V))
    bid, col, par = lat.maps()
    Vb = lat.Vb
    c = col[perm].reshape(-1, Vb)
    b = bid[perm].reshape(-1, Vb)
    p = par[perm].reshape(-1, Vb)
    assert np.all(b == b[:, :1])                      # one block per chunk
    nblack = lat.nblocks // 2
    assert np.all(c[:nblack] == 0) and np.all(c[nblack:] == 1)
    assert np.all(p[:, : Vb // 2] == 0) and np.all(p[:, Vb // 2:] == 1)


def test_active_link_fractions():
    """Sec. 5: about 10% of the links for 4^4 blocks; Sec. 6: 8% for a 6^4
    core inside 8^4 blocks."""
    lat4 = oracle.Lattice((8, 8, 8, 8), B=(4, 4, 4, 4))
    m = oracle.active_links(lat4)
    assert m.sum() == 96 * lat4.nblocks
    assert abs(m.mean() - 0.10) < 0.01
    lat8 = oracle.Lattice((16, 16, 16, 16), B=(8, 8, 8, 8))
    m8 = oracle.active_links(lat8, lo=1, hi=6)
    assert m8.sum() == 1280 * lat8.nblocks
    assert abs(m8.mean() - 0.08) < 0.005


def test_active_links_brute_force():
    """At most one end on the block boundary, both ends in the same block."""
    lat = oracle.Lattice((8, 4, 4, 8), B=(4, 4, 4, 4))
    m = oracle.active_links(lat)
    x = lat.coords()

    def on_boundary(r):
        return np.any((r == 0) | (r == np.array(lat.B) - 1), axis=-1)

    for mu in range(4):
        y = x.copy()
        y[:, mu] += 1
        inside = np.all(y // np.array(lat.B) == x // np.array(lat.B), axis=1) & (y[:, mu] < lat.L[mu])
        rx = x % np.array(lat.B)
        ry = np.where(inside[:, None], y % np.array(lat.B), 0)
        nb = on_boundary(rx).astype(int) + on_boundary(ry).astype(int)
        want = inside & (nb <= 1)
        assert np.array_equal(m[:, mu], want)


def _dense(lat, f):
    return oracle.dense(f, lat.V)


def test_decomposition_sums_to_D():
    lat = oracle.Lattice((4, 4, 4, 4), B=(2, 2, 2, 2))
    U = synth.gauge_field(lat.L, 0.6, 21)
    k = 0.13
    psi = synth.spinor(lat.L, 3)
    parts = (oracle.apply_Dblock(lat, U, k, psi, 2) + oracle.apply_Dhop(lat, U, k, psi, 0)
             + oracle.apply_Dhop(lat, U, k, psi, 1))
    assert np.abs(parts - oracle.apply_D(lat, U, k, psi)).max() < 1e-14


def test_block_operators_are_masked_D():
    """D_b = P_b D P_b (Dirichlet); D_bw, D_wb = the cross-block entries."""
    lat = oracle.Lattice((4, 4, 4, 4), B=(2, 2, 2, 2), bc=(1, 1, 1, -1))
    U = synth.gauge_field(lat.L, 0.6, 22)
    k = 0.12
    bid, col, _ = lat.maps()
    D = _dense(lat, lambda v: oracle.apply_D(lat, U, k, v))
    site = np.repeat(np.arange(lat.V), 12)
    same = bid[site][:, None] == bid[site][None, :]
    for c in (0, 1):
        Db = _dense(lat, lambda v: oracle.apply_Dblock(lat, U, k, v, c))
        rowc = (col[site] == c)[:, None]
        assert np.array_equal(Db, np.where(same & rowc, D, 0))
        Dh = _dense(lat, lambda v: oracle.apply_Dhop(lat, U, k, v, c))
        want = np.where(~same & (col[site] == 1 - c)[:, None] & (col[site] == c)[None, :], D, 0)
        assert np.array_equal(Dh, want)


def test_ddfactor_exact():
    """log|det D| = sum_b log|det D_b| + log|det Dhat| (eq. ddfactor), with
    Dhat = 1 - D_bb^-1 D_bw D_ww^-1 D_wb assembled column by column from the
    oracle's Schur apply."""
    lat = oracle.Lattice((4, 4, 4, 4), B=(2, 2, 2, 2))
    U = synth.gauge_field(lat.L, 0.6, 23)
    k = 0.125
    bid, col, _ = lat.maps()
    D = _dense(lat, lambda v: oracle.apply_D(lat, U, k, v))
    total = 0.0
    Dblk = _dense(lat, lambda v: oracle.apply_Dblock(lat, U, k, v, 2))
    for b in range(lat.nblocks):
        idx = oracle.site_dofs(bid == b)
        total += oracle.log_abs_det(Dblk[np.ix_(idx, idx)])
    black = oracle.site_dofs(col == 0)
    Dhat = oracle.dense(lambda v: oracle.schur_apply(lat, U, k, v), lat.V, cols=black)[black]
    total += oracle.log_abs_det(Dhat)
    assert abs(total - oracle.log_abs_det(D)) < 1e-8


def test_schur_identity_on_black_interior():
    """Sec. 4: Dhat acts non-trivially only through the block boundaries; a
    field on black-block interior sites is left exactly unchanged."""
    lat = oracle.Lattice((8, 8, 8, 8), B=(4, 4, 4, 4))
    U = synth.gauge_field(lat.L, 0.5, 24)
    _, col, _ = lat.maps()
    r = lat.coords() % np.array(lat.B)
    interior = np.all((r > 0) & (r < np.array(lat.B) - 1), axis=1) & (col == 0)
    psi = synth.spinor(lat.L, 9)
    psi[~interior] = 0
    out = oracle.schur_apply(lat, U, 0.135, psi)
    assert np.array_equal(out, psi)
