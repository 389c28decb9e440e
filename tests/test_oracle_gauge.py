"""Pins of the oracle's gauge update (the heat-bath of step 0 of eq. 4step
with the Wilson plaquette action, paper Sec. 5) and of its filter step."""
import numpy as np
import pytest
from scipy import integrate, special, stats

import oracle
from paper_1112_1243_amd import synth


@pytest.mark.parametrize("alpha", [0.7, 3.0, 12.0])
def test_kennedy_pendleton_moments(alpha):
    """Accepted a0 follow sqrt(1 - a0^2) exp(alpha a0): mean I_2/I_1 (Bessel)
    and second moment by quadrature, within 5 standard errors."""
    u = np.random.default_rng(17).random((4, 400000))
    u = 1.0 - u  # (0, 1]
    ok, a0 = oracle.kp_a0(alpha, u)
    a0 = a0[ok]
    assert ok.mean() > 0.3  # the method is least efficient at small alpha
    dens = lambda x: np.sqrt(1 - x * x) * np.exp(alpha * x)
    z = integrate.quad(dens, -1, 1)[0]
    m2 = integrate.quad(lambda x: x * x * dens(x), -1, 1)[0] / z
    m1 = special.iv(2, alpha) / special.iv(1, alpha)
    se = a0.std() / np.sqrt(len(a0))
    assert abs(a0.mean() - m1) < 5 * se
    assert abs((a0 * a0).mean() - m2) < 5 * (a0 * a0).std() / np.sqrt(len(a0))
    assert a0.min() >= -1.0 and a0.max() <= 1.0


def test_one_link_fixed_point():
    """Repeated heat-bath updates of one link with a fixed staple sample
    exp(beta Re tr(U A) / 3) dU: the chain average of Re tr(U A) / 3 equals
    the Haar integral, estimated by reweighting Haar-random SU(3) matrices."""
    beta = 1.5
    A = synth.gauge_field((1, 1, 1, 1), 0.8, 71)[0, :3].sum(axis=0)
    u = np.eye(3, dtype=np.complex128)
    vals = []
    for sw in range(6000):
        u = oracle.heatbath_link(u, A, beta, 72, 5, 1, sw)
        vals.append(np.trace(u @ A).real / 3.0)
    vals = np.array(vals[100:])
    H = stats.unitary_group.rvs(3, size=200000, random_state=73)
    H = H / np.linalg.det(H)[:, None, None] ** (1.0 / 3.0)  # Haar on SU(3)
    f = np.einsum("nab,ba->n", H, A).real / 3.0
    w = np.exp(beta * f)
    want = np.sum(f * w) / np.sum(w)
    # chain error with a generous allowance for autocorrelation
    assert abs(vals.mean() - want) < 6 * vals.std() / np.sqrt(len(vals) / 4)
    assert abs(np.linalg.det(u) - 1) < 1e-12


def test_sweep_keeps_su3_and_the_mask():
    lat = oracle.Lattice((4, 4, 4, 4), B=(2, 2, 2, 2))
    U = synth.gauge_field(lat.L, 0.5, 74)
    mask = synth.bernoulli_links(lat.L, 0.3, 75)
    V = oracle.heatbath(lat, U, 5.8, mask, 76, 0)
    assert np.array_equal(V[~mask], U[~mask])
    W = V[mask]
    assert np.abs(np.einsum("nab,ncb->nac", W, W.conj()) - np.eye(3)).max() < 1e-12
    assert np.abs(np.linalg.det(W) - 1).max() < 1e-12
    assert np.abs(W - U[mask]).min() > 1e-6  # every masked link moved


def test_strong_coupling_plaquette():
    """At small beta, <Re tr U_P / 3> = beta/18 + beta^2/216 + O(beta^3)
    (character expansion with Haar integrals of SU(3))."""
    lat = oracle.Lattice((4, 4, 4, 4), B=(2, 2, 2, 2))
    U = synth.gauge_field(lat.L, 3.0, 77)
    mask = np.ones((lat.V, 4), bool)
    beta, ps = 1.0, []
    for sw in range(25):
        U = oracle.heatbath(lat, U, beta, mask, 78, sw)
        if sw >= 5:
            ps.append(oracle.plaquette(lat, U))
    assert abs(np.mean(ps) - (beta / 18 + beta ** 2 / 216)) < 0.005


def test_filter_step_structure():
    """Accepted blocks take the heat-bath proposal, rejected ones keep their
    links; with nothing to update the step changes nothing and is accepted."""
    lat = oracle.Lattice((4, 4, 4, 4), B=(2, 2, 2, 2))
    U = synth.gauge_field(lat.L, 0.5, 79)
    bid, _, _ = lat.maps()
    x = lat.coords()
    inside = np.zeros((lat.V, 4), bool)
    for mu in range(4):
        y = x.copy()
        y[:, mu] = (y[:, mu] + 1) % lat.L[mu]
        inside[:, mu] = bid == bid[y[:, 0] + 4 * (y[:, 1] + 4 * (y[:, 2] + 4 * y[:, 3]))]
    # at beta 1 the proposal moves far enough for block ratios of -0.6 .. -1.1
    V, acc, log_r, ok = oracle.filter_step(lat, U, 1.0, 0.16, inside, 1, 1, 1, 80, 81)
    prop = oracle.heatbath(lat, U, 1.0, inside, 80, 0)
    assert 0 < acc.sum() < lat.nblocks
    if ok:
        take = acc[0][bid]
        assert np.array_equal(V[take], prop[take]) and np.array_equal(V[~take], U[~take])
    else:
        assert np.array_equal(V, U)
    V, acc, log_r, ok = oracle.filter_step(lat, U, 5.8, 0.12, np.zeros((lat.V, 4), bool), 1, 1, 1, 80, 81)
    assert ok and abs(log_r) < 1e-10 and acc.all() and np.array_equal(V, U)


def test_overrelaxation_keeps_the_action():
    """An over-relaxation sweep is microcanonical: the sum of plaquettes is
    unchanged (every link update keeps Re tr(U A), and links of one class
    share no plaquette), SU(3) is kept, and the links move."""
    lat = oracle.Lattice((4, 4, 4, 4), B=(2, 2, 2, 2))
    U = synth.gauge_field(lat.L, 0.5, 82)
    mask = np.ones((lat.V, 4), bool)
    V = oracle.overrelax(lat, U, mask)
    assert abs(oracle.plaquette(lat, V) - oracle.plaquette(lat, U)) < 1e-13
    assert np.abs(np.einsum("xmab,xmcb->xmac", V, V.conj()) - np.eye(3)).max() < 1e-12
    assert np.abs(V - U).max() > 0.1


def test_overrelaxation_single_subgroup_is_an_involution():
    """For one SU(2) subgroup, X = (v^+)^2 maps the subgroup part k v of W to
    k v^+, whose reflection is X' = v^2: two steps give the identity."""
    A = synth.gauge_field((1, 1, 1, 1), 0.8, 83)[0, :3].sum(axis=0)
    u = synth.gauge_field((1, 1, 1, 1), 0.8, 84)[0, 0]

    def one(u):
        W = u @ A
        a, b = 0.5 * (W[0, 0] + np.conj(W[1, 1])), 0.5 * (W[0, 1] - np.conj(W[1, 0]))
        v = np.array([[a, b], [-np.conj(b), np.conj(a)]]) / np.sqrt(abs(a) ** 2 + abs(b) ** 2)
        E = np.eye(3, dtype=np.complex128)
        E[:2, :2] = v.conj().T @ v.conj().T
        return E @ u
    # the oracle's first subgroup step is this map; applying it twice returns u
    assert np.abs(one(one(u)) - u).max() < 1e-13
    saved = oracle.SUBGROUPS
    try:
        oracle.core.SUBGROUPS = ((0, 1),)
        assert np.abs(oracle.overrelax_link(u, A) - one(u)).max() < 1e-14
    finally:
        oracle.core.SUBGROUPS = saved


def _gauge_transform(lat, U, g):
    x = lat.coords()
    out = np.empty_like(U)
    for mu in range(4):
        y = x.copy()
        y[:, mu] = (y[:, mu] + 1) % lat.L[mu]
        t = y[:, 0] + lat.L[0] * (y[:, 1] + lat.L[1] * (y[:, 2] + lat.L[2] * y[:, 3]))
        out[:, mu] = g @ U[:, mu] @ np.conj(np.swapaxes(g[t], -1, -2))
    return out


def test_relative_gauge_fixing():
    """F never decreases from sweep to sweep; the fixed field has the same
    block determinants (gauge invariance); a random gauge copy of U is driven
    back towards U (F close to its maximum 4 V)."""
    lat = oracle.Lattice((4, 4, 4, 4), B=(2, 2, 2, 2))
    U = synth.gauge_field(lat.L, 0.5, 85)
    Up = synth.redraw(U, synth.bernoulli_links(lat.L, 0.2, 86), 0.5, 86)
    g = synth.gauge_field(lat.L, 0.4, 87)[:, 0]
    Ug = _gauge_transform(lat, Up, g)
    F = [oracle.relative_gauge_functional(U, Ug)]
    V = Ug
    for _ in range(3):
        V = oracle.relative_gauge(lat, U, V, 1)
        F.append(oracle.relative_gauge_functional(U, V))
    assert all(b >= a - 1e-12 for a, b in zip(F, F[1:])) and F[-1] > F[0] + 1.0
    assert np.abs(oracle.block_log_dets(lat, V, 0.13) - oracle.block_log_dets(lat, Ug, 0.13)).max() < 1e-10
    W = oracle.relative_gauge(lat, U, _gauge_transform(lat, U, g), 30)
    assert oracle.relative_gauge_functional(U, W) > 4 * lat.V - 1e-6
