"""Pins of the oracle's Wilson-Dirac operator against closed forms and exact
symmetries (the operator: paper Sec. 5, "plain Wilson-Dirac operator")."""
import itertools

import numpy as np
import pytest

import oracle
from paper_1112_1243_amd import synth


def test_gamma_algebra():
    g = [oracle.gamma(mu) for mu in range(4)]
    eye = np.eye(4)
    for mu in range(4):
        assert np.allclose(g[mu], g[mu].conj().T)
        for nu in range(4):
            assert np.allclose(g[mu] @ g[nu] + g[nu] @ g[mu], 2 * eye * (mu == nu))
    g5 = g[0] @ g[1] @ g[2] @ g[3]
    assert np.allclose(g5, oracle.GAMMA5)


def _plane_wave(lat, p, u):
    x = lat.coords()
    phase = np.exp(1j * (x @ np.asarray(p)))
    return phase[:, None, None] * u[None, :, :], phase


def _Dp(kappa, p):
    """Momentum-space Wilson operator 1 - 2 kappa sum cos p + 2 i kappa sum g sin p."""
    m = (1 - 2 * kappa * np.sum(np.cos(p))) * np.eye(4, dtype=complex)
    for mu in range(4):
        m = m + 2j * kappa * np.sin(p[mu]) * oracle.gamma(mu)
    return m


@pytest.mark.parametrize("bc", [(1, 1, 1, 1), (1, 1, 1, -1)])
def test_free_field_plane_waves(bc):
    lat = oracle.Lattice((4, 6, 4, 8), bc=bc)
    U = synth.unit_gauge(lat.L)
    kappa = 0.137
    rng = np.random.default_rng(1)
    for trial in range(4):
        n = [rng.integers(0, l) for l in lat.L]
        p = np.array([2 * np.pi * (n[mu] + (0.5 if bc[mu] < 0 else 0)) / lat.L[mu] for mu in range(4)])
        u = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
        psi, phase = _plane_wave(lat, p, u)
        out = oracle.apply_D(lat, U, kappa, psi)
        want = phase[:, None, None] * (_Dp(kappa, p) @ u)[None]
        assert np.abs(out - want).max() < 1e-13


def test_u1_background_plane_waves():
    """U_mu(x) = exp(i alpha_mu) 1 shifts the momentum p -> p + alpha (this
    fixes which end of the link carries U and which U^+)."""
    lat = oracle.Lattice((4, 4, 6, 4))
    alpha = np.array([0.3, -0.7, 0.2, 1.1])
    U = synth.unit_gauge(lat.L) * np.exp(1j * alpha)[None, :, None, None]
    kappa = 0.11
    rng = np.random.default_rng(2)
    for trial in range(4):
        n = [rng.integers(0, l) for l in lat.L]
        p = np.array([2 * np.pi * n[mu] / lat.L[mu] for mu in range(4)])
        u = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
        psi, phase = _plane_wave(lat, p, u)
        out = oracle.apply_D(lat, U, kappa, psi)
        want = phase[:, None, None] * (_Dp(kappa, p + alpha) @ u)[None]
        assert np.abs(out - want).max() < 1e-13


def test_free_field_log_det():
    """log|det D| = 6 sum_p log[(1 - 2k sum cos p)^2 + 4 k^2 sum sin^2 p]."""
    lat = oracle.Lattice((4, 4, 4, 4))
    kappa = 0.12
    U = synth.unit_gauge(lat.L)
    D = oracle.dense(lambda v: oracle.apply_D(lat, U, kappa, v), lat.V)
    want = 0.0
    for n in itertools.product(*[range(l) for l in lat.L]):
        p = 2 * np.pi * np.array(n) / np.array(lat.L)
        a = 1 - 2 * kappa * np.cos(p).sum()
        want += 6 * np.log(a * a + 4 * kappa**2 * np.sin(p).dot(np.sin(p)))
    assert abs(oracle.log_abs_det(D) - want) < 1e-9


def test_gamma5_hermiticity():
    lat = oracle.Lattice((4, 4, 4, 6), bc=(1, 1, 1, -1))
    U = synth.gauge_field(lat.L, 0.7, 11)
    kappa = 0.13
    psi = synth.spinor(lat.L, 1)
    chi = synth.spinor(lat.L, 2)
    lhs = np.vdot(chi, oracle.g5(oracle.apply_D(lat, U, kappa, oracle.g5(psi))))
    rhs = np.vdot(oracle.apply_D(lat, U, kappa, chi), psi)
    assert abs(lhs - rhs) < 1e-11 * abs(rhs)


def test_gauge_covariance():
    """D[U^g] (g psi) = g (D[U] psi), U^g_mu(x) = g(x) U_mu(x) g(x+mu)^+."""
    lat = oracle.Lattice((4, 4, 4, 4), bc=(1, 1, 1, -1))
    U = synth.gauge_field(lat.L, 0.8, 3)
    g = synth.gauge_field(lat.L, 2.0, 4)[:, 0]
    x = lat.coords()
    Ug = np.empty_like(U)
    for mu in range(4):
        y = x.copy()
        y[:, mu] = (y[:, mu] + 1) % lat.L[mu]
        t = y[:, 0] + lat.L[0] * (y[:, 1] + lat.L[1] * (y[:, 2] + lat.L[2] * y[:, 3]))
        Ug[:, mu] = g @ U[:, mu] @ np.conj(np.swapaxes(g[t], -1, -2))
    psi = synth.spinor(lat.L, 5)
    gpsi = np.einsum("xab,xsb->xsa", g, psi)
    lhs = oracle.apply_D(lat, Ug, 0.125, gpsi)
    rhs = np.einsum("xab,xsb->xsa", g, oracle.apply_D(lat, U, 0.125, psi))
    assert np.abs(lhs - rhs).max() < 1e-13


def test_even_odd_determinant():
    """det D = det(1 - kappa^2 H_eo H_oe) on the even sites (D_ee = D_oo = 1)."""
    lat = oracle.Lattice((4, 4, 4, 4), B=(2, 2, 2, 2))
    U = synth.gauge_field(lat.L, 0.6, 8)
    kappa = 0.14
    _, _, par = lat.maps()
    ev = oracle.site_dofs(par == 0)
    D = oracle.dense(lambda v: oracle.apply_D(lat, U, kappa, v), lat.V)
    Dee = oracle.dense(lambda v: oracle.apply_Dee(lat, U, kappa, v), lat.V, cols=ev)[ev]
    assert abs(oracle.log_abs_det(D) - oracle.log_abs_det(Dee)) < 1e-9
    # odd rows of the even-odd operator are zero
    Dfull = oracle.dense(lambda v: oracle.apply_Dee(lat, U, kappa, v), lat.V, cols=ev)
    odd = oracle.site_dofs(par == 1)
    assert np.all(Dfull[odd] == 0)
