"""Pins of the oracle's noise: Philox4x64-10 (Salmon et al., SC'11) and the
complex Gaussian / Z2 vectors of the stochastic acceptance step (paper
Sec. 4)."""
import os

import numpy as np

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x64_10_kat.txt")


def test_philox_known_answers():
    rows = [l.split() for l in open(GOLDEN) if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(t, 16) for t in r]
        out = oracle.philox4x64_10(v[0:4], v[4:6])
        assert [int(o) for o in out] == v[6:10]


def test_philox_matches_numpy():
    """numpy's Philox advances its counter before each block of 4 words."""
    rng = np.random.default_rng(0)
    for _ in range(20):
        ctr = [int(c) for c in rng.integers(0, 2**62, 4)]
        key = [int(c) for c in rng.integers(0, 2**62, 2)]
        bg = np.random.Philox(key=key, counter=ctr)
        words = bg.random_raw(8)
        c1 = list(ctr)
        c1[0] += 1
        c2 = list(ctr)
        c2[0] += 2
        assert list(oracle.philox4x64_10(c1, key)) == list(words[:4])
        assert list(oracle.philox4x64_10(c2, key)) == list(words[4:])


def _words(site, step, k, seed, nblk):
    out = []
    for j in range(nblk):
        out.extend(int(w) for w in oracle.philox4x64_10([site, step, k, j], [seed, 3]))
    return out


def test_z2_bits():
    lat = oracle.Lattice((4, 4, 2, 2))
    eta = oracle.noise(lat, oracle.NOISE_Z2, 77, 3, 5)
    for s in (0, 5, 17, lat.V - 1):
        w = _words(s, 3, 5, 77, 1)[0]
        want = np.array([1.0 - 2.0 * ((w >> a) & 1) for a in range(12)])
        assert np.array_equal(eta[s].reshape(-1), want.astype(complex))


def test_gauss_from_words():
    lat = oracle.Lattice((4, 2, 2, 2))
    eta = oracle.noise(lat, oracle.NOISE_GAUSS, 5, 1, 2)
    for s in (0, 9, lat.V - 1):
        w = _words(s, 1, 2, 5, 6)
        u = [((x >> 11) + 0.5) * 2.0**-53 for x in w]
        want = np.array([np.sqrt(-np.log(u[2 * a])) * np.exp(2j * np.pi * u[2 * a + 1]) for a in range(12)])
        assert np.abs(eta[s].reshape(-1) - want).max() < 1e-15


def test_noise_moments_and_mask():
    lat = oracle.Lattice((8, 8, 8, 8))
    e = oracle.noise(lat, oracle.NOISE_GAUSS, 123, 0, 0).reshape(-1)
    n = e.size
    assert abs(np.mean(np.abs(e) ** 2) - 1) < 5 / np.sqrt(n)
    assert abs(np.mean(e)) < 5 / np.sqrt(n)
    assert abs(np.mean(e * e)) < 5 / np.sqrt(n)          # circular: E eta^2 = 0
    z = oracle.noise(lat, oracle.NOISE_Z2, 123, 0, 0).reshape(-1)
    assert set(np.unique(z)) == {-1.0, 1.0}
    assert abs(np.mean(z.real)) < 5 / np.sqrt(n)
    mask = np.zeros(lat.V, bool)
    mask[::3] = True
    em = oracle.noise(lat, oracle.NOISE_GAUSS, 123, 0, 0, support=mask)
    full = oracle.noise(lat, oracle.NOISE_GAUSS, 123, 0, 0)
    assert np.array_equal(em[mask], full[mask]) and np.all(em[~mask] == 0)
    # different (step, k) give independent streams
    e2 = oracle.noise(lat, oracle.NOISE_GAUSS, 123, 0, 1).reshape(-1)
    assert abs(np.vdot(e, e2)) / n < 5 / np.sqrt(n)
