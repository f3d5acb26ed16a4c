"""Pins for the oracle's LJC(linear) law (Table 1, Section 2), CPU only.

Closed forms of the two-body Lennard-Jones and Coulomb(4r) terms, the
Lorentz-Berthelot combining rule, F = -grad U by finite differences, Newton's
third law and translation invariance.
"""
import numpy as np
import pytest

KC = 332.0637
D = 4.0


def _pair(r, q=(0.0, 0.0), sig=(3.4, 3.4), eps=(0.1, 0.1)):
    pos = np.array([[0.0, 0.0, 0.0], [r, 0.0, 0.0]])
    return pos, np.array(q, float), np.array(sig, float), np.array(eps, float)


def test_lj_minimum_and_depth(oracle_mod):
    # u = 4e[(s/r)^12 - (s/r)^6] has its minimum -e at r = 2^(1/6) s.
    s12 = 0.5 * (3.0 + 3.8)
    e12 = np.sqrt(0.05 * 0.2)
    rmin = 2.0 ** (1.0 / 6.0) * s12
    pos, q, sig, eps = _pair(rmin, sig=(3.0, 3.8), eps=(0.05, 0.2))
    f, u = oracle_mod.ljc_linear(pos, q, sig, eps, kc=KC, D=D)
    np.testing.assert_allclose(u, [-e12, -e12], rtol=1e-14)
    assert np.abs(f).max() < 1e-14


def test_lj_force_at_sigma(oracle_mod):
    # at r = s: u = 0 and the force is repulsive with magnitude 24 e / s.
    pos, q, sig, eps = _pair(3.4, sig=(3.4, 3.4), eps=(0.1, 0.1))
    f, u = oracle_mod.ljc_linear(pos, q, sig, eps, kc=KC, D=D)
    np.testing.assert_allclose(u, [0.0, 0.0], atol=1e-16)
    np.testing.assert_allclose(f[0], [-24 * 0.1 / 3.4, 0, 0], rtol=1e-14)
    np.testing.assert_allclose(f[1], [24 * 0.1 / 3.4, 0, 0], rtol=1e-14)


@pytest.mark.parametrize("qq", [(0.5, 0.5), (0.8, -0.3)])
def test_coulomb_linear_dielectric(oracle_mod, qq):
    # dielectric 4r: u = kc q1 q2 / (4 r^2); force magnitude 2 kc q1 q2 / (4 r^3), like charges repel.
    r = 5.0
    pos, q, sig, eps = _pair(r, q=qq, eps=(0.0, 0.0))
    f, u = oracle_mod.ljc_linear(pos, q, sig, eps, kc=KC, D=D)
    uc = KC * qq[0] * qq[1] / (4.0 * r * r)
    fc = 2.0 * KC * qq[0] * qq[1] / (4.0 * r ** 3)
    np.testing.assert_allclose(u, [uc, uc], rtol=1e-14)
    np.testing.assert_allclose(f[0], [-fc, 0, 0], rtol=1e-14)
    np.testing.assert_allclose(f[1], [fc, 0, 0], rtol=1e-14)


def _md(n, seed, box=12.0):
    rng = np.random.default_rng(seed)
    # well-separated random atoms on a jittered lattice
    k = int(np.ceil(n ** (1 / 3)))
    g = np.stack(np.meshgrid(*(np.arange(k),) * 3, indexing="ij"), -1).reshape(-1, 3)[:n]
    pos = g * (box / k) + rng.uniform(-0.4, 0.4, (n, 3))
    q = rng.uniform(-0.8, 0.8, n)
    sig = rng.uniform(3.0, 3.8, n)
    eps = rng.uniform(0.05, 0.2, n)
    return pos, q, sig, eps


def test_force_is_minus_gradient_of_energy(oracle_mod):
    pos, q, sig, eps = _md(10, 4)
    f, _ = oracle_mod.ljc_linear(pos, q, sig, eps, kc=KC, D=D)

    def U(p):
        return 0.5 * oracle_mod.ljc_linear(p, q, sig, eps, kc=KC, D=D)[1].sum()

    h = 1e-5
    fd = np.zeros_like(pos)
    for i in range(pos.shape[0]):
        for c in range(3):
            pp, pm = pos.copy(), pos.copy()
            pp[i, c] += h
            pm[i, c] -= h
            fd[i, c] = -(U(pp) - U(pm)) / (2 * h)
    np.testing.assert_allclose(f, fd, rtol=1e-6, atol=1e-7 * np.abs(f).max())


def test_newton_third_law_and_translation(oracle_mod):
    pos, q, sig, eps = _md(64, 7, box=20.0)
    f, u = oracle_mod.ljc_linear(pos, q, sig, eps, kc=KC, D=D)
    assert np.linalg.norm(f.sum(0)) <= 1e-13 * np.linalg.norm(f, axis=1).sum()
    f2, u2 = oracle_mod.ljc_linear(pos + 3.25, q, sig, eps, kc=KC, D=D)
    np.testing.assert_allclose(f2, f, rtol=1e-8, atol=1e-10 * np.abs(f).max())
    np.testing.assert_allclose(u2, u, rtol=1e-8, atol=1e-10 * np.abs(u).max())


def test_pair_energy_symmetry(oracle_mod):
    # the total energy counts each pair twice in sum_i U_i
    pos, q, sig, eps = _md(3, 1)
    _, u = oracle_mod.ljc_linear(pos, q, sig, eps, kc=KC, D=D)
    pair = np.zeros((3, 3))
    for i in range(3):
        for j in range(3):
            if i != j:
                sub = [i, j]
                pair[i, j] = oracle_mod.ljc_linear(pos[sub], q[sub], sig[sub], eps[sub], kc=KC, D=D)[1][0]
    np.testing.assert_allclose(pair, pair.T, rtol=1e-14)
    np.testing.assert_allclose(u, pair.sum(1), rtol=1e-14)


def test_replication_identity(oracle_mod):
    pos, q, sig, eps = _md(40, 3, box=18.0)
    f, u = oracle_mod.ljc_linear(pos, q, sig, eps)
    fa, ua = oracle_mod.ljc_linear(pos, q, sig, eps, jrange=(0, 13))
    fb, ub = oracle_mod.ljc_linear(pos, q, sig, eps, jrange=(13, 40))
    np.testing.assert_allclose(fa + fb, f, rtol=1e-12, atol=1e-14 * np.abs(f).max())
    np.testing.assert_allclose(ua + ub, u, rtol=1e-12, atol=1e-14 * np.abs(u).max())
