"""Pins for the oracle's LJC(constant) and LJC(sigmoidal) laws (Table 1), CPU only.

* LJC(constant): the two-body Coulomb closed form k q1 q2 / (D r) and its
  force, F = -grad U by finite differences, Newton's third law, and an LJ part
  identical to LJC(linear)'s when the charges vanish.
* LJC(sigmoidal): with zeta(r) = exp(delta) constant it reduces exactly to
  LJC(constant) with D = e^delta; F = -grad U by finite differences for a
  genuinely r-dependent zeta; a two-body value of k q1 q2 / (zeta(r) r).
  The paper gives no constants for zeta, so no paper value pins them.
"""
import numpy as np

KC = 332.0637


def _pair(r, q=(0.5, -0.4), sig=(3.2, 3.6), eps=(0.1, 0.15)):
    pos = np.array([[0.0, 0.0, 0.0], [0.0, r, 0.0]])
    return pos, np.array(q), np.array(sig), np.array(eps)


def _sys(n, seed, box=12.0):
    rng = np.random.default_rng(seed)
    k = int(np.ceil(n ** (1 / 3)))
    g = np.stack(np.meshgrid(*(np.arange(k),) * 3, indexing="ij"), -1).reshape(-1, 3)[:n]
    pos = g * (box / k) + rng.uniform(-0.4, 0.4, (n, 3))
    return pos, rng.uniform(-0.8, 0.8, n), rng.uniform(3.0, 3.8, n), rng.uniform(0.05, 0.2, n)


def _fd_force(energy_fn, pos, h=1e-5):
    fd = np.zeros_like(pos)
    for i in range(pos.shape[0]):
        for c in range(3):
            pp, pm = pos.copy(), pos.copy()
            pp[i, c] += h
            pm[i, c] -= h
            fd[i, c] = -(energy_fn(pp) - energy_fn(pm)) / (2 * h)
    return fd


def test_constant_two_body_coulomb(oracle_mod):
    r, D = 6.0, 4.0
    pos, q, sig, eps = _pair(r, eps=(0.0, 0.0))
    f, u = oracle_mod.ljc_constant(pos, q, sig, eps, kc=KC, D=D)
    uc = KC * 0.5 * -0.4 / (D * r)
    fc = KC * 0.5 * -0.4 / (D * r * r)           # < 0: opposite charges attract
    np.testing.assert_allclose(u, [uc, uc], rtol=1e-14)
    np.testing.assert_allclose(f[0], [0.0, -fc, 0.0], rtol=1e-14, atol=1e-16)
    np.testing.assert_allclose(f[1], [0.0, fc, 0.0], rtol=1e-14, atol=1e-16)


def test_constant_lj_part_matches_linear_law(oracle_mod):
    pos, _, sig, eps = _sys(20, 1)
    q0 = np.zeros(20)
    fa, ua = oracle_mod.ljc_constant(pos, q0, sig, eps)
    fb, ub = oracle_mod.ljc_linear(pos, q0, sig, eps)
    np.testing.assert_allclose(fa, fb, rtol=1e-13, atol=1e-15 * np.abs(fb).max())
    np.testing.assert_allclose(ua, ub, rtol=1e-13, atol=1e-15 * np.abs(ub).max())


def test_constant_force_is_minus_gradient(oracle_mod):
    pos, q, sig, eps = _sys(9, 2)
    f, _ = oracle_mod.ljc_constant(pos, q, sig, eps, kc=KC, D=2.5)
    fd = _fd_force(lambda p: 0.5 * oracle_mod.ljc_constant(p, q, sig, eps, kc=KC, D=2.5)[1].sum(), pos)
    np.testing.assert_allclose(f, fd, rtol=1e-6, atol=1e-7 * np.abs(f).max())
    assert np.linalg.norm(f.sum(0)) <= 1e-13 * np.abs(f).sum()


def test_sigmoidal_reduces_to_constant_dielectric(oracle_mod):
    pos, q, sig, eps = _sys(30, 3)
    D = 7.5
    fs, us = oracle_mod.ljc_sigmoidal(pos, q, sig, eps, (0.0, 0.0, 0.0, np.log(D)), kc=KC)
    fc, uc = oracle_mod.ljc_constant(pos, q, sig, eps, kc=KC, D=D)
    np.testing.assert_allclose(fs, fc, rtol=1e-12, atol=1e-13 * np.abs(fc).max())
    np.testing.assert_allclose(us, uc, rtol=1e-12, atol=1e-13 * np.abs(uc).max())


ZC = (2e-4, -6e-3, 0.25, 0.4)


def test_sigmoidal_two_body_value(oracle_mod):
    r = 5.0
    pos, q, sig, eps = _pair(r, eps=(0.0, 0.0))
    _, u = oracle_mod.ljc_sigmoidal(pos, q, sig, eps, ZC, kc=KC)
    a, b, c, d = ZC
    zeta = np.exp(a * 125.0 + b * 25.0 + c * 5.0 + d)
    np.testing.assert_allclose(u, [KC * 0.5 * -0.4 / (zeta * r)] * 2, rtol=1e-14)


def test_sigmoidal_force_is_minus_gradient(oracle_mod):
    pos, q, sig, eps = _sys(9, 4)
    f, _ = oracle_mod.ljc_sigmoidal(pos, q, sig, eps, ZC, kc=KC)
    fd = _fd_force(lambda p: 0.5 * oracle_mod.ljc_sigmoidal(p, q, sig, eps, ZC, kc=KC)[1].sum(), pos)
    np.testing.assert_allclose(f, fd, rtol=1e-6, atol=1e-7 * np.abs(f).max())
    assert np.linalg.norm(f.sum(0)) <= 1e-13 * np.abs(f).sum()
