"""Pins for the oracle's exclusion lists (Section 5: the LJC kernels read an
exclusion list per particle) and for the bonded-chain workload, CPU only.

* Empty lists reproduce each plain LJC law exactly.
* With lists, F_i equals the plain F_i minus the two-body forces of the
  excluded partners (each from the oracle on the isolated pair), and U_i
  likewise; the masked pairs are therefore exactly the listed ones.
* Symmetric lists keep Newton's third law; F = -grad U by finite differences.
* The LJC(linear) adjoint with exclusions matches finite differences of
  L = g . F(r) and of the parameter derivatives.
* The chain generator: bond lengths, the minimum separation of non-bonded
  atoms, and symmetric 1-2 / 1-3 lists.
"""
import numpy as np
import pytest

from paper_0706_3060_amd import workloads as W

KC, D = 332.0637, 4.0
ZC = (2e-4, -6e-3, 0.25, 0.4)


def _plain(oracle_mod, kind, pos, q, s, e):
    if kind == 1:
        return oracle_mod.ljc_linear(pos, q, s, e, kc=KC, D=D)
    if kind == 2:
        return oracle_mod.ljc_constant(pos, q, s, e, kc=KC, D=D)
    return oracle_mod.ljc_sigmoidal(pos, q, s, e, ZC, kc=KC)


def _chains(n_chains=6, chain_len=7, seed=3):
    sy, eo, ei = W.bonded_chains(n_chains, chain_len, seed, box=18.0)
    return sy, eo, ei


@pytest.mark.parametrize("kind", [1, 2, 3])
def test_empty_lists_are_the_plain_law(oracle_mod, kind):
    sy, _, _ = _chains()
    eo = np.zeros(sy.n + 1, dtype=np.int64)
    f, u = oracle_mod.ljc_excl(kind, sy.pos, sy.q, sy.sigma, sy.epsilon, eo, [], kc=KC, D=D, zeta_coef=ZC)
    fr, ur = _plain(oracle_mod, kind, sy.pos, sy.q, sy.sigma, sy.epsilon)
    np.testing.assert_array_equal(f, fr)
    np.testing.assert_array_equal(u, ur)


@pytest.mark.parametrize("kind", [1, 2, 3])
def test_excluded_pairs_are_exactly_the_listed_ones(oracle_mod, kind):
    sy, eo, ei = _chains()
    f, u = oracle_mod.ljc_excl(kind, sy.pos, sy.q, sy.sigma, sy.epsilon, eo, ei, kc=KC, D=D, zeta_coef=ZC)
    fr, ur = _plain(oracle_mod, kind, sy.pos, sy.q, sy.sigma, sy.epsilon)
    fx, ux = fr.copy(), ur.copy()
    for i in range(sy.n):
        for j in ei[eo[i]:eo[i + 1]]:
            idx = [i, int(j)]
            f2, u2 = _plain(oracle_mod, kind, sy.pos[idx], sy.q[idx], sy.sigma[idx], sy.epsilon[idx])
            fx[i] -= f2[0]
            ux[i] -= u2[0]
    scale = np.abs(fr).max()
    np.testing.assert_allclose(f, fx, rtol=0, atol=1e-12 * scale)
    np.testing.assert_allclose(u, ux, rtol=0, atol=1e-12 * np.abs(ur).max())
    # the bonded partners are close: excluding them changes the forces a lot
    assert np.abs(f - fr).max() > 0.1 * np.abs(f).max()


@pytest.mark.parametrize("kind", [1, 2, 3])
def test_symmetric_lists_conserve_momentum_and_force_is_gradient(oracle_mod, kind):
    sy, eo, ei = _chains(3, 5, 7)
    f, _ = oracle_mod.ljc_excl(kind, sy.pos, sy.q, sy.sigma, sy.epsilon, eo, ei, kc=KC, D=D, zeta_coef=ZC)
    assert np.linalg.norm(f.sum(0)) <= 1e-12 * np.abs(f).sum()

    def energy(p):
        return 0.5 * oracle_mod.ljc_excl(kind, p, sy.q, sy.sigma, sy.epsilon, eo, ei, kc=KC, D=D,
                                         zeta_coef=ZC)[1].sum()

    h = 1e-6
    fd = np.zeros_like(sy.pos)
    for i in range(sy.n):
        for c in range(3):
            pp, pm = sy.pos.copy(), sy.pos.copy()
            pp[i, c] += h
            pm[i, c] -= h
            fd[i, c] = -(energy(pp) - energy(pm)) / (2 * h)
    np.testing.assert_allclose(f, fd, rtol=1e-6, atol=1e-6 * np.abs(f).max())


def test_adjoint_with_exclusions_matches_finite_differences(oracle_mod):
    sy, eo, ei = _chains(3, 5, 9)
    g = W.unit_cotangent(sy.n, 4)
    gp, gq, gs, ge = oracle_mod.ljc_adjoint_excl(sy.pos, sy.q, sy.sigma, sy.epsilon, g, eo, ei, kc=KC, D=D)

    def loss(pos=sy.pos, q=sy.q, s=sy.sigma, e=sy.epsilon):
        return (g * oracle_mod.ljc_excl(1, pos, q, s, e, eo, ei, kc=KC, D=D)[0]).sum()

    h = 1e-6
    for i in (0, 4, 9, 14):
        for c in range(3):
            pp, pm = sy.pos.copy(), sy.pos.copy()
            pp[i, c] += h
            pm[i, c] -= h
            fd = (loss(pos=pp) - loss(pos=pm)) / (2 * h)
            assert abs(gp[i, c] - fd) <= 1e-5 * max(1.0, abs(fd)), (i, c, gp[i, c], fd)
        base = {"q": sy.q, "s": sy.sigma, "e": sy.epsilon}
        for name, grad in (("q", gq), ("s", gs), ("e", ge)):
            kp, km = dict(base), dict(base)
            kp[name], km[name] = base[name].copy(), base[name].copy()
            kp[name][i] += h
            km[name][i] -= h
            fd = (loss(**kp) - loss(**km)) / (2 * h)
            assert abs(grad[i] - fd) <= 1e-5 * max(1.0, abs(fd)), (name, i, grad[i], fd)
    # empty lists: the plain adjoint
    eo0 = np.zeros(sy.n + 1, dtype=np.int64)
    a = oracle_mod.ljc_adjoint_excl(sy.pos, sy.q, sy.sigma, sy.epsilon, g, eo0, [], kc=KC, D=D)
    b = oracle_mod.ljc_adjoint(sy.pos, sy.q, sy.sigma, sy.epsilon, g, kc=KC, D=D)
    for x, y in zip(a, b):
        np.testing.assert_array_equal(x, y)


def test_bonded_chain_geometry():
    sy, eo, ei = W.bonded_chains(40, 12, 5)
    n, L = sy.n, 12
    ch = np.arange(n) // L
    bonds = np.linalg.norm(sy.pos[1:] - sy.pos[:-1], axis=1)[(ch[1:] == ch[:-1])]
    np.testing.assert_allclose(bonds, 1.53, rtol=1e-12)
    d = np.linalg.norm(sy.pos[:, None] - sy.pos[None], axis=-1)
    I, J = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    bonded = (ch[I] == ch[J]) & (np.abs(I - J) == 1)
    assert d[(I != J) & ~bonded].min() >= 2.5
    pairs = {(i, int(j)) for i in range(n) for j in ei[eo[i]:eo[i + 1]]}
    assert all((j, i) in pairs for (i, j) in pairs)
    assert all(ch[i] == ch[j] and 1 <= abs(i - j) <= 2 for (i, j) in pairs)
    assert len(pairs) == 40 * (2 * (L - 1) + 2 * (L - 2))
