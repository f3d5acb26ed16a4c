"""Pins for the oracle's softened-gravity law (Eq. 1, Section 3.3), CPU only.

Each test checks the oracle against something other than itself: hand-worked
closed forms, a textbook symmetric configuration, Newton's third law, the
gradient of the potential by finite differences, invariances, and the
replication identity of Section 3.4.
"""
import numpy as np
import pytest
from hypothesis import given, settings, strategies as st


def test_two_body_closed_form(oracle_mod):
    # r1 = 0, r2 = (3,4,0): |d| = 5.  a1 = G m2 d / s^3, phi1 = -G m2 / s.
    pos = np.array([[0.0, 0.0, 0.0], [3.0, 4.0, 0.0]])
    mass = np.array([7.0, 2.0])
    acc, phi = oracle_mod.gravity(pos, mass, G=1.5, eps=0.0)
    np.testing.assert_allclose(acc[0], [0.072, 0.096, 0.0], rtol=1e-15, atol=1e-17)
    np.testing.assert_allclose(phi[0], -0.6, rtol=1e-15)
    # the other body feels G m1 (-d) / s^3
    np.testing.assert_allclose(acc[1], [-1.5 * 7 * 3 / 125, -1.5 * 7 * 4 / 125, 0.0], rtol=1e-15)
    # softening eps = 12: s = sqrt(25 + 144) = 13
    acc, phi = oracle_mod.gravity(pos, mass, G=1.5, eps=12.0)
    np.testing.assert_allclose(acc[0], [3.0 * 3 / 2197, 3.0 * 4 / 2197, 0.0], rtol=1e-15, atol=1e-18)
    np.testing.assert_allclose(phi[0], -3.0 / 13.0, rtol=1e-15)


@pytest.mark.parametrize("n", [3, 4, 7, 16])
def test_regular_polygon(oracle_mod, n):
    # n equal masses on a circle of radius R: the pull on each vertex is radial,
    # |a| = G m / (4 R^2) * sum_k csc(pi k / n), phi = -G m / (2R) * sum_k csc(pi k / n).
    R, m, G = 2.5, 0.3, 1.7
    th = 2 * np.pi * np.arange(n) / n + 0.1
    pos = np.stack([R * np.cos(th), R * np.sin(th), np.full(n, 0.4)], axis=1)
    acc, phi = oracle_mod.gravity(pos, np.full(n, m), G=G)
    csc = (1.0 / np.sin(np.pi * np.arange(1, n) / n)).sum()
    rhat = np.stack([np.cos(th), np.sin(th), np.zeros(n)], axis=1)
    np.testing.assert_allclose(acc, -(G * m / (4 * R * R)) * csc * rhat, rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(phi, -(G * m / (2 * R)) * csc, rtol=1e-14)


def _rand_system(n, seed, spread=1.0):
    rng = np.random.default_rng(seed)
    return rng.normal(0, spread, (n, 3)), rng.uniform(0.1, 2.0, n)


def test_newton_third_law(oracle_mod):
    pos, mass = _rand_system(300, 11)
    acc, _ = oracle_mod.gravity(pos, mass, eps=0.05)
    net = (mass[:, None] * acc).sum(0)
    scale = (mass * np.linalg.norm(acc, axis=1)).sum()
    assert np.linalg.norm(net) <= 1e-14 * scale


def test_force_is_minus_gradient_of_potential(oracle_mod):
    # a_i = -(1/m_i) dU/dr_i with U = 1/2 sum_i m_i phi_i
    pos, mass = _rand_system(12, 5)
    G, eps, h = 1.3, 0.2, 1e-5
    acc, _ = oracle_mod.gravity(pos, mass, G=G, eps=eps)

    def U(p):
        return 0.5 * (mass * oracle_mod.gravity(p, mass, G=G, eps=eps)[1]).sum()

    fd = np.zeros_like(pos)
    for i in range(pos.shape[0]):
        for c in range(3):
            pp, pm = pos.copy(), pos.copy()
            pp[i, c] += h
            pm[i, c] -= h
            fd[i, c] = -(U(pp) - U(pm)) / (2 * h) / mass[i]
    np.testing.assert_allclose(acc, fd, rtol=1e-7, atol=1e-8 * np.abs(acc).max())


@settings(max_examples=25, deadline=None)
@given(seed=st.integers(0, 10_000), n=st.integers(2, 40))
def test_permutation_invariance(oracle_mod, seed, n):
    pos, mass = _rand_system(n, seed)
    perm = np.random.default_rng(seed + 1).permutation(n)
    acc, phi = oracle_mod.gravity(pos, mass, eps=0.01)
    acc_p, phi_p = oracle_mod.gravity(pos[perm], mass[perm], eps=0.01)
    np.testing.assert_allclose(acc_p, acc[perm], rtol=1e-12, atol=1e-14 * np.abs(acc).max())
    np.testing.assert_allclose(phi_p, phi[perm], rtol=1e-13)


def test_translation_invariance(oracle_mod):
    pos, mass = _rand_system(64, 3)
    acc, phi = oracle_mod.gravity(pos, mass, eps=0.01)
    acc_t, phi_t = oracle_mod.gravity(pos + np.array([0.25, -0.5, 0.125]), mass, eps=0.01)
    np.testing.assert_allclose(acc_t, acc, rtol=1e-9, atol=1e-12 * np.abs(acc).max())
    np.testing.assert_allclose(phi_t, phi, rtol=1e-12)


def test_replication_identity(oracle_mod):
    # Section 3.4: forces from disjoint halves of the j range add up to the force.
    pos, mass = _rand_system(101, 8)
    acc, phi = oracle_mod.gravity(pos, mass, eps=0.02)
    a1, p1 = oracle_mod.gravity(pos, mass, eps=0.02, jrange=(0, 50))
    a2, p2 = oracle_mod.gravity(pos, mass, eps=0.02, jrange=(50, 101))
    np.testing.assert_allclose(a1 + a2, acc, rtol=1e-12, atol=1e-14 * np.abs(acc).max())
    np.testing.assert_allclose(p1 + p2, phi, rtol=1e-13)


def test_subset_rows_match_full(oracle_mod):
    pos, mass = _rand_system(200, 9)
    acc, phi = oracle_mod.gravity(pos, mass, eps=0.01)
    il = np.array([199, 0, 17, 17, 101])
    a, p = oracle_mod.gravity(pos, mass, eps=0.01, ilist=il)
    np.testing.assert_array_equal(a, acc[il])
    np.testing.assert_array_equal(p, phi[il])


def test_self_term_excluded_and_degenerate_sizes(oracle_mod):
    a, p = oracle_mod.gravity(np.array([[1.0, 2.0, 3.0]]), np.array([5.0]), eps=0.1)
    assert np.all(a == 0) and np.all(p == 0)
    a, p = oracle_mod.gravity(np.zeros((0, 3)), np.zeros(0))
    assert a.shape == (0, 3) and p.shape == (0,)
    # coincident bodies without softening: the pair term is undefined (inf/nan)
    a, p = oracle_mod.gravity(np.zeros((2, 3)), np.ones(2), eps=0.0)
    assert not np.all(np.isfinite(a)) and not np.all(np.isfinite(p))


def test_thread_count_does_not_change_results(oracle_mod):
    pos, mass = _rand_system(500, 21)
    a1, p1 = oracle_mod.gravity(pos, mass, eps=0.01, nthreads=1)
    a4, p4 = oracle_mod.gravity(pos, mass, eps=0.01, nthreads=4)
    np.testing.assert_array_equal(a1, a4)
    np.testing.assert_array_equal(p1, p4)


def test_thread_request_does_not_stick(oracle_mod):
    """A one-thread request applies to that call only: a later request for all threads
    gets the initial count back (the bench times the oracle both ways)."""
    full = oracle_mod.threads(0)
    assert oracle_mod.threads(1) == 1
    assert oracle_mod.threads(0) == full
