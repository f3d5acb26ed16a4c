"""Pins for the oracle's update step and the adjoints, CPU only.

Leapfrog (the force-then-update cycle of Section 1, read as kick-drift-kick):
a circular two-body orbit, second-order energy error, time reversibility.
Adjoints (derivatives of Eq. 1 and of the LJC(linear) law): finite
differences, the dot-product test, the translation sum rule and the exact
Euler (homogeneity) identities of the LJC law.
"""
import numpy as np
import pytest

KC = 332.0637
D = 4.0


def test_circular_binary_orbit(oracle_mod):
    # two masses 1/2 at separation 1 (G = 1, no softening) circle their centre of
    # mass with omega = 1, speed 1/2; after one period they return to the start.
    pos = np.array([[0.5, 0.0, 0.0], [-0.5, 0.0, 0.0]])
    vel = np.array([[0.0, 0.5, 0.0], [0.0, -0.5, 0.0]])
    mass = np.array([0.5, 0.5])
    acc, _ = oracle_mod.gravity(pos, mass)
    np.testing.assert_allclose(acc, [[-0.5, 0, 0], [0.5, 0, 0]], rtol=1e-15)
    nsteps = 2000
    dt = 2 * np.pi / nsteps
    x, v, a, pot = oracle_mod.leapfrog(oracle_mod.GRAVITY, pos, vel, acc, mass, dt, nsteps)
    np.testing.assert_allclose(np.linalg.norm(x, axis=1), 0.5, rtol=1e-5)
    # leapfrog's phase error per period is ~ 2 pi (omega dt)^2 / 24 ~ 2.6e-6
    np.testing.assert_allclose(x, pos, atol=2e-5)
    np.testing.assert_allclose(v, vel, atol=2e-5)
    np.testing.assert_allclose(pot, [-0.5, -0.5], rtol=1e-5)   # phi = -G m_j / r, m_j = 1/2


def _energy(oracle_mod, x, v, m, eps):
    _, phi = oracle_mod.gravity(x, m, eps=eps)
    return 0.5 * (m * (v * v).sum(1)).sum() + 0.5 * (m * phi).sum()


def _max_energy_error(oracle_mod, pos, vel, m, eps, dt, t_end):
    acc, _ = oracle_mod.gravity(pos, m, eps=eps)
    e0 = _energy(oracle_mod, pos, vel, m, eps)
    x, v, a = pos, vel, acc
    worst = 0.0
    nout = 8
    for _ in range(nout):
        x, v, a, _ = oracle_mod.leapfrog(oracle_mod.GRAVITY, x, v, a, m, dt,
                                         int(round(t_end / nout / dt)), eps=eps)
        worst = max(worst, abs(_energy(oracle_mod, x, v, m, eps) - e0) / abs(e0))
    return worst


def test_energy_error_is_second_order(oracle_mod):
    from paper_0706_3060_amd.workloads import plummer
    pos, vel, m = plummer(64, 17)
    eps = 0.1
    e1 = _max_energy_error(oracle_mod, pos, vel, m, eps, 1 / 64, 1.0)
    e2 = _max_energy_error(oracle_mod, pos, vel, m, eps, 1 / 128, 1.0)
    assert e1 < 1e-3
    assert 3.0 < e1 / e2 < 5.0, (e1, e2)


def test_time_reversibility(oracle_mod):
    from paper_0706_3060_amd.workloads import plummer
    pos, vel, m = plummer(32, 5)
    eps = 0.05
    acc, _ = oracle_mod.gravity(pos, m, eps=eps)
    x, v, a, _ = oracle_mod.leapfrog(oracle_mod.GRAVITY, pos, vel, acc, m, 1e-3, 200, eps=eps)
    x2, v2, a2, _ = oracle_mod.leapfrog(oracle_mod.GRAVITY, x, -v, a, m, 1e-3, 200, eps=eps)
    np.testing.assert_allclose(x2, pos, atol=1e-12)
    np.testing.assert_allclose(-v2, vel, atol=1e-11)


def test_ljc_leapfrog_with_masses_conserves_energy(oracle_mod):
    # two atoms released from rest inside the LJ well oscillate; kinetic energy
    # uses the masses passed as inverse masses.
    pos = np.array([[0.0, 0.0, 0.0], [4.2, 0.0, 0.0]])
    vel = np.zeros((2, 3))
    par = np.array([[0.0, 3.4, 0.2], [0.0, 3.4, 0.2]])
    mass = np.array([12.0, 16.0])
    inv_mass = 1.0 / mass
    f, u = oracle_mod.ljc_linear(pos, par[:, 0], par[:, 1], par[:, 2])
    e0 = 0.5 * u.sum()
    acc = f * inv_mass[:, None]
    x, v, a, pot = oracle_mod.leapfrog(oracle_mod.LJC_LINEAR, pos, vel, acc, par, 0.01, 3000,
                                       inv_mass=inv_mass)
    e1 = 0.5 * (mass * (v * v).sum(1)).sum() + 0.5 * pot.sum()
    assert abs(e1 - e0) < 1e-4 * abs(e0)
    np.testing.assert_allclose((mass[:, None] * v).sum(0), 0, atol=1e-12)   # momentum
    assert np.abs(v).max() > 1e-3   # it did move


# ------------------------------------------------------------------ adjoints

def _grav_sys(n, seed):
    rng = np.random.default_rng(seed)
    return rng.normal(0, 1, (n, 3)), rng.uniform(0.2, 2.0, n)


def test_gravity_adjoint_matches_fd_jvp(oracle_mod):
    pos, m = _grav_sys(10, 2)
    G, eps = 1.2, 0.15
    rng = np.random.default_rng(3)
    u = rng.normal(size=pos.shape)
    v = rng.normal(size=pos.shape)
    h = 1e-5
    ap, _ = oracle_mod.gravity(pos + h * v, m, G=G, eps=eps)
    am, _ = oracle_mod.gravity(pos - h * v, m, G=G, eps=eps)
    jv = (ap - am) / (2 * h)
    adj = oracle_mod.gravity_adjoint(pos, m, u, G=G, eps=eps)
    lhs = (u * jv).sum()
    rhs = (adj * v).sum()
    assert abs(lhs - rhs) <= 1e-8 * (abs(lhs) + np.abs(u * jv).sum())
    # full Jacobian-transpose check, column by column
    J = np.zeros((pos.size, pos.size))
    for k in range(pos.size):
        e = np.zeros(pos.size)
        e[k] = h
        J[:, k] = (oracle_mod.gravity(pos + e.reshape(-1, 3), m, G=G, eps=eps)[0]
                   - oracle_mod.gravity(pos - e.reshape(-1, 3), m, G=G, eps=eps)[0]).ravel() / (2 * h)
    np.testing.assert_allclose(adj.ravel(), J.T @ u.ravel(), rtol=1e-6, atol=1e-8 * np.abs(adj).max())


def test_gravity_adjoint_sum_rule_and_symmetry(oracle_mod):
    pos, m = _grav_sys(50, 4)
    g = np.random.default_rng(5).normal(size=pos.shape)
    adj = oracle_mod.gravity_adjoint(pos, m, g, eps=0.05)
    assert np.linalg.norm(adj.sum(0)) <= 1e-13 * np.abs(adj).sum()
    # equal masses make the Jacobian symmetric: <u, J^T w> = <w, J^T u>
    me = np.full(50, 0.02)
    w = np.random.default_rng(6).normal(size=pos.shape)
    a1 = (g * oracle_mod.gravity_adjoint(pos, me, w, eps=0.05)).sum()
    a2 = (w * oracle_mod.gravity_adjoint(pos, me, g, eps=0.05)).sum()
    assert abs(a1 - a2) <= 1e-12 * abs(a1)


def _ljc_sys(n, seed, box=11.0):
    rng = np.random.default_rng(seed)
    k = int(np.ceil(n ** (1 / 3)))
    grid = np.stack(np.meshgrid(*(np.arange(k),) * 3, indexing="ij"), -1).reshape(-1, 3)[:n]
    pos = grid * (box / k) + rng.uniform(-0.3, 0.3, (n, 3))
    return pos, rng.uniform(-0.8, 0.8, n), rng.uniform(3.0, 3.8, n), rng.uniform(0.05, 0.2, n)


def _L(oracle_mod, g, pos, q, s, e):
    return (g * oracle_mod.ljc_linear(pos, q, s, e, kc=KC, D=D)[0]).sum()


def test_ljc_adjoint_matches_finite_differences(oracle_mod):
    pos, q, s, e = _ljc_sys(8, 9)
    g = np.random.default_rng(10).normal(size=pos.shape)
    gp, gq, gs, ge = oracle_mod.ljc_adjoint(pos, q, s, e, g, kc=KC, D=D)

    def fd(fun, x, h):
        out = np.zeros_like(x)
        for idx in np.ndindex(x.shape):
            xp, xm = x.copy(), x.copy()
            xp[idx] += h
            xm[idx] -= h
            out[idx] = (fun(xp) - fun(xm)) / (2 * h)
        return out

    np.testing.assert_allclose(gp, fd(lambda p: _L(oracle_mod, g, p, q, s, e), pos, 1e-5),
                               rtol=1e-6, atol=1e-7 * np.abs(gp).max())
    np.testing.assert_allclose(gq, fd(lambda x: _L(oracle_mod, g, pos, x, s, e), q, 1e-6),
                               rtol=1e-6, atol=1e-7 * np.abs(gq).max())
    np.testing.assert_allclose(gs, fd(lambda x: _L(oracle_mod, g, pos, q, x, e), s, 1e-6),
                               rtol=1e-6, atol=1e-7 * np.abs(gs).max())
    np.testing.assert_allclose(ge, fd(lambda x: _L(oracle_mod, g, pos, q, s, x), e, 1e-7),
                               rtol=1e-6, atol=1e-7 * np.abs(ge).max())


def test_ljc_euler_identities(oracle_mod):
    # F_C is quadratic in q, F_LJ is linear in eps, and scaling r and sigma by
    # lambda scales F_LJ by 1/lambda and F_C by 1/lambda^3.
    pos, q, s, e = _ljc_sys(27, 12, box=14.0)
    g = np.random.default_rng(13).normal(size=pos.shape)
    gp, gq, gs, ge = oracle_mod.ljc_adjoint(pos, q, s, e, g, kc=KC, D=D)
    fc = oracle_mod.ljc_linear(pos, q, s, np.zeros_like(e), kc=KC, D=D)[0]
    flj = oracle_mod.ljc_linear(pos, np.zeros_like(q), s, e, kc=KC, D=D)[0]
    gfc, gflj = (g * fc).sum(), (g * flj).sum()
    scale = np.abs(g * fc).sum() + np.abs(g * flj).sum()
    assert abs((q * gq).sum() - 2 * gfc) <= 1e-11 * scale
    assert abs((e * ge).sum() - gflj) <= 1e-11 * scale
    assert abs((s * gs).sum() + (pos * gp).sum() + gflj + 3 * gfc) <= 1e-10 * scale


def test_ljc_adjoint_sum_rule(oracle_mod):
    pos, q, s, e = _ljc_sys(30, 14, box=15.0)
    g = np.random.default_rng(15).normal(size=pos.shape)
    gp = oracle_mod.ljc_adjoint(pos, q, s, e, g)[0]
    assert np.linalg.norm(gp.sum(0)) <= 1e-12 * np.abs(gp).sum()


def test_adjoint_subset_rows(oracle_mod):
    pos, q, s, e = _ljc_sys(20, 16, box=13.0)
    g = np.random.default_rng(17).normal(size=pos.shape)
    full = oracle_mod.ljc_adjoint(pos, q, s, e, g)
    il = np.array([3, 19, 0])
    sub = oracle_mod.ljc_adjoint(pos, q, s, e, g, ilist=il)
    for a, b in zip(full, sub):
        np.testing.assert_array_equal(a[il], b)
    pg, mg = _grav_sys(20, 18)
    gg = oracle_mod.gravity_adjoint(pg, mg, g, eps=0.1)
    np.testing.assert_array_equal(oracle_mod.gravity_adjoint(pg, mg, g, eps=0.1, ilist=il), gg[il])


def test_ljc_constant_leapfrog_conserves_energy(oracle_mod):
    # an ion pair (opposite charges, constant dielectric) bound against the LJ
    # wall: energy, momentum conserved over many oscillations
    pos = np.array([[0.0, 0.0, 0.0], [0.0, 4.6, 0.3]])
    vel = np.zeros((2, 3))
    par = np.array([[0.4, 3.2, 0.1], [-0.4, 3.6, 0.15]])
    mass = np.array([23.0, 35.5])
    inv_mass = 1.0 / mass
    f, u = oracle_mod.ljc_constant(pos, par[:, 0], par[:, 1], par[:, 2], D=4.0)
    e0 = 0.5 * u.sum()
    x, v, a, pot = oracle_mod.leapfrog(oracle_mod.LJC_CONSTANT, pos, vel, f * inv_mass[:, None], par,
                                       0.005, 4000, inv_mass=inv_mass, D=4.0)
    e1 = 0.5 * (mass * (v * v).sum(1)).sum() + 0.5 * pot.sum()
    assert abs(e1 - e0) < 1e-4 * abs(e0)
    np.testing.assert_allclose((mass[:, None] * v).sum(0), 0, atol=1e-12)
    assert np.abs(v).max() > 1e-2
    # one step equals the hand-written kick-drift-kick around the oracle's forces
    x1, v1, a1, _ = oracle_mod.leapfrog(oracle_mod.LJC_CONSTANT, pos, vel, f * inv_mass[:, None], par,
                                        0.005, 1, inv_mass=inv_mass, D=4.0)
    vh = vel + 0.0025 * f * inv_mass[:, None]
    xe = pos + 0.005 * vh
    fe, _ = oracle_mod.ljc_constant(xe, par[:, 0], par[:, 1], par[:, 2], D=4.0)
    np.testing.assert_allclose(x1, xe, rtol=0, atol=1e-15)
    np.testing.assert_allclose(v1, vh + 0.0025 * fe * inv_mass[:, None], rtol=1e-13, atol=1e-16)
