"""Pins for the oracle's acceleration-and-jerk law (Table 1 "Gravity (accel &
jerk)") and the fourth-order Hermite integrators built on it, CPU only.

* jerk: the time derivative of the acceleration along the motion (central
  differences of a(x + v h)), two-body closed forms for transverse and radial
  relative motion, and sum_i m_i jerk_i = 0 (Newton's third law, differentiated);
  the acceleration and potential agree with the plain gravity oracle.
* Hermite, shared step: a circular Kepler orbit against the exact solution,
  with the error falling 16x when the step halves (fourth order), and energy
  conservation on a softened Plummer sphere.
* Hermite, block steps: when every particle's criterion allows the largest
  step the block scheme is the shared-step scheme (bitwise); with real steps
  the schedule keeps every t_i a multiple of its power-of-two step, and energy
  is conserved at the synchronisation points.
"""
import numpy as np

from paper_0706_3060_amd import workloads as W


def test_jerk_is_time_derivative_of_acceleration(oracle_mod):
    x, v, m = W.plummer(40, 3)
    eps = 0.05
    _, jerk, _ = oracle_mod.gravity_jerk(x, v, m, eps=eps)
    h = 1e-5
    ap, _ = oracle_mod.gravity(x + h * v, m, eps=eps)
    am, _ = oracle_mod.gravity(x - h * v, m, eps=eps)
    fd = (ap - am) / (2 * h)
    np.testing.assert_allclose(jerk, fd, rtol=1e-6, atol=1e-8 * np.abs(jerk).max())


def test_jerk_two_body_closed_forms(oracle_mod):
    r, w, m1 = 2.0, 0.3, 0.7
    pos = np.array([[0.0, 0.0, 0.0], [r, 0.0, 0.0]])
    mass = np.array([1.3, m1])
    # transverse relative velocity: d . w = 0, jerk_0 = m1 w / r^3
    vel = np.array([[0.0, 0.0, 0.0], [0.0, w, 0.0]])
    a, j, phi = oracle_mod.gravity_jerk(pos, vel, mass)
    np.testing.assert_allclose(a[0], [m1 / r ** 2, 0, 0], rtol=1e-15)
    np.testing.assert_allclose(j[0], [0, m1 * w / r ** 3, 0], rtol=1e-15, atol=1e-18)
    # radial relative velocity: jerk_0 = m1 (w / r^3 - 3 w / r^3) = -2 m1 w / r^3 along x
    vel = np.array([[0.0, 0.0, 0.0], [w, 0.0, 0.0]])
    _, j, _ = oracle_mod.gravity_jerk(pos, vel, mass)
    np.testing.assert_allclose(j[0], [-2 * m1 * w / r ** 3, 0, 0], rtol=1e-15, atol=1e-18)
    np.testing.assert_allclose(phi, [-m1 / r, -1.3 / r], rtol=1e-15)


def test_jerk_momentum_and_agreement_with_gravity(oracle_mod):
    x, v, m = W.plummer(50, 4)
    m = m * np.random.default_rng(2).uniform(0.5, 1.5, 50)
    a, j, phi = oracle_mod.gravity_jerk(x, v, m, G=1.7, eps=0.02)
    mj = (m[:, None] * j).sum(0)
    assert np.abs(mj).max() <= 1e-14 * (m[:, None] * np.abs(j)).sum()
    ag, pg = oracle_mod.gravity(x, m, G=1.7, eps=0.02)
    np.testing.assert_allclose(a, ag, rtol=1e-14, atol=1e-16)
    np.testing.assert_allclose(phi, pg, rtol=1e-14)
    il = np.array([7, 0, 49, 7])
    a2, j2, _ = oracle_mod.gravity_jerk(x, v, m, G=1.7, eps=0.02, ilist=il)
    np.testing.assert_array_equal(j2, j[il])


def _kepler_circular():
    # equal masses 1/2 at separation 1: relative angular velocity sqrt(G M / r^3) = 1
    pos = np.array([[-0.5, 0.0, 0.0], [0.5, 0.0, 0.0]])
    vel = np.array([[0.0, -0.5, 0.0], [0.0, 0.5, 0.0]])
    return pos, vel, np.array([0.5, 0.5])


def test_hermite_kepler_orbit_is_fourth_order(oracle_mod):
    pos, vel, m = _kepler_circular()
    a, j, _ = oracle_mod.gravity_jerk(pos, vel, m)
    T = 1.0
    exact = np.array([[-0.5 * np.cos(T), -0.5 * np.sin(T), 0.0], [0.5 * np.cos(T), 0.5 * np.sin(T), 0.0]])
    errs = []
    for k in (32, 64, 128):
        x, v, _, _ = oracle_mod.hermite(pos, vel, a, j, m, T / k, k)
        errs.append(np.abs(x - exact).max())
    assert errs[-1] < 1e-9
    for e1, e2 in zip(errs, errs[1:]):
        assert 13.0 < e1 / e2 < 19.0, errs


def test_hermite_conserves_energy_on_plummer(oracle_mod):
    x, v, m = W.plummer(32, 7)
    eps = 0.05

    def energy(x, v):
        _, phi = oracle_mod.gravity(x, m, eps=eps)
        return 0.5 * (m * (v * v).sum(1)).sum() + 0.5 * (m * phi).sum()

    a, j, _ = oracle_mod.gravity_jerk(x, v, m, eps=eps)
    e0 = energy(x, v)
    x1, v1, a1, j1 = oracle_mod.hermite(x, v, a, j, m, 1.0 / 512, 256, eps=eps)
    assert abs(energy(x1, v1) - e0) < 1e-7 * abs(e0)
    # acc / jerk on exit are those of the last predicted state
    ar, jr, _ = oracle_mod.gravity_jerk(x1, v1, m, eps=eps)
    assert np.abs(a1 - ar).max() < 1e-6 * np.abs(ar).max()


def test_block_steps_reduce_to_shared_step(oracle_mod):
    x, v, m = W.plummer(24, 8)
    eps, dt_max = 0.05, 1.0 / 256
    a, j, _ = oracle_mod.gravity_jerk(x, v, m, eps=eps)
    t, dt = oracle_mod.hermite_block_init(a, j, 1e6, dt_max)
    assert np.all(t == 0) and np.all(dt == dt_max)
    xb, vb, ab, jb, tb, dtb, act, tn = oracle_mod.hermite_block(x, v, a, j, t, dt, m, 6, 1e6, dt_max,
                                                                eps=eps)
    xs, vs, as_, js = oracle_mod.hermite(x, v, a, j, m, dt_max, 6, eps=eps)
    assert np.all(act == 24) and tn == 6 * dt_max and np.all(tb == tn)
    np.testing.assert_array_equal(xb, xs)
    np.testing.assert_array_equal(vb, vs)
    np.testing.assert_array_equal(ab, as_)
    np.testing.assert_array_equal(jb, js)


def test_block_schedule_invariants_and_energy(oracle_mod):
    x, v, m = W.plummer(64, 9)
    eps, dt_max, eta = 0.01, 1.0 / 16, 0.02

    def energy(x, v):
        _, phi = oracle_mod.gravity(x, m, eps=eps)
        return 0.5 * (m * (v * v).sum(1)).sum() + 0.5 * (m * phi).sum()

    a, j, _ = oracle_mod.gravity_jerk(x, v, m, eps=eps)
    t, dt = oracle_mod.hermite_block_init(a, j, 0.01, dt_max)
    e0 = energy(x, v)
    state = (x, v, a, j, t, dt)
    t_now, steps, actives = 0.0, 0, []
    while t_now < 2 * dt_max:
        xs, vs, as_, js, ts, dts, act, t_now = oracle_mod.hermite_block(*state, m, 1, eta, dt_max, eps=eps)
        state = (xs, vs, as_, js, ts, dts)
        actives.append(int(act[0]))
        steps += 1
        k = np.log2(dt_max / dts)
        assert np.all(k == np.round(k)) and np.all(k >= 0)          # power-of-two fractions
        assert np.all(np.fmod(ts, dts) == 0)                         # commensurate
        assert np.all(ts <= t_now) and np.all(ts + dts > t_now)
    assert t_now == 2 * dt_max and np.all(state[4] == t_now)          # synchronised
    assert len(set(np.round(np.log2(dt_max / state[5])))) > 1       # genuinely individual steps
    assert min(actives) >= 1 and max(actives) == 64 and steps > 2
    assert abs(energy(state[0], state[1]) - e0) < 1e-6 * abs(e0)
