"""Pins of the oracle's compensated sums and of its block-step criterion, CPU only.

Compensated sums (the FP64 j-sums the <= 1e-12 gates rest on):

* exact terms: one particle at the origin and its partners on the coordinate
  axes at distances R = 2^k (no softening), so that every pair term of gravity
  (m_j d / R^3, m_j / R) and of Coulomb with the linear dielectric
  (2 k q_i q_j d / (D R^4), k q_i q_j / (D R^2)) is an exact double.  Partners
  come in opposite pairs with nearly equal weights, so the sums cancel by
  factors of 1e3 and more.  The exact sum (rational arithmetic) rounded once
  is then the only correct FP64 answer: the oracle must return it to within
  one unit in the last place, and a plain left-to-right FP64 sum of the same
  terms misses it by far more.
* realistic terms: a Plummer sphere with particles placed in opposite pairs
  around a few centres (high cancellation on those rows), against a reference
  whose pair terms are computed in 80-bit extended precision and summed
  exactly; the oracle's error must stay within the FP64 rounding of the terms
  themselves and well below that of a plain FP64 sum.

Block-step criterion (the fourth-order Hermite scheme with block steps): the
initial estimate eta_s |a| / |j|, Aarseth's criterion and the power-of-two
quantisation on hand-computed values, and on a circular two-body orbit whose
derivatives are known in closed form (|d^k a / dt^k| = w^(k+2) R).
"""
import math
from fractions import Fraction

import numpy as np

from paper_0706_3060_amd import workloads as W

ULP = np.spacing


def _axis_points():
    """Points 2^k e_a on the three coordinate axes, k = -10 .. 10 (one of each +-pair)."""
    pts = []
    for k in range(-10, 11):
        for a in range(3):
            p = [0.0, 0.0, 0.0]
            p[a] = 2.0 ** k
            pts.append(p)
    return np.array(pts)


def _opposed_weights(rng, k, lo_exp, hi_exp, rel_bits):
    """k weights with 30-bit mantissas over a wide exponent range, and partners that differ from
    them by a few units at 2^-rel_bits relative (exact), so that opposite terms nearly cancel."""
    mant = rng.integers(1 << 29, 1 << 30, size=k).astype(np.float64)
    e = rng.integers(lo_exp, hi_exp, size=k)
    w = np.ldexp(mant, e - 30)
    dw = np.ldexp(rng.integers(-8, 8, size=k).astype(np.float64), e - rel_bits)
    return w, w + dw


def _exact_round(terms):
    s = sum((Fraction(float(t)) for t in terms), Fraction(0))
    return float(s)


def _plain(terms):
    s = 0.0
    for t in terms:
        s += float(t)
    return s


def _axis_system(rng, rel_bits, signed=False):
    half = _axis_points()
    k = half.shape[0]
    w1, w2 = _opposed_weights(rng, k, -12, 12, rel_bits)
    if signed:                                          # one sign per opposite pair
        sg = np.where(rng.random(k) < 0.5, -1.0, 1.0)
        w1, w2 = w1 * sg, w2 * sg
    pos = np.concatenate([np.zeros((1, 3)), half, -half])
    w = np.concatenate([[1.0], w1, w2])
    perm = 1 + rng.permutation(2 * k)                  # partners in random j order
    pos = np.concatenate([pos[:1], pos[perm]])
    w = np.concatenate([w[:1], w[perm]])
    return pos, w


def test_gravity_sums_are_correctly_rounded_on_exact_terms(oracle_mod):
    rng = np.random.default_rng(101)
    worst_or, worst_plain, kappa_min = 0.0, 0.0, np.inf
    for trial in range(6):
        pos, m = _axis_system(rng, 16)
        a, phi = oracle_mod.gravity(pos, m, ilist=np.array([0]))
        d, mj = pos[1:], m[1:]
        R = np.linalg.norm(d, axis=1)
        for c in range(3):
            terms = mj * d[:, c] / R ** 3                      # exact: m_j d / R^3 with R = 2^k
            ref = _exact_round(terms)
            kappa_min = min(kappa_min, np.abs(terms).sum() / abs(ref))
            err_or = abs(a[0, c] - ref) / ULP(abs(ref))
            err_pl = abs(_plain(terms) - ref) / ULP(abs(ref))
            assert err_or <= 1.0, (trial, c, err_or)
            worst_or = max(worst_or, err_or)
            worst_plain = max(worst_plain, err_pl)
        pterms = -mj / R
        ref = _exact_round(pterms)
        assert abs(phi[0] - ref) <= ULP(abs(ref)), (trial, phi[0], ref)
    assert kappa_min > 1e3, kappa_min
    # the compensated sums are not a plain sum in disguise
    assert worst_plain >= 5.0 * max(worst_or, 1.0), (worst_plain, worst_or)


def test_ljc_linear_sums_are_correctly_rounded_on_exact_terms(oracle_mod):
    # pure Coulomb with the linear dielectric (epsilon = 0 keeps every term exact),
    # k = 1 and D = 4: F_0 = sum_j 2 k q_0 q_j (r_0 - r_j) / (D r^4), U_0 = sum_j k q_0 q_j / (D r^2)
    rng = np.random.default_rng(102)
    worst_or, worst_plain, kappa_min = 0.0, 0.0, np.inf
    for trial in range(6):
        pos, q = _axis_system(rng, 16, signed=True)
        q[0] = 0.75
        n = q.size
        sig = np.full(n, 2.0)
        eps = np.zeros(n)
        f, u = oracle_mod.ljc_linear(pos, q, sig, eps, kc=1.0, D=4.0, ilist=np.array([0]))
        d = -pos[1:]                                           # r_0 - r_j
        R = np.linalg.norm(d, axis=1)
        qq = q[0] * q[1:]
        for c in range(3):
            terms = 2.0 * qq / 4.0 / R ** 4 * d[:, c]
            ref = _exact_round(terms)
            kappa_min = min(kappa_min, np.abs(terms).sum() / abs(ref))
            err_or = abs(f[0, c] - ref) / ULP(abs(ref))
            worst_or = max(worst_or, err_or)
            worst_plain = max(worst_plain, abs(_plain(terms) - ref) / ULP(abs(ref)))
            assert err_or <= 1.0, (trial, c, err_or)
        eterms = qq / 4.0 / R ** 2
        ref = _exact_round(eterms)
        assert abs(u[0] - ref) <= ULP(abs(ref)), (trial, u[0], ref)
    assert kappa_min > 1e3, kappa_min
    assert worst_plain >= 5.0 * max(worst_or, 1.0), (worst_plain, worst_or)


def _ld_reference_gravity(pos, m, eps, i):
    """a_i and phi_i with pair terms in 80-bit extended precision, summed exactly."""
    P = pos.astype(np.longdouble)
    M = m.astype(np.longdouble)
    d = P - P[i]
    s2 = (d * d).sum(1) + np.longdouble(eps) * np.longdouble(eps)
    s = np.sqrt(s2)
    w = M / (s2 * s)
    mask = np.arange(len(m)) != i
    out = []
    for c in range(3):
        t = (w * d[:, c])[mask]
        out.append(sum((Fraction(*x.as_integer_ratio()) for x in t), Fraction(0)))
    ph = -sum((Fraction(*x.as_integer_ratio()) for x in (M / s)[mask]), Fraction(0))
    absf = np.array([float(np.abs(w * d[:, c])[mask].sum()) for c in range(3)])
    return np.array([float(x) for x in out]), float(ph), absf


def test_gravity_against_extended_precision_at_high_cancellation(oracle_mod):
    # 400 particles: 4 centres, each surrounded by 99 particles in opposite pairs at equal masses
    # plus one unpaired particle, so that the centres' forces cancel by large factors
    rng = np.random.default_rng(103)
    x, _, _ = W.plummer(200, 21)
    centres = x[:4] * 0.5
    pts = [centres]
    for c in range(4):
        off = x[4 + 49 * c: 4 + 49 * (c + 1)] * 0.01
        pts += [centres[c] + off, centres[c] - off]
    pts.append(x[-4:])
    pos = np.concatenate(pts)
    m = rng.uniform(0.5, 1.5, pos.shape[0]) / pos.shape[0]
    for c in range(4):                                   # opposite partners carry equal masses
        b = 4 + 98 * c
        m[b + 49: b + 98] = m[b: b + 49]
    eps = 1e-3
    a, phi = oracle_mod.gravity(pos, m, eps=eps, ilist=np.arange(4))
    u = 2.0 ** -53
    plain_worse = 0
    for i in range(4):
        ref, ph_ref, absf = _ld_reference_gravity(pos, m, eps, i)
        kappa = absf.sum() / np.abs(ref).sum()
        assert kappa > 1e3, kappa
        # FP64 rounding of the pair terms (a few u each) bounds the oracle's error normwise
        err = np.abs(a[i] - ref)
        assert np.all(err <= 8 * u * absf), (i, err, absf)
        assert abs(phi[i] - ph_ref) <= 8 * u * abs(ph_ref)
        # a plain FP64 sum of the FP64 terms, in the same j order
        d = pos - pos[i]
        s2 = (d * d).sum(1) + eps * eps
        s = np.sqrt(s2)
        w = m / (s2 * s)
        for c in range(3):
            t = (w * d[:, c])[np.arange(len(m)) != i]
            if abs(_plain(t) - ref[c]) > 5 * abs(a[i, c] - ref[c]):
                plain_worse += 1
    # on most of the 12 cancelling components the plain sum is at least 5x further from the reference
    assert plain_worse >= 8, plain_worse


def test_ljc_linear_against_extended_precision(oracle_mod):
    sysm = W.md_system(300, 5, box=(32.0 * 300) ** (1.0 / 3.0))
    pos, q, sig, eps = sysm.pos, sysm.q, sysm.sigma, sysm.epsilon
    rows = np.array([0, 17, 123, 299])
    f, u = oracle_mod.ljc_linear(pos, q, sig, eps, ilist=rows)
    kc, D = 332.0637, 4.0
    uu = 2.0 ** -53
    for k, i in enumerate(rows):
        P = pos.astype(np.longdouble)
        r = P[i] - P
        r2 = (r * r).sum(1)
        mask = np.arange(len(q)) != i
        r2[~mask] = 1
        sij = (np.longdouble(sig[i]) + sig.astype(np.longdouble)) / 2
        eij = np.sqrt(np.longdouble(eps[i]) * eps.astype(np.longdouble))
        sr6 = (sij * sij / r2) ** 3
        coul = np.longdouble(kc) * np.longdouble(q[i]) * q.astype(np.longdouble) / np.longdouble(D)
        Wt = 2 * coul / (r2 * r2) + 24 * eij / r2 * (2 * sr6 * sr6 - sr6)
        for c in range(3):
            t = (Wt * r[:, c])[mask]
            ref = float(sum((Fraction(*x.as_integer_ratio()) for x in t), Fraction(0)))
            bound = 16 * uu * float(np.abs(t).sum())
            assert abs(f[k, c] - ref) <= bound, (i, c, f[k, c], ref, bound)
        et = (coul / r2 + 4 * eij * (sr6 * sr6 - sr6))[mask]
        eref = float(sum((Fraction(*x.as_integer_ratio()) for x in et), Fraction(0)))
        assert abs(u[k] - eref) <= 16 * uu * float(np.abs(et).sum())


# ------------------------------------------------------------------ step criterion
def test_initial_step_hand_values(oracle_mod):
    # |a| = |(3, 4, 0)| = 5, |j| = |(0, 0, 2)| = 2: eta_s |a| / |j| = 0.01 * 5 / 2 = 0.025
    assert oracle_mod.initial_step([3, 4, 0], [0, 0, 2], 0.01, 1.0) == 0.025
    # zero jerk: the largest step
    assert oracle_mod.initial_step([3, 4, 0], [0, 0, 0], 0.01, 0.5) == 0.5
    # quantised at t = 0: the largest 2^-k <= 0.025 is 2^-6 = 0.015625
    t, dt = oracle_mod.hermite_block_init(np.array([[3.0, 4, 0]]), np.array([[0.0, 0, 2]]), 0.01, 1.0)
    assert t[0] == 0.0 and dt[0] == 0.015625


def test_aarseth_criterion_hand_values(oracle_mod):
    # |a| = 5, |j| = 2, |a2| = |(1, 2, 2)| = 3, |a3| = |(2, 3, 6)| = 7, eta = 0.02:
    # (|a||a2| + |j|^2) / (|j||a3| + |a2|^2) = (15 + 4) / (14 + 9) = 19 / 23
    dt = oracle_mod.aarseth_step([3, 4, 0], [0, 0, 2], [1, 2, 2], [2, 3, 6], 0.02, 1.0)
    assert abs(dt - math.sqrt(0.02 * 19.0 / 23.0)) <= 2e-16
    assert abs(dt - 0.1285369173834303) <= 2e-16            # sqrt(0.38 / 23) = sqrt(0.016521739130434782)
    # the same magnitudes in other places give other values (no symmetric mix-up):
    # a <-> j: (2*3 + 25) / (5*7 + 9) = 31 / 44; a2 <-> a3: (5*7 + 4) / (2*3 + 49) = 39 / 55
    assert abs(oracle_mod.aarseth_step([0, 0, 2], [3, 4, 0], [1, 2, 2], [2, 3, 6], 0.02, 1.0)
               - math.sqrt(0.02 * 31.0 / 44.0)) <= 2e-16
    assert abs(oracle_mod.aarseth_step([3, 4, 0], [0, 0, 2], [2, 3, 6], [1, 2, 2], 0.02, 1.0)
               - math.sqrt(0.02 * 39.0 / 55.0)) <= 2e-16
    # vanishing denominator: the largest step
    assert oracle_mod.aarseth_step([3, 4, 0], [0, 0, 0], [0, 0, 0], [2, 3, 6], 0.02, 0.25) == 0.25


def test_quantise_step_branches(oracle_mod):
    Q = oracle_mod.quantise_step
    # largest dt_max / 2^k not above the estimate
    assert Q(0.3, 1.0, 0.0, 0.0) == 0.25
    assert Q(0.25, 1.0, 0.0, 0.0) == 0.25
    assert Q(5.0, 1.0, 0.0, 0.0) == 1.0
    # at most twice the old step
    assert Q(0.3, 1.0, 0.0, 1.0 / 16) == 0.125
    assert Q(0.3, 1.0, 0.0, 0.25) == 0.25
    # commensurate with the new time: t = 3/8 is a multiple of 1/8 but not of 1/4
    assert Q(0.3, 1.0, 0.375, 0.25) == 0.125
    assert Q(0.3, 1.0, 0.5, 0.25) == 0.25
    # both: cap to 2 * 1/16 = 1/8, then t = 1/16 forces 1/16
    assert Q(0.3, 1.0, 0.0625, 1.0 / 16) == 0.0625


def _circular(omega):
    # two equal masses M/2 at separation 1 with G = 1: relative angular velocity sqrt(M) = omega;
    # each moves on a circle of radius R = 1/2
    M = omega * omega
    pos = np.array([[-0.5, 0.0, 0.0], [0.5, 0.0, 0.0]])
    vel = np.array([[0.0, -0.5 * omega, 0.0], [0.0, 0.5 * omega, 0.0]])
    return pos, vel, np.array([M / 2, M / 2])


def test_block_steps_on_a_circular_orbit(oracle_mod):
    # |a| = w^2 R, |j| = w^3 R, |a2| = w^4 R, |a3| = w^5 R with w = 2, R = 1/2:
    # initial estimate eta_s |a| / |j| = eta_s / w; Aarseth's criterion sqrt(eta (2 w^6 R^2) / (2 w^8 R^2))
    # = sqrt(eta) / w
    pos, vel, m = _circular(2.0)
    a, j, _ = oracle_mod.gravity_jerk(pos, vel, m)
    np.testing.assert_allclose(np.linalg.norm(a, axis=1), [2.0, 2.0], rtol=1e-15)
    np.testing.assert_allclose(np.linalg.norm(j, axis=1), [4.0, 4.0], rtol=1e-15)
    # eta_s = 0.04: 0.02 -> 1/64
    t, dt = oracle_mod.hermite_block_init(a, j, 0.04, 1.0)
    assert np.all(dt == 1.0 / 64)
    # eta = 0.005: sqrt(0.005) / 2 = 0.0354 lies in [1/32, 1/16).  First step (t = 1/64): capped at
    # 2 * 1/64 = 1/32, which does not divide 1/64, so 1/64 again.  Second step (t = 1/32): 1/32.
    # (with a2 and a3 swapped the criterion gives sqrt(0.005 / 6) = 0.0289 < 1/32.)
    state = (pos, vel, a, j, t, dt)
    seen = []
    for _ in range(2):
        x, v, a1, j1, ts, dts, act, tn = oracle_mod.hermite_block(*state, m, 1, 0.005, 1.0)
        state = (x, v, a1, j1, ts, dts)
        seen.append((tn, dts[0], dts[1]))
    assert seen == [(1.0 / 64, 1.0 / 64, 1.0 / 64), (1.0 / 32, 1.0 / 32, 1.0 / 32)], seen


def test_energy_scale_hand_values(oracle_mod):
    # k = 4, D = 4, charges (1, 1, -1), epsilon = 0 at distances 2 and 4 from particle 0:
    # linear dielectric u = k q q / (D r^2): +1/4 and -1/16, so S_0 = 5/16 while U_0 = 3/16;
    # constant dielectric u = k q q / (D r): +1/2 and -1/4, S_0 = 3/4; the sigmoidal law with
    # zeta = exp(ln 4) = 4 is the constant one
    pos = np.array([[0.0, 0, 0], [2.0, 0, 0], [0.0, -4.0, 0]])
    q = np.array([1.0, 1.0, -1.0])
    sig = np.full(3, 2.0)
    eps = np.zeros(3)
    s1 = oracle_mod.ljc_energy_abs(1, pos, q, sig, eps, kc=4.0, D=4.0)
    s2 = oracle_mod.ljc_energy_abs(2, pos, q, sig, eps, kc=4.0, D=4.0)
    s3 = oracle_mod.ljc_energy_abs(3, pos, q, sig, eps, kc=4.0, zeta_coef=[0, 0, 0, math.log(4.0)])
    assert s1[0] == 0.3125 and s2[0] == 0.75 and abs(s3[0] - 0.75) <= 1e-15
    _, u1 = oracle_mod.ljc_linear(pos, q, sig, eps, kc=4.0, D=4.0)
    assert u1[0] == 0.1875
    # Lennard-Jones minimum r = 2^(1/6) sigma, no charges: u = -epsilon, S = epsilon
    r = 2.0 ** (1.0 / 6.0) * 3.0
    pos2 = np.array([[0.0, 0, 0], [r, 0, 0]])
    s = oracle_mod.ljc_energy_abs(1, pos2, np.zeros(2), np.full(2, 3.0), np.full(2, 0.2))
    np.testing.assert_allclose(s, [0.2, 0.2], rtol=1e-14)
    # an excluded partner drops out of the scale
    s1x = oracle_mod.ljc_energy_abs(1, pos, q, sig, eps, kc=4.0, D=4.0,
                                    excl_offsets=np.array([0, 1, 1, 1]), excl_index=np.array([2]))
    assert s1x[0] == 0.25
