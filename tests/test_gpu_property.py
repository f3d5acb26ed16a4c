"""Property-based GPU parity: random small systems and ensembles, laws, precisions and
forced launch configurations against the FP64 oracle.

Each example draws a size (0 to 700 particles, so ragged tails of every kind), a law, a
precision and a launch configuration (block, rows per lane, j tile, j split, j staging;
the library clamps each to what the kernels support for that law and size), runs the
forward through the C ABI, and compares with the oracle on the same inputs:
FP64 paths to 1e-12 per row, FP32 paths median <= 1e-5 and maximum <= 1e-3 (against
the oracle fed the FP32-rounded inputs).  Row errors are taken relative to
max(|F_i|, 1e-3 max_j |F_j|), so that a row whose force nearly cancels is held to the
scale of the system rather than to its own tiny norm; potentials are held normwise, row by
row, to S_i = sum_j |u_ij| (see check_potential), at every size.  The batched test draws ensembles of
up to 24 systems of 0 to 400 particles (empty and one-particle systems included) for the
persistent launch and compares each system with its own oracle call; the adjoint and the
acceleration-and-jerk, exclusion-list and integrator tests, and the batched adjoint over random
ensembles, do the same for those paths.
Examples are drawn
from a fixed seed (derandomize), so every run checks the same cases.
"""
import numpy as np
import pytest
import torch
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

import oracle
from paper_0706_3060_amd import workloads as W

pytestmark = pytest.mark.gpu

ZC = (2e-4, -6e-3, 0.25, 0.4)
EPS = 0.01


@pytest.fixture(scope="module")
def nb():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_0706_3060_amd import nbody
    return nbody


def dev(a):
    return torch.tensor(np.asarray(a), dtype=torch.float64, device="cuda")


def host(t):
    return t.detach().cpu().numpy()


def row_errors(f, ref):
    nref = np.linalg.norm(ref, axis=1)
    floor = 1e-3 * nref.max() if nref.size else 0.0
    return np.linalg.norm(f - ref, axis=1) / np.maximum(nref, max(floor, 1e-300))


# Potentials are held normwise, row by row: |U_i - U_i^ref| / S_i with S_i = sum_j |u_ij| (the
# oracle's plain loop over the same pair energies).  A rounding error of the sum is a small
# multiple of the unit roundoff times S_i, whatever the cancellation: an LJC potential can be
# the near-cancelling sum of a Coulomb attraction and a Lennard-Jones repulsion (e.g. -2.898 +
# 2.915 kcal/mol in a three-particle system), whose FP32 error relative to the small total is a
# property of FP32 arithmetic.  Gravity's pair energies all have one sign, so S_i = |phi_i|.
KINDS = {"ljc_linear": 1, "ljc_constant": 2, "ljc_sigmoidal": 3}


def potential_scale(law, x, par, prec, eoff=None, eidx=None):
    """S_i for the oracle inputs of `reference` (None for gravity: |phi_i| itself)."""
    if law == "gravity":
        return None
    if prec != "fp64":
        x, par = W.round_to_f32(x), W.round_to_f32(par)
    return oracle.ljc_energy_abs(KINDS[law], x, par[:, 0], par[:, 1], par[:, 2], zeta_coef=ZC,
                                 excl_offsets=eoff, excl_index=eidx)


def check_potential(got, ref, prec, scale, what):
    s = np.abs(ref) if scale is None else scale
    tiny = 1e-300 if s.size == 0 else max(1e-300, 1e-30 * s.max())
    e = np.abs(got - ref) / np.maximum(s, tiny)
    if e.size == 0:
        return
    if prec == "fp64":
        assert e.max() <= 1e-12, (e.max(), what)
    else:
        assert np.median(e) <= 1e-5 and e.max() <= 1e-3, (np.median(e), e.max(), what)


def inputs(law, n, seed):
    if law == "gravity":
        x, _, m = W.plummer(n, seed)
        return x, m
    s = W.md_system(n, seed, box=(32.0 * n) ** (1.0 / 3.0))
    return s.pos, s.params()


def reference(law, x, par, prec):
    if prec != "fp64":
        x, par = W.round_to_f32(x), W.round_to_f32(par)
    if law == "gravity":
        return oracle.gravity(x, par, eps=EPS)
    q, sg, ep = par[:, 0], par[:, 1], par[:, 2]
    if law == "ljc_linear":
        return oracle.ljc_linear(x, q, sg, ep)
    if law == "ljc_constant":
        return oracle.ljc_constant(x, q, sg, ep)
    return oracle.ljc_sigmoidal(x, q, sg, ep, ZC)


def gpu_law(nb, law, prec):
    if law == "gravity":
        return nb.gravity(prec, softening=EPS)
    if law == "ljc_linear":
        return nb.ljc_linear(prec)
    if law == "ljc_constant":
        return nb.ljc_constant(prec)
    return nb.ljc_sigmoidal(ZC, prec)


@settings(max_examples=300, deadline=None, derandomize=True, database=None,
          suppress_health_check=[HealthCheck.too_slow, HealthCheck.function_scoped_fixture])
@given(n=st.integers(min_value=0, max_value=700),
       law=st.sampled_from(["gravity", "ljc_linear", "ljc_constant", "ljc_sigmoidal"]),
       prec=st.sampled_from(["fp64", "fp32_kahan", "fp32_fp64acc"]),
       block=st.sampled_from([64, 128, 192, 256]),
       ipl=st.sampled_from([1, 2, 4, 8]),
       j_tile=st.sampled_from([64, 128, 256, 512]),
       j_split=st.integers(min_value=1, max_value=64),
       j_stage=st.sampled_from([0, 1, 2]),
       potential=st.booleans(),
       seed=st.integers(min_value=0, max_value=10 ** 6))
def test_random_systems_and_configurations(nb, n, law, prec, block, ipl, j_tile, j_split, j_stage,
                                           potential, seed):
    lw = gpu_law(nb, law, prec)
    if n == 0:
        x, par = np.zeros((0, 3)), (np.zeros(0) if law == "gravity" else np.zeros((0, 3)))
    else:
        x, par = inputs(law, n, seed)
    try:
        nb.set_config(nb.API_FORCES, block, ipl, j_tile, j_split, j_stage)
        f, p = nb.forces(dev(x), dev(par), lw, potential=potential)
    finally:
        nb.clear_config(nb.API_FORCES)
    assert tuple(f.shape) == (n, 3)
    assert (p is not None) == potential
    if n == 0:
        return
    fr, pr = reference(law, x, par, prec)
    e = row_errors(host(f), fr)
    if prec == "fp64":
        assert e.max() <= 1e-12, (e.max(), n, law, prec)
    else:
        assert np.median(e) <= 1e-5 and e.max() <= 1e-3, (np.median(e), e.max(), n, law, prec)
    if potential:
        check_potential(host(p), pr, prec, potential_scale(law, x, par, prec), (n, law, prec))


def ensemble(law, sizes, seed):
    """Concatenated independent systems of the given sizes (empty ones included)."""
    xs, ps = [], []
    for k, n in enumerate(sizes):
        if n == 0:
            xs.append(np.zeros((0, 3)))
            ps.append(np.zeros(0) if law == "gravity" else np.zeros((0, 3)))
        else:
            x, par = inputs(law, n, seed + k)
            xs.append(x)
            ps.append(np.asarray(par))
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    if not sizes:
        return off, np.zeros((0, 3)), (np.zeros(0) if law == "gravity" else np.zeros((0, 3)))
    return off, np.concatenate(xs), np.concatenate(ps)


@settings(max_examples=80, deadline=None, derandomize=True, database=None,
          suppress_health_check=[HealthCheck.too_slow, HealthCheck.function_scoped_fixture])
@given(sizes=st.lists(st.integers(min_value=0, max_value=400), min_size=0, max_size=24),
       law=st.sampled_from(["gravity", "ljc_linear", "ljc_constant", "ljc_sigmoidal"]),
       prec=st.sampled_from(["fp64", "fp32_kahan", "fp32_fp64acc"]),
       block=st.sampled_from([64, 128, 256]),
       ipl=st.sampled_from([1, 2, 4]),
       j_tile=st.sampled_from([64, 256]),
       j_stage=st.sampled_from([0, 1, 2]),
       per_wave=st.sampled_from([1, 8, 64]),
       seed=st.integers(min_value=0, max_value=10 ** 6))
def test_random_batches(nb, sizes, law, prec, block, ipl, j_tile, j_stage, per_wave, seed):
    """The persistent batched launch over random ensembles (empty and one-particle systems
    included) with a forced configuration equals the oracle system by system.  The work-unit
    target per wave (the batched j_split) decides how far large systems are cut into parts;
    j_stage 2 selects the symmetric tiles (every law with FP32 pair arithmetic; with FP64 it
    reads as 1)."""
    lw = gpu_law(nb, law, prec)
    off, x, par = ensemble(law, sizes, seed)
    try:
        nb.set_config(nb.API_BATCHED, block, ipl, j_tile, per_wave, j_stage)
        f, p = nb.forces_batched(off, dev(x), dev(par), lw)
    finally:
        nb.clear_config(nb.API_BATCHED)
    assert tuple(f.shape) == (int(off[-1]), 3)
    f, p = host(f), host(p)
    for s in range(len(sizes)):
        a, b = int(off[s]), int(off[s + 1])
        if b - a == 0:
            continue
        if b - a == 1:
            assert np.all(f[a:b] == 0) and np.all(p[a:b] == 0)
            continue
        fr, pr = reference(law, x[a:b], par[a:b], prec)
        e = row_errors(f[a:b], fr)
        if prec == "fp64":
            assert e.max() <= 1e-12, (s, e.max(), law, prec)
        else:
            assert np.median(e) <= 1e-5 and e.max() <= 1e-3, (s, np.median(e), e.max(), law, prec)
        check_potential(p[a:b], pr, prec, potential_scale(law, x[a:b], par[a:b], prec), (s, law, prec))


def rel_to_max(got, ref):
    return np.abs(got - ref) / max(np.abs(ref).max(), 1e-300)


@settings(max_examples=60, deadline=None, derandomize=True, database=None,
          suppress_health_check=[HealthCheck.too_slow, HealthCheck.function_scoped_fixture])
@given(sizes=st.lists(st.integers(min_value=0, max_value=400), min_size=0, max_size=16),
       law=st.sampled_from(["gravity", "ljc_linear"]),
       prec=st.sampled_from(["fp64", "fp32_kahan", "fp32_fp64acc"]),
       ipl=st.sampled_from([1, 2]),
       j_stage=st.sampled_from([0, 1, 2]),
       per_wave=st.sampled_from([1, 8]),
       seed=st.integers(min_value=0, max_value=10 ** 6))
def test_random_batched_adjoints(nb, sizes, law, prec, ipl, j_stage, per_wave, seed):
    """The batched adjoint over random ensembles (empty and one-particle systems included)
    under a forced configuration equals the oracle's analytic adjoint system by system (as the
    single-system adjoints).  j_stage 2 selects the adjoint's symmetric tiles for FP32 pair
    arithmetic (with FP64 it reads as 1)."""
    lw = gpu_law(nb, law, prec)
    off, x, par = ensemble(law, sizes, seed)
    n = int(off[-1])
    g = W.unit_cotangent(n, seed + 3) if n else np.zeros((0, 3))
    try:
        nb.set_config(nb.API_BACKWARD_BATCHED, 256, ipl, 256, per_wave, j_stage)
        gp, gq, _ = nb.forces_backward_batched(off, dev(x), dev(par), dev(g), lw)
    finally:
        nb.clear_config(nb.API_BACKWARD_BATCHED)
    gp = host(gp)
    gq = host(gq) if gq is not None else None
    for s in range(len(sizes)):
        a, b = int(off[s]), int(off[s + 1])
        if b - a < 2:
            assert np.all(gp[a:b] == 0) and (gq is None or np.all(gq[a:b] == 0))
            continue
        xs, ps = x[a:b], par[a:b]
        xr = xs if prec == "fp64" else W.round_to_f32(xs)
        if law == "gravity":
            refs = [(gp[a:b], oracle.gravity_adjoint(xr, ps, g[a:b], eps=EPS), True)]
        else:
            rp, rq, rs, re = oracle.ljc_adjoint(xr, ps[:, 0], ps[:, 1], ps[:, 2], g[a:b])
            refs = [(gp[a:b], rp, True), (gq[a:b, 0], rq, False), (gq[a:b, 1], rs, False),
                    (gq[a:b, 2], re, False)]
        for got, ref, rows in refs:
            e = row_errors(got, ref) if rows else rel_to_max(got, ref)
            if prec == "fp64":
                assert e.max() <= 1e-10, (s, e.max(), law, prec)
            else:
                assert np.median(e) <= 1e-5 and e.max() <= 1e-3, (s, np.median(e), e.max(), law, prec)


@settings(max_examples=80, deadline=None, derandomize=True, database=None,
          suppress_health_check=[HealthCheck.too_slow, HealthCheck.function_scoped_fixture])
@given(n=st.integers(min_value=2, max_value=400),
       law=st.sampled_from(["gravity", "ljc_linear"]),
       prec=st.sampled_from(["fp64", "fp32_kahan", "fp32_fp64acc"]),
       block=st.sampled_from([64, 128, 256]),
       ipl=st.sampled_from([1, 2]),
       j_tile=st.sampled_from([64, 256]),
       j_split=st.integers(min_value=1, max_value=16),
       j_stage=st.sampled_from([0, 1, 2]),
       seed=st.integers(min_value=0, max_value=10 ** 6))
def test_random_adjoints(nb, n, law, prec, block, ipl, j_tile, j_split, j_stage, seed):
    """The adjoint (gravity: dL/dpos; LJC(linear): dL/dpos and dL/d(q, sigma, eps)) on random
    systems under a forced configuration against the oracle's analytic adjoint (FP64:
    1e-10 of the scale, the cancelling sums of the adjoint; FP32 as the forward).  j_stage 2
    selects the symmetric tiles for the FP32 adjoints (gravity's position adjoint over the block
    grid, LJC(linear)'s over 256-record blocks; with FP64 it reads as 1)."""
    lw = gpu_law(nb, law, prec)
    x, par = inputs(law, n, seed)
    g = W.unit_cotangent(n, seed + 1)
    try:
        nb.set_config(nb.API_BACKWARD, block, ipl, j_tile, j_split, j_stage)
        gp, gq, _ = nb.forces_backward(dev(x), dev(par), dev(g), lw)
    finally:
        nb.clear_config(nb.API_BACKWARD)
    xr = x if prec == "fp64" else W.round_to_f32(x)
    if law == "gravity":
        assert gq is None
        refs = [(host(gp), oracle.gravity_adjoint(xr, par, g, eps=EPS), True)]
    else:
        rp, rq, rs, re = oracle.ljc_adjoint(xr, par[:, 0], par[:, 1], par[:, 2], g)
        gq = host(gq)
        refs = [(host(gp), rp, True), (gq[:, 0], rq, False), (gq[:, 1], rs, False), (gq[:, 2], re, False)]
    for got, ref, rows in refs:
        e = row_errors(got, ref) if rows else rel_to_max(got, ref)
        if prec == "fp64":
            assert e.max() <= 1e-10, (e.max(), n, law, prec)
        else:
            assert np.median(e) <= 1e-5 and e.max() <= 1e-3, (np.median(e), e.max(), n, law, prec)


@settings(max_examples=80, deadline=None, derandomize=True, database=None,
          suppress_health_check=[HealthCheck.too_slow, HealthCheck.function_scoped_fixture])
@given(n=st.integers(min_value=1, max_value=500),
       prec=st.sampled_from(["fp64", "fp32_kahan", "fp32_fp64acc"]),
       block=st.sampled_from([64, 128, 256]),
       ipl=st.sampled_from([1, 2]),
       j_tile=st.sampled_from([64, 256]),
       j_split=st.integers(min_value=1, max_value=32),
       j_stage=st.sampled_from([0, 1, 2]),
       potential=st.booleans(),
       subset=st.booleans(),
       seed=st.integers(min_value=0, max_value=10 ** 6))
def test_random_jerk(nb, n, prec, block, ipl, j_tile, j_split, j_stage, potential, subset, seed):
    """Acceleration, jerk and potential (Table 1 "Gravity (accel & jerk)") on random Plummer
    spheres, for all rows or a random row subset, under a forced configuration (the symmetric
    tiles for whole systems with FP32 pair arithmetic, one-sided otherwise), against the oracle."""
    x, v, m = W.plummer(n, seed)
    rows = None
    if subset:
        rng = np.random.default_rng(seed + 2)
        rows = np.sort(rng.choice(n, max(1, n // 3), replace=False)).astype(np.int64)
    lw = nb.gravity(prec, softening=EPS)
    try:
        nb.set_config(nb.API_JERK, block, ipl, j_tile, j_split, j_stage)
        a, j, p = nb.forces_jerk(dev(x), dev(v), dev(m), lw,
                                 ilist=None if rows is None else torch.tensor(rows, device="cuda"),
                                 potential=potential)
    finally:
        nb.clear_config(nb.API_JERK)
    assert (p is not None) == potential
    if prec == "fp64":
        ra, rj, rp = oracle.gravity_jerk(x, v, m, eps=EPS, ilist=rows)
    else:
        ra, rj, rp = oracle.gravity_jerk(W.round_to_f32(x), W.round_to_f32(v), W.round_to_f32(m),
                                         eps=EPS, ilist=rows)
    checks = [row_errors(host(a), ra), row_errors(host(j), rj)]
    if potential:
        check_potential(host(p), rp, prec, None, (n, prec))
    for e in checks:
        if prec == "fp64":
            assert e.max() <= 1e-12, (e.max(), n, prec)
        else:
            assert np.median(e) <= 1e-5 and e.max() <= 1e-3, (np.median(e), e.max(), n, prec)



@settings(max_examples=80, deadline=None, derandomize=True, database=None,
          suppress_health_check=[HealthCheck.too_slow, HealthCheck.function_scoped_fixture])
@given(n=st.integers(min_value=2, max_value=300),
       law=st.sampled_from(["ljc_linear", "ljc_constant", "ljc_sigmoidal"]),
       prec=st.sampled_from(["fp64", "fp32_kahan", "fp32_fp64acc"]),
       max_partners=st.integers(min_value=0, max_value=12),
       block=st.sampled_from([64, 128, 256]),
       ipl=st.sampled_from([1, 2, 4]),
       j_tile=st.sampled_from([64, 256]),
       j_split=st.integers(min_value=1, max_value=16),
       seed=st.integers(min_value=0, max_value=10 ** 6))
def test_random_exclusions(nb, n, law, prec, max_partners, block, ipl, j_tile, j_split, seed):
    """LJC forces with random per-particle exclusion lists (uneven lengths, empty lists,
    repeated entries and the particle itself included) under a forced configuration,
    against the oracle with the same lists."""
    x, par = inputs(law, n, seed)
    rng = np.random.default_rng(seed + 3)
    lists = []
    for i in range(n):
        k = int(rng.integers(0, max_partners + 1))
        lst = list(rng.integers(0, n, k))
        if k and rng.random() < 0.2:
            lst.append(i)                      # the particle itself
        if k and rng.random() < 0.2:
            lst.append(lst[0])                 # a repeated entry
        lists.append(lst)
    eoff = np.concatenate([[0], np.cumsum([len(l) for l in lists])]).astype(np.int64)
    eidx = np.array([j for l in lists for j in l], dtype=np.int64)
    excl = nb.Exclusions(torch.tensor(eoff, device="cuda"),
                         torch.tensor(eidx, device="cuda") if eidx.size else None)
    try:
        nb.set_config(nb.API_FORCES, block, ipl, j_tile, j_split, 1)
        f, p = nb.forces(dev(x), dev(par), gpu_law(nb, law, prec), exclusions=excl)
    finally:
        nb.clear_config(nb.API_FORCES)
    xr = x if prec == "fp64" else W.round_to_f32(x)
    fr, pr = oracle.ljc_excl(KINDS[law], xr, par[:, 0], par[:, 1], par[:, 2], eoff, eidx,
                             zeta_coef=ZC)
    e = row_errors(host(f), fr)
    if prec == "fp64":
        assert e.max() <= 1e-12, (e.max(), n, law, prec)
    else:
        assert np.median(e) <= 1e-5 and e.max() <= 1e-3, (np.median(e), e.max(), n, law, prec)
    sc = oracle.ljc_energy_abs(KINDS[law], xr, par[:, 0], par[:, 1], par[:, 2], zeta_coef=ZC,
                               excl_offsets=eoff, excl_index=eidx)
    check_potential(host(p), pr, prec, sc, (n, law, prec))


@settings(max_examples=60, deadline=None, derandomize=True, database=None,
          suppress_health_check=[HealthCheck.too_slow, HealthCheck.function_scoped_fixture])
@given(n=st.integers(min_value=2, max_value=300),
       law=st.sampled_from(["gravity", "ljc_linear", "ljc_constant"]),
       nsteps=st.integers(min_value=1, max_value=4),
       with_inv_mass=st.booleans(),
       j_split=st.integers(min_value=1, max_value=16),
       j_stage=st.sampled_from([0, 1]),
       seed=st.integers(min_value=0, max_value=10 ** 6))
def test_random_leapfrog(nb, n, law, nsteps, with_inv_mass, j_split, j_stage, seed):
    """FP64 kick-drift-kick steps (the update of the simulation cycle) on random systems
    under a forced configuration against the oracle's: positions and velocities to 1e-12
    of their scale, accelerations and potentials as the forward."""
    x, par = inputs(law, n, seed)
    rng = np.random.default_rng(seed + 4)
    if law == "gravity":
        v, dt, inv = rng.normal(0.0, 0.3, (n, 3)), 1e-3, None
    else:
        v, dt = rng.normal(0.0, 0.01, (n, 3)), 2e-4
        inv = rng.uniform(1.0 / 16.0, 1.0 / 12.0, n) if with_inv_mass else None
    lw = gpu_law(nb, law, "fp64")
    okind = {"gravity": oracle.GRAVITY, "ljc_linear": oracle.LJC_LINEAR,
             "ljc_constant": oracle.LJC_CONSTANT}[law]
    a0, _ = reference(law, x, par, "fp64")
    if inv is not None:
        a0 = a0 * inv[:, None]
    X, V, A = dev(x), dev(v), dev(a0)
    try:
        nb.set_config(nb.API_LEAPFROG, 256, 1, 256, j_split, j_stage)
        pot = nb.leapfrog(X, V, A, dev(par), lw, dt, nsteps,
                          inv_mass=None if inv is None else dev(inv), potential=True)
    finally:
        nb.clear_config(nb.API_LEAPFROG)
    xr, vr, ar, pr = oracle.leapfrog(okind, x, v, a0, par, dt, nsteps, inv_mass=inv, eps=EPS)
    assert np.abs(host(X) - xr).max() <= 1e-12 * np.abs(xr).max()
    assert np.abs(host(V) - vr).max() <= 1e-12 * max(np.abs(vr).max(), 1e-300)
    assert row_errors(host(A), ar).max() <= 1e-12
    check_potential(host(pot), pr, "fp64", potential_scale(law, xr, par, "fp64"), (n, law))


@settings(max_examples=40, deadline=None, derandomize=True, database=None,
          suppress_health_check=[HealthCheck.too_slow, HealthCheck.function_scoped_fixture])
@given(n=st.integers(min_value=2, max_value=300),
       nsteps=st.integers(min_value=1, max_value=4),
       j_split=st.integers(min_value=1, max_value=16),
       seed=st.integers(min_value=0, max_value=10 ** 6))
def test_random_hermite(nb, n, nsteps, j_split, seed):
    """FP64 shared-step Hermite steps on random Plummer spheres under a forced split against
    the oracle's."""
    x, v, m = W.plummer(n, seed)
    lw = nb.gravity("fp64", softening=EPS)
    a0, j0, _ = oracle.gravity_jerk(x, v, m, eps=EPS)
    X, V, A, J = dev(x), dev(v), dev(a0), dev(j0)
    try:
        nb.set_config(nb.API_HERMITE, 256, 1, 1024, j_split, 0)
        nb.hermite(X, V, A, J, dev(m), lw, 1.0 / 1024, nsteps)
    finally:
        nb.clear_config(nb.API_HERMITE)
    xr, vr, ar, jr = oracle.hermite(x, v, a0, j0, m, 1.0 / 1024, nsteps, eps=EPS)
    assert np.abs(host(X) - xr).max() <= 1e-12 * np.abs(xr).max()
    assert np.abs(host(V) - vr).max() <= 1e-12 * np.abs(vr).max()
    assert row_errors(host(A), ar).max() <= 1e-11
    assert row_errors(host(J), jr).max() <= 1e-10
