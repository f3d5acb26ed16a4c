"""GPU parity of the acceleration-and-jerk tiles over unordered pairs (Table 1's "Gravity (accel &
jerk)" with each pair evaluated once and its terms applied to both particles) against the FP64
oracle on the FP32-rounded state.

Ragged sizes around the chunk (64) and block (1024 records) edges, both tile-sum precisions, one
or two j parts, with and without the potential (the acceleration and jerk bitwise the same); the
rule's choice at N = 40,000, 70,000 and 300,000 (bitwise repeatable, equal to the one-sided kernel to the FP32 bar,
sampled rows against the oracle); shared Hermite steps through the tiles against the one-sided
kernel's and the oracle's FP64 trajectory; and row lists, which the tiles do not take, falling back
to the one-sided kernel.  Bars as for the other FP32 paths: per-particle relative error of the
acceleration, the jerk and the potential median <= 1e-5 and max <= 1e-3.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_0706_3060_amd import workloads as W

pytestmark = pytest.mark.gpu

SIZES = [2, 3, 63, 64, 65, 1000, 1023, 1024, 1025, 2047, 2049, 3001]
EPS, G = 0.01, 1.7
ONE_SIDED = (256, 1, 256, 24, 0)


@pytest.fixture(scope="module")
def nb():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_0706_3060_amd import nbody
    return nbody


def dev(a):
    return torch.tensor(np.asarray(a), dtype=torch.float64, device="cuda")


def host(t):
    return None if t is None else t.detach().cpu().numpy()


def rel_rows(x, ref):
    return np.linalg.norm(x - ref, axis=1) / np.linalg.norm(ref, axis=1)


def check(got, ref, rows=None):
    (a, j, p), (ar, jr, pr) = got, ref
    if rows is not None:
        a, j, p = a[rows], j[rows], None if p is None else p[rows]
    errs = [rel_rows(a, ar), rel_rows(j, jr)]
    if p is not None:
        errs.append(np.abs(p - pr) / np.abs(pr))
    for e in errs:
        assert np.median(e) <= 1e-5 and e.max() <= 1e-3, (np.median(e), e.max())


def oracle32(x, v, m, rows=None, eps=EPS, g=G):
    return oracle.gravity_jerk(W.round_to_f32(x), W.round_to_f32(v), W.round_to_f32(m), G=g, eps=eps,
                               ilist=rows)


def run(nb, cfg, *args, **kw):
    try:
        nb.set_config(nb.API_JERK, *cfg)
        return nb.forces_jerk(*args, **kw)
    finally:
        nb.clear_config(nb.API_JERK)


@pytest.mark.parametrize("split", [1, 2])
@pytest.mark.parametrize("prec", ["fp32_kahan", "fp32_fp64acc"])
def test_jerk_tiles_ragged_sizes(nb, prec, split):
    law = nb.gravity(prec, softening=EPS, G=G)
    for k, n in enumerate(SIZES):
        x, v, m = W.plummer(n, 400 + k)
        X, V, M = dev(x), dev(v), dev(m)
        try:
            nb.set_config(nb.API_JERK, 256, 4, 2048, split, 2)
            c = nb.get_config(nb.API_JERK, n, law)
            assert (c["j_stage"], c["block"], c["i_per_lane"], c["j_tile"], c["j_split"]) == \
                (2, 512, 2, 1024, split), c
            a, j, p = nb.forces_jerk(X, V, M, law)
            a2, j2, p2 = nb.forces_jerk(X, V, M, law, potential=False)
        finally:
            nb.clear_config(nb.API_JERK)
        check((host(a), host(j), host(p)), oracle32(x, v, m))
        assert p2 is None and torch.equal(a, a2) and torch.equal(j, j2), n


@pytest.mark.parametrize("n,parts", [(40000, 2), (70000, 2), (300000, 1)])
def test_jerk_tiles_are_the_rule_and_repeat_bitwise(nb, n, parts):
    x, v, m = W.plummer(n, 77)
    law = nb.gravity("fp32_kahan", softening=EPS, G=G)
    c = nb.get_config(nb.API_JERK, n, law)
    assert (c["j_stage"], c["block"], c["j_tile"], c["j_split"]) == (2, 512, 1024, parts), c
    X, V, M = dev(x), dev(v), dev(m)
    r1 = nb.forces_jerk(X, V, M, law)
    r2 = nb.forces_jerk(X, V, M, law)
    assert all(torch.equal(s, t) for s, t in zip(r1, r2))
    r3 = run(nb, ONE_SIDED, X, V, M, law)
    check(tuple(host(t) for t in r1), tuple(host(t) for t in r3))
    rows = np.sort(np.random.default_rng(7).choice(n, 256, replace=False))
    check(tuple(host(t) for t in r1), oracle32(x, v, m, rows), rows)


def test_hermite_shared_steps_through_the_tiles(nb):
    n, dt, steps, eps = 3001, 1.0 / 1024, 4, 0.05
    x, v, m = W.plummer(n, 78)
    a0, j0, _ = oracle.gravity_jerk(x, v, m, eps=eps)
    law = nb.gravity("fp32_kahan", softening=eps)
    out = {}
    for name, cfg in (("tiles", (512, 2, 1024, 2, 2)), ("one", ONE_SIDED)):
        X, V, A, J = dev(x), dev(v), dev(a0), dev(j0)
        try:
            nb.set_config(nb.API_JERK, *cfg)
            assert (nb.get_config(nb.API_JERK, n, law)["j_stage"] == 2) == (name == "tiles")
            nb.hermite(X, V, A, J, dev(m), law, dt, steps)
        finally:
            nb.clear_config(nb.API_JERK)
        out[name] = tuple(host(t) for t in (X, V, A, J))
    xr, vr, ar, jr = oracle.hermite(x, v, a0, j0, m, dt, steps, eps=eps)
    amax, jmax = np.abs(a0).max(), np.abs(j0).max()
    # each step's FP32 acceleration and jerk (bar 1e-3 relative per particle) enter the
    # corrector with weights h / 2 (velocity) and h^2 / 12 (position, jerk term of the velocity)
    for X, V, A, J in out.values():
        assert np.abs(X - xr).max() <= steps * dt * dt * 1e-3 * amax + 1e-12 * np.abs(xr).max()
        assert np.abs(V - vr).max() <= steps * dt * 1e-3 * (amax + dt * jmax)
    # the new accelerations and jerks against the oracle's (their evaluation states differ by the
    # trajectories' differences above, far below the bar)
    check((out["tiles"][2], out["tiles"][3], None), (ar, jr, None))
    check((out["tiles"][2], out["tiles"][3], None), (out["one"][2], out["one"][3], None))


def test_row_lists_fall_back_to_one_sided(nb):
    n = 3001
    x, v, m = W.plummer(n, 79)
    rows = np.random.default_rng(3).integers(0, n, 500)
    law = nb.gravity("fp32_kahan", softening=EPS, G=G)
    a, j, p = run(nb, (512, 2, 1024, 2, 2), dev(x), dev(v), dev(m), law,
                  ilist=torch.tensor(rows, device="cuda"))
    check((host(a), host(j), host(p)), oracle32(x, v, m, rows))
