"""GPU parity of the symmetric pair tiles for the LJC laws of Table 1 (linear, constant and
sigmoidal dielectric), each unordered pair evaluated once and applied to both atoms, against the
FP64 oracle on the FP32-rounded positions.

Ragged sizes around the chunk (64) and block (1024, 2048 records) edges, both workgroup shapes,
both tile-sum precisions, energies on and off; the rule's choice at N = 70,000 (bitwise
repeatable, and equal to the one-sided kernel to the FP32 bar); a leapfrog step through the
tiles (the linear and constant dielectrics, whose oracle integrates them); shares of the tile
triangle adding up to the whole; and exclusion lists, which the tiles do not take, falling back
to the one-sided kernel.  Bars as for the other FP32 paths: per-atom relative force error
median <= 1e-5 and max <= 1e-3; energies relative to the largest |U_i|.  The sigmoidal
coefficients are those of the per-law tests: zeta(r) rises from about 4 at contact to about 100
at 20 A.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_0706_3060_amd import workloads as W

pytestmark = pytest.mark.gpu

SIZES = [2, 3, 63, 64, 65, 1000, 1023, 1025, 2047, 2049, 3001]
KINDS = ["linear", "constant", "sigmoidal"]
ZC = (2e-4, -6e-3, 0.25, 0.4)
D_CONST = 4.0


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


def gpu_law(nb, kind, prec):
    if kind == "linear":
        return nb.ljc_linear(prec)
    if kind == "constant":
        return nb.ljc_constant(prec, dielectric=D_CONST)
    return nb.ljc_sigmoidal(ZC, prec)


def oracle_law(kind, pos, s, ilist=None):
    if kind == "linear":
        return oracle.ljc_linear(pos, s.q, s.sigma, s.epsilon, ilist=ilist)
    if kind == "constant":
        return oracle.ljc_constant(pos, s.q, s.sigma, s.epsilon, D=D_CONST, ilist=ilist)
    return oracle.ljc_sigmoidal(pos, s.q, s.sigma, s.epsilon, ZC, ilist=ilist)


@pytest.fixture(scope="module")
def big():
    return system(70000, 71)


def system(n, seed):
    # the MD box at the density of the throughput workload (1/32 atoms per cubic Angstrom)
    return W.md_system(n, seed, box=(32.0 * n) ** (1.0 / 3.0) + 3.0)


def check(f, u, fr, ur, potential=True):
    e = np.linalg.norm(f - fr, axis=1) / np.linalg.norm(fr, axis=1)
    assert np.median(e) <= 1e-5 and e.max() <= 1e-3, (np.median(e), e.max())
    if potential:
        eu = np.abs(u - ur) / np.abs(ur).max()
        assert np.median(eu) <= 1e-5 and eu.max() <= 1e-3, (np.median(eu), eu.max())


@pytest.mark.parametrize("shape", [(512, 2), (256, 4)])
@pytest.mark.parametrize("j_tile", [1024, 2048])
@pytest.mark.parametrize("prec", ["fp32_kahan", "fp32_fp64acc"])
@pytest.mark.parametrize("kind", KINDS)
def test_ljc_symmetric_ragged_sizes(nb, kind, shape, j_tile, prec):
    law = gpu_law(nb, kind, prec)
    for k, n in enumerate(SIZES):
        s = system(n, 300 + k)
        fr, ur = oracle_law(kind, W.round_to_f32(s.pos), s)
        nb.set_config(nb.API_FORCES, shape[0], shape[1], j_tile, 1, 2)
        try:
            c = nb.get_config(nb.API_FORCES, n, law)
            assert (c["j_stage"], c["block"], c["i_per_lane"]) == (2,) + shape, c
            for potential in (True, False):
                f, u = nb.forces(dev(s.pos), dev(s.params()), law, potential=potential)
                check(host(f), None if u is None else host(u), fr, ur, potential)
                assert potential or u is None
        finally:
            nb.clear_config(nb.API_FORCES)


@pytest.mark.parametrize("kind", KINDS)
def test_ljc_symmetric_j_parts(nb, kind):
    # each tile's j chunks in 4 parts, one workgroup each
    law = gpu_law(nb, kind, "fp32_kahan")
    for k, n in enumerate([65, 2049, 3001]):
        s = system(n, 330 + k)
        fr, ur = oracle_law(kind, W.round_to_f32(s.pos), s)
        nb.set_config(nb.API_FORCES, 256, 4, 1024, 4, 2)
        try:
            assert nb.get_config(nb.API_FORCES, n, law)["j_split"] == 4
            f, u = nb.forces(dev(s.pos), dev(s.params()), law)
        finally:
            nb.clear_config(nb.API_FORCES)
        check(host(f), host(u), fr, ur)


@pytest.mark.parametrize("kind", KINDS)
def test_ljc_symmetric_is_the_rule_and_repeats_bitwise(nb, big, kind):
    s, n = big, 70000
    law = gpu_law(nb, kind, "fp32_kahan")
    c = nb.get_config(nb.API_FORCES, n, law)
    assert (c["j_stage"], c["j_tile"], c["block"], c["i_per_lane"]) == (2, 1024, 512, 2), c
    X, P = dev(s.pos), dev(s.params())
    f1, u1 = nb.forces(X, P, law)
    f2, u2 = nb.forces(X, P, law)
    assert torch.equal(f1, f2) and torch.equal(u1, u2)
    nb.set_config(nb.API_FORCES, 256, 1, 256, 32, 1)                # the one-sided kernel
    try:
        f3, u3 = nb.forces(X, P, law)
    finally:
        nb.clear_config(nb.API_FORCES)
    check(host(f1), host(u1), host(f3), host(u3))
    rows = np.sort(np.random.default_rng(7).choice(n, 256, replace=False))
    fr, ur = oracle_law(kind, W.round_to_f32(s.pos), s, ilist=rows)
    e = np.linalg.norm(host(f1)[rows] - fr, axis=1) / np.linalg.norm(fr, axis=1)
    assert np.median(e) <= 1e-5 and e.max() <= 1e-3, (np.median(e), e.max())
    # energies relative to the largest |U_i| of the whole system (the one-sided kernel's)
    eu = np.abs(host(u1)[rows] - ur) / np.abs(host(u3)).max()
    assert np.median(eu) <= 1e-5 and eu.max() <= 1e-3, (np.median(eu), eu.max())


def test_ljc_symmetric_rule_below_65536(nb):
    # from 32,768 atoms the rule takes the tiles (the 8-wave shape with the energies, in two j
    # parts, the most it takes), against the one-sided kernel and sampled oracle rows
    n = 40000
    s = system(n, 72)
    law = gpu_law(nb, "linear", "fp32_kahan")
    c = nb.get_config(nb.API_FORCES, n, law)
    assert (c["j_stage"], c["j_tile"], c["block"], c["i_per_lane"], c["j_split"]) == (2, 1024, 512, 2, 2), c
    X, P = dev(s.pos), dev(s.params())
    f1, u1 = nb.forces(X, P, law)
    nb.set_config(nb.API_FORCES, 256, 1, 256, 32, 1)                # the one-sided kernel
    try:
        f3, u3 = nb.forces(X, P, law)
    finally:
        nb.clear_config(nb.API_FORCES)
    check(host(f1), host(u1), host(f3), host(u3))
    rows = np.sort(np.random.default_rng(8).choice(n, 256, replace=False))
    fr, ur = oracle_law("linear", W.round_to_f32(s.pos), s, ilist=rows)
    e = np.linalg.norm(host(f1)[rows] - fr, axis=1) / np.linalg.norm(fr, axis=1)
    assert np.median(e) <= 1e-5 and e.max() <= 1e-3, (np.median(e), e.max())


@pytest.mark.parametrize("shape", [(512, 2), (256, 4)])
@pytest.mark.parametrize("kind", ["linear", "constant"])
def test_ljc_symmetric_leapfrog_step(nb, kind, shape):
    n, dt = 2049, 2e-3
    s = system(n, 81)
    rng = np.random.default_rng(82)
    v = rng.standard_normal((n, 3)) * 0.01
    im = 1.0 / rng.uniform(1.0, 16.0, n)                              # atom masses 1 .. 16
    par = np.stack([s.q, s.sigma, s.epsilon], axis=1)
    f0, _ = oracle_law(kind, s.pos, s)
    a0 = f0 * im[:, None]
    law = gpu_law(nb, kind, "fp32_kahan")
    X, V, A = dev(s.pos), dev(v), dev(a0)
    nb.set_config(nb.API_LEAPFROG, shape[0], shape[1], 1024, 1, 2)
    try:
        u = nb.leapfrog(X, V, A, dev(s.params()), law, dt, 2, inv_mass=dev(im), potential=True)
    finally:
        nb.clear_config(nb.API_LEAPFROG)
    # accelerations at the final positions against the oracle there (FP32 bar)
    fr, ur = oracle_law(kind, W.round_to_f32(host(X)), s)
    check(host(A) / im[:, None], host(u), fr, ur)
    # the trajectory against the oracle's FP64 leapfrog
    code = oracle.LJC_LINEAR if kind == "linear" else oracle.LJC_CONSTANT
    xr, vr, _, _ = oracle.leapfrog(code, s.pos, v, a0, par, dt, 2, inv_mass=im, D=D_CONST)
    amax = np.abs(a0).max()
    assert np.abs(host(X) - xr).max() <= 4 * dt * dt * 1e-3 * amax + 1e-12 * np.abs(xr).max()
    assert np.abs(host(V) - vr).max() <= 4 * dt * 1e-3 * amax


@pytest.mark.parametrize("kind", KINDS)
def test_ljc_shares_add_up_to_the_forces(nb, kind):
    n = 3001
    s = system(n, 91)
    law = gpu_law(nb, kind, "fp32_fp64acc")
    X, P = dev(s.pos), dev(s.params())
    nb.set_config(nb.API_FORCES, 256, 4, 1024, 1, 2)
    try:
        f_full, u_full = nb.forces(X, P, law)
        f1, u1 = nb.forces_share(X, P, law, 0, 1)
        assert torch.equal(f1, f_full) and torch.equal(u1, u_full)
        fs, us = torch.zeros_like(f_full), torch.zeros_like(u_full)
        for sh in range(3):
            f, u = nb.forces_share(X, P, law, sh, 3)
            fs += f
            us += u
    finally:
        nb.clear_config(nb.API_FORCES)
    # shares add up to the whole up to the rounding of the FP64 additions (the forces of
    # neighbouring atoms cancel to far below the largest term, hence the bar on the largest)
    assert (fs - f_full).abs().max().item() <= 1e-12 * f_full.abs().max().item()
    assert (us - u_full).abs().max().item() <= 1e-12 * u_full.abs().max().item()
    fr, ur = oracle_law(kind, W.round_to_f32(s.pos), s)
    check(host(fs), host(us), fr, ur)


def test_ljc_exclusions_fall_back_to_one_sided(nb):
    # the tiles take no exclusion lists: a forced symmetric configuration runs one-sided
    s, off, idx = W.bonded_chains(40, 50, 61)
    law = nb.ljc_linear("fp32_kahan")
    fr, ur = oracle.ljc_excl(oracle.LJC_LINEAR, W.round_to_f32(s.pos), s.q, s.sigma, s.epsilon, off, idx)
    nb.set_config(nb.API_FORCES, 256, 4, 1024, 1, 2)
    try:
        ex = nb.Exclusions(torch.tensor(off, dtype=torch.int64, device="cuda"),
                           torch.tensor(idx, dtype=torch.int64, device="cuda"))
        f, u = nb.forces(dev(s.pos), dev(s.params()), law, exclusions=ex)
    finally:
        nb.clear_config(nb.API_FORCES)
    check(host(f), host(u), fr, ur)
