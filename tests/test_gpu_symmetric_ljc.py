"""GPU parity of the symmetric pair tiles for LJC with the linear dielectric (Table 1), each
unordered pair evaluated once and applied to both atoms, against the FP64 oracle on the
FP32-rounded positions.

Ragged sizes around the chunk (64) and block (1024, 2048 records) edges, both workgroup shapes,
both tile-sum precisions, energies on and off; the rule's choice at N = 70,000 (bitwise
repeatable, and equal to the one-sided kernel to the FP32 bar); a leapfrog step through the
tiles; shares of the tile triangle adding up to the whole; and exclusion lists, which the tiles
do not take, falling back to the one-sided kernel.  Bars as for the other FP32 paths: per-atom
relative force error median <= 1e-5 and max <= 1e-3; energies relative to the largest |U_i|.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_0706_3060_amd import workloads as W

pytestmark = pytest.mark.gpu

SIZES = [2, 3, 63, 64, 65, 1000, 1023, 1025, 2047, 2049, 3001]


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
def test_ljc_symmetric_ragged_sizes(nb, shape, j_tile, prec):
    law = nb.ljc_linear(prec)
    for k, n in enumerate(SIZES):
        s = system(n, 300 + k)
        fr, ur = oracle.ljc_linear(W.round_to_f32(s.pos), s.q, s.sigma, s.epsilon)
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


def test_ljc_symmetric_is_the_rule_and_repeats_bitwise(nb):
    n = 70000
    s = system(n, 71)
    law = nb.ljc_linear("fp32_kahan")
    c = nb.get_config(nb.API_FORCES, n, law)
    assert (c["j_stage"], c["j_tile"], c["block"], c["i_per_lane"]) == (2, 1024, 256, 4), c
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
    fr, ur = oracle.ljc_linear(W.round_to_f32(s.pos), s.q, s.sigma, s.epsilon, ilist=rows)
    e = np.linalg.norm(host(f1)[rows] - fr, axis=1) / np.linalg.norm(fr, axis=1)
    assert np.median(e) <= 1e-5 and e.max() <= 1e-3, (np.median(e), e.max())
    # energies relative to the largest |U_i| of the whole system (the one-sided kernel's)
    eu = np.abs(host(u1)[rows] - ur) / np.abs(host(u3)).max()
    assert np.median(eu) <= 1e-5 and eu.max() <= 1e-3, (np.median(eu), eu.max())


@pytest.mark.parametrize("shape", [(512, 2), (256, 4)])
def test_ljc_symmetric_leapfrog_step(nb, shape):
    n, dt = 2049, 2e-3
    s = system(n, 81)
    rng = np.random.default_rng(82)
    v = rng.standard_normal((n, 3)) * 0.01
    im = 1.0 / rng.uniform(1.0, 16.0, n)                              # atom masses 1 .. 16
    par = np.stack([s.q, s.sigma, s.epsilon], axis=1)
    f0, _ = oracle.ljc_linear(s.pos, s.q, s.sigma, s.epsilon)
    a0 = f0 * im[:, None]
    law = nb.ljc_linear("fp32_kahan")
    X, V, A = dev(s.pos), dev(v), dev(a0)
    nb.set_config(nb.API_LEAPFROG, shape[0], shape[1], 1024, 1, 2)
    try:
        u = nb.leapfrog(X, V, A, dev(s.params()), law, dt, 2, inv_mass=dev(im), potential=True)
    finally:
        nb.clear_config(nb.API_LEAPFROG)
    # accelerations at the final positions against the oracle there (FP32 bar)
    fr, ur = oracle.ljc_linear(W.round_to_f32(host(X)), s.q, s.sigma, s.epsilon)
    check(host(A) / im[:, None], host(u), fr, ur)
    # the trajectory against the oracle's FP64 leapfrog
    xr, vr, _, _ = oracle.leapfrog(oracle.LJC_LINEAR, s.pos, v, a0, par, dt, 2, inv_mass=im)
    amax = np.abs(a0).max()
    assert np.abs(host(X) - xr).max() <= 4 * dt * dt * 1e-3 * amax + 1e-12 * np.abs(xr).max()
    assert np.abs(host(V) - vr).max() <= 4 * dt * 1e-3 * amax


def test_ljc_shares_add_up_to_the_forces(nb):
    n = 3001
    s = system(n, 91)
    law = nb.ljc_linear("fp32_fp64acc")
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
    fr, ur = oracle.ljc_linear(W.round_to_f32(s.pos), s.q, s.sigma, s.epsilon)
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
