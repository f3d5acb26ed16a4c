"""GPU parity of the LJC(constant) and LJC(sigmoidal) laws (Table 1) against the
FP64 CPU oracle, and of the launch-configuration space of the adjoint.

Tolerances as for the other laws: FP64 paths <= 1e-12 in the maximum
per-particle relative force error (energies relative to the largest |U_i|);
FP32 paths median <= 1e-5 and maximum <= 1e-3 against the oracle fed the
FP32-rounded positions.  The sigmoidal constants are not given by the paper;
ZC below makes zeta(r) rise from about 4 at contact to about 100 at 20 A, the
shape of a sigmoidal solvent screening, and the sigmoidal law with a constant
zeta = e^d must reproduce LJC(constant) with D = e^d.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_0706_3060_amd import workloads as W

pytestmark = pytest.mark.gpu

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


def rel_rows(x, ref):
    return np.linalg.norm(x - ref, axis=1) / np.linalg.norm(ref, axis=1)


def gpu_law(nb, kind, prec):
    if kind == "constant":
        return nb.ljc_constant(prec, dielectric=D_CONST)
    return nb.ljc_sigmoidal(ZC, prec)


def oracle_law(kind, pos, q, sigma, eps, ilist=None):
    if kind == "constant":
        return oracle.ljc_constant(pos, q, sigma, eps, D=D_CONST, ilist=ilist)
    return oracle.ljc_sigmoidal(pos, q, sigma, eps, ZC, ilist=ilist)


def check(prec, f, u, fr, ur):
    e = rel_rows(f, fr)
    eu = np.abs(u - ur) / np.abs(ur).max()
    if prec == "fp64":
        assert e.max() <= 1e-12, e.max()
        assert eu.max() <= 1e-12, eu.max()
    else:
        assert np.median(e) <= 1e-5 and e.max() <= 1e-3, (np.median(e), e.max())
        assert np.median(eu) <= 1e-5 and eu.max() <= 1e-3, (np.median(eu), eu.max())


@pytest.mark.parametrize("kind", ["constant", "sigmoidal"])
@pytest.mark.parametrize("prec", ["fp64", "fp32_kahan", "fp32_fp64acc"])
@pytest.mark.parametrize("n", [2000, 65, 2])
def test_forward_matches_oracle(nb, kind, prec, n):
    s = W.md_system(n, 21 + n, box=40.0 * (n / 2000.0) ** (1 / 3) + 5.0)
    f, u = nb.forces(dev(s.pos), dev(s.params()), gpu_law(nb, kind, prec))
    x = s.pos if prec == "fp64" else W.round_to_f32(s.pos)
    fr, ur = oracle_law(kind, x, s.q, s.sigma, s.epsilon)
    check(prec, host(f), host(u), fr, ur)


def test_sigmoidal_with_constant_zeta_is_constant_law(nb):
    s = W.md_system(1500, 31, box=36.0)
    d = float(np.log(7.5))
    fs, us = nb.forces(dev(s.pos), dev(s.params()), nb.ljc_sigmoidal((0.0, 0.0, 0.0, d), "fp64"))
    fc, uc = nb.forces(dev(s.pos), dev(s.params()), nb.ljc_constant("fp64", dielectric=7.5))
    assert rel_rows(host(fs), host(fc)).max() <= 1e-12
    assert (np.abs(host(us) - host(uc)) / np.abs(host(uc)).max()).max() <= 1e-12


@pytest.mark.parametrize("kind", ["constant", "sigmoidal"])
def test_subset_rows(nb, kind):
    s = W.md_system(3000, 41, box=45.0)
    il = np.random.default_rng(3).integers(0, 3000, 333)
    f, u = nb.forces_subset(dev(s.pos), dev(s.params()), torch.tensor(il, device="cuda"),
                            gpu_law(nb, kind, "fp64"))
    fr, ur = oracle_law(kind, s.pos, s.q, s.sigma, s.epsilon, ilist=il)
    check("fp64", host(f), host(u), fr, ur)


CONFIGS = [(64, 1, 64, 1, 0), (256, 2, 256, 3, 0), (128, 1, 1024, 9, 0), (256, 1, 256, 1, 1),
           (128, 2, 64, 5, 1), (64, 2, 512, 64, 1)]


@pytest.mark.parametrize("cfg", CONFIGS)
@pytest.mark.parametrize("kind", ["constant", "sigmoidal"])
def test_launch_configurations(nb, cfg, kind):
    block, ipl, jt, js, stage = cfg
    s = W.md_system(2500, 51, box=43.0)
    x32 = W.round_to_f32(s.pos)
    ref32 = oracle_law(kind, x32, s.q, s.sigma, s.epsilon)
    ref64 = oracle_law(kind, s.pos, s.q, s.sigma, s.epsilon)
    try:
        nb.set_config(nb.API_FORCES, block, ipl, jt, js, stage)
        out64 = nb.forces(dev(s.pos), dev(s.params()), gpu_law(nb, kind, "fp64"))
        out32 = nb.forces(dev(s.pos), dev(s.params()), gpu_law(nb, kind, "fp32_kahan"))
    finally:
        nb.clear_config(nb.API_FORCES)
    check("fp64", host(out64[0]), host(out64[1]), *ref64)
    check("fp32_kahan", host(out32[0]), host(out32[1]), *ref32)


SIZES = [0, 1, 2, 63, 64, 65, 300, 0, 777, 1500, 129, 5]


@pytest.fixture(scope="module")
def ensemble():
    return W.batched_md(len(SIZES), seed=7, sizes=SIZES, workers=1)


@pytest.mark.parametrize("kind", ["constant", "sigmoidal"])
@pytest.mark.parametrize("prec", ["fp64", "fp32_kahan"])
def test_batched_matches_per_system_oracle(nb, ensemble, kind, prec):
    off, pos, par, systems = ensemble
    f, u = nb.forces_batched(off, dev(pos), dev(par), gpu_law(nb, kind, prec))
    f, u = host(f), host(u)
    for s, sy in enumerate(systems):
        a, b = off[s], off[s + 1]
        if b - a == 0:
            continue
        if b - a == 1:
            assert np.all(f[a:b] == 0) and np.all(u[a:b] == 0)
            continue
        x = sy.pos if prec == "fp64" else W.round_to_f32(sy.pos)
        fr, ur = oracle_law(kind, x, sy.q, sy.sigma, sy.epsilon)
        check(prec, f[a:b], u[a:b], fr, ur)


def test_constant_law_leapfrog_step(nb):
    # one KDK step with per-atom masses, FP64, against the oracle's leapfrog
    s = W.md_system(1000, 61, box=32.0)
    mass = np.random.default_rng(5).uniform(12.0, 32.0, s.n)
    vel = np.random.default_rng(6).normal(0.0, 0.01, (s.n, 3))
    law = nb.ljc_constant("fp64", dielectric=D_CONST)
    f0, _ = oracle.ljc_constant(s.pos, s.q, s.sigma, s.epsilon, D=D_CONST)
    a0 = f0 / mass[:, None]
    x, v, a = dev(s.pos), dev(vel), dev(a0)
    u1 = nb.leapfrog(x, v, a, dev(s.params()), law, 2e-3, 2, inv_mass=dev(1.0 / mass), potential=True)
    xr, vr, ar, ur = oracle.leapfrog(oracle.LJC_CONSTANT, s.pos, vel, a0, s.params(), 2e-3, 2,
                                     inv_mass=1.0 / mass, D=D_CONST)
    assert np.abs(host(x) - xr).max() <= 1e-12 * np.abs(xr).max()
    assert np.abs(host(v) - vr).max() <= 1e-12 * np.abs(vr).max()
    assert rel_rows(host(a), ar).max() <= 1e-12
    assert (np.abs(host(u1) - ur) / np.abs(ur).max()).max() <= 1e-12


# ------------------------------------------------- adjoint configurations
ADJ_CONFIGS = [(256, 1, 256, 1, 0), (128, 2, 512, 3, 0), (256, 1, 256, 4, 1), (64, 2, 64, 7, 1),
               (256, 4, 256, 2, 1)]


@pytest.mark.parametrize("cfg", ADJ_CONFIGS)
def test_adjoint_launch_configurations(nb, cfg):
    block, ipl, jt, js, stage = cfg
    pos, _, m = W.plummer(2100, 71)
    g = W.unit_cotangent(2100, 72)
    s = W.md_system(1300, 73, box=35.0)
    gl = W.unit_cotangent(s.n, 74)
    ref_g = oracle.gravity_adjoint(pos, m, g, eps=0.01)
    ref_g32 = oracle.gravity_adjoint(W.round_to_f32(pos), m, g, eps=0.01)
    rp, rq, rs, re = oracle.ljc_adjoint(s.pos, s.q, s.sigma, s.epsilon, gl)
    rp32 = oracle.ljc_adjoint(W.round_to_f32(s.pos), s.q, s.sigma, s.epsilon, gl)[0]
    try:
        nb.set_config(nb.API_BACKWARD, block, ipl, jt, js, stage)
        g64, _, _ = nb.forces_backward(dev(pos), dev(m), dev(g), nb.gravity("fp64", softening=0.01))
        g32, _, _ = nb.forces_backward(dev(pos), dev(m), dev(g), nb.gravity("fp32_kahan", softening=0.01))
        l64, q64, _ = nb.forces_backward(dev(s.pos), dev(s.params()), dev(gl), nb.ljc_linear("fp64"))
        l32, _, _ = nb.forces_backward(dev(s.pos), dev(s.params()), dev(gl), nb.ljc_linear("fp32_fp64acc"))
    finally:
        nb.clear_config(nb.API_BACKWARD)
    assert rel_rows(host(g64), ref_g).max() <= 1e-11
    e = rel_rows(host(g32), ref_g32)
    assert np.median(e) <= 1e-5 and e.max() <= 1e-3, (np.median(e), e.max())
    e = rel_rows(host(l64), rp)
    assert np.median(e) <= 1e-12 and e.max() <= 1e-10, (np.median(e), e.max())
    q64 = host(q64)
    for got, ref in ((q64[:, 0], rq), (q64[:, 1], rs), (q64[:, 2], re)):
        assert (np.abs(got - ref) / np.abs(ref).max()).max() <= 1e-10
    e = rel_rows(host(l32), rp32)
    assert np.median(e) <= 1e-5 and e.max() <= 1e-3, (np.median(e), e.max())
