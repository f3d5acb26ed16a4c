"""GPU parity of exclusion lists (Section 5: the LJC kernels read an exclusion
list per particle) and of the batched adjoint, against the FP64 oracle.

Workload: synthetic bonded chains (1-2 and 1-3 pairs excluded), the stand-in
for a bonded molecule.  Tolerances as elsewhere: FP64 <= 1e-12 per row
(adjoint position rows 1e-10), FP32 median <= 1e-5 and max <= 1e-3 against the
oracle fed FP32-rounded positions.  Empty lists reproduce the plain kernels
bitwise under the same launch configuration.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_0706_3060_amd import workloads as W

pytestmark = pytest.mark.gpu

ZC = (2e-4, -6e-3, 0.25, 0.4)
KINDS = {"linear": 1, "constant": 2, "sigmoidal": 3}


@pytest.fixture(scope="module")
def nb():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_0706_3060_amd import nbody
    return nbody


def dev(a, dtype=torch.float64):
    return torch.tensor(np.asarray(a), dtype=dtype, device="cuda")


def host(t):
    return t.detach().cpu().numpy()


def rel_rows(x, ref):
    return np.linalg.norm(x - ref, axis=1) / np.linalg.norm(ref, axis=1)


def gpu_law(nb, kind, prec):
    if kind == "linear":
        return nb.ljc_linear(prec)
    if kind == "constant":
        return nb.ljc_constant(prec)
    return nb.ljc_sigmoidal(ZC, prec)


def check(prec, f, u, fr, ur, tol64=1e-12):
    e = rel_rows(f, fr)
    eu = np.abs(u - ur) / np.abs(ur).max()
    if prec == "fp64":
        assert e.max() <= tol64 and eu.max() <= tol64, (e.max(), eu.max())
    else:
        assert np.median(e) <= 1e-5 and e.max() <= 1e-3, (np.median(e), e.max())
        assert np.median(eu) <= 1e-5 and eu.max() <= 1e-3, (np.median(eu), eu.max())


@pytest.fixture(scope="module")
def chains():
    return W.bonded_chains(80, 24, 21)          # 1920 atoms (ragged: 30 x 64)


@pytest.mark.parametrize("kind", ["linear", "constant", "sigmoidal"])
@pytest.mark.parametrize("prec", ["fp64", "fp32_kahan", "fp32_fp64acc"])
def test_forces_with_exclusions_match_oracle(nb, chains, kind, prec):
    sy, eo, ei = chains
    excl = nb.Exclusions(dev(eo, torch.int64), dev(ei, torch.int64))
    f, u = nb.forces(dev(sy.pos), dev(sy.params()), gpu_law(nb, kind, prec), exclusions=excl)
    x = sy.pos if prec == "fp64" else W.round_to_f32(sy.pos)
    fr, ur = oracle.ljc_excl(KINDS[kind], x, sy.q, sy.sigma, sy.epsilon, eo, ei, zeta_coef=ZC)
    check(prec, host(f), host(u), fr, ur)


CONFIGS = [(64, 1, 64, 1), (256, 2, 256, 3), (128, 1, 1024, 7), (256, 1, 256, 30)]


@pytest.mark.parametrize("cfg", CONFIGS)
def test_exclusion_configurations(nb, chains, cfg):
    sy, eo, ei = chains
    block, ipl, jt, js = cfg
    excl = nb.Exclusions(dev(eo, torch.int64), dev(ei, torch.int64))
    fr, ur = oracle.ljc_excl(1, sy.pos, sy.q, sy.sigma, sy.epsilon, eo, ei)
    try:
        nb.set_config(nb.API_FORCES, block, ipl, jt, js, 1)
        f, u = nb.forces(dev(sy.pos), dev(sy.params()), nb.ljc_linear("fp64"), exclusions=excl)
        # empty lists: the plain kernel, bitwise, under the same configuration
        empty = nb.Exclusions(dev(np.zeros(sy.n + 1), torch.int64), None)
        f0, u0 = nb.forces(dev(sy.pos), dev(sy.params()), nb.ljc_linear("fp32_kahan"), exclusions=empty)
        f1, u1 = nb.forces(dev(sy.pos), dev(sy.params()), nb.ljc_linear("fp32_kahan"))
    finally:
        nb.clear_config(nb.API_FORCES)
    check("fp64", host(f), host(u), fr, ur)
    assert torch.equal(f0, f1) and torch.equal(u0, u1)


def _bonded_ensemble(counts, seed):
    systems, eos, eis = [], [], []
    base = 0
    offs = [0]
    for k, nc in enumerate(counts):
        if nc == 0:
            systems.append(None)
            offs.append(base)
            continue
        sy, eo, ei = W.bonded_chains(nc, 9, seed + k)
        systems.append((sy, eo, ei))
        base += sy.n
        offs.append(base)
    n = base
    pos = np.concatenate([s[0].pos for s in systems if s]) if n else np.zeros((0, 3))
    par = np.concatenate([s[0].params() for s in systems if s]) if n else np.zeros((0, 3))
    types = np.concatenate([s[0].types for s in systems if s]) if n else np.zeros(0, np.int32)
    # global CSR over the concatenated rows
    lists = []
    for s, o in zip(systems, offs[:-1]):
        if s is None:
            continue
        _, eo, ei = s
        for i in range(s[0].n):
            lists.append(ei[eo[i]:eo[i + 1]] + o)
    geo = np.zeros(n + 1, dtype=np.int64)
    geo[1:] = np.cumsum([len(l) for l in lists])
    gei = np.concatenate(lists).astype(np.int64) if lists else np.zeros(0, np.int64)
    return np.array(offs, dtype=np.int64), pos, par, types, geo, gei, systems


@pytest.mark.parametrize("prec", ["fp64", "fp32_kahan"])
def test_batched_with_exclusions(nb, prec):
    off, pos, par, _, geo, gei, systems = _bonded_ensemble([3, 0, 20, 7, 1, 45, 12], 31)
    excl = nb.Exclusions(dev(geo, torch.int64), dev(gei, torch.int64))
    f, u = nb.forces_batched(off, dev(pos), dev(par), nb.ljc_linear(prec), exclusions=excl)
    f, u = host(f), host(u)
    for s, sysd in enumerate(systems):
        if sysd is None:
            continue
        sy, eo, ei = sysd
        a, b = off[s], off[s + 1]
        x = sy.pos if prec == "fp64" else W.round_to_f32(sy.pos)
        fr, ur = oracle.ljc_excl(1, x, sy.q, sy.sigma, sy.epsilon, eo, ei)
        check(prec, f[a:b], u[a:b], fr, ur)


@pytest.mark.parametrize("prec", ["fp64", "fp32_fp64acc", "fp32_kahan"])
def test_adjoint_with_exclusions(nb, chains, prec):
    sy, eo, ei = chains
    g = W.unit_cotangent(sy.n, 61)
    excl = nb.Exclusions(dev(eo, torch.int64), dev(ei, torch.int64))
    gp, gq, gt = nb.forces_backward(dev(sy.pos), dev(sy.params()), dev(g), nb.ljc_linear(prec),
                                    types=dev(sy.types, torch.int32), n_types=4, exclusions=excl)
    x = sy.pos if prec == "fp64" else W.round_to_f32(sy.pos)
    rp, rq, rs, re = oracle.ljc_adjoint_excl(x, sy.q, sy.sigma, sy.epsilon, g, eo, ei)
    tol_med, tol_max = (1e-12, 1e-10) if prec == "fp64" else (1e-5, 1e-3)
    e = rel_rows(host(gp), rp)
    assert np.median(e) <= tol_med and e.max() <= tol_max, (np.median(e), e.max())
    gq = host(gq)
    for got, ref in ((gq[:, 0], rq), (gq[:, 1], rs), (gq[:, 2], re)):
        err = np.abs(got - ref) / np.abs(ref).max()
        assert np.median(err) <= tol_med and err.max() <= tol_max, (np.median(err), err.max())
    gt = host(gt)
    for t in range(4):
        sel = sy.types == t
        np.testing.assert_allclose(gt[t], [gq[sel, 1].sum(), gq[sel, 2].sum()], rtol=1e-12,
                                   atol=1e-12 * np.abs(gq).sum())


@pytest.mark.parametrize("prec", ["fp64", "fp32_kahan"])
def test_batched_adjoint(nb, prec):
    # LJC(linear), plain and with exclusions, and gravity: one persistent launch
    off, pos, par, types, geo, gei, systems = _bonded_ensemble([4, 0, 17, 1, 30, 9], 41)
    n = pos.shape[0]
    g = W.unit_cotangent(n, 62)
    law = nb.ljc_linear(prec)
    tol_med, tol_max = (1e-12, 1e-10) if prec == "fp64" else (1e-5, 1e-3)
    excl = nb.Exclusions(dev(geo, torch.int64), dev(gei, torch.int64))
    for ex in (None, excl):
        gp, gq, gt = nb.forces_backward_batched(off, dev(pos), dev(par), dev(g), law,
                                                types=dev(types, torch.int32), n_types=4,
                                                exclusions=ex)
        gp, gq, gt = host(gp), host(gq), host(gt)
        for s, sysd in enumerate(systems):
            if sysd is None:
                continue
            sy, eo, ei = sysd
            a, b = off[s], off[s + 1]
            x = sy.pos if prec == "fp64" else W.round_to_f32(sy.pos)
            if ex is None:
                rp, rq, rs, re = oracle.ljc_adjoint(x, sy.q, sy.sigma, sy.epsilon, g[a:b])
            else:
                rp, rq, rs, re = oracle.ljc_adjoint_excl(x, sy.q, sy.sigma, sy.epsilon, g[a:b], eo, ei)
            if b - a == 1:
                continue
            e = rel_rows(gp[a:b], rp)
            assert np.median(e) <= tol_med and e.max() <= tol_max, (s, np.median(e), e.max())
            for got, ref in ((gq[a:b, 0], rq), (gq[a:b, 1], rs), (gq[a:b, 2], re)):
                err = np.abs(got - ref) / np.abs(ref).max()
                assert np.median(err) <= tol_med and err.max() <= tol_max
        for t in range(4):
            sel = types == t
            np.testing.assert_allclose(gt[t], [gq[sel, 1].sum(), gq[sel, 2].sum()], rtol=1e-12,
                                       atol=1e-12 * np.abs(gq).sum())
    # gravity: the Hessian-vector product of every system in one launch
    sizes = [100, 0, 513, 64, 1, 900]
    offg = np.concatenate([[0], np.cumsum(sizes)])
    pg = np.concatenate([W.plummer(k, 200 + i)[0] if k else np.zeros((0, 3)) for i, k in enumerate(sizes)])
    mg = np.random.default_rng(5).uniform(0.5, 1.5, pg.shape[0]) / pg.shape[0]
    gg = W.unit_cotangent(pg.shape[0], 63)
    gpg, _, _ = nb.forces_backward_batched(offg, dev(pg), dev(mg), dev(gg), nb.gravity(prec, softening=0.01))
    gpg = host(gpg)
    for s in range(len(sizes)):
        a, b = offg[s], offg[s + 1]
        if b - a < 2:
            continue
        x = pg[a:b] if prec == "fp64" else W.round_to_f32(pg[a:b])
        ref = oracle.gravity_adjoint(x, mg[a:b], gg[a:b], eps=0.01)
        e = rel_rows(gpg[a:b], ref)
        assert np.median(e) <= tol_med and e.max() <= (1e-11 if prec == "fp64" else 1e-3), (s, e.max())


def test_autograd_with_exclusions_and_batched(nb):
    # gradcheck (FP64) of the exclusion-aware and the batched autograd Functions
    sy, eo, ei = W.bonded_chains(2, 4, 71, box=9.0)
    law = nb.ljc_linear("fp64")
    excl = nb.Exclusions(dev(eo, torch.int64), dev(ei, torch.int64))
    pos = dev(sy.pos).requires_grad_(True)
    par = dev(sy.params()).requires_grad_(True)
    assert torch.autograd.gradcheck(lambda x, p: nb.NBodyForcesFn.apply(x, p, law, excl), (pos, par),
                                    eps=1e-6, atol=1e-6, rtol=1e-6)
    off, pos2, par2, _, geo, gei, _ = _bonded_ensemble([1, 0, 2], 81)
    ex2 = nb.Exclusions(dev(geo, torch.int64), dev(gei, torch.int64))
    x2 = dev(pos2).requires_grad_(True)
    p2 = dev(par2).requires_grad_(True)
    assert torch.autograd.gradcheck(lambda x, p: nb.NBodyBatchedForcesFn.apply(x, p, off, law, ex2),
                                    (x2, p2), eps=1e-6, atol=1e-6, rtol=1e-6)
    # typed force matching through the exclusion-aware Function equals the oracle's gradient
    t = W.perturbed(sy, 5)
    ft, _ = nb.forces(dev(sy.pos), dev(t.params()), law, exclusions=excl)
    x3 = dev(sy.pos).requires_grad_(True)
    q = dev(sy.q).requires_grad_(True)
    st = dev(sy.sigma_t).requires_grad_(True)
    et = dev(sy.eps_t).requires_grad_(True)
    F = nb.LJCTypedForcesFn.apply(x3, q, st, et, dev(sy.types, torch.int32), law, excl)
    ((F - ft) ** 2).sum().backward()
    g = 2.0 * (host(F) - host(ft))
    rp, rq, rs, re = oracle.ljc_adjoint_excl(sy.pos, sy.q, sy.sigma, sy.epsilon, g, eo, ei)
    np.testing.assert_allclose(host(x3.grad), rp, rtol=1e-9, atol=1e-11 * np.abs(rp).max())
    np.testing.assert_allclose(host(q.grad), rq, rtol=1e-9, atol=1e-11 * np.abs(rq).max())
    for k in range(4):
        sel = sy.types == k
        if sel.any():
            np.testing.assert_allclose(host(st.grad)[k], rs[sel].sum(), rtol=1e-9, atol=1e-12)
            np.testing.assert_allclose(host(et.grad)[k], re[sel].sum(), rtol=1e-9, atol=1e-12)
