"""GPU parity of the batched adjoint over unordered pairs (batched backward with j_stage 2: one
wave per tile of two 256-record blocks of a system, each unordered pair's adjoint terms applied
to both particles) against the FP64 oracle's analytic derivatives, system by system.

System sizes are ragged around the chunk (64) and block (256) edges and reach the largest system
the tiles take (8192), with empty and one-particle systems between them, so that off-diagonal,
diagonal and padded tiles all occur.  Gravity (the Hessian-vector product, G != 1, unequal
masses) and LJC(linear) (positions, charges, sigma and epsilon, and the per-type sums), both FP32
tile-sum precisions.  The result repeats bit for bit and agrees with the one-sided persistent
adjoint; a system above 8192 particles and exclusion lists fall back to the one-sided launch.
Bars as for the other FP32 adjoints: per-particle relative position-gradient error median
<= 1e-5 and max <= 1e-3; parameter gradients relative to their largest magnitude.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_0706_3060_amd import workloads as W

pytestmark = pytest.mark.gpu

SIZES = [300, 0, 1, 2, 63, 64, 65, 255, 256, 257, 700, 1, 1024, 1500, 2049, 4000]
BSYM = (256, 4, 256, 1, 2)
ONE_SIDED = (256, 1, 256, 8, 1)
EPS, G = 0.01, 1.7


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


def row_errors(f, ref):
    nref = np.linalg.norm(ref, axis=1)
    floor = 1e-3 * nref.max() if nref.size else 0.0
    return np.linalg.norm(f - ref, axis=1) / np.maximum(nref, max(floor, 1e-300))


def ensemble(law, sizes, seed):
    if law == "gravity":
        xs, ms = [], []
        for k, n in enumerate(sizes):
            if n == 0:
                xs.append(np.zeros((0, 3)))
                ms.append(np.zeros(0))
                continue
            x, _, m = W.plummer(n, seed + k) if n > 1 else (np.zeros((1, 3)), None, np.ones(1))
            xs.append(x)
            ms.append(m * np.random.default_rng(seed + k).uniform(0.5, 1.5, n))
        off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
        return off, np.concatenate(xs), np.concatenate(ms), None
    off, pos, par, systems = W.batched_md(len(sizes), seed=seed, sizes=sizes, workers=1)
    types = np.concatenate([sy.types for sy in systems]).astype(np.int32)
    return off, pos, par, types


def gpu_law(nb, law, prec):
    return nb.gravity(prec, softening=EPS, G=G) if law == "gravity" else nb.ljc_linear(prec)


def backward(nb, off, x, par, g, lw, cfg, types=None):
    try:
        nb.set_config(nb.API_BACKWARD_BATCHED, *cfg)
        ty = torch.tensor(types, device="cuda") if types is not None else None
        return nb.forces_backward_batched(off, dev(x), dev(par), dev(g), lw, types=ty,
                                          n_types=4 if types is not None else 0)
    finally:
        nb.clear_config(nb.API_BACKWARD_BATCHED)


def check_system(law, x, par, g, gp, gq):
    n = x.shape[0]
    if n == 0:
        return
    if n == 1:
        assert np.all(gp == 0) and (gq is None or np.all(gq == 0))
        return
    xr, pr, gr = W.round_to_f32(x), W.round_to_f32(par), W.round_to_f32(g)
    if law == "gravity":
        rp = oracle.gravity_adjoint(xr, pr, gr, G=G, eps=EPS)
    else:
        rp, rq, rs, re = oracle.ljc_adjoint(xr, pr[:, 0], pr[:, 1], pr[:, 2], gr)
    e = row_errors(gp, rp)
    assert np.median(e) <= 1e-5 and e.max() <= 1e-3, (n, np.median(e), e.max())
    if law != "gravity":
        for got, ref in ((gq[:, 0], rq), (gq[:, 1], rs), (gq[:, 2], re)):
            err = np.abs(got - ref) / np.abs(ref).max()
            assert np.median(err) <= 1e-5 and err.max() <= 1e-3, (n, np.median(err), err.max())


@pytest.mark.parametrize("law", ["gravity", "ljc_linear"])
@pytest.mark.parametrize("prec", ["fp32_kahan", "fp32_fp64acc"])
def test_batched_symmetric_adjoint_against_the_oracle(nb, law, prec):
    off, x, par, types = ensemble(law, SIZES, 950)
    g = W.unit_cotangent(x.shape[0], 951)
    lw = gpu_law(nb, law, prec)
    gp, gq, gt = backward(nb, off, x, par, g, lw, BSYM, types)
    gp, gq, gt = host(gp), host(gq), host(gt)
    for s in range(len(SIZES)):
        a, b = int(off[s]), int(off[s + 1])
        check_system(law, x[a:b], par[a:b], g[a:b], gp[a:b], gq[a:b] if gq is not None else None)
    if types is not None:
        # per-type sums of dL/dsigma and dL/depsilon over all systems
        for t in range(4):
            sel = types == t
            for col, k in ((1, 0), (2, 1)):
                np.testing.assert_allclose(gt[t, k], gq[sel, col].sum(), rtol=1e-12,
                                           atol=1e-12 * np.abs(gq[:, col]).sum())


@pytest.mark.parametrize("law", ["gravity", "ljc_linear"])
def test_batched_symmetric_adjoint_repeats_and_matches_one_sided(nb, law):
    off, x, par, _ = ensemble(law, [8192, 3000, 517, 5000], 960)
    g = W.unit_cotangent(x.shape[0], 961)
    lw = gpu_law(nb, law, "fp32_kahan")
    p1, q1, _ = backward(nb, off, x, par, g, lw, BSYM)
    p2, q2, _ = backward(nb, off, x, par, g, lw, BSYM)
    assert torch.equal(p1, p2) and (q1 is None or torch.equal(q1, q2))
    p3, q3, _ = backward(nb, off, x, par, g, lw, ONE_SIDED)
    e = row_errors(host(p1), host(p3))
    assert np.median(e) <= 1e-5 and e.max() <= 1e-3
    if q1 is not None:
        err = (q1 - q3).abs().max(dim=0).values / q3.abs().max(dim=0).values
        assert err.max().item() <= 1e-3
    # the oracle on sampled rows of the 8192 system
    rows = np.sort(np.random.default_rng(5).choice(8192, 128, replace=False))
    xr, pr, gr = W.round_to_f32(x[:8192]), W.round_to_f32(par[:8192]), W.round_to_f32(g[:8192])
    if law == "gravity":
        rp = oracle.gravity_adjoint(xr, pr, gr, G=G, eps=EPS, ilist=rows)
    else:
        rp = oracle.ljc_adjoint(xr, pr[:, 0], pr[:, 1], pr[:, 2], gr, ilist=rows)[0]
    e = row_errors(host(p1)[rows], rp)
    assert np.median(e) <= 1e-5 and e.max() <= 1e-3


def test_batched_symmetric_adjoint_falls_back(nb):
    # a system above 8192 particles: the whole launch runs one-sided; so does one with exclusions
    off, x, par, _ = ensemble("ljc_linear", [9000, 300], 970)
    g = W.unit_cotangent(x.shape[0], 971)
    lw = gpu_law(nb, "ljc_linear", "fp32_kahan")
    gp, gq, _ = backward(nb, off, x, par, g, lw, BSYM)
    check_system("ljc_linear", x[9000:], par[9000:], g[9000:], host(gp)[9000:], host(gq)[9000:])
    sy, eoff, eidx = W.bonded_chains(16, 32, 5)
    n = sy.pos.shape[0]
    offs = np.arange(0, n + 1, 64, dtype=np.int64)
    ge = W.unit_cotangent(n, 972)
    ex = nb.Exclusions(torch.tensor(eoff, dtype=torch.int64, device="cuda"),
                       torch.tensor(eidx, dtype=torch.int64, device="cuda"))
    out = {}
    for name, cfg in (("sym", BSYM), ("one", ONE_SIDED)):
        try:
            nb.set_config(nb.API_BACKWARD_BATCHED, *cfg)
            out[name] = nb.forces_backward_batched(offs, dev(sy.pos), dev(sy.params()), dev(ge), lw,
                                                   exclusions=ex)
        finally:
            nb.clear_config(nb.API_BACKWARD_BATCHED)
    assert torch.equal(out["sym"][0], out["one"][0]) and torch.equal(out["sym"][1], out["one"][1])
