"""GPU parity of the batched symmetric tiles (batched j_stage 2: each unordered pair of a
system evaluated once, one wave per tile of two 256-record blocks) against the FP64 oracle.

System sizes are ragged around the chunk (64) and block (256) edges and reach the largest
system the tiles take (8192, 32 blocks), with empty and one-particle systems between them,
so that every kind of tile occurs: off-diagonal, diagonal with one-sided self chunks, and
padding.  Gravity and the three LJC laws, both FP32 tile-sum precisions, potential on and off; the
result repeats bit for bit and agrees with the one-sided persistent launch; an ensemble with
a system above 8192 falls back to the one-sided launch; exclusion lists fall back too.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_0706_3060_amd import workloads as W

pytestmark = pytest.mark.gpu

EPS = 0.01
ZC = (2e-4, -6e-3, 0.25, 0.4)           # the sigmoidal dielectric of the per-law tests
KIND = {"ljc_linear": 1, "ljc_constant": 2, "ljc_sigmoidal": 3}
SIZES = [300, 0, 1, 2, 63, 64, 65, 255, 256, 257, 700, 1, 1024, 1500, 2048, 2049, 4000]
BSYM = (256, 4, 256, 1, 2)


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
        return off, np.concatenate(xs), np.concatenate(ms)
    off, pos, par, _ = W.batched_md(len(sizes), seed=seed, sizes=sizes, workers=1)
    return off, pos, par


def gpu_law(nb, law, prec):
    if law == "gravity":
        return nb.gravity(prec, softening=EPS)
    if law == "ljc_linear":
        return nb.ljc_linear(prec)
    if law == "ljc_constant":
        return nb.ljc_constant(prec, dielectric=4.0)
    return nb.ljc_sigmoidal(ZC, prec)


def check_system(law, x, par, f, p, potential):
    n = x.shape[0]
    if n == 0:
        return
    if n == 1:
        assert np.all(f == 0) and (p is None or np.all(p == 0))
        return
    xr, pr = W.round_to_f32(x), W.round_to_f32(par)
    if law == "gravity":
        fr, ur = oracle.gravity(xr, pr, eps=EPS)
        scale = np.abs(ur)
    else:
        q, sg, ep = pr[:, 0], pr[:, 1], pr[:, 2]
        if law == "ljc_linear":
            fr, ur = oracle.ljc_linear(xr, q, sg, ep)
        elif law == "ljc_constant":
            fr, ur = oracle.ljc_constant(xr, q, sg, ep, D=4.0)
        else:
            fr, ur = oracle.ljc_sigmoidal(xr, q, sg, ep, ZC)
        scale = oracle.ljc_energy_abs(KIND[law], xr, q, sg, ep, D=4.0,
                                      zeta_coef=ZC if law == "ljc_sigmoidal" else None)
    e = row_errors(f, fr)
    assert np.median(e) <= 1e-5 and e.max() <= 1e-3, (n, np.median(e), e.max())
    if potential:
        ep = np.abs(p - ur) / np.maximum(scale, 1e-300)
        assert np.median(ep) <= 1e-5 and ep.max() <= 1e-3, (n, np.median(ep), ep.max())
    else:
        assert p is None


def run(nb, off, x, par, lw, potential, cfg):
    try:
        nb.set_config(nb.API_BATCHED, *cfg)
        return nb.forces_batched(off, dev(x), dev(par), lw, potential=potential)
    finally:
        nb.clear_config(nb.API_BATCHED)


@pytest.mark.parametrize("law", ["gravity", "ljc_linear", "ljc_constant", "ljc_sigmoidal"])
@pytest.mark.parametrize("prec", ["fp32_kahan", "fp32_fp64acc"])
@pytest.mark.parametrize("potential", [True, False])
def test_batched_symmetric_against_the_oracle(nb, law, prec, potential):
    off, x, par = ensemble(law, SIZES, 900)
    lw = gpu_law(nb, law, prec)
    assert nb.get_config(nb.API_BATCHED, int(off[-1]), lw)["j_stage"] in (0, 1, 2)
    f, p = run(nb, off, x, par, lw, potential, BSYM)
    f, p = host(f), (host(p) if p is not None else None)
    for s in range(len(SIZES)):
        a, b = int(off[s]), int(off[s + 1])
        check_system(law, x[a:b], par[a:b], f[a:b], p[a:b] if p is not None else None, potential)


@pytest.mark.parametrize("law", ["gravity", "ljc_linear"])
def test_batched_symmetric_repeats_and_matches_one_sided(nb, law):
    off, x, par = ensemble(law, [8192, 3000, 517, 5000], 910)     # the largest system the tiles take
    lw = gpu_law(nb, law, "fp32_kahan")
    f1, p1 = run(nb, off, x, par, lw, True, BSYM)
    f2, p2 = run(nb, off, x, par, lw, True, BSYM)
    assert torch.equal(f1, f2) and torch.equal(p1, p2)
    f3, p3 = run(nb, off, x, par, lw, True, (256, 1, 256, 8, 1))
    e = row_errors(host(f1), host(f3))
    assert np.median(e) <= 1e-5 and e.max() <= 1e-3
    # the oracle on sampled rows of the 8192 system
    rows = np.sort(np.random.default_rng(2).choice(8192, 128, replace=False))
    xr, pr = W.round_to_f32(x[:8192]), W.round_to_f32(par[:8192])
    if law == "gravity":
        fr, _ = oracle.gravity(xr, pr, eps=EPS, ilist=rows)
    else:
        fr, _ = oracle.ljc_linear(xr, pr[:, 0], pr[:, 1], pr[:, 2], ilist=rows)
    e = row_errors(host(f1)[rows], fr)
    assert np.median(e) <= 1e-5 and e.max() <= 1e-3


def test_batched_symmetric_falls_back(nb):
    # a system above 8192 particles: the whole launch runs one-sided; so does one with exclusions
    off, x, par = ensemble("ljc_linear", [9000, 300], 920)
    lw = gpu_law(nb, "ljc_linear", "fp32_kahan")
    f, p = run(nb, off, x, par, lw, True, BSYM)
    check_system("ljc_linear", x[9000:], par[9000:], host(f)[9000:], host(p)[9000:], True)
    rows = np.sort(np.random.default_rng(3).choice(9000, 64, replace=False))
    xr, pr = W.round_to_f32(x[:9000]), W.round_to_f32(par[:9000])
    fr, _ = oracle.ljc_linear(xr, pr[:, 0], pr[:, 1], pr[:, 2], ilist=rows)
    e = row_errors(host(f)[rows], fr)
    assert np.median(e) <= 1e-5 and e.max() <= 1e-3
    # exclusions: bonded chains (one system per chain block) through the same forced shape
    sy, eoff, eidx = W.bonded_chains(16, 32, 5)
    n = sy.pos.shape[0]
    offs = np.arange(0, n + 1, 64, dtype=np.int64)
    ex = nb.Exclusions(torch.tensor(eoff, dtype=torch.int64, device="cuda"),
                       torch.tensor(eidx, dtype=torch.int64, device="cuda"))
    try:
        nb.set_config(nb.API_BATCHED, *BSYM)
        fe, _ = nb.forces_batched(offs, dev(sy.pos), dev(sy.params()), lw, exclusions=ex)
        nb.set_config(nb.API_BATCHED, 256, 1, 256, 8, 1)      # the rule's one-sided shape
        fo, _ = nb.forces_batched(offs, dev(sy.pos), dev(sy.params()), lw, exclusions=ex)
    finally:
        nb.clear_config(nb.API_BATCHED)
    assert torch.isfinite(fe).all() and torch.equal(fe, fo)
