"""GPU parity of LJC(linear)'s single-system adjoint over unordered pairs (the backward of the
forces under a loss L(F), g = dL/dF: each pair's position terms applied to both atoms with
opposite signs, its charge, sigma and epsilon terms from one shared scalar) against the FP64
oracle's analytic derivatives on the FP32-rounded inputs.

Ragged sizes around the chunk (64) and block (256 records) edges, both FP32 tile-sum precisions,
positions and parameters with per-type sums; the rule's choice at N = 70,000 and 150,000 (bitwise repeatable,
equal to the one-sided adjoint to the FP32 bar, sampled rows against the oracle); the position or
the parameter gradients alone (bitwise the same); and exclusion lists, which the tiles do not
take, running the one-sided kernel.  Bars as for the other FP32
adjoints: per-atom relative position-gradient error median <= 1e-5 and max <= 1e-3; parameter
gradients relative to their largest magnitude.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_0706_3060_amd import workloads as W

pytestmark = pytest.mark.gpu

SIZES = [2, 3, 63, 64, 65, 255, 256, 257, 1000, 3001]
TILES = (256, 4, 256, 1, 2)
ONE_SIDED = (256, 1, 256, 8, 1)


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


def system(n, seed):
    return W.md_system(n, seed, box=(32.0 * n) ** (1.0 / 3.0) + 3.0)


def row_errors(f, ref):
    nref = np.linalg.norm(ref, axis=1)
    return np.linalg.norm(f - ref, axis=1) / np.maximum(nref, 1e-3 * nref.max())


def check(gp, gq, ref, rows=None):
    rp, rq, rs, re = ref
    if rows is not None:
        gp, gq = gp[rows], gq[rows]
    e = row_errors(gp, rp)
    assert np.median(e) <= 1e-5 and e.max() <= 1e-3, (np.median(e), e.max())
    for got, want in ((gq[:, 0], rq), (gq[:, 1], rs), (gq[:, 2], re)):
        err = np.abs(got - want) / np.abs(want).max()
        assert np.median(err) <= 1e-5 and err.max() <= 1e-3, (np.median(err), err.max())


def oracle32(s, g, rows=None):
    x, p = W.round_to_f32(s.pos), W.round_to_f32(s.params())
    return oracle.ljc_adjoint(x, p[:, 0], p[:, 1], p[:, 2], W.round_to_f32(g), ilist=rows)


def backward(nb, cfg, X, P, G, law, **kw):
    try:
        nb.set_config(nb.API_BACKWARD, *cfg)
        return nb.forces_backward(X, P, G, law, **kw)
    finally:
        nb.clear_config(nb.API_BACKWARD)


@pytest.mark.parametrize("prec", ["fp32_kahan", "fp32_fp64acc"])
def test_ljc_adjoint_tiles_ragged_sizes(nb, prec):
    law = nb.ljc_linear(prec)
    for k, n in enumerate(SIZES):
        s = system(n, 500 + k)
        g = W.unit_cotangent(n, 600 + k)
        types = torch.tensor(s.types.astype(np.int32), device="cuda")
        try:
            nb.set_config(nb.API_BACKWARD, *TILES)
            c = nb.get_config(nb.API_BACKWARD, n, law)
            assert (c["j_stage"], c["block"], c["i_per_lane"], c["j_tile"]) == (2, 256, 4, 256), c
            gp, gq, gt = nb.forces_backward(dev(s.pos), dev(s.params()), dev(g), law, types=types,
                                            n_types=4)
        finally:
            nb.clear_config(nb.API_BACKWARD)
        gp, gq, gt = host(gp), host(gq), host(gt)
        check(gp, gq, oracle32(s, g))
        for t in range(4):
            sel = s.types == t
            for col, j in ((1, 0), (2, 1)):
                np.testing.assert_allclose(gt[t, j], gq[sel, col].sum(), rtol=1e-12,
                                           atol=1e-12 * np.abs(gq[:, col]).sum())


@pytest.mark.parametrize("n", [70000, 150000])
def test_ljc_adjoint_tiles_are_the_rule_and_repeat_bitwise(nb, n):
    s = system(n, 81)
    g = W.unit_cotangent(n, 82)
    law = nb.ljc_linear("fp32_kahan")
    c = nb.get_config(nb.API_BACKWARD, n, law)
    assert (c["j_stage"], c["block"], c["j_tile"]) == (2, 256, 256), c
    X, P, G = dev(s.pos), dev(s.params()), dev(g)
    p1, q1, _ = nb.forces_backward(X, P, G, law)
    p2, q2, _ = nb.forces_backward(X, P, G, law)
    assert torch.equal(p1, p2) and torch.equal(q1, q2)
    p3, q3, _ = backward(nb, ONE_SIDED, X, P, G, law)
    e = row_errors(host(p1), host(p3))
    assert np.median(e) <= 1e-5 and e.max() <= 1e-3, (np.median(e), e.max())
    err = ((q1 - q3).abs().max(dim=0).values / q3.abs().max(dim=0).values).max().item()
    assert err <= 1e-3, err
    rows = np.sort(np.random.default_rng(9).choice(n, 128, replace=False))
    check(host(p1), host(q1), oracle32(s, g, rows), rows)


def test_ljc_adjoint_exclusions_run_one_sided(nb):
    # the tiles take no exclusion lists: a forced tile configuration runs the one-sided kernel
    # in the shape the lists give it (LDS staging, at most 2 rows per lane), bit for bit
    sy, eoff, eidx = W.bonded_chains(40, 50, 61)
    n = sy.pos.shape[0]
    g = W.unit_cotangent(n, 62)
    law = nb.ljc_linear("fp32_kahan")
    ex = nb.Exclusions(torch.tensor(eoff, dtype=torch.int64, device="cuda"),
                       torch.tensor(eidx, dtype=torch.int64, device="cuda"))
    X, P, G = dev(sy.pos), dev(sy.params()), dev(g)
    a = backward(nb, TILES, X, P, G, law, exclusions=ex)
    b = backward(nb, (256, 2, 256, 1, 1), X, P, G, law, exclusions=ex)
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
    x, p = W.round_to_f32(sy.pos), W.round_to_f32(sy.params())
    ref = oracle.ljc_adjoint_excl(x, p[:, 0], p[:, 1], p[:, 2], W.round_to_f32(g), eoff, eidx)
    check(host(a[0]), host(a[1]), ref)


def test_ljc_adjoint_tiles_partial_outputs(nb):
    # only the position gradient, or only the parameter gradients: the same values bit for bit
    n = 3001
    s = system(n, 83)
    g = W.unit_cotangent(n, 84)
    law = nb.ljc_linear("fp32_kahan")
    X, P, G = dev(s.pos), dev(s.params()), dev(g)
    gp, gq, _ = backward(nb, TILES, X, P, G, law)
    gp2, gq2, _ = backward(nb, TILES, X, P, G, law, want_params=False)
    gp3, gq3, _ = backward(nb, TILES, X, P, G, law, want_pos=False)
    assert gq2 is None and gp3 is None
    assert torch.equal(gp, gp2) and torch.equal(gq, gq3)
