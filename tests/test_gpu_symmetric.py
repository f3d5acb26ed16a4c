"""GPU parity of the symmetric pair tiles (j_stage 2: each unordered pair evaluated once and applied
to both particles) against the FP64 oracle on the same FP32-rounded inputs.

Sizes are ragged around the chunk (64) and block (1024, 2048 records) edges, so the tiles cover
padding, diagonal tiles with one-sided self chunks, and off-diagonal tiles; both block edges,
both tile-sum precisions, potential on and off, no softening, G != 1, one leapfrog step through
the symmetric path, and the paths that fall back to the one-sided kernel (row subsets, the
allocation-free entry point when the tiles do not fit its area).  A pair counted twice or missed
shows up as an error of order one in the affected rows.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_0706_3060_amd import workloads as W

pytestmark = pytest.mark.gpu

SIZES = [1, 2, 3, 63, 64, 65, 127, 1000, 1023, 1024, 1025, 2047, 2048, 2049, 3001, 5000]


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


def check(f, p, x, m, eps, G, potential):
    a_ref, phi_ref = oracle.gravity(W.round_to_f32(x), W.round_to_f32(m), G=G, eps=eps)
    e = row_errors(host(f), a_ref)
    assert np.median(e) <= 1e-5 and e.max() <= 1e-3, (np.median(e), e.max())
    if potential:
        ep = np.abs(host(p) - phi_ref) / np.abs(phi_ref)
        assert np.median(ep) <= 1e-5 and ep.max() <= 1e-3, (np.median(ep), ep.max())
    else:
        assert p is None


@pytest.mark.parametrize("shape", [(512, 2), (256, 4)])
@pytest.mark.parametrize("j_tile", [1024, 2048])
@pytest.mark.parametrize("prec", ["fp32_kahan", "fp32_fp64acc"])
def test_symmetric_ragged_sizes(nb, j_tile, prec, shape):
    # two workgroup shapes: 8 waves of 2 i chunks, 4 waves of 4 i chunks
    law = nb.gravity(prec, softening=0.01)
    for k, n in enumerate(SIZES):
        x, _, m = W.plummer(n, 500 + k) if n > 1 else (np.zeros((1, 3)), None, np.ones(1))
        m = m * np.random.default_rng(k).uniform(0.5, 1.5, n)         # unequal masses
        try:
            nb.set_config(nb.API_FORCES, shape[0], shape[1], j_tile, 1, 2)
            c = nb.get_config(nb.API_FORCES, n, law)
            assert (c["j_stage"], c["block"], c["i_per_lane"]) == (2,) + shape, c
            for potential in (True, False):
                f, p = nb.forces(dev(x), dev(m), law, potential=potential)
                if n == 1:
                    assert np.all(host(f) == 0) and (p is None or np.all(host(p) == 0))
                    continue
                check(f, p, x, m, 0.01, 1.0, potential)
        finally:
            nb.clear_config(nb.API_FORCES)


# (workgroup shape, j_tile, j parts per tile): every allowed combination (a part needs at least
# as many chunks as the workgroup has waves)
PART_CASES = [((512, 2), 1024, 2), ((512, 2), 2048, 2), ((512, 2), 2048, 4), ((256, 4), 1024, 2),
              ((256, 4), 1024, 4), ((256, 4), 2048, 2), ((256, 4), 2048, 4)]


@pytest.mark.parametrize("shape,j_tile,split", PART_CASES)
def test_symmetric_j_parts(nb, shape, j_tile, split):
    """The j chunks of each tile cut into 2 or 4 parts, one workgroup each (j_split with
    j_stage 2): each part writes its own i-side slot and the j-side slot of its own rows, and the
    reduction adds a row's slots in order.  Ragged sizes against the oracle, potential on and
    off, both tile-sum precisions, G != 1; a single-block system is one diagonal tile in parts."""
    for prec in ("fp32_kahan", "fp32_fp64acc"):
        law = nb.gravity(prec, softening=0.01, G=1.3)
        for k, n in enumerate([2, 65, 1025, 2049, 3001, 5000]):
            x, _, m = W.plummer(n, 540 + k)
            m = m * np.random.default_rng(k).uniform(0.5, 1.5, n)
            nb.set_config(nb.API_FORCES, shape[0], shape[1], j_tile, split, 2)
            try:
                c = nb.get_config(nb.API_FORCES, n, law)
                assert (c["j_stage"], c["j_split"], c["block"]) == (2, split, shape[0]), c
                for potential in (True, False):
                    f, p = nb.forces(dev(x), dev(m), law, potential=potential)
                    check(f, p, x, m, 0.01, 1.3, potential)
            finally:
                nb.clear_config(nb.API_FORCES)


def test_symmetric_j_parts_repeat_and_match_whole_tiles(nb):
    # at N = 70,000 with 4 parts per tile: bit-for-bit repeatable, and equal to whole tiles to
    # the FP32 bar (the parts group the j sums differently)
    n = 70000
    x, _, m = W.plummer(n, 545)
    law = nb.gravity("fp32_kahan", softening=0.01)
    X, M = dev(x), dev(m)
    out = {}
    for split in (1, 4):
        nb.set_config(nb.API_FORCES, 256, 4, 1024, split, 2)
        try:
            out[split] = [nb.forces(X, M, law) for _ in range(2)]
        finally:
            nb.clear_config(nb.API_FORCES)
    (f1, p1), (f2, p2) = out[4]
    assert torch.equal(f1, f2) and torch.equal(p1, p2)
    e = row_errors(host(f1), host(out[1][0][0]))
    assert np.median(e) <= 1e-5 and e.max() <= 1e-3


@pytest.mark.parametrize("shape", [(512, 2), (256, 4)])
def test_symmetric_without_softening_and_with_G(nb, shape):
    # eps = 0: the self pair of every diagonal chunk must be masked, not evaluated at r = 0
    law = nb.gravity("fp32_kahan", softening=0.0, G=6.674e-3)
    for n in (65, 1500, 4096):
        x, _, m = W.plummer(n, 600 + n)
        nb.set_config(nb.API_FORCES, shape[0], shape[1], 1024, 1, 2)
        try:
            f, p = nb.forces(dev(x), dev(m), law)
        finally:
            nb.clear_config(nb.API_FORCES)
        assert torch.isfinite(f).all() and torch.isfinite(p).all()
        check(f, p, x, m, 0.0, 6.674e-3, True)


@pytest.mark.parametrize("n,parts", [(40000, 4), (70000, 2)])
def test_symmetric_is_the_rule_and_repeats_bitwise(nb, n, parts):
    # from 32,768 particles; four j parts below 65,536, two up to 2^17
    x, _, m = W.plummer(n, 77)
    law = nb.gravity("fp32_kahan", softening=0.01)
    c = nb.get_config(nb.API_FORCES, n, law)
    assert (c["j_stage"], c["j_tile"], c["i_per_lane"], c["block"], c["j_split"]) == (2, 1024, 4, 256, parts), c
    X, M = dev(x), dev(m)
    f1, p1 = nb.forces(X, M, law)
    f2, p2 = nb.forces(X, M, law)
    assert torch.equal(f1, f2) and torch.equal(p1, p2)
    # the one-sided kernel agrees to the FP32 bar
    nb.set_config(nb.API_FORCES, 256, 1, 256, 32, 1)
    try:
        f3, p3 = nb.forces(X, M, law)
    finally:
        nb.clear_config(nb.API_FORCES)
    e = row_errors(host(f1), host(f3))
    assert np.median(e) <= 1e-5 and e.max() <= 1e-3
    # the oracle on sampled rows
    rows = np.sort(np.random.default_rng(7).choice(n, 256, replace=False))
    a_ref, phi_ref = oracle.gravity(W.round_to_f32(x), W.round_to_f32(m), eps=0.01, ilist=rows)
    e = row_errors(host(f1)[rows], a_ref)
    assert np.median(e) <= 1e-5 and e.max() <= 1e-3


@pytest.mark.parametrize("shape", [(512, 2), (256, 4)])
@pytest.mark.parametrize("j_tile", [1024, 2048])
def test_symmetric_leapfrog_step(nb, j_tile, shape):
    n, eps, dt = 3001, 0.01, 1e-3
    x, v, m = W.plummer(n, 88)
    law = nb.gravity("fp32_kahan", softening=eps)
    a0, _ = oracle.gravity(x, m, eps=eps)
    X, V, A, M = dev(x), dev(v), dev(a0), dev(m)
    nb.set_config(nb.API_LEAPFROG, shape[0], shape[1], j_tile, 1, 2)
    try:
        pot = nb.leapfrog(X, V, A, M, law, dt, 2, potential=True)
    finally:
        nb.clear_config(nb.API_LEAPFROG)
    # the FP64 drift from the GPU's own accelerations is exact up to rounding; compare the
    # accelerations at the final positions with the oracle there (FP32 bar)
    a_ref, phi_ref = oracle.gravity(W.round_to_f32(host(X)), W.round_to_f32(m), eps=eps)
    e = row_errors(host(A), a_ref)
    assert np.median(e) <= 1e-5 and e.max() <= 1e-3
    ep = np.abs(host(pot) - phi_ref) / np.abs(phi_ref)
    assert np.median(ep) <= 1e-5 and ep.max() <= 1e-3
    # and the trajectory against the oracle's FP64 leapfrog
    # (two steps; the FP32 accelerations are within 1e-3 of max |a| row by row)
    xr, vr, ar, _ = oracle.leapfrog(oracle.GRAVITY, x, v, a0, m, dt, 2, eps=eps)
    amax = np.abs(a0).max()
    assert np.abs(host(X) - xr).max() <= 4 * dt * dt * 1e-3 * amax + 1e-12 * np.abs(xr).max()
    assert np.abs(host(V) - vr).max() <= 4 * dt * 1e-3 * amax


@pytest.mark.parametrize("shape", [(512, 2), (256, 4)])
def test_subset_and_noalloc_fall_back(nb, shape):
    n = 5000
    x, _, m = W.plummer(n, 99)
    law = nb.gravity("fp32_kahan", softening=0.01)
    X, M = dev(x), dev(m)
    rows = np.sort(np.random.default_rng(3).choice(n, 300, replace=False)).astype(np.int64)
    a_ref, _ = oracle.gravity(W.round_to_f32(x), W.round_to_f32(m), eps=0.01, ilist=rows)
    nb.set_config(nb.API_FORCES, shape[0], shape[1], 1024, 1, 2)
    try:
        fs, _ = nb.forces_subset(X, M, torch.tensor(rows, device="cuda"), law)
        e = row_errors(host(fs), a_ref)
        assert np.median(e) <= 1e-5 and e.max() <= 1e-3
        fn, pn = nb.forces_noalloc(X, M, law)
        e = row_errors(host(fn)[rows], a_ref)
        assert np.median(e) <= 1e-5 and e.max() <= 1e-3
    finally:
        nb.clear_config(nb.API_FORCES)
    # a size whose symmetric tiles do not fit the scratch area (the one-sided kernel runs)
    n = 300000
    x, _, m = W.plummer(n, 101)
    fn, _ = nb.forces_noalloc(dev(x), dev(m), law)
    rows = np.sort(np.random.default_rng(4).choice(n, 64, replace=False))
    a_ref, _ = oracle.gravity(W.round_to_f32(x), W.round_to_f32(m), eps=0.01, ilist=rows)
    e = row_errors(host(fn)[rows], a_ref)
    assert np.median(e) <= 1e-5 and e.max() <= 1e-3


@pytest.mark.parametrize("n,G,shape,split", [(3001, 1.0, (512, 2), 1), (70000, 2.5, (256, 4), 1),
                                              (5000, 1.0, (256, 4), 4)])
def test_shares_add_up_to_the_forces(nb, n, G, shape, split):
    """nbody_forces_share: the shares of the tile triangle (what each of several GPUs would
    evaluate) add up to the whole evaluation; one share is the whole evaluation bit for bit.
    The sum of 8 shares also meets the oracle on sampled rows."""
    x, _, m = W.plummer(n, 710 + n % 97)
    law = nb.gravity("fp32_kahan", softening=0.01, G=G)
    X, M = dev(x), dev(m)
    nb.set_config(nb.API_FORCES, shape[0], shape[1], 1024, split, 2)
    try:
        f_full, p_full = nb.forces(X, M, law)
        f1, p1 = nb.forces_share(X, M, law, 0, 1)
        assert torch.equal(f1, f_full) and torch.equal(p1, p_full)
        fmax, pmax = f_full.abs().max().item(), p_full.abs().max().item()
        for shares in (2, 3, 8):
            fs = torch.zeros_like(f_full)
            ps = torch.zeros_like(p_full)
            for sh in range(shares):
                f, p = nb.forces_share(X, M, law, sh, shares)
                fs += f
                ps += p
            assert (fs - f_full).abs().max().item() <= 1e-12 * fmax, shares
            assert (ps - p_full).abs().max().item() <= 1e-12 * pmax, shares
    finally:
        nb.clear_config(nb.API_FORCES)
    rows = np.sort(np.random.default_rng(8).choice(n, 200, replace=False))
    a_ref, phi_ref = oracle.gravity(W.round_to_f32(x), W.round_to_f32(m), G=G, eps=0.01, ilist=rows)
    e = row_errors(host(fs)[rows], a_ref)
    assert np.median(e) <= 1e-5 and e.max() <= 1e-3
    ep = np.abs(host(ps)[rows] - phi_ref) / np.abs(phi_ref)
    assert np.median(ep) <= 1e-5 and ep.max() <= 1e-3


def test_share_more_shares_than_tiles(nb):
    # 5 particles make one tile: every share but the one holding it returns zeros
    x, _, m = W.plummer(5, 720)
    law = nb.gravity("fp32_kahan", softening=0.01)
    X, M = dev(x), dev(m)
    f_full, _ = nb.forces(X, M, law)
    total = torch.zeros_like(f_full)
    nonzero = 0
    for sh in range(4):
        f, _ = nb.forces_share(X, M, law, sh, 4)
        nonzero += int(bool((f != 0).any()))
        total += f
    assert nonzero == 1
    assert (total - f_full).abs().max().item() <= 1e-5 * f_full.abs().max().item()


@pytest.mark.parametrize("shape,split", [((512, 2), 1), ((256, 4), 1), ((256, 4), 4)])
@pytest.mark.parametrize("prec", ["fp32_kahan", "fp32_fp64acc"])
def test_symmetric_position_adjoint(nb, shape, split, prec):
    """Gravity's position adjoint (the Hessian-vector product) over unordered pairs: the pair's
    term for one particle is minus its term for the other.  Ragged sizes against the oracle's
    adjoint, with G != 1 and unequal masses; the rule's choice repeats bit for bit."""
    law = nb.gravity(prec, softening=0.01, G=1.7)
    for k, n in enumerate([2, 63, 65, 1023, 1025, 2049, 3001]):
        x, _, m = W.plummer(n, 930 + k)
        m = m * np.random.default_rng(k).uniform(0.5, 1.5, n)
        g = np.random.default_rng(40 + k).standard_normal((n, 3))
        nb.set_config(nb.API_BACKWARD, shape[0], shape[1], 1024, split, 2)
        try:
            c = nb.get_config(nb.API_BACKWARD, n, law)
            assert (c["j_stage"], c["block"], c["i_per_lane"], c["j_split"]) == (2,) + shape + (split,), c
            gp, _, _ = nb.forces_backward(dev(x), dev(m), dev(g), law)
        finally:
            nb.clear_config(nb.API_BACKWARD)
        ref = oracle.gravity_adjoint(W.round_to_f32(x), W.round_to_f32(m), W.round_to_f32(g), G=1.7, eps=0.01)
        e = row_errors(host(gp), ref)
        assert np.median(e) <= 1e-5 and e.max() <= 1e-3, (n, np.median(e), e.max())


@pytest.mark.parametrize("n,parts", [(40000, 2), (70000, 2)])
def test_symmetric_position_adjoint_is_the_rule(nb, n, parts):
    # from 32,768 particles (8 waves of 2 chunks without a potential: two j parts at most)
    x, _, m = W.plummer(n, 940)
    g = np.random.default_rng(41).standard_normal((n, 3))
    law = nb.gravity("fp32_fp64acc", softening=0.01)
    c = nb.get_config(nb.API_BACKWARD, n, law)
    assert (c["j_stage"], c["j_split"]) == (2, parts), c
    X, M, Gd = dev(x), dev(m), dev(g)
    g1, _, _ = nb.forces_backward(X, M, Gd, law)
    g2, _, _ = nb.forces_backward(X, M, Gd, law)
    assert torch.equal(g1, g2)
    nb.set_config(nb.API_BACKWARD, 256, 1, 256, 8, 1)               # the one-sided adjoint
    try:
        g3, _, _ = nb.forces_backward(X, M, Gd, law)
    finally:
        nb.clear_config(nb.API_BACKWARD)
    e = row_errors(host(g1), host(g3))
    assert np.median(e) <= 1e-5 and e.max() <= 1e-3
    rows = np.sort(np.random.default_rng(9).choice(n, 128, replace=False))
    ref = oracle.gravity_adjoint(W.round_to_f32(x), W.round_to_f32(m), W.round_to_f32(g), eps=0.01, ilist=rows)
    e = row_errors(host(g1)[rows], ref)
    assert np.median(e) <= 1e-5 and e.max() <= 1e-3
