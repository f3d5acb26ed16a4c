"""The allocation-free forward entry point (nbody_forces_noalloc) against nbody_forces.

The entry point keeps its records and split partials in the library's device scratch area
instead of a caller workspace; its j split may be smaller than the workspace path's, so the two
agree to the parity bar of the precision (FP64 1e-12 per row, FP32 median 1e-5 and max 1e-3),
not bit for bit.  Each case makes two calls in a row, the second on a smaller system, so the
second runs over what the first left in the shared scratch area.  Sizes beyond the area are
refused before anything is enqueued.
"""
import numpy as np
import pytest
import torch

from paper_0706_3060_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def nb():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_0706_3060_amd import nbody
    return nbody


def dev(a):
    return torch.tensor(np.asarray(a), dtype=torch.float64, device="cuda")


def inputs(law_name, n, seed):
    if law_name == "gravity":
        x, _, m = W.plummer(n, seed)
        return x, m
    s = W.md_system(n, seed, box=(32.0 * n) ** (1.0 / 3.0))
    return s.pos, s.params()


def law_of(nb, law_name, prec):
    return nb.gravity(prec, softening=0.01) if law_name == "gravity" else nb.ljc_linear(prec)


@pytest.mark.parametrize("law_name,prec,sizes", [
    ("gravity", "fp32_kahan", (200000, 3001)),
    ("gravity", "fp64", (65536, 1000)),
    ("ljc_linear", "fp32_fp64acc", (20000, 777)),
    ("ljc_linear", "fp64", (6000, 700)),
])
def test_noalloc_matches_workspace_entry_point(nb, law_name, prec, sizes):
    law = law_of(nb, law_name, prec)
    for k, n in enumerate(sizes):
        x, par = inputs(law_name, n, 40 + k)
        X, P = dev(x), dev(par)
        f0, p0 = nb.forces(X, P, law)
        f1, p1 = nb.forces_noalloc(X, P, law)
        torch.cuda.synchronize()
        f0, p0, f1, p1 = (t.cpu().numpy() for t in (f0, p0, f1, p1))
        e = np.linalg.norm(f1 - f0, axis=1) / np.linalg.norm(f0, axis=1)
        ep = np.abs(p1 - p0) / np.abs(p0)
        if prec == "fp64":
            assert e.max() <= 1e-12 and ep.max() <= 1e-12, (n, e.max(), ep.max())
        else:
            assert np.median(e) <= 1e-5 and e.max() <= 1e-3, (n, np.median(e), e.max())
            assert np.median(ep) <= 1e-5 and ep.max() <= 1e-3, (n, np.median(ep), ep.max())
        # without the potential
        f2, p2 = nb.forces_noalloc(X, P, law, potential=False)
        assert p2 is None
        assert np.linalg.norm(f2.cpu().numpy() - f0, axis=1).max() <= 1e-3 * np.linalg.norm(f0, axis=1).max()


def test_noalloc_refuses_sizes_beyond_its_area(nb):
    from paper_0706_3060_amd import _native as N
    law = nb.ljc_linear("fp64")                    # 64-byte records: at most 2^26 / 64 - 64 particles
    limit = (64 << 20) // 64 - 64
    n = limit + 1
    X = torch.zeros((n, 3), dtype=torch.float64, device="cuda")
    P = torch.zeros((n, 3), dtype=torch.float64, device="cuda")
    f = torch.full((n, 3), 7.0, dtype=torch.float64, device="cuda")
    with pytest.raises(N.NBodyError) as ei:
        nb.forces_noalloc(X, P, law, out=(f, None))
    assert ei.value.code == N.NBODY_EINVAL and "limit" in str(ei.value)
    torch.cuda.synchronize()
    assert bool((f == 7.0).all())                 # refused before anything was enqueued
    # a size within the limit runs
    x, par = inputs("ljc_linear", 64, 5)
    f3, _ = nb.forces_noalloc(dev(x), dev(par), law)
    assert torch.isfinite(f3).all()
