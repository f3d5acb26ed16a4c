"""The forward and the leapfrog captured in a HIP graph (through torch.cuda.graph) and
replayed: every launch of these paths is a kernel on the caller's stream, with no host
synchronisation, memset or host copy inside, so a captured call can be replayed.

Each test replays the graph several times, with eager work of the library and
synchronisations between the replays, and checks every replay bit for bit against the
same computation run eagerly.
"""
import numpy as np
import pytest
import torch

from paper_0706_3060_amd import workloads as W

pytestmark = pytest.mark.gpu

EPS = 0.01


@pytest.fixture(scope="module")
def nb():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_0706_3060_amd import nbody
    return nbody


def dev(a):
    return torch.tensor(np.asarray(a), dtype=torch.float64, device="cuda")


def warm_on_side_stream(fn):
    """Run fn once on a side stream (the library's workspace for a new stream is allocated
    outside the capture), as torch recommends before capturing."""
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        fn()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()


@pytest.mark.parametrize("prec", ["fp32_kahan", "fp64"])
def test_forces_replay(nb, prec):
    x, _, m = W.plummer(5000, 71)
    X, M = dev(x), dev(m)
    law = nb.gravity(prec, softening=EPS)
    f_ref, p_ref = nb.forces(X, M, law)
    torch.cuda.synchronize()
    warm_on_side_stream(lambda: nb.forces(X, M, law))
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        f_g, p_g = nb.forces(X, M, law)
    for _ in range(4):
        f_g.fill_(float("nan"))
        p_g.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(f_g, f_ref) and torch.equal(p_g, p_ref)
        f_e, _ = nb.forces(X, M, law)          # eager work between replays
        torch.cuda.synchronize()
        assert torch.equal(f_e, f_ref)


def test_leapfrog_replay(nb):
    x, v, m = W.plummer(3000, 72)
    law = nb.gravity("fp32_kahan", softening=EPS)
    M = dev(m)
    a0, _ = nb.forces(dev(x), M, law)
    torch.cuda.synchronize()
    # eager reference: three calls of five steps
    Xe, Ve, Ae = dev(x), dev(v), a0.clone()
    refs = []
    for _ in range(3):
        nb.leapfrog(Xe, Ve, Ae, M, law, 1e-3, 5)
        torch.cuda.synchronize()
        refs.append((Xe.clone(), Ve.clone(), Ae.clone()))
    # captured: one call of five steps, replayed three times on the same state
    Xg, Vg, Ag = dev(x), dev(v), a0.clone()
    Xw, Vw, Aw = dev(x), dev(v), a0.clone()
    warm_on_side_stream(lambda: nb.leapfrog(Xw, Vw, Aw, M, law, 1e-3, 5))
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        nb.leapfrog(Xg, Vg, Ag, M, law, 1e-3, 5)
    assert torch.equal(Xg, dev(x))                   # capture itself runs nothing
    for k in range(3):
        g.replay()
        torch.cuda.synchronize()
        for got, want in zip((Xg, Vg, Ag), refs[k]):
            assert torch.equal(got, want), k
        nb.forces(Xw, M, law)                        # eager work between replays
        torch.cuda.synchronize()
