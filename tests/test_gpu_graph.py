"""The forward, the leapfrog, the shared Hermite step and the batched forward and adjoint
captured in a HIP graph (through torch.cuda.graph) and replayed: every launch of these paths is
a kernel on the caller's stream, with no host synchronisation, memset or host copy inside (the
batched paths read their plan tables from device memory made at an ensemble's first launch), so
a captured call can be replayed.

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


@pytest.mark.parametrize("tiles", [False, True])
def test_hermite_replay(nb, tiles):
    """Shared Hermite steps (the predictor's pack, the acceleration and jerk, one-sided or over
    unordered pairs with their slot reduction, and the corrector) captured and replayed."""
    x, v, m = W.plummer(3000, 73)
    law = nb.gravity("fp32_kahan", softening=0.05)
    M = dev(m)
    dt, steps = 1.0 / 1024, 2
    try:
        nb.set_config(nb.API_JERK, *((512, 2, 1024, 2, 2) if tiles else (256, 1, 256, 4, 0)))
        a0, j0, _ = nb.forces_jerk(dev(x), dev(v), M, law, potential=False)
        torch.cuda.synchronize()
        # eager reference: three calls of two steps
        Xe, Ve, Ae, Je = dev(x), dev(v), a0.clone(), j0.clone()
        refs = []
        for _ in range(3):
            nb.hermite(Xe, Ve, Ae, Je, M, law, dt, steps)
            torch.cuda.synchronize()
            refs.append((Xe.clone(), Ve.clone(), Ae.clone(), Je.clone()))
        # captured: one call of two steps, replayed three times on the same state
        Xg, Vg, Ag, Jg = dev(x), dev(v), a0.clone(), j0.clone()
        Xw, Vw, Aw, Jw = dev(x), dev(v), a0.clone(), j0.clone()
        warm_on_side_stream(lambda: nb.hermite(Xw, Vw, Aw, Jw, M, law, dt, steps))
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            nb.hermite(Xg, Vg, Ag, Jg, M, law, dt, steps)
        assert torch.equal(Xg, dev(x))                   # capture itself runs nothing
        for k in range(3):
            g.replay()
            torch.cuda.synchronize()
            for got, want in zip((Xg, Vg, Ag, Jg), refs[k]):
                assert torch.equal(got, want), k
            nb.forces_jerk(Xw, Vw, M, law)                # eager work between replays
            torch.cuda.synchronize()
    finally:
        nb.clear_config(nb.API_JERK)


def _ensemble(sizes, seed):
    off, pos, par, _ = W.batched_md(len(sizes), seed=seed, sizes=sizes, workers=1)
    return off, dev(pos), dev(par)


# uneven systems, two of them large enough to be cut into j parts (the part-sum
# reduction is then part of the captured work), one empty
SIZES_A = [700, 0, 3000, 45, 1800, 9000, 128, 2500, 64, 6000]
SIZES_B = [300, 1200, 65, 2000]


@pytest.mark.parametrize("prec,shape", [("fp32_kahan", None), ("fp64", None), ("fp32_kahan", (256, 4, 256, 1, 2))])
def test_forces_batched_replay(nb, prec, shape):
    """The batched forward keeps each ensemble's plan tables in device memory after its
    first launch, so later launches copy nothing from the host and can be captured.
    Between replays the same workspace serves another ensemble eagerly."""
    # the symmetric tiles take systems of up to 8192 particles
    off, X, P = _ensemble(SIZES_A if shape is None else [s if s <= 8192 else 8000 for s in SIZES_A], 81)
    offb, Xb, Pb = _ensemble(SIZES_B, 82)
    law = nb.ljc_linear(prec)
    if shape is not None:                    # the symmetric tiles
        nb.set_config(nb.API_BATCHED, *shape)
    try:
        _replay_batched(nb, off, X, P, offb, Xb, Pb, law)
    finally:
        nb.clear_config(nb.API_BATCHED)


def _replay_batched(nb, off, X, P, offb, Xb, Pb, law):
    f_ref, p_ref = nb.forces_batched(off, X, P, law)
    fb_ref, _ = nb.forces_batched(offb, Xb, Pb, law)
    torch.cuda.synchronize()
    warm_on_side_stream(lambda: nb.forces_batched(off, X, P, law))
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        f_g, p_g = nb.forces_batched(off, X, P, law)
    for _ in range(4):
        f_g.fill_(float("nan"))
        p_g.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(f_g, f_ref) and torch.equal(p_g, p_ref)
        fb, _ = nb.forces_batched(offb, Xb, Pb, law)       # another ensemble, eagerly
        torch.cuda.synchronize()
        assert torch.equal(fb, fb_ref)


@pytest.mark.parametrize("tiles", [False, True])
def test_backward_batched_replay(nb, tiles):
    # the rule takes the adjoint's symmetric tiles when every system fits 8192 particles; with
    # the 9000-particle system the launch runs one-sided
    off, X, P = _ensemble(SIZES_A if not tiles else [s if s <= 8192 else 8000 for s in SIZES_A], 83)
    g_in = dev(np.random.default_rng(5).standard_normal((int(off[-1]), 3)))
    law = nb.ljc_linear("fp32_kahan")
    c = nb.get_config(nb.API_BACKWARD_BATCHED, int(off[-1]), law, n_systems=len(off) - 1)
    assert c["j_stage"] == 2, c                     # the rule (a 9000-particle system runs one-sided)
    ref = nb.forces_backward_batched(off, X, P, g_in, law)
    torch.cuda.synchronize()
    warm_on_side_stream(lambda: nb.forces_backward_batched(off, X, P, g_in, law))
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        out = nb.forces_backward_batched(off, X, P, g_in, law)
    for _ in range(3):
        out[0].fill_(float("nan"))
        out[1].fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out[0], ref[0]) and torch.equal(out[1], ref[1])
        nb.forces_batched(off, X, P, law)                   # eager work between replays
        torch.cuda.synchronize()


def test_backward_single_system_tiles_replay(nb):
    """LJC(linear)'s single-system adjoint over unordered pairs (pack, tiles, slot reduction,
    per-type sums) captured and replayed: its tile order is arithmetic, with no plan tables."""
    s = W.md_system(3001, 84, box=48.0)
    X, P = dev(s.pos), dev(s.params())
    g_in = dev(np.random.default_rng(6).standard_normal((3001, 3)))
    types = torch.tensor(s.types.astype(np.int32), device="cuda")
    law = nb.ljc_linear("fp32_kahan")
    try:
        nb.set_config(nb.API_BACKWARD, 256, 4, 256, 1, 2)
        ref = nb.forces_backward(X, P, g_in, law, types=types, n_types=4)
        torch.cuda.synchronize()
        warm_on_side_stream(lambda: nb.forces_backward(X, P, g_in, law, types=types, n_types=4))
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            out = nb.forces_backward(X, P, g_in, law, types=types, n_types=4)
        for _ in range(3):
            for t in out:
                t.fill_(float("nan"))
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            assert all(torch.equal(a, b) for a, b in zip(out, ref))
            nb.forces(X, P, law)                                # eager work between replays
            torch.cuda.synchronize()
    finally:
        nb.clear_config(nb.API_BACKWARD)


def test_first_batched_launch_refused_under_capture(nb):
    """A new ensemble's first launch uploads its plan tables, which a capture cannot hold:
    the call is refused before anything is enqueued, and the ensemble works eagerly after."""
    from paper_0706_3060_amd import _native as N
    off, X, P = _ensemble([500, 1500, 77, 2300], 84)
    law = nb.ljc_linear("fp32_kahan")
    g = torch.cuda.CUDAGraph()
    with pytest.raises(N.NBodyError, match="cannot be captured"):
        with torch.cuda.graph(g):
            nb.forces_batched(off, X, P, law)
    torch.cuda.synchronize()
    f, _ = nb.forces_batched(off, X, P, law)
    f2, _ = nb.forces_batched(off, X, P, law)
    torch.cuda.synchronize()
    assert torch.isfinite(f).all() and torch.equal(f, f2)
