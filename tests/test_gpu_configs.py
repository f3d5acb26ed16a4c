"""The five measured workloads at their full sizes, on the GPU, against the oracle.

Where the oracle cannot evaluate every output in seconds, it evaluates sampled
rows one by one (seeded samples) and the rest is checked against the FP64 GPU
pass, which is itself pinned to the oracle.

1. gravity, Plummer N=4096, FP64: forward + one KDK step            (tests/test_gpu_forward.py)
2. gravity, Plummer N=65,536, FP32 + FP64/Kahan sums, 100 KDK steps: force error at t=0 and
   t=100, relative energy drift next to the FP64 trajectory's
3. LJC(linear), N=8192 MD box, FP32 forward + force-matching backward; FD and Euler checks
4. 256 LJC systems, N_s in [500, 5000], one persistent launch vs per-system FP64
5. gravity, Plummer N=1,048,576, eps=0.005, FP32 + Kahan vs the FP64 GPU pass, oracle on
   sampled rows; Hessian-vector product at N=262,144
"""
import numpy as np
import pytest
import torch

import oracle
from paper_0706_3060_amd import workloads as W

pytestmark = pytest.mark.gpu

# The forced alternative shapes of the full-size case: the one-sided kernel with 32 j parts over
# XCD-ordered blocks and LDS staging, and with one j part and scalar staging.
ALT_CFG = {"sym_8x2": (512, 2, 2048, 1, 2), "one_sided": (256, 1, 256, 32, 1), "scalar": (256, 1, 256, 1, 0)}


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


def energy(nb, x, v, m, eps):
    """Total energy with the potential from the FP64 pass (so FP32 potential error is not
    counted as drift)."""
    _, phi = nb.forces(x, m, nb.gravity("fp64", softening=eps))
    return float((0.5 * m * (v * v).sum(1)).sum() + 0.5 * (m * phi).sum())


@pytest.mark.parametrize("prec", ["fp32_kahan", "fp32_fp64acc"])
def test_config2_plummer_65536_100_steps(nb, prec):
    n, eps, dt = 65536, 0.01, 1e-3
    pos, vel, m = W.plummer(n, 2)
    law = nb.gravity(prec, softening=eps)
    law64 = nb.gravity("fp64", softening=eps)
    x, v, mm = dev(pos), dev(vel), dev(m)
    a, _ = nb.forces(x, mm, law)
    # t = 0 against the full oracle on the FP32-rounded inputs
    a_ref, _ = oracle.gravity(W.round_to_f32(pos), W.round_to_f32(m), eps=eps)
    e0 = rel_rows(host(a), a_ref)
    assert np.median(e0) <= 1e-5 and e0.max() <= 1e-3, (np.median(e0), e0.max())
    E0 = energy(nb, x, v, mm, eps)
    nb.leapfrog(x, v, a, mm, law, dt, 100)
    # FP64 trajectory from the same state
    x64, v64 = dev(pos), dev(vel)
    a64, _ = nb.forces(x64, mm, law64)
    nb.leapfrog(x64, v64, a64, mm, law64, dt, 100)
    drift32 = abs(energy(nb, x, v, mm, eps) - E0) / abs(E0)
    drift64 = abs(energy(nb, x64, v64, mm, eps) - E0) / abs(E0)
    assert drift64 < 1e-4
    assert abs(drift32 - drift64) <= 1e-6 + 0.05 * drift64, (drift32, drift64)
    # t = 100: oracle at the GPU's own positions, 4096 sampled rows
    rows = np.sort(np.random.default_rng(22).choice(n, 4096, replace=False))
    xr = W.round_to_f32(host(x))
    a100_ref, _ = oracle.gravity(xr, W.round_to_f32(m), eps=eps, ilist=rows)
    e100 = rel_rows(host(a)[rows], a100_ref)
    assert np.median(e100) <= 1e-5 and e100.max() <= 1e-3, (np.median(e100), e100.max())


def _md_target(nb):
    s = W.md_system(8192, 3)
    t = W.perturbed(s, 33)
    return s, t


def test_config3_md_8192_forward_and_force_matching_gradient(nb):
    s, t = _md_target(nb)
    law = nb.ljc_linear("fp32_fp64acc")
    law64 = nb.ljc_linear("fp64")
    x = dev(s.pos)
    f, u = nb.forces(x, dev(s.params()), law)
    f_ref, u_ref = oracle.ljc_linear(W.round_to_f32(s.pos), s.q, s.sigma, s.epsilon)
    e = rel_rows(host(f), f_ref)
    assert np.median(e) <= 1e-5 and e.max() <= 1e-3, (np.median(e), e.max())
    # backward of L = ||F - F_target||^2 through the typed autograd Function
    ftarget, _ = nb.forces(x, dev(t.params()), law64)
    pos = x.clone().requires_grad_(True)
    q = dev(s.q).requires_grad_(True)
    st = dev(s.sigma_t).requires_grad_(True)
    et = dev(s.eps_t).requires_grad_(True)
    types = torch.tensor(s.types, device="cuda")
    F = nb.LJCTypedForcesFn.apply(pos, q, st, et, types, law)
    L = ((F - ftarget) ** 2).sum()
    L.backward()
    g = 2.0 * (host(F) - host(ftarget))
    rp, rq, rs, re = oracle.ljc_adjoint(W.round_to_f32(s.pos), s.q, s.sigma, s.epsilon, g)
    ep = rel_rows(host(pos.grad), rp)
    assert np.median(ep) <= 1e-5 and ep.max() <= 1e-3, (np.median(ep), ep.max())
    eq = np.abs(host(q.grad) - rq) / np.abs(rq).max()
    assert np.median(eq) <= 1e-5 and eq.max() <= 1e-3
    for k in range(4):
        sel = s.types == k
        assert abs(host(st.grad)[k] - rs[sel].sum()) <= 1e-5 * np.abs(rs[sel]).sum()
        assert abs(host(et.grad)[k] - re[sel].sum()) <= 1e-5 * np.abs(re[sel]).sum()


def test_config3_gradient_finite_differences_fp64(nb):
    # FD of L(theta) on the FP64 GPU path against the FP64 GPU adjoint
    s, t = _md_target(nb)
    law = nb.ljc_linear("fp64")
    x = dev(s.pos)
    types = torch.tensor(s.types, device="cuda")
    ftarget, _ = nb.forces(x, dev(t.params()), law)

    def L(pos, q, st, et):
        par = torch.stack([q, st[types.long()], et[types.long()]], 1)
        f, _ = nb.forces(pos, par, law, potential=False)
        return float(((f - ftarget) ** 2).sum())

    pos = x.clone().requires_grad_(True)
    q = dev(s.q).requires_grad_(True)
    st = dev(s.sigma_t).requires_grad_(True)
    et = dev(s.eps_t).requires_grad_(True)
    F = nb.LJCTypedForcesFn.apply(pos, q, st, et, types, law)
    ((F - ftarget) ** 2).sum().backward()
    rng = np.random.default_rng(3)
    base = (x, dev(s.q), dev(s.sigma_t), dev(s.eps_t))
    grads = (pos.grad, q.grad, st.grad, et.grad)
    checks = [(0, (int(i), int(c))) for i, c in zip(rng.integers(0, 8192, 6), rng.integers(0, 3, 6))]
    checks += [(1, (int(i),)) for i in rng.integers(0, 8192, 4)]
    checks += [(2, (k,)) for k in range(4)] + [(3, (k,)) for k in range(4)]
    for which, idx in checks:
        h = 1e-5 * max(1.0, abs(float(base[which][idx])))
        plus = [b.clone() for b in base]
        minus = [b.clone() for b in base]
        plus[which][idx] += h
        minus[which][idx] -= h
        fd = (L(*plus) - L(*minus)) / (2 * h)
        an = float(grads[which][idx])
        assert abs(fd - an) <= 1e-5 * max(abs(an), 1e-3 * float(grads[which].abs().max())), (which, idx, fd, an)


def test_config3_euler_identities_on_gpu(nb):
    s, _ = _md_target(nb)
    law = nb.ljc_linear("fp64")
    x = dev(s.pos)
    g = W.unit_cotangent(s.n, 57)
    gp, gpar, _ = nb.forces_backward(x, dev(s.params()), dev(g), law)
    p0 = s.params()
    pc, plj = p0.copy(), p0.copy()
    pc[:, 2] = 0.0
    plj[:, 0] = 0.0
    fc, _ = nb.forces(x, dev(pc), law)
    flj, _ = nb.forces(x, dev(plj), law)
    gfc, gflj = float((g * host(fc)).sum()), float((g * host(flj)).sum())
    gp, gpar = host(gp), host(gpar)
    scale = np.abs(g * host(fc)).sum() + np.abs(g * host(flj)).sum()
    assert abs((s.q * gpar[:, 0]).sum() - 2 * gfc) <= 1e-10 * scale
    assert abs((s.epsilon * gpar[:, 2]).sum() - gflj) <= 1e-10 * scale
    assert abs((s.sigma * gpar[:, 1]).sum() + (s.pos * gp).sum() + gflj + 3 * gfc) <= 1e-9 * scale


# The default rule, and four forced shapes of the persistent launch over the full ensemble: one
# row per lane with scalar staging and two rows per lane with LDS staging.  Under the forced
# shapes the planner cuts the large systems into j parts whose slots and unit table reach the
# limits of the workspace layout (a unit table once sized below the planner's maximum made such
# launches fault; the CPU test of the planner checks the layout for every occupancy); the fourth
# shape aims at 64 work units per wave, the most parts the planner makes, and the last runs the
# symmetric tiles (each unordered pair of a system once).
@pytest.mark.parametrize("shape", [None, (256, 1, 256, 8, 0), (256, 2, 256, 8, 1), (128, 1, 64, 64, 1),
                                   (256, 4, 256, 1, 2)])
def test_config4_full_ensemble(nb, full_ensemble, shape):
    off, pos, par, systems = full_ensemble
    S = len(systems)
    x, p = dev(pos), dev(par)
    law = nb.ljc_linear("fp32_kahan")
    law64 = nb.ljc_linear("fp64")
    try:
        if shape is not None:
            nb.set_config(nb.API_BATCHED, *shape)
        fb, ub = nb.forces_batched(off, x, p, law)
    finally:
        nb.clear_config(nb.API_BATCHED)
    fb, ub = host(fb), host(ub)
    meds = []
    for s in range(S):
        a, b = off[s], off[s + 1]
        f64, u64 = nb.forces(x[a:b], p[a:b], law64)
        e = rel_rows(fb[a:b], host(f64))
        meds.append(np.median(e))
        assert e.max() <= 1e-3, (s, e.max())
    assert max(meds) <= 1e-5, max(meds)
    if shape is not None:
        return
    # the oracle on 8 sampled systems, 64 sampled rows each
    rng = np.random.default_rng(44)
    for s in rng.choice(S, 8, replace=False):
        a, b = off[s], off[s + 1]
        sy = systems[s]
        rows = np.sort(rng.choice(b - a, min(64, b - a), replace=False))
        fr, _ = oracle.ljc_linear(W.round_to_f32(sy.pos), sy.q, sy.sigma, sy.epsilon, ilist=rows)
        e = rel_rows(fb[a:b][rows], fr)
        assert np.median(e) <= 1e-5 and e.max() <= 1e-3


@pytest.mark.parametrize("shape", ["rule", "sym_8x2", "one_sided", "scalar"])
def test_config5_plummer_1m(nb, shape):
    """Gravity at N = 2^20, FP32 + Kahan, against the FP64 GPU pass over all rows and the oracle
    on sampled rows.  "rule" runs the configuration the benchmark times (the library's rule for
    this size: the symmetric pair tiles with 2048-record blocks, 4-wave workgroups of 4 i chunks
    per wave, and the slot-ordered partial reduction), through both timed entry points: the
    forward and one kick-drift-kick step.  "sym_8x2" forces the other symmetric shape (8 waves
    of 2 i chunks); "one_sided" forces the one-sided kernel with 32 j parts over XCD-ordered blocks and LDS
    staging, "scalar" one j part with scalar staging."""
    n, eps, dt = 1 << 20, 0.005, 1e-3
    pos, vel, m = W.plummer(n, 5)
    x, mm = dev(pos), dev(m)
    law = nb.gravity("fp32_kahan", softening=eps)
    law64 = nb.gravity("fp64", softening=eps)
    if shape == "rule":
        for api in (nb.API_FORCES, nb.API_LEAPFROG):
            c = nb.get_config(api, n, law)
            assert (c["j_stage"], c["j_tile"], c["i_per_lane"], c["block"]) == (2, 2048, 4, 256), (api, c)
    try:
        if shape != "rule":
            for api in (nb.API_FORCES, nb.API_LEAPFROG):
                nb.set_config(api, *ALT_CFG[shape])
        f32, p32 = nb.forces(x, mm, law)
        # one step of the timed loop: a(t) from the forward, kick-drift, forces at x(t+dt), kick
        X, V, A = x.clone(), dev(vel), f32.clone()
        pot1 = nb.leapfrog(X, V, A, mm, law, dt, 1, potential=True)
    finally:
        nb.clear_config(nb.API_FORCES)
        nb.clear_config(nb.API_LEAPFROG)
    f64, p64 = nb.forces(x, mm, law64)
    f32, f64, p32, p64 = host(f32), host(f64), host(p32), host(p64)
    e = rel_rows(f32, f64)
    assert np.median(e) <= 1e-5 and e.max() <= 1e-3, (np.median(e), e.max())
    ep = np.abs(p32 - p64) / np.abs(p64)
    assert np.median(ep) <= 1e-5 and ep.max() <= 1e-3
    rows = np.sort(np.random.default_rng(55).choice(n, 512, replace=False))
    a_ref, phi_ref = oracle.gravity(pos, m, eps=eps, ilist=rows)
    assert rel_rows(f64[rows], a_ref).max() <= 1e-12
    assert (np.abs(p64[rows] - phi_ref) / np.abs(phi_ref)).max() <= 1e-12
    a32_ref, p32_ref = oracle.gravity(W.round_to_f32(pos), W.round_to_f32(m), eps=eps, ilist=rows)
    e32 = rel_rows(f32[rows], a32_ref)
    assert np.median(e32) <= 1e-5 and e32.max() <= 1e-3
    ep32 = np.abs(p32[rows] - p32_ref) / np.abs(p32_ref)
    assert np.median(ep32) <= 1e-5 and ep32.max() <= 1e-3
    # the step: FP64 kick-drift from the same a(t) (so x(t+dt) agrees to FP64 rounding), then the
    # FP32 forces at x(t+dt) against the oracle there, on the same rows
    xh, vh = host(X), host(V)
    v_half = vel + 0.5 * dt * f32
    x1 = pos + dt * v_half
    assert np.abs(xh - x1).max() <= 1e-14 * np.abs(x1).max()
    a1_ref, phi1_ref = oracle.gravity(W.round_to_f32(xh), W.round_to_f32(m), eps=eps, ilist=rows)
    e1 = rel_rows(host(A)[rows], a1_ref)
    assert np.median(e1) <= 1e-5 and e1.max() <= 1e-3, (np.median(e1), e1.max())
    np.testing.assert_allclose(vh[rows], v_half[rows] + 0.5 * dt * host(A)[rows], rtol=0, atol=1e-14)
    ep1 = np.abs(host(pot1)[rows] - phi1_ref) / np.abs(phi1_ref)
    assert np.median(ep1) <= 1e-5 and ep1.max() <= 1e-3


def test_config5_hvp_262144(nb):
    n, eps = 262144, 0.005
    pos, _, m = W.plummer(n, 6)
    g = W.unit_cotangent(n, 56)
    x, mm, gg = dev(pos), dev(m), dev(g)
    h32, _, _ = nb.forces_backward(x, mm, gg, nb.gravity("fp32_fp64acc", softening=eps))
    h64, _, _ = nb.forces_backward(x, mm, gg, nb.gravity("fp64", softening=eps))
    h32, h64 = host(h32), host(h64)
    e = rel_rows(h32, h64)
    assert np.median(e) <= 1e-5 and e.max() <= 1e-3, (np.median(e), e.max())
    rows = np.sort(np.random.default_rng(56).choice(n, 256, replace=False))
    ref = oracle.gravity_adjoint(pos, m, g, eps=eps, ilist=rows)
    assert rel_rows(h64[rows], ref).max() <= 1e-11
    ref32 = oracle.gravity_adjoint(W.round_to_f32(pos), W.round_to_f32(m), W.round_to_f32(g),
                                   eps=eps, ilist=rows)
    e32 = rel_rows(h32[rows], ref32)
    assert np.median(e32) <= 1e-5 and e32.max() <= 1e-3
