"""Non-finite inputs and checkpoint/resume on the GPU.

* A NaN in one particle's position reaches every row of the force and the
  potential through the pair sums, as in the oracle.  A NaN in one particle's
  mass reaches every other row, while that particle's own row (which its mass
  does not enter: the self pair is skipped) stays finite and equal to the
  oracle's.
* An integrator stopped, written to a file with save_state, read back with
  load_state into fresh tensors and continued gives bit for bit the state of
  the uninterrupted run (leapfrog: 50 + 50 = 100 steps; block-step Hermite:
  20 + 20 = 40 block steps).
"""
import numpy as np
import pytest
import torch

import oracle
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


def host(t):
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("prec", ["fp64", "fp32_kahan"])
def test_nan_position_reaches_every_row(nb, prec):
    x, _, m = W.plummer(1000, 41)
    k = 417
    x[k, 1] = np.nan
    f, p = nb.forces(dev(x), dev(m), nb.gravity(prec, softening=EPS))
    a_ref, phi_ref = oracle.gravity(x, m, eps=EPS)
    assert np.isnan(a_ref).any(axis=1).all() and np.isnan(phi_ref).all()
    assert torch.isnan(f).any(dim=1).all() and torch.isnan(p).all()
    s = W.md_system(600, 42, box=30.0)
    pos = s.pos.copy()
    pos[5, 0] = np.nan
    fl, ul = nb.forces(dev(pos), dev(s.params()), nb.ljc_linear(prec))
    assert torch.isnan(fl).any(dim=1).all() and torch.isnan(ul).all()


@pytest.mark.parametrize("prec", ["fp64", "fp32_kahan"])
def test_nan_mass_spares_only_its_own_row(nb, prec):
    x, _, m = W.plummer(1000, 43)
    k = 123
    m[k] = np.nan
    f, p = nb.forces(dev(x), dev(m), nb.gravity(prec, softening=EPS))
    # the FP32 path is checked against the oracle fed the FP32-rounded inputs
    xr, mr = (x, m) if prec == "fp64" else (W.round_to_f32(x), W.round_to_f32(m))
    a_ref, phi_ref = oracle.gravity(xr, mr, eps=EPS)
    others = np.arange(len(m)) != k
    assert np.isnan(a_ref[others]).all() and np.isfinite(a_ref[k]).all()
    fh, ph = host(f), host(p)
    assert np.isnan(fh[others]).any(axis=1).all() and np.isnan(ph[others]).all()
    assert np.isfinite(fh[k]).all() and np.isfinite(ph[k])
    tol = 1e-12 if prec == "fp64" else 1e-4
    assert np.linalg.norm(fh[k] - a_ref[k]) <= tol * np.linalg.norm(a_ref[k])
    assert abs(ph[k] - phi_ref[k]) <= tol * abs(phi_ref[k])


@pytest.mark.parametrize("case", ["gravity_fp32_kahan", "ljc_linear_fp64"])
def test_leapfrog_resume_is_bitwise(nb, case, tmp_path):
    dt = 1e-3
    if case.startswith("gravity"):
        x, v, m = W.plummer(4096, 44)
        law, par, inv_mass = nb.gravity("fp32_kahan", softening=EPS), m, None
    else:
        s = W.md_system(1200, 45, box=36.0)
        x, v = s.pos, np.random.default_rng(46).normal(0.0, 0.01, (1200, 3))
        law, par, inv_mass = nb.ljc_linear("fp64"), s.params(), np.full(1200, 1.0 / 12.0)
        dt = 1e-4
    a0, _ = nb.forces(dev(x), dev(par), law)
    im = None if inv_mass is None else dev(inv_mass)
    if im is not None:
        a0 = a0 * im[:, None]
    X, V, A = dev(x), dev(v), a0.clone()
    nb.leapfrog(X, V, A, dev(par), law, dt, 100, inv_mass=im)
    Xr, Vr, Ar = dev(x), dev(v), a0.clone()
    nb.leapfrog(Xr, Vr, Ar, dev(par), law, dt, 50, inv_mass=im)
    path = tmp_path / "leapfrog_state.npz"
    nb.save_state(path, pos=Xr, vel=Vr, acc=Ar, t=50 * dt, step=50, seed=44)
    del Xr, Vr, Ar
    st = nb.load_state(path)
    assert st["step"] == 50 and st["t"] == 50 * dt and st["seed"] == 44
    nb.leapfrog(st["pos"], st["vel"], st["acc"], dev(par), law, dt, 50, inv_mass=im)
    for got, want in ((st["pos"], X), (st["vel"], V), (st["acc"], A)):
        assert torch.equal(got, want)


@pytest.mark.parametrize("prec", ["fp64", "fp32_kahan"])
def test_block_steps_resume_is_bitwise(nb, prec, tmp_path):
    x, v, m = W.plummer(2048, 47)
    eta, dt_max = 0.02, 1.0 / 16
    law = nb.gravity(prec, softening=0.02)
    A0, J0, _ = nb.forces_jerk(dev(x), dev(v), dev(m), law, potential=False)
    T0, DT0 = nb.hermite_block_init(A0.clone(), J0.clone(), 0.01, dt_max)
    full = [dev(x), dev(v), A0.clone(), J0.clone(), T0.clone(), DT0.clone()]
    c_full, t_full = nb.hermite_block(*full, dev(m), law, eta, dt_max, 40)
    part = [dev(x), dev(v), A0.clone(), J0.clone(), T0.clone(), DT0.clone()]
    c1, t1 = nb.hermite_block(*part, dev(m), law, eta, dt_max, 20)
    names = ("pos", "vel", "acc", "jerk", "t_i", "dt_i")
    path = tmp_path / "block_state.npz"
    nb.save_state(path, t=t1, **dict(zip(names, part)))
    del part
    st = nb.load_state(path)
    assert st["t"] == t1
    c2, t2 = nb.hermite_block(*(st[k] for k in names), dev(m), law, eta, dt_max, 20)
    assert np.array_equal(np.concatenate([c1, c2]), c_full) and t2 == t_full
    for k, want in zip(names, full):
        assert torch.equal(st[k], want), k
