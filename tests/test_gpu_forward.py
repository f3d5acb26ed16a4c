"""GPU parity of the forward all-pairs path (C ABI via the torch binding) against
the FP64 CPU oracle.

Tolerances: FP64 paths <= 1e-12 in the maximum per-particle relative error;
FP32 paths median <= 1e-5 and maximum <= 1e-3, measured against the oracle fed
the FP32-rounded inputs (so input quantisation is not counted).
"""
import os

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


def rel_rows(x, ref):
    return np.linalg.norm(x - ref, axis=1) / np.linalg.norm(ref, axis=1)


def rel_scalar(x, ref):
    return np.abs(x - ref) / np.abs(ref)


def test_library_is_native_and_single_runtime(nb):
    from paper_0706_3060_amd import _native
    assert _native.lib()._name.endswith("libnbody.so")
    assert "torch" in _native.runtime_path()


# ------------------------------------------------------------------ FP64
@pytest.mark.parametrize("n", [4096, 1000, 63, 64, 65, 2])
def test_gravity_fp64_matches_oracle(nb, n):
    pos, _, m = W.plummer(n, 1)
    f, p = nb.forces(dev(pos), dev(m), nb.gravity("fp64", softening=EPS))
    a_ref, phi_ref = oracle.gravity(pos, m, eps=EPS)
    assert rel_rows(host(f), a_ref).max() <= 1e-12
    assert rel_scalar(host(p), phi_ref).max() <= 1e-12


def test_gravity_fp64_one_leapfrog_step(nb):
    # N=4096 Plummer, eps=0.01, dt=1e-3: a0, phi0, then one KDK step (x1, v1, a1)
    pos, vel, m = W.plummer(4096, 1)
    law = nb.gravity("fp64", softening=EPS)
    x, v = dev(pos), dev(vel)
    a, _ = nb.forces(x, dev(m), law)
    a0_ref, _ = oracle.gravity(pos, m, eps=EPS)
    phi1 = nb.leapfrog(x, v, a, dev(m), law, 1e-3, 1, potential=True)
    xr, vr, ar, pr = oracle.leapfrog(oracle.GRAVITY, pos, vel, a0_ref, m, 1e-3, 1, eps=EPS)
    assert np.abs(host(x) - xr).max() <= 1e-12 * np.abs(xr).max()
    assert np.abs(host(v) - vr).max() <= 1e-12 * np.abs(vr).max()
    assert rel_rows(host(a), ar).max() <= 1e-12
    assert rel_scalar(host(phi1), pr).max() <= 1e-12


def test_ljc_fp64_matches_oracle(nb):
    s = W.md_system(1500, 3, box=36.0)
    f, u = nb.forces(dev(s.pos), dev(s.params()), nb.ljc_linear("fp64"))
    f_ref, u_ref = oracle.ljc_linear(s.pos, s.q, s.sigma, s.epsilon)
    assert rel_rows(host(f), f_ref).max() <= 1e-12
    assert (np.abs(host(u) - u_ref) / np.abs(u_ref).max()).max() <= 1e-12


# ------------------------------------------------------------------ FP32
@pytest.mark.parametrize("prec", ["fp32_kahan", "fp32_fp64acc"])
@pytest.mark.parametrize("n", [4096, 20000, 777])
def test_gravity_fp32_matches_oracle(nb, prec, n):
    pos, _, m = W.plummer(n, 2)
    f, p = nb.forces(dev(pos), dev(m), nb.gravity(prec, softening=EPS))
    a_ref, phi_ref = oracle.gravity(W.round_to_f32(pos), W.round_to_f32(m), eps=EPS)
    e = rel_rows(host(f), a_ref)
    ep = rel_scalar(host(p), phi_ref)
    assert np.median(e) <= 1e-5 and e.max() <= 1e-3, (np.median(e), e.max())
    assert np.median(ep) <= 1e-5 and ep.max() <= 1e-3


@pytest.mark.parametrize("prec", ["fp32_kahan", "fp32_fp64acc"])
def test_ljc_fp32_matches_oracle(nb, prec):
    s = W.md_system(3000, 5, box=45.0)
    f, u = nb.forces(dev(s.pos), dev(s.params()), nb.ljc_linear(prec))
    f_ref, u_ref = oracle.ljc_linear(W.round_to_f32(s.pos), s.q, s.sigma, s.epsilon)
    e = rel_rows(host(f), f_ref)
    assert np.median(e) <= 1e-5 and e.max() <= 1e-3, (np.median(e), e.max())
    eu = np.abs(host(u) - u_ref) / np.abs(u_ref).max()
    assert np.median(eu) <= 1e-5


def test_fp32_plain_ablation_runs(nb):
    pos, _, m = W.plummer(20000, 3)
    f, _ = nb.forces(dev(pos), dev(m), nb.gravity("fp32_plain", softening=EPS))
    a_ref, _ = oracle.gravity(W.round_to_f32(pos), W.round_to_f32(m), eps=EPS)
    e = rel_rows(host(f), a_ref)
    assert np.median(e) <= 1e-4


# ------------------------------------------------------- configurations
# splits that are multiples of 8 take the XCD-ordered block mapping (8, 24, 32, 64), the
# others the plain (row block, part) grid
CONFIGS = [(64, 1, 64, 1, 0), (256, 2, 256, 3, 0), (128, 4, 128, 7, 0), (256, 8, 512, 2, 0),
           (64, 1, 1024, 64, 0), (256, 1, 256, 1, 1), (128, 2, 64, 5, 1), (256, 4, 512, 2, 1),
           (64, 1, 64, 64, 1), (256, 1, 256, 24, 1), (128, 2, 256, 8, 0), (256, 1, 256, 32, 1)]


@pytest.mark.parametrize("cfg", CONFIGS)
def test_launch_configurations_agree(nb, cfg):
    block, ipl, jt, js, stage = cfg
    pos, _, m = W.plummer(3001, 4)
    x, mm = dev(pos), dev(m)
    law64 = nb.gravity("fp64", softening=EPS)
    law32 = nb.gravity("fp32_fp64acc", softening=EPS)
    a_ref, phi_ref = oracle.gravity(pos, m, eps=EPS)
    try:
        nb.set_config(nb.API_FORCES, block, ipl, jt, js, stage)
        f64, p64 = nb.forces(x, mm, law64)
        f32, _ = nb.forces(x, mm, law32)
        s = W.md_system(700, 12, box=30.0)
        fl, ul = nb.forces(dev(s.pos), dev(s.params()), nb.ljc_linear("fp32_kahan"))
    finally:
        nb.clear_config(nb.API_FORCES)
    assert rel_rows(host(f64), a_ref).max() <= 1e-12
    assert rel_scalar(host(p64), phi_ref).max() <= 1e-12
    a32_ref, _ = oracle.gravity(W.round_to_f32(pos), W.round_to_f32(m), eps=EPS)
    e = rel_rows(host(f32), a32_ref)
    assert np.median(e) <= 1e-5 and e.max() <= 1e-3
    fl_ref, ul_ref = oracle.ljc_linear(W.round_to_f32(s.pos), s.q, s.sigma, s.epsilon)
    el = rel_rows(host(fl), fl_ref)
    assert np.median(el) <= 1e-5 and el.max() <= 1e-3
    assert np.median(np.abs(host(ul) - ul_ref) / np.abs(ul_ref).max()) <= 1e-5


def test_j_stages_agree(nb):
    # both ways of bringing j records to the arithmetic give the same sums
    pos, _, m = W.plummer(4000, 9)
    x, mm = dev(pos), dev(m)
    law = nb.gravity("fp64", softening=EPS)
    out = []
    for stage in (0, 1):
        try:
            nb.set_config(nb.API_FORCES, 256, 1, 256, 1, stage)
            out.append(nb.forces(x, mm, law))
        finally:
            nb.clear_config(nb.API_FORCES)
    assert (out[0][0] - out[1][0]).abs().max().item() <= 1e-14 * out[0][0].abs().max().item()


def test_deterministic(nb):
    pos, _, m = W.plummer(5000, 5)
    law = nb.gravity("fp32_kahan", softening=EPS)
    f1, p1 = nb.forces(dev(pos), dev(m), law)
    f2, p2 = nb.forces(dev(pos), dev(m), law)
    assert torch.equal(f1, f2) and torch.equal(p1, p2)


def test_subset_rows(nb):
    pos, _, m = W.plummer(6000, 6)
    il = np.random.default_rng(0).integers(0, 6000, 700)
    f, p = nb.forces_subset(dev(pos), dev(m), torch.tensor(il, device="cuda"),
                            nb.gravity("fp64", softening=EPS))
    a_ref, phi_ref = oracle.gravity(pos, m, eps=EPS, ilist=il)
    assert rel_rows(host(f), a_ref).max() <= 1e-12
    assert rel_scalar(host(p), phi_ref).max() <= 1e-12


def test_edge_cases(nb):
    law = nb.gravity("fp64", softening=EPS)
    f, p = nb.forces(dev(np.zeros((0, 3))), dev(np.zeros(0)), law)
    assert f.shape == (0, 3)
    f, p = nb.forces(dev([[1.0, 2.0, 3.0]]), dev([2.0]), law)
    assert torch.all(f == 0) and torch.all(p == 0)
    # coincident particles with zero softening: undefined, as in the oracle
    f, p = nb.forces(dev(np.zeros((2, 3))), dev([1.0, 1.0]), nb.gravity("fp64", softening=0.0))
    assert not torch.isfinite(f).all()


def test_issue_rate_probe(nb):
    """The issue-rate probes behind the roofline ceiling return plausible figures: a
    wave64 FP32 FMA issues in 2 to 4 shader cycles with VGPR operands, no faster with
    an SGPR operand, v_rsq_f32 at a fraction of that rate, at a clock within the
    part's range."""
    r = nb.probe_issue_rates()
    assert 1.8 <= r["fma_cycles"] <= 4.0, r
    assert r["fma_sgpr_cycles"] >= 0.9 * r["fma_cycles"], r
    assert 2.0 * r["fma_cycles"] <= r["rsq_cycles"] <= 40.0, r
    assert 0.5 <= r["clock_ghz"] <= 3.0 and r["wall_counter_mhz"] > 0, r
    # a group of one rsq and 13 FMAs costs at least the 13 FMAs; distinct operands change
    # the FMA rate by little; the cross-lane moves cost at least a VALU slot
    assert r["rsq_13fma_cycles"] >= 12.0 * r["fma_cycles"], r
    assert 0.7 * r["fma_cycles"] <= r["fma_distinct_cycles"] <= 1.5 * r["fma_cycles"], r
    assert r["dpp_mov_cycles"] >= 0.9 * r["fma_cycles"] and r["bpermute_cycles"] > 0, r


def test_tuning_cache_round_trip(nb, tmp_path):
    """A tuned configuration saved on this GPU loads back; the same file relabelled for
    another architecture is refused."""
    x, _, m = W.plummer(2048, 21)
    law = nb.gravity("fp32_kahan", softening=0.01)
    cfg, ms = nb.autotune(dev(x), dev(m), law)
    assert ms > 0
    path = tmp_path / "tune.json"
    nb.tune_save(path)
    text = path.read_text()
    assert '"arch": "gfx950"' in text and '"device_cus": %d' % torch.cuda.get_device_properties(0).multi_processor_count in text
    nb.tune_load(path)
    other = tmp_path / "other.json"
    other.write_text(text.replace('"arch": "gfx950"', '"arch": "gfx942"'))
    with pytest.raises(RuntimeError):
        nb.tune_load(other)


@pytest.mark.parametrize("law_name", ["gravity", "ljc_linear"])
def test_permutation_and_translation_invariance(nb, law_name):
    """Permuting the particles permutes the outputs, and translating every position
    leaves them unchanged, to FP64 rounding (FP64 path; the GPU sums in another order
    after a permutation, so the comparison is to 1e-12 rather than bitwise)."""
    if law_name == "gravity":
        x, _, m = W.plummer(1500, 31)
        par = m
        law = nb.gravity("fp64", softening=EPS)
        shift = np.array([3.5, -2.25, 7.0])
    else:
        s = W.md_system(1500, 32, box=36.0)
        x, par = s.pos, s.params()
        law = nb.ljc_linear("fp64")
        shift = np.array([40.0, -25.0, 11.0])
    f0, p0 = nb.forces(dev(x), dev(par), law)
    perm = np.random.default_rng(33).permutation(len(x))
    f1, p1 = nb.forces(dev(x[perm]), dev(np.asarray(par)[perm]), law)
    f0h, p0h = host(f0), host(p0)
    assert rel_rows(host(f1), f0h[perm]).max() <= 1e-12
    assert rel_scalar(host(p1), p0h[perm]).max() <= 1e-12
    f2, p2 = nb.forces(dev(x + shift), dev(par), law)
    scale = np.abs(f0h).max()
    assert np.abs(host(f2) - f0h).max() <= 1e-12 * scale
    assert rel_scalar(host(p2), p0h).max() <= 1e-11


def test_tune_cache_environment_variable_carries_over(nb, tmp_path):
    """With NBODY_TUNE_CACHE set, an autotuning run writes the file and a later process
    reads it back: its lookup returns the tuned configuration (two child processes,
    one after the other)."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    cache = tmp_path / "cache.json"
    common = ("import sys; sys.path.insert(0, %r)\n"
              "import torch\n"
              "from paper_0706_3060_amd import nbody as nb, workloads as W\n"
              "law = nb.gravity('fp32_kahan', softening=0.01)\n" % root)
    tune = common + ("x, _, m = W.plummer(3000, 61)\n"
                     "cfg, ms = nb.autotune(torch.tensor(x, device='cuda'), torch.tensor(m, device='cuda'), law)\n"
                     "print(sorted(cfg.items()))\n")
    look = common + "print(sorted(nb.get_config(nb.API_FORCES, 3000, law).items()))\n"
    env = dict(os.environ, NBODY_TUNE_CACHE=str(cache))
    r1 = subprocess.run([sys.executable, "-c", tune], capture_output=True, text=True, env=env, timeout=240)
    assert r1.returncode == 0, r1.stderr[-2000:]
    assert cache.exists() and '"arch": "gfx950"' in cache.read_text()
    r2 = subprocess.run([sys.executable, "-c", look], capture_output=True, text=True, env=env, timeout=240)
    assert r2.returncode == 0, r2.stderr[-2000:]
    assert r2.stdout.split() == r1.stdout.split()
