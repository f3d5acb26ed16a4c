"""Synthetic-input generators and the paper's printed numbers, CPU only.

* Plummer sphere: the virial ratio, the potential energy against the model's
  closed form W = -3 pi / 32 (G = M = a = 1) and the cumulative mass profile
  M(<r) = r^3 / (1 + r^2)^(3/2).
* MD boxes: minimum separation, box bounds, neutral charge, type tables.
* Golden fixtures transcribed from the paper (Appendix flop accounting,
  Tables 1 and 2) pin the flop and interaction-count conventions the
  benchmark reports with.
"""
import os

import numpy as np
import pytest

from paper_0706_3060_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rows(name):
    out = []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                out.append(line.split())
    return out


def test_plummer_virial_and_potential(oracle_mod):
    pos, vel, m = W.plummer(8192, 1)
    assert np.allclose(m, 1.0 / 8192)
    np.testing.assert_allclose((m[:, None] * pos).sum(0), 0, atol=1e-12)
    np.testing.assert_allclose((m[:, None] * vel).sum(0), 0, atol=1e-12)
    _, phi = oracle_mod.gravity(pos, m, eps=1e-4)
    Wpot = 0.5 * (m * phi).sum()
    T = 0.5 * (m * (vel * vel).sum(1)).sum()
    assert abs(Wpot - (-3 * np.pi / 32)) < 0.03 * 3 * np.pi / 32
    assert abs(2 * T / abs(Wpot) - 1.0) < 0.06


def test_plummer_mass_profile():
    from scipy import stats
    pos, _, _ = W.plummer(20000, 2)
    r = np.linalg.norm(pos, axis=1)
    cdf = lambda x: (x ** 3 / (1 + x * x) ** 1.5) / 0.999
    assert stats.kstest(r, cdf).pvalue > 1e-3


def test_plummer_is_seeded():
    a = W.plummer(100, 7)
    b = W.plummer(100, 7)
    c = W.plummer(100, 8)
    for x, y in zip(a, b):
        np.testing.assert_array_equal(x, y)
    assert not np.array_equal(a[0], c[0])


def test_md_system_constraints():
    from scipy.spatial.distance import pdist
    s = W.md_system(1500, 3, box=36.0)
    assert s.pos.shape == (1500, 3)
    assert s.pos.min() >= 0 and s.pos.max() < 36.0
    assert pdist(s.pos).min() >= 2.5
    assert abs(s.q.sum()) < 1e-12 and np.abs(s.q).max() <= 1.6
    np.testing.assert_allclose(s.sigma_t, [3.0, 3.0 + 0.8 / 3, 3.0 + 1.6 / 3, 3.8])
    np.testing.assert_allclose(s.eps_t, [0.05, 0.1, 0.15, 0.2])
    p = s.params()
    np.testing.assert_array_equal(p[:, 1], s.sigma_t[s.types])
    t = W.perturbed(s, 33)
    assert np.all(np.abs(t.q / s.q - 1) <= 0.05 + 1e-12)
    assert np.all(np.abs(t.sigma_t / s.sigma_t - 1) <= 0.05 + 1e-12)


def test_batched_md_layout():
    off, pos, par, systems = W.batched_md(5, seed=4, n_min=20, n_max=60, workers=1)
    assert off[0] == 0 and np.all(np.diff(off) >= 20) and off[-1] == pos.shape[0] == par.shape[0]
    for s, sy in enumerate(systems):
        np.testing.assert_array_equal(pos[off[s]:off[s + 1]], sy.pos)
        assert abs(sy.box ** 3 / sy.n - 32.0) < 1e-9


def test_unit_cotangent():
    g = W.unit_cotangent(1000, 56)
    assert g.shape == (1000, 3)
    np.testing.assert_allclose(np.linalg.norm(g), 1.0, rtol=1e-14)


def test_appendix_flop_accounting():
    rows = _rows("appendix_ga_flops.txt")
    total = sum(int(r[1]) for r in rows)
    assert total == 76 and total / 4 == 19


def test_table1_transcription():
    for name, flops, _, _, _, _, gflops, gint, _ in _rows("table1_kernels.txt"):
        assert abs(float(flops) * float(gint) - float(gflops)) <= 0.012 * float(gflops), name


def test_table2_interaction_convention():
    # N^2 interactions per force evaluation, one evaluation per 2 fs step
    for name, mint, nsday, atoms in _rows("table2_md.txt"):
        steps_per_s = float(mint) * 1e6 / float(atoms) ** 2
        assert abs(steps_per_s * 86400 * 2e-6 - float(nsday)) <= 0.01 * float(nsday), name
