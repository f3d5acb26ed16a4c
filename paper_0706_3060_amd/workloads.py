"""Seeded synthetic inputs shaped like the paper's two workloads.

This module only draws inputs: it holds none of the force, potential, update
or adjoint arithmetic, and it imports neither the HIP binding nor the oracle,
so that both sides can be fed the very same arrays.  Everything is drawn with
numpy's PCG64 (``numpy.random.default_rng(seed)``).

* Stellar dynamics (Section 1; the gravity kernels of Table 1): a Plummer
  sphere of scale radius 1 with equal masses 1/N, sampled with the method of
  Aarseth, Henon and Wielen (1974), G = M = a = 1, radii truncated at mass
  fraction 0.999, equilibrium velocities, centre of mass at rest at the origin.
* Continuum-solvent molecular dynamics (Section 2; the LJC kernels of
  Table 1): atoms placed uniformly in a cube by random sequential addition
  with a minimum pair separation, four Lennard-Jones types, charges uniform in
  [-qmax, qmax] shifted to zero net charge.
"""
from __future__ import annotations

import multiprocessing
import os
import sys
from dataclasses import dataclass

import numpy as np

COULOMB_K = 332.0637        # kcal * Angstrom / (mol * e^2)


def _unit_vectors(rng, n):
    z = rng.uniform(-1.0, 1.0, n)
    phi = rng.uniform(0.0, 2.0 * np.pi, n)
    s = np.sqrt(1.0 - z * z)
    return np.stack([s * np.cos(phi), s * np.sin(phi), z], axis=1)


def plummer(n: int, seed: int, max_mass_fraction: float = 0.999):
    """Plummer sphere (G = M = a = 1): returns (pos [n,3], vel [n,3], mass [n])."""
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.0, max_mass_fraction, n)
    x = np.maximum(x, 1e-300)
    r = 1.0 / np.sqrt(x ** (-2.0 / 3.0) - 1.0)
    pos = r[:, None] * _unit_vectors(rng, n)
    # speed fraction q from the density q^2 (1 - q^2)^(7/2) by rejection (bound 0.1)
    q = np.empty(n)
    filled = 0
    while filled < n:
        m = max(2 * (n - filled), 64)
        a = rng.uniform(0.0, 1.0, m)
        b = rng.uniform(0.0, 0.1, m)
        ok = a[b < a * a * (1.0 - a * a) ** 3.5]
        take = min(ok.size, n - filled)
        q[filled:filled + take] = ok[:take]
        filled += take
    vesc = np.sqrt(2.0) * (1.0 + r * r) ** (-0.25)
    vel = (q * vesc)[:, None] * _unit_vectors(rng, n)
    mass = np.full(n, 1.0 / n)
    pos -= (mass[:, None] * pos).sum(0) / mass.sum()
    vel -= (mass[:, None] * vel).sum(0) / mass.sum()
    return pos, vel, mass


def random_sequential_addition(n: int, box: float, min_sep: float, rng, batch: int = 1024,
                               max_tries: int = 100_000_000):
    """n points uniform in [0, box)^3 with no pair closer than ``min_sep`` (open box).

    Random sequential addition: candidates are drawn uniformly and accepted in
    draw order when they keep the minimum separation from every point accepted
    before them.  Candidates are handled in batches only for speed; the
    acceptance rule is the sequential one."""
    cell = min_sep / np.sqrt(3.0)          # a cell holds at most one point
    nc = max(int(np.floor(box / cell)), 1)
    cell = box / nc
    reach = int(np.ceil(min_sep / cell))
    grid = -np.ones((nc + 2 * reach,) * 3, dtype=np.int64)
    pts = np.zeros((n, 3))
    count = 0
    tries = 0
    off = np.arange(-reach, reach + 1)
    ox, oy, oz = np.meshgrid(off, off, off, indexing="ij")
    offs = np.stack([ox.ravel(), oy.ravel(), oz.ravel()], axis=1)
    d2min = min_sep * min_sep
    while count < n:
        if tries > max_tries:
            raise RuntimeError("random sequential addition jammed at %d of %d points" % (count, n))
        cand = rng.uniform(0.0, box, (batch, 3))
        tries += batch
        ci = np.minimum((cand / cell).astype(np.int64), nc - 1) + reach
        nb = ci[:, None, :] + offs[None, :, :]
        occ = grid[nb[..., 0], nb[..., 1], nb[..., 2]]
        has = occ >= 0
        other = pts[np.where(has, occ, 0)]
        d2 = ((other - cand[:, None, :]) ** 2).sum(-1)
        keep = np.nonzero(~(has & (d2 < d2min)).any(1))[0]
        if keep.size == 0:
            continue
        c = cand[keep]
        dd = ((c[:, None, :] - c[None, :, :]) ** 2).sum(-1)
        earlier = np.tril(dd < d2min, k=-1)          # earlier[b, a]: a < b and too close
        accepted = np.ones(keep.size, dtype=bool)
        for b in np.nonzero(earlier.any(1))[0]:
            accepted[b] = not (earlier[b] & accepted).any()
        idx = keep[accepted][: n - count]
        k = idx.size
        pts[count:count + k] = cand[idx]
        grid[ci[idx, 0], ci[idx, 1], ci[idx, 2]] = np.arange(count, count + k)
        count += k
    return pts


@dataclass
class MDSystem:
    """One continuum-solvent LJC system: positions [n,3], per-atom (q, sigma, eps) and types."""
    pos: np.ndarray
    q: np.ndarray
    types: np.ndarray
    sigma_t: np.ndarray
    eps_t: np.ndarray
    box: float

    @property
    def n(self):
        return self.pos.shape[0]

    @property
    def sigma(self):
        return self.sigma_t[self.types]

    @property
    def epsilon(self):
        return self.eps_t[self.types]

    def params(self):
        """Per-atom parameter rows (q, sigma, epsilon) as an [n,3] FP64 array."""
        return np.ascontiguousarray(np.stack([self.q, self.sigma, self.epsilon], axis=1))


def md_system(n: int, seed: int, box: float = 64.0, min_sep: float = 2.5, qmax: float = 0.8,
              n_types: int = 4) -> MDSystem:
    """Uniform atoms in a cube (random sequential addition), 4 LJ types, neutral charges."""
    rng = np.random.default_rng(seed)
    pos = random_sequential_addition(n, box, min_sep, rng)
    types = rng.integers(0, n_types, n)
    q = rng.uniform(-qmax, qmax, n)
    if n:
        q -= q.mean()
    sig = np.linspace(3.0, 3.8, n_types)
    eps = np.linspace(0.05, 0.2, n_types)
    return MDSystem(pos=pos, q=q, types=types.astype(np.int32), sigma_t=sig, eps_t=eps, box=box)


def bonded_chains(n_chains: int, chain_len: int, seed: int, box: float = None,
                  density: float = 1.0 / 32.0, bond: float = 1.53, angle_deg: float = 111.0,
                  min_sep: float = 2.5, qmax: float = 0.8, n_types: int = 4, excl_depth: int = 2):
    """Synthetic bonded molecules: ``n_chains`` linear chains of ``chain_len`` atoms in a cube.

    Each chain grows as a fixed-bond, fixed-angle walk (bond length ``bond`` A, bond angle
    ``angle_deg``, uniformly random dihedral) and every new atom keeps ``min_sep`` from every
    atom placed before it except its own bonded predecessor.  Atoms are numbered chain by
    chain.  The exclusion list of atom i holds the atoms of its chain within ``excl_depth``
    bonds (1-2 and 1-3 pairs for depth 2), so the lists are symmetric.  Types, charges and the
    per-type sigma / epsilon follow the md_system recipe.
    Returns (MDSystem, excl_offsets [n+1] int64, excl_index [nnz] int64)."""
    rng = np.random.default_rng(seed)
    n = n_chains * chain_len
    if box is None:
        box = (max(n, 1) / density) ** (1.0 / 3.0)
    cell = min_sep
    grid = {}
    pts = np.zeros((n, 3))
    d2min = min_sep * min_sep
    cos_t, sin_t = np.cos(np.radians(angle_deg)), np.sin(np.radians(angle_deg))

    def clear(p, skip):
        c = np.floor(p / cell).astype(np.int64)
        for dx in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dz in (-1, 0, 1):
                    for k in grid.get((c[0] + dx, c[1] + dy, c[2] + dz), ()):
                        if k != skip and ((pts[k] - p) ** 2).sum() < d2min:
                            return False
        return True

    def put(k, p):
        pts[k] = p
        c = np.floor(p / cell).astype(np.int64)
        grid.setdefault((c[0], c[1], c[2]), []).append(k)

    def unit(v):
        return v / np.linalg.norm(v)

    k = 0
    for _ in range(n_chains):
        for attempt in range(1000):
            start = k
            placed = []
            ok = True
            for a in range(chain_len):
                for _try in range(100):
                    if a == 0:
                        p = rng.uniform(0.0, box, 3)
                    elif a == 1:
                        p = pts[k - 1] + bond * unit(rng.standard_normal(3))
                    else:
                        b1 = unit(pts[k - 1] - pts[k - 2])
                        e1 = unit(np.cross(b1, rng.standard_normal(3)))
                        # the next bond makes angle_deg with the previous one (reversed)
                        p = pts[k - 1] + bond * (-cos_t * b1 + sin_t * e1)
                    if clear(p, k - 1 if a > 0 else -1):
                        break
                else:
                    ok = False
                    break
                put(k, p)
                placed.append(k)
                k += 1
            if ok:
                break
            for idx in placed:                      # undo the failed chain
                c = np.floor(pts[idx] / cell).astype(np.int64)
                grid[(c[0], c[1], c[2])].remove(idx)
            k = start
        else:
            raise RuntimeError("could not place a chain")
    types = rng.integers(0, n_types, n).astype(np.int32)
    q = rng.uniform(-qmax, qmax, n)
    if n:
        q -= q.mean()
    sys_ = MDSystem(pos=pts, q=q, types=types, sigma_t=np.linspace(3.0, 3.8, n_types),
                    eps_t=np.linspace(0.05, 0.2, n_types), box=box)
    lists = []
    for i in range(n):
        c0 = (i // chain_len) * chain_len
        lists.append([j for j in range(max(c0, i - excl_depth), min(c0 + chain_len, i + excl_depth + 1))
                      if j != i])
    eoff = np.zeros(n + 1, dtype=np.int64)
    eoff[1:] = np.cumsum([len(l) for l in lists])
    eidx = np.array([j for l in lists for j in l], dtype=np.int64)
    return sys_, eoff, eidx


def perturbed(sys: MDSystem, seed: int, rel: float = 0.05) -> MDSystem:
    """Same atoms, parameters scaled by (1 + rel*xi), xi ~ U[-1, 1] (charges per atom,
    sigma and epsilon per type)."""
    rng = np.random.default_rng(seed)
    q = sys.q * (1.0 + rel * rng.uniform(-1.0, 1.0, sys.n))
    st = sys.sigma_t * (1.0 + rel * rng.uniform(-1.0, 1.0, sys.sigma_t.size))
    et = sys.eps_t * (1.0 + rel * rng.uniform(-1.0, 1.0, sys.eps_t.size))
    return MDSystem(pos=sys.pos, q=q, types=sys.types, sigma_t=st, eps_t=et, box=sys.box)


def ensemble_sizes(n_systems: int = 256, seed: int = 4, n_min: int = 500, n_max: int = 5000):
    """The system sizes of batched_md's ensemble: N_s ~ U{n_min .. n_max}, int64 [n_systems]."""
    rng = np.random.default_rng(seed)
    return rng.integers(n_min, n_max + 1, n_systems).astype(np.int64)


def batched_md(n_systems: int = 256, seed: int = 4, n_min: int = 500, n_max: int = 5000,
               density: float = 1.0 / 32.0, sizes=None, workers=None):
    """Ensemble of independent LJC systems at constant density.

    System s is drawn with seed ``seed*1000 + s`` in a cube of side (N_s/density)^(1/3).
    Systems are independent, so they are drawn in a fork pool of ``workers``
    processes when no GPU context exists yet in this process (a forked child of
    a process holding a GPU context is not safe).
    Returns (offsets [S+1] int64, pos [sum N,3], params [sum N,3], systems)."""
    if sizes is None:
        sizes = ensemble_sizes(n_systems, seed, n_min, n_max)
    sizes = np.asarray(sizes, dtype=np.int64)
    jobs = [(int(ns), seed * 1000 + s, (ns / density) ** (1.0 / 3.0) if ns > 0 else 1.0)
            for s, ns in enumerate(sizes)]
    if workers is None:
        workers = min(16, os.cpu_count() or 1)
    if workers > 1 and len(jobs) > 1 and _fork_is_safe():
        ctx = multiprocessing.get_context("fork")
        with ctx.Pool(min(workers, len(jobs))) as pool:
            systems = pool.starmap(_md_job, jobs)
    else:
        systems = [_md_job(*j) for j in jobs]
    offsets = np.zeros(len(sizes) + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(sizes)
    pos = np.concatenate([m.pos for m in systems]) if len(systems) else np.zeros((0, 3))
    params = np.concatenate([m.params() for m in systems]) if len(systems) else np.zeros((0, 3))
    return offsets, np.ascontiguousarray(pos), np.ascontiguousarray(params), systems


def _md_job(n, seed, box):
    return md_system(n, seed, box=box)


def _fork_is_safe():
    torch = sys.modules.get("torch")
    if torch is None:
        return True
    try:
        return not torch.cuda.is_initialized()
    except Exception:
        return False


def unit_cotangent(n: int, seed: int):
    """g ~ N(0, I_{3n}) scaled to unit 2-norm, shaped [n,3]."""
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((n, 3))
    nrm = np.linalg.norm(g)
    return g / nrm if nrm > 0 else g


def round_to_f32(a):
    """The FP64 values an FP32 path actually sees (inputs rounded once to nearest FP32)."""
    return np.asarray(a, dtype=np.float64).astype(np.float32).astype(np.float64)
