"""FP64 CPU oracle for the all-pairs N-body force evaluation.

TEST INFRASTRUCTURE ONLY.  The only callers allowed are the test suite
(``tests/``), the smoke check in ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py``.  The product package never imports this
module and this module never imports the product package: the two share no
code, header, helper or constant, and meet only at the seeded input arrays.

The arithmetic lives in ``oracle.c`` (plain C, IEEE double, compensated sums
over j, OpenMP over i).  This file only builds and loads it and converts
numpy arrays to pointers.  Every function here follows the paper passage its C
counterpart cites:

* :func:`gravity` -- Eq. 1 (Section 3.3), Table 1 "Gravity (accel)", plus the
  softened potential whose negative gradient is Eq. 1;
* :func:`ljc_linear` -- Table 1 "LJC (linear)" (Coulomb with dielectric D*r
  plus Lennard-Jones), read potential-consistently;
* :func:`ljc_constant`, :func:`ljc_sigmoidal` -- Table 1 "LJC (constant)" and
  "LJC (sigmoidal)" (the latter with caller-given dielectric constants);
* :func:`leapfrog` -- the force-then-update cycle of Section 1 as
  kick-drift-kick leapfrog;
* :func:`gravity_adjoint`, :func:`ljc_adjoint` -- derivatives of the two laws
  (not in the paper; written out from the definitions above);
* :func:`ljc_excl`, :func:`ljc_adjoint_excl` -- the LJC laws and the LJC(linear)
  adjoint with per-particle exclusion lists (Section 5);
* :func:`gravity_jerk` -- Table 1 "Gravity (accel & jerk)", the GAJ kernel of
  Section 2;
* :func:`hermite`, :func:`hermite_block_init`, :func:`hermite_block` -- the
  fourth-order Hermite scheme that consumes acceleration and jerk, with a
  shared step or with block individual steps (the particle-subset setting of
  Section 3.4).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

GRAVITY = 0
LJC_LINEAR = 1
LJC_CONSTANT = 2


def build(force: bool = True) -> str:
    """Compile ``oracle.c`` into ``liboracle.so`` with gcc (IEEE, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
               "-shared", "-Wall", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build(force=False)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        I64 = ctypes.c_int64
        D = ctypes.c_double
        I = ctypes.c_int
        lib.oracle_initial_step.argtypes = [P, P, D, D]
        lib.oracle_initial_step.restype = D
        lib.oracle_aarseth_step.argtypes = [P, P, P, P, D, D]
        lib.oracle_aarseth_step.restype = D
        lib.oracle_quantise_step.argtypes = [D, D, D, D]
        lib.oracle_quantise_step.restype = D
        lib.oracle_ljc_energy_abs.argtypes = [I, P, P, P, P, I64, D, D, P, P, P, P, I]
        lib.oracle_threads.argtypes = [I]
        lib.oracle_threads.restype = I
        lib.oracle_gravity.argtypes = [P, P, I64, D, D, P, I64, I64, I64, P, P, I]
        lib.oracle_ljc_linear.argtypes = [P, P, P, P, I64, D, D, P, I64, I64, I64, P, P, I]
        lib.oracle_ljc_constant.argtypes = [P, P, P, P, I64, D, D, P, I64, P, P, I]
        lib.oracle_ljc_sigmoidal.argtypes = [P, P, P, P, I64, D, P, P, I64, P, P, I]
        lib.oracle_leapfrog.argtypes = [I, P, P, P, P, P, I64, D, D, D, ctypes.c_int32, P, I]
        lib.oracle_gravity_adjoint.argtypes = [P, P, I64, D, D, P, P, I64, P, I]
        lib.oracle_ljc_adjoint.argtypes = [P, P, P, P, I64, D, D, P, P, I64, P, P, P, P, I]
        lib.oracle_ljc_excl.argtypes = [I, P, P, P, P, I64, D, D, P, P, P, P, P, I]
        lib.oracle_ljc_adjoint_excl.argtypes = [P, P, P, P, I64, D, D, P, P, P, P, P, P, P, I]
        lib.oracle_gravity_jerk.argtypes = [P, P, P, I64, D, D, P, I64, P, P, P, I]
        lib.oracle_hermite.argtypes = [P, P, P, P, P, I64, D, D, D, ctypes.c_int32, I]
        lib.oracle_hermite_block_init.argtypes = [P, P, I64, D, D, P, P]
        lib.oracle_hermite_block.argtypes = [P, P, P, P, P, P, P, I64, D, D, D, D,
                                             ctypes.c_int32, P, P, I]
        for f in (lib.oracle_gravity, lib.oracle_ljc_linear, lib.oracle_ljc_constant,
                  lib.oracle_ljc_sigmoidal, lib.oracle_leapfrog,
                  lib.oracle_gravity_adjoint, lib.oracle_ljc_adjoint, lib.oracle_gravity_jerk,
                  lib.oracle_hermite, lib.oracle_hermite_block_init, lib.oracle_hermite_block,
                  lib.oracle_ljc_excl, lib.oracle_ljc_adjoint_excl):
            f.restype = I
        _lib = lib
    return _lib


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None and a.shape != shape:
        raise ValueError("expected shape %s, got %s" % (shape, a.shape))
    return a


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _ilist(ilist, n):
    if ilist is None:
        return None, n
    il = np.ascontiguousarray(ilist, dtype=np.int64)
    if il.size and (il.min() < 0 or il.max() >= n):
        raise ValueError("ilist out of range")
    return il, il.size


def threads(nthreads: int = 0) -> int:
    """Threads the oracle's OpenMP loops use for a request of ``nthreads`` (0 = all)."""
    return int(_load().oracle_threads(int(nthreads)))


def gravity(pos, mass, G=1.0, eps=0.0, ilist=None, jrange=None, nthreads=0):
    """Softened gravity of Eq. 1: returns (acc [ni,3], phi [ni]) in FP64.

    ``ilist`` restricts the rows (i-subset); ``jrange=(j0, j1)`` restricts the
    sources to a contiguous j range (for the replication identity of
    Section 3.4)."""
    pos = _f64(pos)
    n = pos.shape[0]
    pos = _f64(pos, (n, 3))
    mass = _f64(mass, (n,))
    il, ni = _ilist(ilist, n)
    j0, j1 = (0, n) if jrange is None else (int(jrange[0]), int(jrange[1]))
    acc = np.empty((ni, 3))
    phi = np.empty(ni)
    rc = _load().oracle_gravity(_ptr(pos), _ptr(mass), n, float(G), float(eps), _ptr(il), ni,
                                j0, j1, _ptr(acc), _ptr(phi), int(nthreads))
    if rc:
        raise ValueError("oracle_gravity rc=%d" % rc)
    return acc, phi


def ljc_linear(pos, q, sigma, epsilon, kc=332.0637, D=4.0, ilist=None, jrange=None, nthreads=0):
    """LJ + Coulomb(dielectric D*r) of Table 1: returns (force [ni,3], U_i [ni])."""
    pos = _f64(pos)
    n = pos.shape[0]
    pos = _f64(pos, (n, 3))
    q = _f64(q, (n,))
    sigma = _f64(sigma, (n,))
    epsilon = _f64(epsilon, (n,))
    il, ni = _ilist(ilist, n)
    j0, j1 = (0, n) if jrange is None else (int(jrange[0]), int(jrange[1]))
    f = np.empty((ni, 3))
    u = np.empty(ni)
    rc = _load().oracle_ljc_linear(_ptr(pos), _ptr(q), _ptr(sigma), _ptr(epsilon), n, float(kc),
                                   float(D), _ptr(il), ni, j0, j1, _ptr(f), _ptr(u), int(nthreads))
    if rc:
        raise ValueError("oracle_ljc_linear rc=%d" % rc)
    return f, u


def _ljc_args(pos, q, sigma, epsilon, ilist):
    pos = _f64(pos)
    n = pos.shape[0]
    pos = _f64(pos, (n, 3))
    q = _f64(q, (n,))
    sigma = _f64(sigma, (n,))
    epsilon = _f64(epsilon, (n,))
    il, ni = _ilist(ilist, n)
    return pos, q, sigma, epsilon, n, il, ni


def ljc_constant(pos, q, sigma, epsilon, kc=332.0637, D=4.0, ilist=None, nthreads=0):
    """LJ + Coulomb with constant dielectric D (Table 1 LJC(constant)): (force, U_i)."""
    pos, q, sigma, epsilon, n, il, ni = _ljc_args(pos, q, sigma, epsilon, ilist)
    f = np.empty((ni, 3))
    u = np.empty(ni)
    rc = _load().oracle_ljc_constant(_ptr(pos), _ptr(q), _ptr(sigma), _ptr(epsilon), n, float(kc),
                                     float(D), _ptr(il), ni, _ptr(f), _ptr(u), int(nthreads))
    if rc:
        raise ValueError("oracle_ljc_constant rc=%d" % rc)
    return f, u


def ljc_sigmoidal(pos, q, sigma, epsilon, zeta_coef, kc=332.0637, ilist=None, nthreads=0):
    """LJ + Coulomb with dielectric zeta(r) = exp(a r^3 + b r^2 + c r + d), zeta_coef = (a, b, c, d)
    (Table 1 LJC(sigmoidal), read potential-consistently): (force, U_i)."""
    pos, q, sigma, epsilon, n, il, ni = _ljc_args(pos, q, sigma, epsilon, ilist)
    zc = _f64(zeta_coef, (4,))
    f = np.empty((ni, 3))
    u = np.empty(ni)
    rc = _load().oracle_ljc_sigmoidal(_ptr(pos), _ptr(q), _ptr(sigma), _ptr(epsilon), n, float(kc),
                                      _ptr(zc), _ptr(il), ni, _ptr(f), _ptr(u), int(nthreads))
    if rc:
        raise ValueError("oracle_ljc_sigmoidal rc=%d" % rc)
    return f, u


def leapfrog(law, pos, vel, acc, params, dt, nsteps, inv_mass=None, G=1.0, eps=0.0,
             kc=332.0637, D=4.0, nthreads=0):
    """Kick-drift-kick leapfrog in FP64.  Returns (pos, vel, acc, pot) after ``nsteps``.

    ``params`` is the mass [n] for gravity, or an [n,3] array of (q, sigma,
    epsilon) for LJC(linear) and LJC(constant).  ``acc`` is a(t) on entry."""
    pos = _f64(pos).copy()
    n = pos.shape[0]
    vel = _f64(vel, (n, 3)).copy()
    acc = _f64(acc, (n, 3)).copy()
    if law == GRAVITY:
        par = _f64(params, (n,))
        c0, c1 = float(G), float(eps)
    elif law in (LJC_LINEAR, LJC_CONSTANT):
        par = np.ascontiguousarray(_f64(params, (n, 3)).T)  # q | sigma | eps blocks
        c0, c1 = float(kc), float(D)
    else:
        raise ValueError("law")
    im = None if inv_mass is None else _f64(inv_mass, (n,))
    pot = np.empty(n)
    rc = _load().oracle_leapfrog(int(law), _ptr(pos), _ptr(vel), _ptr(acc), _ptr(par), _ptr(im), n,
                                 c0, c1, float(dt), int(nsteps), _ptr(pot), int(nthreads))
    if rc:
        raise ValueError("oracle_leapfrog rc=%d" % rc)
    return pos, vel, acc, pot


def gravity_adjoint(pos, mass, g, G=1.0, eps=0.0, ilist=None, nthreads=0):
    """dL/dr for L with dL/da = g under Eq. 1 (the Hessian-vector product)."""
    pos = _f64(pos)
    n = pos.shape[0]
    pos = _f64(pos, (n, 3))
    mass = _f64(mass, (n,))
    g = _f64(g, (n, 3))
    il, ni = _ilist(ilist, n)
    out = np.empty((ni, 3))
    rc = _load().oracle_gravity_adjoint(_ptr(pos), _ptr(mass), n, float(G), float(eps), _ptr(g),
                                        _ptr(il), ni, _ptr(out), int(nthreads))
    if rc:
        raise ValueError("oracle_gravity_adjoint rc=%d" % rc)
    return out


def ljc_adjoint(pos, q, sigma, epsilon, g, kc=332.0637, D=4.0, ilist=None, nthreads=0):
    """(dL/dr [ni,3], dL/dq [ni], dL/dsigma [ni], dL/depsilon [ni]) for dL/dF = g."""
    pos = _f64(pos)
    n = pos.shape[0]
    pos = _f64(pos, (n, 3))
    q = _f64(q, (n,))
    sigma = _f64(sigma, (n,))
    epsilon = _f64(epsilon, (n,))
    g = _f64(g, (n, 3))
    il, ni = _ilist(ilist, n)
    gp = np.empty((ni, 3))
    gq = np.empty(ni)
    gs = np.empty(ni)
    ge = np.empty(ni)
    rc = _load().oracle_ljc_adjoint(_ptr(pos), _ptr(q), _ptr(sigma), _ptr(epsilon), n, float(kc),
                                    float(D), _ptr(g), _ptr(il), ni, _ptr(gp), _ptr(gq), _ptr(gs),
                                    _ptr(ge), int(nthreads))
    if rc:
        raise ValueError("oracle_ljc_adjoint rc=%d" % rc)
    return gp, gq, gs, ge


def gravity_jerk(pos, vel, mass, G=1.0, eps=0.0, ilist=None, nthreads=0):
    """(acc [ni,3], jerk [ni,3], phi [ni]) of Table 1's "Gravity (accel & jerk)"."""
    pos = _f64(pos)
    n = pos.shape[0]
    pos = _f64(pos, (n, 3))
    vel = _f64(vel, (n, 3))
    mass = _f64(mass, (n,))
    il, ni = _ilist(ilist, n)
    acc = np.empty((ni, 3))
    jerk = np.empty((ni, 3))
    phi = np.empty(ni)
    rc = _load().oracle_gravity_jerk(_ptr(pos), _ptr(vel), _ptr(mass), n, float(G), float(eps),
                                     _ptr(il), ni, _ptr(acc), _ptr(jerk), _ptr(phi), int(nthreads))
    if rc:
        raise ValueError("oracle_gravity_jerk rc=%d" % rc)
    return acc, jerk, phi


def hermite(pos, vel, acc, jerk, mass, dt, nsteps, G=1.0, eps=0.0, nthreads=0):
    """Shared-step fourth-order Hermite: returns (pos, vel, acc, jerk) after nsteps."""
    pos = _f64(pos).copy()
    n = pos.shape[0]
    vel = _f64(vel, (n, 3)).copy()
    acc = _f64(acc, (n, 3)).copy()
    jerk = _f64(jerk, (n, 3)).copy()
    mass = _f64(mass, (n,))
    rc = _load().oracle_hermite(_ptr(pos), _ptr(vel), _ptr(acc), _ptr(jerk), _ptr(mass), n,
                                float(G), float(eps), float(dt), int(nsteps), int(nthreads))
    if rc:
        raise ValueError("oracle_hermite rc=%d" % rc)
    return pos, vel, acc, jerk


def initial_step(a, j, eta_s, dt_max):
    """The block scheme's initial step estimate for one particle (before quantisation)."""
    a, j = _f64(a, (3,)), _f64(j, (3,))
    return float(_load().oracle_initial_step(_ptr(a), _ptr(j), float(eta_s), float(dt_max)))


def aarseth_step(a, j, a2, a3, eta, dt_max):
    """Aarseth's step criterion from a and its first three derivatives (before quantisation)."""
    a, j, a2, a3 = (_f64(v, (3,)) for v in (a, j, a2, a3))
    return float(_load().oracle_aarseth_step(_ptr(a), _ptr(j), _ptr(a2), _ptr(a3), float(eta),
                                             float(dt_max)))


def quantise_step(dts, dt_max, t, dt_old):
    """The block scheme's step: a power-of-two fraction of dt_max, at most dts (and at most twice
    dt_old when dt_old > 0), that divides t."""
    return float(_load().oracle_quantise_step(float(dts), float(dt_max), float(t), float(dt_old)))


def hermite_block_init(acc, jerk, eta_s, dt_max):
    """Initial block steps (t_i = 0, dt_i quantised from eta_s |a| / |jerk|)."""
    acc = _f64(acc)
    n = acc.shape[0]
    jerk = _f64(jerk, (n, 3))
    t = np.empty(n)
    dt = np.empty(n)
    rc = _load().oracle_hermite_block_init(_ptr(acc), _ptr(jerk), n, float(eta_s), float(dt_max),
                                           _ptr(t), _ptr(dt))
    if rc:
        raise ValueError("oracle_hermite_block_init rc=%d" % rc)
    return t, dt


def hermite_block(pos, vel, acc, jerk, t_i, dt_i, mass, nblocks, eta, dt_max, G=1.0, eps=0.0,
                  nthreads=0):
    """nblocks block steps of the individual-step Hermite scheme.  Returns
    (pos, vel, acc, jerk, t_i, dt_i, active_counts [nblocks], t_now)."""
    pos = _f64(pos).copy()
    n = pos.shape[0]
    vel = _f64(vel, (n, 3)).copy()
    acc = _f64(acc, (n, 3)).copy()
    jerk = _f64(jerk, (n, 3)).copy()
    t_i = _f64(t_i, (n,)).copy()
    dt_i = _f64(dt_i, (n,)).copy()
    mass = _f64(mass, (n,))
    active = np.zeros(max(int(nblocks), 1), dtype=np.int64)
    t_now = ctypes.c_double(0.0)
    rc = _load().oracle_hermite_block(_ptr(pos), _ptr(vel), _ptr(acc), _ptr(jerk), _ptr(t_i),
                                      _ptr(dt_i), _ptr(mass), n, float(G), float(eps), float(eta),
                                      float(dt_max), int(nblocks), _ptr(active),
                                      ctypes.byref(t_now), int(nthreads))
    if rc:
        raise ValueError("oracle_hermite_block rc=%d" % rc)
    return pos, vel, acc, jerk, t_i, dt_i, active[:int(nblocks)], t_now.value


def _excl(eoff, eidx, n):
    eoff = np.ascontiguousarray(eoff, dtype=np.int64)
    eidx = np.ascontiguousarray(eidx, dtype=np.int64)
    if eoff.shape != (n + 1,) or eoff[0] != 0 or np.any(np.diff(eoff) < 0) or eoff[-1] != eidx.size:
        raise ValueError("bad exclusion offsets")
    if eidx.size and (eidx.min() < 0 or eidx.max() >= n):
        raise ValueError("exclusion index out of range")
    if eidx.size == 0:
        eidx = np.zeros(1, dtype=np.int64)     # a valid pointer; never read
    return eoff, eidx


def ljc_excl(kind, pos, q, sigma, epsilon, excl_offsets, excl_index, kc=332.0637, D=4.0,
             zeta_coef=(0.0, 0.0, 0.0, 0.0), nthreads=0):
    """LJC law `kind` (LJC_LINEAR, LJC_CONSTANT or 3 = sigmoidal) with exclusion lists:
    pair (i, j) is left out of atom i's sums when j is in its list.  (force, U_i)."""
    pos, q, sigma, epsilon, n, _, _ = _ljc_args(pos, q, sigma, epsilon, None)
    eoff, eidx = _excl(excl_offsets, excl_index, n)
    zc = _f64(zeta_coef, (4,))
    f = np.empty((n, 3))
    u = np.empty(n)
    rc = _load().oracle_ljc_excl(int(kind), _ptr(pos), _ptr(q), _ptr(sigma), _ptr(epsilon), n,
                                 float(kc), float(D), _ptr(zc), _ptr(eoff), _ptr(eidx), _ptr(f),
                                 _ptr(u), int(nthreads))
    if rc:
        raise ValueError("oracle_ljc_excl rc=%d" % rc)
    return f, u


def ljc_energy_abs(kind, pos, q, sigma, epsilon, kc=332.0637, D=4.0, zeta_coef=None,
                   excl_offsets=None, excl_index=None, nthreads=0):
    """S_i = sum_{j != i} |u_ij| for LJC law `kind` (1 linear, 2 constant, 3 sigmoidal): the scale
    that bounds the rounding error of the energy sum U_i (a plain loop over the same pair energies)."""
    pos = _f64(pos)
    n = pos.shape[0]
    pos = _f64(pos, (n, 3))
    q, sigma, epsilon = _f64(q, (n,)), _f64(sigma, (n,)), _f64(epsilon, (n,))
    zc = None if zeta_coef is None else _f64(zeta_coef, (4,))
    if excl_offsets is not None:
        eoff, eidx = _excl(excl_offsets, excl_index, n)
    else:
        eoff = eidx = None
    out = np.empty(n)
    rc = _load().oracle_ljc_energy_abs(int(kind), _ptr(pos), _ptr(q), _ptr(sigma), _ptr(epsilon), n,
                                       float(kc), float(D), _ptr(zc), _ptr(eoff), _ptr(eidx),
                                       _ptr(out), int(nthreads))
    if rc:
        raise ValueError("oracle_ljc_energy_abs rc=%d" % rc)
    return out


def ljc_adjoint_excl(pos, q, sigma, epsilon, g, excl_offsets, excl_index, kc=332.0637, D=4.0,
                     nthreads=0):
    """LJC(linear) adjoint with (symmetric) exclusion lists: (dL/dr, dL/dq, dL/dsigma, dL/deps)."""
    pos, q, sigma, epsilon, n, _, _ = _ljc_args(pos, q, sigma, epsilon, None)
    g = _f64(g, (n, 3))
    eoff, eidx = _excl(excl_offsets, excl_index, n)
    gp = np.empty((n, 3))
    gq = np.empty(n)
    gs = np.empty(n)
    ge = np.empty(n)
    rc = _load().oracle_ljc_adjoint_excl(_ptr(pos), _ptr(q), _ptr(sigma), _ptr(epsilon), n,
                                         float(kc), float(D), _ptr(g), _ptr(eoff), _ptr(eidx),
                                         _ptr(gp), _ptr(gq), _ptr(gs), _ptr(ge), int(nthreads))
    if rc:
        raise ValueError("oracle_ljc_adjoint_excl rc=%d" % rc)
    return gp, gq, gs, ge
