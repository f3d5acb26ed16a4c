"""Torch-facing binding of libnbody.so: argument marshalling only.

Every step of the computation (packing, the all-pairs kernels, reductions,
the leapfrog update, the adjoint, the per-type gradient sums) runs in the HIP
kernels of libnbody.so.  PyTorch supplies device memory (inputs, outputs and
the workspace) and the current stream.  There is no CPU or PyTorch fallback:
when the library is missing, or a tensor is not on a GPU, the call raises.

Laws (see include/nbody.h for the full statement and citations):
  gravity:       Eq. 1 softened gravity, params = masses [N]; with forces_jerk
                 also its time derivative (Table 1 "Gravity (accel & jerk)")
  ljc_linear, ljc_constant, ljc_sigmoidal:
                 Table 1's LJC laws, params = [N, 3] rows (q, sigma, epsilon)
Integrators: leapfrog (kick-drift-kick), hermite (fourth-order Hermite, shared
step) and hermite_block (Hermite with block individual steps).
Checkpoints: save_state / load_state write and read an integrator's state as a
plain .npz file.
"""
from __future__ import annotations

import ctypes
import math
from dataclasses import dataclass

import numpy as np
import torch

from . import _native as N

GRAVITY, LJC_LINEAR, LJC_CONSTANT, LJC_SIGMOIDAL = 0, 1, 2, 3
FP64, FP32_KAHAN, FP32_FP64ACC, FP32_PLAIN = 0, 1, 2, 3
API_FORCES, API_BATCHED, API_BACKWARD, API_LEAPFROG = (N.API_FORCES, N.API_BATCHED,
                                                       N.API_BACKWARD, N.API_LEAPFROG)
API_JERK, API_HERMITE, API_BACKWARD_BATCHED = N.API_JERK, N.API_HERMITE, N.API_BACKWARD_BATCHED


@dataclass
class Exclusions:
    """Per-particle exclusion lists (bonded pairs left out of the LJC sums; Section 5):
    particle x excludes index[offsets[x]:offsets[x+1]].  `offsets` [n+1] and `index`
    [count] are int64 GPU tensors (index may be None when there are no entries)."""
    offsets: torch.Tensor
    index: torch.Tensor = None

    def c(self, n):
        off = self.offsets
        if not (isinstance(off, torch.Tensor) and off.is_cuda and off.dtype == torch.int64
                and off.is_contiguous() and tuple(off.shape) == (n + 1,)):
            raise ValueError("exclusion offsets must be a contiguous int64 GPU tensor of shape (%d,)"
                             % (n + 1))
        idx = self.index
        count = 0
        if idx is not None:
            if not (isinstance(idx, torch.Tensor) and idx.is_cuda and idx.dtype == torch.int64
                    and idx.is_contiguous() and idx.dim() == 1):
                raise ValueError("exclusion index must be a contiguous 1-d int64 GPU tensor")
            count = idx.numel()
        return N.NBodyExclusions(_ptr(off), _ptr(idx) if count else None, count)
PRECISIONS = {"fp64": FP64, "fp32_kahan": FP32_KAHAN, "fp32_fp64acc": FP32_FP64ACC,
              "fp32_plain": FP32_PLAIN}


@dataclass(frozen=True)
class Law:
    kind: int = GRAVITY
    precision: int = FP32_FP64ACC
    G: float = 1.0
    softening: float = 0.0
    coulomb_k: float = 332.0637
    dielectric: float = 4.0
    zeta: tuple = (0.0, 0.0, 0.0, 0.0)

    def c(self) -> N.NBodyLaw:
        return N.NBodyLaw(self.kind, self.precision, self.G, self.softening, self.coulomb_k,
                          self.dielectric, (ctypes.c_double * 4)(*[float(z) for z in self.zeta]))

    @property
    def n_params(self) -> int:
        return 1 if self.kind == GRAVITY else 3


def gravity(precision=FP32_FP64ACC, G=1.0, softening=0.0) -> Law:
    return Law(GRAVITY, PRECISIONS.get(precision, precision), float(G), float(softening))


def ljc_linear(precision=FP32_FP64ACC, coulomb_k=332.0637, dielectric=4.0) -> Law:
    """Table 1 LJC(linear): Coulomb with dielectric D r plus Lennard-Jones."""
    return Law(LJC_LINEAR, PRECISIONS.get(precision, precision), 1.0, 0.0, float(coulomb_k),
               float(dielectric))


def ljc_constant(precision=FP32_FP64ACC, coulomb_k=332.0637, dielectric=4.0) -> Law:
    """Table 1 LJC(constant): Coulomb with a constant dielectric D plus Lennard-Jones."""
    return Law(LJC_CONSTANT, PRECISIONS.get(precision, precision), 1.0, 0.0, float(coulomb_k),
               float(dielectric))


def ljc_sigmoidal(zeta, precision=FP32_FP64ACC, coulomb_k=332.0637) -> Law:
    """Table 1 LJC(sigmoidal): dielectric zeta(r) = exp(z0 r^3 + z1 r^2 + z2 r + z3)."""
    z = tuple(float(v) for v in zeta)
    if len(z) != 4:
        raise ValueError("zeta needs four coefficients")
    return Law(LJC_SIGMOIDAL, PRECISIONS.get(precision, precision), 1.0, 0.0, float(coulomb_k),
               1.0, z)


# ------------------------------------------------------------------ helpers
def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _raw_stream(device) -> int:
    """The handle of torch's current stream on `device` (the raw value, without building a
    torch Stream object, which costs tens of microseconds per call)."""
    idx = device.index if isinstance(device, torch.device) else device
    if idx is None:
        idx = torch.cuda.current_device()
    return torch._C._cuda_getCurrentRawStream(idx)


def _stream(device):
    return ctypes.c_void_p(_raw_stream(device))


def _dev_f64(t, shape, name, device=None):
    if not isinstance(t, torch.Tensor):
        t = torch.as_tensor(t, dtype=torch.float64, device=device)
    if not t.is_cuda:
        raise ValueError("%s must be a GPU tensor (got %s)" % (name, t.device))
    if t.dtype != torch.float64:
        t = t.to(torch.float64)
    t = t.contiguous()
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError("%s must have shape %s, got %s" % (name, tuple(shape), tuple(t.shape)))
    return t


def _params(params, n, law, device):
    p = params if isinstance(params, torch.Tensor) else torch.as_tensor(params, device=device)
    if law.kind == GRAVITY and p.dim() == 1:
        p = p.reshape(n, 1)
    return _dev_f64(p, (n, law.n_params), "params")


_ws = {}


def workspace(api, n_total, n_systems, law: Law, device) -> torch.Tensor:
    """A cached uint8 device buffer at least nbody_workspace_bytes() long (per device and stream)."""
    nbytes = N.lib().nbody_workspace_bytes(api, int(n_total), int(n_systems), ctypes.byref(law.c()))
    if nbytes == 0 and n_total > 0:
        raise ValueError("invalid workspace request")
    dev = torch.device(device)
    key = (dev.index, _raw_stream(dev))
    buf = _ws.get(key)
    if buf is None or buf.numel() < nbytes:
        buf = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=dev)
        _ws[key] = buf
    return buf


def clear_workspace_cache():
    _ws.clear()


# --------------------------------------------------------------- forward
def forces(pos, params, law: Law, potential: bool = True, out=None, exclusions: Exclusions = None):
    """All-pairs forces (gravity: accelerations) and optionally potentials, with optional
    exclusion lists (LJC laws).

    Returns (force [N,3] float64, potential [N] float64 or None)."""
    pos = _dev_f64(pos, None, "pos")
    n = pos.shape[0]
    pos = _dev_f64(pos, (n, 3), "pos")
    par = _params(params, n, law, pos.device)
    f = out if out is not None else torch.empty((n, 3), dtype=torch.float64, device=pos.device)
    p = torch.empty(n, dtype=torch.float64, device=pos.device) if potential else None
    ws = workspace(API_FORCES, n, 1, law, pos.device)
    if exclusions is None:
        N.check(N.lib().nbody_forces(_ptr(pos), _ptr(par), n, ctypes.byref(law.c()), _ptr(f), _ptr(p),
                                     _ptr(ws), ws.numel(), _stream(pos.device)))
    else:
        ex = exclusions.c(n)
        N.check(N.lib().nbody_forces_excl(_ptr(pos), _ptr(par), n, ctypes.byref(ex),
                                          ctypes.byref(law.c()), _ptr(f), _ptr(p), _ptr(ws),
                                          ws.numel(), _stream(pos.device)))
    return f, p


def forces_noalloc(pos, params, law: Law, potential: bool = True, out=None):
    """forces() through the allocation-free entry point: no workspace, the library's device
    scratch area instead (n limited by its size; calls overlapping on one GPU race).  ``out``
    optionally gives preallocated (force [n,3], potential [n] or None) tensors, so that a
    caller under graph capture allocates nothing either."""
    pos = _dev_f64(pos, None, "pos")
    n = pos.shape[0]
    pos = _dev_f64(pos, (n, 3), "pos")
    par = _params(params, n, law, pos.device)
    if out is None:
        f = torch.empty((n, 3), dtype=torch.float64, device=pos.device)
        p = torch.empty(n, dtype=torch.float64, device=pos.device) if potential else None
    else:
        f, p = out
    N.check(N.lib().nbody_forces_noalloc(_ptr(pos), _ptr(par), n, ctypes.byref(law.c()), _ptr(f),
                                         _ptr(p), _stream(pos.device)))
    return f, p


def forces_subset(pos, params, ilist, law: Law, potential: bool = True):
    """Forces on particles ilist (int64 indices) against all particles (block time step)."""
    pos = _dev_f64(pos, None, "pos")
    n = pos.shape[0]
    pos = _dev_f64(pos, (n, 3), "pos")
    par = _params(params, n, law, pos.device)
    il = torch.as_tensor(ilist, device=pos.device).to(torch.int64).contiguous()
    ni = il.numel()
    if ni and _checks_values() and (int(il.min()) < 0 or int(il.max()) >= n):
        raise ValueError("ilist indices must lie in [0, %d)" % n)
    f = torch.empty((ni, 3), dtype=torch.float64, device=pos.device)
    p = torch.empty(ni, dtype=torch.float64, device=pos.device) if potential else None
    ws = workspace(API_FORCES, max(n, ni), 1, law, pos.device)
    N.check(N.lib().nbody_forces_subset(_ptr(pos), _ptr(par), n, _ptr(il), ni,
                                        ctypes.byref(law.c()), _ptr(f), _ptr(p), _ptr(ws),
                                        ws.numel(), _stream(pos.device)))
    return f, p


def forces_share(pos, params, law: Law, share: int, n_shares: int, potential: bool = True):
    """Share `share` of `n_shares` of a gravity or LJC(linear) evaluation over unordered pairs (what one of
    n_shares GPUs would evaluate): per-row partial sums of every row; the shares' outputs add
    up to forces()."""
    pos = _dev_f64(pos, None, "pos")
    n = pos.shape[0]
    pos = _dev_f64(pos, (n, 3), "pos")
    par = _params(params, n, law, pos.device)
    f = torch.empty((n, 3), dtype=torch.float64, device=pos.device)
    p = torch.empty(n, dtype=torch.float64, device=pos.device) if potential else None
    ws = workspace(API_FORCES, n, 1, law, pos.device)
    N.check(N.lib().nbody_forces_share(_ptr(pos), _ptr(par), n, ctypes.byref(law.c()), int(share),
                                       int(n_shares), _ptr(f), _ptr(p), _ptr(ws), ws.numel(),
                                       _stream(pos.device)))
    return f, p


def _host_offsets(offsets):
    if isinstance(offsets, torch.Tensor):
        offsets = offsets.detach().cpu().numpy()
    return np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))


def forces_batched(offsets, pos, params, law: Law, potential: bool = True,
                   exclusions: Exclusions = None):
    """Forces of independent systems (rows offsets[s]..offsets[s+1]) in one persistent launch,
    with optional exclusion lists over the concatenated rows."""
    off = _host_offsets(offsets)
    S = off.size - 1
    pos = _dev_f64(pos, None, "pos")
    n = pos.shape[0]
    if S < 0 or (S >= 0 and off[-1] != n):
        raise ValueError("offsets[-1] must equal the number of rows of pos")
    pos = _dev_f64(pos, (n, 3), "pos")
    par = _params(params, n, law, pos.device)
    f = torch.empty((n, 3), dtype=torch.float64, device=pos.device)
    p = torch.empty(n, dtype=torch.float64, device=pos.device) if potential else None
    ws = workspace(API_BATCHED, n, S, law, pos.device)
    if exclusions is None:
        N.check(N.lib().nbody_forces_batched(off.ctypes.data_as(ctypes.c_void_p), S, _ptr(pos),
                                             _ptr(par), ctypes.byref(law.c()), _ptr(f), _ptr(p),
                                             _ptr(ws), ws.numel(), _stream(pos.device)))
    else:
        ex = exclusions.c(n)
        N.check(N.lib().nbody_forces_batched_excl(off.ctypes.data_as(ctypes.c_void_p), S, _ptr(pos),
                                                  _ptr(par), ctypes.byref(ex), ctypes.byref(law.c()),
                                                  _ptr(f), _ptr(p), _ptr(ws), ws.numel(),
                                                  _stream(pos.device)))
    return f, p


# --------------------------------------------------------------- adjoint
def _checks_values():
    """Whether a value check may read device data back: not while a stream is captured (the
    library keeps such inputs in bounds itself: out-of-range types are not counted, row indices
    are clamped to the records)."""
    return not torch.cuda.is_current_stream_capturing()


def _types(types, n, n_types, dev):
    if types is None:
        return None, None
    ty = torch.as_tensor(types, device=dev).to(torch.int32).contiguous()
    if ty.shape != (n,):
        raise ValueError("types must have shape (%d,)" % n)
    if n and _checks_values() and (int(ty.min()) < 0 or int(ty.max()) >= n_types):
        raise ValueError("types must lie in [0, n_types)")
    return ty, torch.empty((int(n_types), 2), dtype=torch.float64, device=dev)


def forces_backward_batched(offsets, pos, params, grad_force, law: Law, want_pos=True,
                            want_params=None, types=None, n_types=0, exclusions: Exclusions = None):
    """Adjoint of forces_batched() (optionally with exclusion lists), every system in one
    persistent launch: (dL/dpos [N,3] or None, dL/dparams [N,P] or None, per-type
    (dL/dsigma, dL/depsilon) [n_types, 2] summed over all systems, or None)."""
    off = _host_offsets(offsets)
    S = off.size - 1
    pos = _dev_f64(pos, None, "pos")
    n = pos.shape[0]
    if S < 0 or off[-1] != n:
        raise ValueError("offsets[-1] must equal the number of rows of pos")
    pos = _dev_f64(pos, (n, 3), "pos")
    par = _params(params, n, law, pos.device)
    g = _dev_f64(grad_force, (n, 3), "grad_force")
    if want_params is None:
        want_params = law.kind != GRAVITY
    dev = pos.device
    gp = torch.empty((n, 3), dtype=torch.float64, device=dev) if want_pos else None
    gq = torch.empty((n, law.n_params), dtype=torch.float64, device=dev) if want_params else None
    ty, gt = _types(types, n, n_types, dev)
    ex = exclusions.c(n) if exclusions is not None else None
    ws = workspace(API_BACKWARD_BATCHED, n, S, law, dev)
    N.check(N.lib().nbody_forces_backward_batched(
        off.ctypes.data_as(ctypes.c_void_p), S, _ptr(pos), _ptr(par),
        ctypes.byref(ex) if ex is not None else None, ctypes.byref(law.c()), _ptr(g), _ptr(gp),
        _ptr(gq), _ptr(ty), int(n_types), _ptr(gt), _ptr(ws), ws.numel(), _stream(dev)))
    return gp, gq, gt


def forces_backward(pos, params, grad_force, law: Law, want_pos=True, want_params=None,
                    types=None, n_types=0, exclusions: Exclusions = None):
    """Adjoint of forces(): returns (dL/dpos [N,3] or None, dL/dparams [N,P] or None,
    per-type (dL/dsigma, dL/depsilon) [n_types, 2] or None)."""
    pos = _dev_f64(pos, None, "pos")
    n = pos.shape[0]
    pos = _dev_f64(pos, (n, 3), "pos")
    par = _params(params, n, law, pos.device)
    g = _dev_f64(grad_force, (n, 3), "grad_force")
    if want_params is None:
        want_params = law.kind != GRAVITY
    dev = pos.device
    gp = torch.empty((n, 3), dtype=torch.float64, device=dev) if want_pos else None
    gq = torch.empty((n, law.n_params), dtype=torch.float64, device=dev) if want_params else None
    ty, gt = _types(types, n, n_types, dev)
    ws = workspace(API_BACKWARD, n, 1, law, dev)
    if exclusions is None:
        N.check(N.lib().nbody_forces_backward(_ptr(pos), _ptr(par), n, ctypes.byref(law.c()), _ptr(g),
                                              _ptr(gp), _ptr(gq), _ptr(ty), int(n_types), _ptr(gt),
                                              _ptr(ws), ws.numel(), _stream(dev)))
    else:
        ex = exclusions.c(n)
        N.check(N.lib().nbody_forces_backward_excl(_ptr(pos), _ptr(par), n, ctypes.byref(ex),
                                                   ctypes.byref(law.c()), _ptr(g), _ptr(gp), _ptr(gq),
                                                   _ptr(ty), int(n_types), _ptr(gt), _ptr(ws),
                                                   ws.numel(), _stream(dev)))
    return gp, gq, gt


# --------------------------------------------------------------- leapfrog
def leapfrog(pos, vel, acc, params, law: Law, dt: float, nsteps: int, inv_mass=None,
             potential: bool = False):
    """nsteps kick-drift-kick steps, updating pos, vel and acc IN PLACE (FP64 tensors on the
    GPU).  Returns the potential at the final positions, or None."""
    for t, name in ((pos, "pos"), (vel, "vel"), (acc, "acc")):
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64
                and t.is_contiguous()):
            raise ValueError("%s must be a contiguous float64 GPU tensor (updated in place)" % name)
    n = pos.shape[0]
    for t, name in ((pos, "pos"), (vel, "vel"), (acc, "acc")):
        if tuple(t.shape) != (n, 3):
            raise ValueError("%s must have shape (%d, 3)" % (name, n))
    par = _params(params, n, law, pos.device)
    im = None if inv_mass is None else _dev_f64(inv_mass, (n,), "inv_mass")
    p = torch.empty(n, dtype=torch.float64, device=pos.device) if potential else None
    ws = workspace(API_LEAPFROG, n, 1, law, pos.device)
    N.check(N.lib().leapfrog_step(_ptr(pos), _ptr(vel), _ptr(acc), _ptr(par), _ptr(im), n,
                                  ctypes.byref(law.c()), float(dt), int(nsteps), _ptr(p),
                                  _ptr(ws), ws.numel(), _stream(pos.device)))
    return p


# ------------------------------------------------------------ checkpoints
def save_state(path, **state):
    """Write an integrator's state to the .npz file ``path``: tensors are copied to the
    host with their dtype, plain numbers (time, step count, seeds) are stored as 0-d
    arrays.  The integrators carry everything they need across calls (the leapfrog
    a(t); the block scheme a, jerk, t_i and dt_i), and the kernels sum in a fixed
    order, so a run resumed from such a file continues bit for bit."""
    arrays = {}
    for key, val in state.items():
        arr = val.detach().cpu().numpy() if isinstance(val, torch.Tensor) else np.asarray(val)
        if arr.dtype == object:
            raise ValueError("state entry %r is neither a tensor nor a number" % key)
        arrays[key] = arr
    with open(path, "wb") as f:
        np.savez(f, **arrays)


def load_state(path, device=None):
    """Read a file written by save_state: arrays come back as contiguous tensors on
    ``device`` (default: the current GPU), 0-d entries as Python numbers.  Nothing
    in the file is executed (no pickled objects are accepted)."""
    device = torch.device("cuda", torch.cuda.current_device()) if device is None else device
    out = {}
    with np.load(path, allow_pickle=False) as z:
        for key in z.files:
            arr = z[key]
            out[key] = (arr.item() if arr.ndim == 0
                        else torch.from_numpy(np.ascontiguousarray(arr)).to(device))
    return out


# ------------------------------------------------------- jerk and Hermite
def _vec3(t, n, name):
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64
            and t.is_contiguous()):
        raise ValueError("%s must be a contiguous float64 GPU tensor (updated in place)" % name)
    if tuple(t.shape) != (n, 3):
        raise ValueError("%s must have shape (%d, 3)" % (name, n))
    return t


def forces_jerk(pos, vel, mass, law: Law, ilist=None, potential: bool = True):
    """Acceleration, jerk and (optionally) potential of softened gravity for every
    particle, or for the int64 indices `ilist`.  Returns (acc, jerk, phi or None)."""
    if law.kind != GRAVITY:
        raise ValueError("the jerk is provided for gravity")
    pos = _dev_f64(pos, None, "pos")
    n = pos.shape[0]
    pos = _dev_f64(pos, (n, 3), "pos")
    vel = _dev_f64(vel, (n, 3), "vel", pos.device)
    m = _dev_f64(mass, (n,), "mass", pos.device)
    il = None
    ni = n
    if ilist is not None:
        il = torch.as_tensor(ilist, device=pos.device).to(torch.int64).contiguous()
        ni = il.numel()
        if ni and _checks_values() and (int(il.min()) < 0 or int(il.max()) >= n):
            raise ValueError("ilist indices must lie in [0, %d)" % n)
    dev = pos.device
    a = torch.empty((ni, 3), dtype=torch.float64, device=dev)
    j = torch.empty((ni, 3), dtype=torch.float64, device=dev)
    p = torch.empty(ni, dtype=torch.float64, device=dev) if potential else None
    ws = workspace(API_JERK, max(n, ni), 1, law, dev)
    N.check(N.lib().nbody_forces_jerk(_ptr(pos), _ptr(vel), _ptr(m), n, _ptr(il), ni,
                                      ctypes.byref(law.c()), _ptr(a), _ptr(j), _ptr(p), _ptr(ws),
                                      ws.numel(), _stream(dev)))
    return a, j, p


def hermite(pos, vel, acc, jerk, mass, law: Law, dt: float, nsteps: int):
    """nsteps shared fourth-order Hermite steps, updating pos, vel, acc, jerk IN PLACE
    (acc and jerk must hold the values at the entry state, e.g. from forces_jerk)."""
    n = pos.shape[0]
    for t, name in ((pos, "pos"), (vel, "vel"), (acc, "acc"), (jerk, "jerk")):
        _vec3(t, n, name)
    m = _dev_f64(mass, (n,), "mass", pos.device)
    ws = workspace(API_HERMITE, n, 1, law, pos.device)
    N.check(N.lib().hermite_step(_ptr(pos), _ptr(vel), _ptr(acc), _ptr(jerk), _ptr(m), n,
                                 ctypes.byref(law.c()), float(dt), int(nsteps), _ptr(ws), ws.numel(),
                                 _stream(pos.device)))


def hermite_block_init(acc, jerk, eta_s: float, dt_max: float):
    """Initial block steps: (t_i, dt_i) float64 GPU tensors [N]."""
    n = acc.shape[0]
    a = _dev_f64(acc, (n, 3), "acc")
    j = _dev_f64(jerk, (n, 3), "jerk", a.device)
    t = torch.empty(n, dtype=torch.float64, device=a.device)
    dt = torch.empty(n, dtype=torch.float64, device=a.device)
    N.check(N.lib().hermite_block_init(_ptr(a), _ptr(j), n, float(eta_s), float(dt_max), _ptr(t),
                                       _ptr(dt), _stream(a.device)))
    return t, dt


def hermite_block(pos, vel, acc, jerk, t_i, dt_i, mass, law: Law, eta: float, dt_max: float,
                  nblocks: int, t_end: float = math.inf):
    """Up to nblocks block steps of the individual-step Hermite scheme, updating
    pos, vel, acc, jerk, t_i, dt_i IN PLACE; a block step whose time would pass
    t_end is not taken, nor is any after it.  Returns (due count of each block step
    [nblocks] int64 numpy array, 0 for steps not taken; time of the last block step
    taken, or nan if none was)."""
    n = pos.shape[0]
    for t, name in ((pos, "pos"), (vel, "vel"), (acc, "acc"), (jerk, "jerk")):
        _vec3(t, n, name)
    for t, name in ((t_i, "t_i"), (dt_i, "dt_i")):
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64
                and t.is_contiguous() and tuple(t.shape) == (n,)):
            raise ValueError("%s must be a contiguous float64 GPU tensor of shape (%d,)" % (name, n))
    m = _dev_f64(mass, (n,), "mass", pos.device)
    counts = np.zeros(max(int(nblocks), 1), dtype=np.int64)
    t_now = ctypes.c_double(math.nan)
    ws = workspace(API_HERMITE, n, 1, law, pos.device)
    N.check(N.lib().hermite_block_steps(_ptr(pos), _ptr(vel), _ptr(acc), _ptr(jerk), _ptr(t_i),
                                        _ptr(dt_i), _ptr(m), n, ctypes.byref(law.c()), float(eta),
                                        float(dt_max), float(t_end), int(nblocks),
                                        counts.ctypes.data_as(ctypes.c_void_p), ctypes.byref(t_now),
                                        _ptr(ws), ws.numel(), _stream(pos.device)))
    return counts[:int(nblocks)], t_now.value


def probe_issue_rates(device=None):
    """Shader cycles a SIMD spends per wave64 instruction on this GPU, at eight waves per SIMD:
    a dict with fma_cycles (FP32 FMA, VGPR operands), fma_sgpr_cycles (one SGPR operand),
    rsq_cycles (v_rsq_f32), clock_ghz and wall_counter_mhz (the shader clock during the FMA
    probe and the fixed counter's rate), rsq_13fma_cycles (one rsq interleaved with 13
    independent FMAs, per group of 14), fma_distinct_cycles (multiplier and addend in distinct
    VGPRs rotating over the chains), dpp_mov_cycles (a DPP row rotation on the VALU) and
    bpermute_cycles (ds_bpermute through the LDS crossbar).  Synchronises the device's current
    stream."""
    dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
    nbytes = int(N.lib().nbody_probe_workspace_bytes())
    ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    out = (ctypes.c_double * 9)()
    N.check(N.lib().nbody_probe_issue_rates(out, 9, _ptr(ws), nbytes, _stream(dev)))
    keys = ("fma_cycles", "fma_sgpr_cycles", "rsq_cycles", "clock_ghz", "wall_counter_mhz",
            "rsq_13fma_cycles", "fma_distinct_cycles", "dpp_mov_cycles", "bpermute_cycles")
    return dict(zip(keys, [float(v) for v in out]))


def autotune_jerk(pos, vel, mass, law: Law, potential=True):
    """Measure launch configurations of the jerk kernel on this problem and remember
    the fastest (also used by the Hermite steps).  Returns (config dict, ms)."""
    pos = _dev_f64(pos, None, "pos")
    n = pos.shape[0]
    vel = _dev_f64(vel, (n, 3), "vel", pos.device)
    m = _dev_f64(mass, (n,), "mass", pos.device)
    dev = pos.device
    a = torch.empty((n, 3), dtype=torch.float64, device=dev)
    j = torch.empty((n, 3), dtype=torch.float64, device=dev)
    p = torch.empty(n, dtype=torch.float64, device=dev) if potential else None
    ws = workspace(API_JERK, n, 1, law, dev)
    best = N.NBodyConfig()
    ms = ctypes.c_double()
    N.check(N.lib().nbody_autotune_jerk(_ptr(pos), _ptr(vel), _ptr(m), n, ctypes.byref(law.c()),
                                        _ptr(a), _ptr(j), _ptr(p), _ptr(ws), ws.numel(), _stream(dev),
                                        ctypes.byref(best), ctypes.byref(ms)))
    return (dict(block=best.block, i_per_lane=best.i_per_lane, j_tile=best.j_tile,
                 j_split=best.j_split, j_stage=best.j_stage), ms.value)


# ------------------------------------------------------------- tuning etc.
def set_config(api, block=256, i_per_lane=1, j_tile=256, j_split=1, j_stage=0):
    cfg = N.NBodyConfig(block, i_per_lane, j_tile, j_split, j_stage)
    N.check(N.lib().nbody_set_config(api, ctypes.byref(cfg)))


def clear_config(api):
    N.check(N.lib().nbody_set_config(api, None))


def get_config(api, n, law: Law, n_systems=1):
    cfg = N.NBodyConfig()
    N.check(N.lib().nbody_get_config(api, int(n), int(n_systems), ctypes.byref(law.c()),
                                     ctypes.byref(cfg)))
    return dict(block=cfg.block, i_per_lane=cfg.i_per_lane, j_tile=cfg.j_tile, j_split=cfg.j_split,
                j_stage=cfg.j_stage)


def autotune(pos, params, law: Law, offsets=None, potential=True):
    """Measure candidate launch configurations on this problem and remember the fastest.
    Returns (config dict, milliseconds)."""
    pos = _dev_f64(pos, None, "pos")
    n = pos.shape[0]
    par = _params(params, n, law, pos.device)
    f = torch.empty((n, 3), dtype=torch.float64, device=pos.device)
    p = torch.empty(n, dtype=torch.float64, device=pos.device) if potential else None
    best = N.NBodyConfig()
    ms = ctypes.c_double()
    if offsets is None:
        ws = workspace(API_FORCES, n, 1, law, pos.device)
        N.check(N.lib().nbody_autotune(API_FORCES, None, 0, _ptr(pos), _ptr(par), n,
                                       ctypes.byref(law.c()), _ptr(f), _ptr(p), _ptr(ws), ws.numel(),
                                       _stream(pos.device), ctypes.byref(best), ctypes.byref(ms)))
    else:
        off = _host_offsets(offsets)
        S = off.size - 1
        ws = workspace(API_BATCHED, n, S, law, pos.device)
        N.check(N.lib().nbody_autotune(API_BATCHED, off.ctypes.data_as(ctypes.c_void_p), S,
                                       _ptr(pos), _ptr(par), n, ctypes.byref(law.c()), _ptr(f),
                                       _ptr(p), _ptr(ws), ws.numel(), _stream(pos.device),
                                       ctypes.byref(best), ctypes.byref(ms)))
    return (dict(block=best.block, i_per_lane=best.i_per_lane, j_tile=best.j_tile,
                 j_split=best.j_split, j_stage=best.j_stage), ms.value)


def tune_save(path):
    N.check(N.lib().nbody_tune_save(str(path).encode()))


def tune_load(path):
    N.check(N.lib().nbody_tune_load(str(path).encode()))


def timing_enable(on=True):
    N.check(N.lib().nbody_timing_enable(1 if on else 0))


def timing_read(reset=True):
    """(total milliseconds, launches) of the all-pairs kernels since the last reset."""
    ms = ctypes.c_double()
    cnt = ctypes.c_int64()
    N.check(N.lib().nbody_timing_read(ctypes.byref(ms), ctypes.byref(cnt), 1 if reset else 0))
    return ms.value, cnt.value


def flops_per_pair(api, law_kind, with_potential):
    return int(N.lib().nbody_flops_per_pair(api, law_kind, 1 if with_potential else 0))


# ---------------------------------------------------------------- autograd
def _refuse_param_grad(ctx, law: Law, what):
    """The parameter adjoint exists for LJC(linear) only (per-atom q, sigma, epsilon): a params
    tensor that requires a gradient under another law is refused rather than left without one."""
    if ctx.needs_input_grad[1] and law.kind != LJC_LINEAR:
        name = {GRAVITY: "gravity masses", LJC_CONSTANT: "LJC(constant) parameters",
                LJC_SIGMOIDAL: "LJC(sigmoidal) parameters"}.get(law.kind, "these parameters")
        raise NotImplementedError("%s: no gradient with respect to %s (only positions, and the "
                                  "LJC(linear) q / sigma / epsilon); pass params.detach()" % (what, name))


class NBodyForcesFn(torch.autograd.Function):
    """F = forces(pos, params) with a hand-written adjoint (nbody_forces_backward), optionally
    with exclusion lists (LJC).

    Gradients: pos always; params for LJC(linear) (per-atom q, sigma, epsilon).  A params
    tensor that requires a gradient under another law raises NotImplementedError."""

    @staticmethod
    def forward(ctx, pos, params, law: Law, exclusions: Exclusions = None):
        _refuse_param_grad(ctx, law, "NBodyForcesFn")
        f, _ = forces(pos, params, law, potential=False, exclusions=exclusions)
        ctx.save_for_backward(pos, params)
        ctx.law = law
        ctx.exclusions = exclusions
        return f

    @staticmethod
    def backward(ctx, grad_f):
        pos, params = ctx.saved_tensors
        law = ctx.law
        need_pos = ctx.needs_input_grad[0]
        need_par = ctx.needs_input_grad[1] and law.kind == LJC_LINEAR
        gp, gq, _ = forces_backward(pos.detach(), params.detach(), grad_f.contiguous(), law,
                                    want_pos=need_pos, want_params=need_par,
                                    exclusions=ctx.exclusions)
        if gq is not None:
            gq = gq.reshape(params.shape)
        return gp, gq, None, None


class NBodyBatchedForcesFn(torch.autograd.Function):
    """Forces of a batch of independent systems (rows offsets[s]..offsets[s+1]) in one
    persistent launch, with the batched adjoint (nbody_forces_backward_batched) as backward;
    optional exclusion lists over the concatenated rows."""

    @staticmethod
    def forward(ctx, pos, params, offsets, law: Law, exclusions: Exclusions = None):
        _refuse_param_grad(ctx, law, "NBodyBatchedForcesFn")
        f, _ = forces_batched(offsets, pos, params, law, potential=False, exclusions=exclusions)
        ctx.save_for_backward(pos, params)
        ctx.offsets = _host_offsets(offsets)
        ctx.law = law
        ctx.exclusions = exclusions
        return f

    @staticmethod
    def backward(ctx, grad_f):
        pos, params = ctx.saved_tensors
        law = ctx.law
        need_pos = ctx.needs_input_grad[0]
        need_par = ctx.needs_input_grad[1] and law.kind == LJC_LINEAR
        gp, gq, _ = forces_backward_batched(ctx.offsets, pos.detach(), params.detach(),
                                            grad_f.contiguous(), law, want_pos=need_pos,
                                            want_params=need_par, exclusions=ctx.exclusions)
        if gq is not None:
            gq = gq.reshape(params.shape)
        return gp, gq, None, None, None


class LJCTypedForcesFn(torch.autograd.Function):
    """LJC(linear) forces with per-type sigma/epsilon tables (optionally with exclusion lists);
    the per-type gradient sums are reduced on the GPU in a fixed order."""

    @staticmethod
    def forward(ctx, pos, q, sigma_t, eps_t, types, law: Law, exclusions: Exclusions = None):
        types = types.to(torch.int64)
        params = torch.stack([q, sigma_t[types], eps_t[types]], dim=1).contiguous()
        f, _ = forces(pos, params, law, potential=False, exclusions=exclusions)
        ctx.save_for_backward(pos, params, types)
        ctx.law = law
        ctx.n_types = sigma_t.shape[0]
        ctx.exclusions = exclusions
        return f

    @staticmethod
    def backward(ctx, grad_f):
        pos, params, types = ctx.saved_tensors
        gp, gq, gt = forces_backward(pos, params, grad_f.contiguous(), ctx.law, want_pos=True,
                                     want_params=True, types=types, n_types=ctx.n_types,
                                     exclusions=ctx.exclusions)
        return (gp, gq[:, 0].contiguous(), gt[:, 0].contiguous(), gt[:, 1].contiguous(), None, None,
                None)
