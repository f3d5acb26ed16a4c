"""The C ABI boundary on a machine without a GPU.

* libnbody.so loads (after torch, so it binds to torch's HIP runtime) and
  exports every function include/nbody.h declares.
* Host-side validation returns the documented error codes before any work is
  enqueued (these calls return before any HIP call is made).
* nbody_workspace_bytes / nbody_flops_per_pair / nbody_version are pure host
  functions.
No kernel is launched here.
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nbody.h")


@pytest.fixture(scope="module")
def N():
    from paper_0706_3060_amd import _native
    if os.environ.get("NBODY_TEST_LIB"):
        # a sanitizer build of the same sources (tests/test_host_sanitize.py)
        _native.LIB_PATH = os.environ["NBODY_TEST_LIB"]
    elif not os.path.exists(_native.LIB_PATH):
        from paper_0706_3060_amd import build
        build.build(verbose=False)
    _native.lib()
    assert any(_native.LIB_PATH in l for l in open("/proc/self/maps"))
    return _native


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(\w+)\s*\(", text, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while", "return")))


def test_header_declares_the_boundary():
    fns = declared_functions()
    for name in ("nbody_forces", "nbody_forces_batched", "nbody_forces_backward", "leapfrog_step",
                 "nbody_workspace_bytes", "nbody_last_error"):
        assert name in fns


def test_library_exports_every_declared_symbol(N):
    lib = N.lib()
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert set(declared_functions()) == set(N.EXPORTED)


def test_single_hip_runtime(N):
    maps = [l.split()[-1] for l in open("/proc/self/maps") if "libamdhip64" in l]
    assert len(set(maps)) == 1, set(maps)
    assert "torch" in maps[0]


def law(N, kind=0, prec=2, G=1.0, eps=0.01, k=332.0637, D=4.0):
    return N.NBodyLaw(kind, prec, G, eps, k, D)


def test_workspace_bytes(N):
    lib = N.lib()
    g = law(N)
    a = lib.nbody_workspace_bytes(0, 1 << 20, 1, ctypes.byref(g))
    assert a >= (1 << 20) * 16            # FP32 gravity records alone
    assert lib.nbody_workspace_bytes(0, 0, 1, ctypes.byref(g)) > 0
    assert lib.nbody_workspace_bytes(0, -1, 1, ctypes.byref(g)) == 0
    assert lib.nbody_workspace_bytes(9, 100, 1, ctypes.byref(g)) == 0
    assert lib.nbody_workspace_bytes(0, 100, 1, None) == 0
    bad = law(N, kind=7)
    assert lib.nbody_workspace_bytes(0, 100, 1, ctypes.byref(bad)) == 0
    f64 = law(N, prec=0)
    assert lib.nbody_workspace_bytes(0, 4096, 1, ctypes.byref(f64)) > \
        lib.nbody_workspace_bytes(0, 4096, 1, ctypes.byref(g)) - 4096 * 16
    assert lib.nbody_workspace_bytes(1, 10000, 50, ctypes.byref(law(N, kind=1))) > 10000 * 32
    assert lib.nbody_workspace_bytes(2, 8192, 1, ctypes.byref(law(N, kind=1))) >= 8192 * 64
    assert lib.nbody_workspace_bytes(3, 8192, 1, ctypes.byref(g)) > \
        lib.nbody_workspace_bytes(0, 8192, 1, ctypes.byref(g))


def fake(addr=0x1000):
    # a non-NULL pointer value that validation never dereferences
    return ctypes.c_void_p(addr)


def call_forces(N, n, lw, ws_bytes=1 << 30, pos=True, out=True):
    return N.lib().nbody_forces(fake() if pos else None, fake(), n,
                                ctypes.byref(lw) if lw is not None else None,
                                fake() if out else None, None, fake(), ws_bytes, None)


def test_forces_validation(N):
    lib = N.lib()
    assert call_forces(N, 10, None) == N.NBODY_EINVAL
    assert b"law is NULL" in lib.nbody_last_error()
    assert call_forces(N, -1, law(N)) == N.NBODY_EINVAL
    assert call_forces(N, 10, law(N, kind=5)) == N.NBODY_EINVAL
    assert call_forces(N, 10, law(N, prec=9)) == N.NBODY_EINVAL
    assert call_forces(N, 10, law(N, eps=-1.0)) == N.NBODY_EINVAL
    assert call_forces(N, 10, law(N, eps=float("nan"))) == N.NBODY_EINVAL
    assert call_forces(N, 10, law(N, kind=1, D=0.0)) == N.NBODY_EINVAL
    assert call_forces(N, 10, law(N), pos=False) == N.NBODY_EINVAL
    assert call_forces(N, 10, law(N), out=False) == N.NBODY_EINVAL
    assert call_forces(N, 10, law(N), ws_bytes=16) == N.NBODY_EWORKSPACE
    assert b"workspace too small" in lib.nbody_last_error()
    assert lib.nbody_forces(fake(), fake(), 10, ctypes.byref(law(N)), fake(), None, None, 1 << 30,
                            None) == N.NBODY_EWORKSPACE
    # N = 0 is a no-op that needs no pointers at all
    assert lib.nbody_forces(None, None, 0, ctypes.byref(law(N)), None, None, None, 0, None) == 0


def test_share_validation(N):
    lib = N.lib()

    def share(n, lw, sh, nsh, ws_bytes=1 << 40, out=True):
        return lib.nbody_forces_share(fake(), fake(), n, ctypes.byref(lw) if lw is not None else None,
                                      sh, nsh, fake() if out else None, None, fake(), ws_bytes, None)

    g = law(N, prec=2)
    assert share(10, None, 0, 1) == N.NBODY_EINVAL
    for sh, nsh in [(-1, 4), (4, 4), (0, 0), (0, -3)]:
        assert share(10, g, sh, nsh) == N.NBODY_EINVAL, (sh, nsh)
        assert b"share" in lib.nbody_last_error()
    # FP64 and plain FP32 shard by rows; the symmetric tiles stop at 2^21 particles
    for kind in (1, 2, 3):
        for prec in (0, 3):
            assert share(10, law(N, kind=kind, prec=prec), 0, 2) == N.NBODY_ENOTSUP, (kind, prec)
        assert share((1 << 21) + 1, law(N, kind=kind), 0, 2) == N.NBODY_ENOTSUP, kind
    assert share(10, law(N, prec=0), 0, 2) == N.NBODY_ENOTSUP
    assert share(10, law(N, prec=3), 0, 2) == N.NBODY_ENOTSUP
    assert share((1 << 21) + 1, g, 0, 2) == N.NBODY_ENOTSUP
    assert share(10, g, 0, 2, out=False) == N.NBODY_EINVAL
    assert share(10, g, 1, 2, ws_bytes=16) == N.NBODY_EWORKSPACE
    assert lib.nbody_forces_share(None, None, 0, ctypes.byref(g), 0, 1, None, None, None, 0, None) == 0


def test_batched_validation(N):
    lib = N.lib()
    lw = law(N, kind=1)

    def off(vals):
        a = (ctypes.c_int64 * len(vals))(*vals)
        return ctypes.cast(a, ctypes.c_void_p), a

    p, keep = off([0, 5, 3])
    assert lib.nbody_forces_batched(p, 2, fake(), fake(), ctypes.byref(lw), fake(), None, fake(),
                                    1 << 30, None) == N.NBODY_EINVAL
    p, keep = off([1, 5])
    assert lib.nbody_forces_batched(p, 1, fake(), fake(), ctypes.byref(lw), fake(), None, fake(),
                                    1 << 30, None) == N.NBODY_EINVAL
    assert lib.nbody_forces_batched(None, 1, fake(), fake(), ctypes.byref(lw), fake(), None, fake(),
                                    1 << 30, None) == N.NBODY_EINVAL
    p, keep = off([0, 0, 0])       # only empty systems: nothing to do
    assert lib.nbody_forces_batched(p, 2, None, None, ctypes.byref(lw), None, None, None, 0,
                                    None) == 0
    p, keep = off([0, 100])
    assert lib.nbody_forces_batched(p, 1, fake(), fake(), ctypes.byref(lw), fake(), None, fake(),
                                    64, None) == N.NBODY_EWORKSPACE


def test_backward_and_leapfrog_validation(N):
    lib = N.lib()
    g = law(N)
    assert lib.nbody_forces_backward(fake(), fake(), 10, ctypes.byref(g), fake(), fake(), fake(),
                                     None, 0, None, fake(), 1 << 30, None) == N.NBODY_EINVAL
    plain = law(N, prec=3)
    assert lib.nbody_forces_backward(fake(), fake(), 10, ctypes.byref(plain), fake(), fake(), None,
                                     None, 0, None, fake(), 1 << 30, None) == N.NBODY_ENOTSUP
    lj = law(N, kind=1)
    assert lib.nbody_forces_backward(fake(), fake(), 10, ctypes.byref(lj), fake(), fake(), fake(),
                                     fake(), 0, fake(), fake(), 1 << 30, None) == N.NBODY_EINVAL
    assert lib.leapfrog_step(fake(), fake(), fake(), fake(), None, 10, ctypes.byref(g),
                             float("inf"), 1, None, fake(), 1 << 30, None) == N.NBODY_EINVAL
    assert lib.leapfrog_step(fake(), fake(), fake(), fake(), None, 10, ctypes.byref(g), 1e-3, -1,
                             None, fake(), 1 << 30, None) == N.NBODY_EINVAL
    # zero steps and no potential requested: nothing to do
    assert lib.leapfrog_step(fake(), fake(), fake(), fake(), None, 10, ctypes.byref(g), 1e-3, 0,
                             None, None, 0, None) == 0


def test_config_validation(N):
    lib = N.lib()
    good = N.NBodyConfig(256, 1, 256, 4, 1)
    assert lib.nbody_set_config(0, ctypes.byref(good)) == 0
    assert lib.nbody_set_config(0, None) == 0
    # the symmetric pair tiles (j_stage 2) take the 512-thread workgroup
    for ok in [N.NBodyConfig(512, 2, 2048, 1, 2), N.NBodyConfig(256, 1, 1024, 1, 2)]:
        assert lib.nbody_set_config(0, ctypes.byref(ok)) == 0
        assert lib.nbody_set_config(0, None) == 0
    for bad in [N.NBodyConfig(96, 1, 256, 1, 0), N.NBodyConfig(256, 3, 256, 1, 0),
                N.NBodyConfig(256, 1, 100, 1, 0), N.NBodyConfig(256, 1, 256, 65, 0),
                N.NBodyConfig(256, 1, 256, 1, 3), N.NBodyConfig(512, 1, 256, 1, 0),
                N.NBodyConfig(1024, 2, 2048, 1, 2)]:
        assert lib.nbody_set_config(0, ctypes.byref(bad)) == N.NBODY_EINVAL
    assert lib.nbody_set_config(7, ctypes.byref(good)) == N.NBODY_EINVAL
    # a forced symmetric configuration (512-thread workgroups) stays one where the symmetric
    # tiles apply, and elsewhere reads as a one-sided shape with a workgroup of at most 256
    # threads, which the other kernels are built for
    sym = N.NBodyConfig(512, 2, 2048, 1, 2)
    grav = lambda prec: N.NBodyLaw(0, prec, 1.0, 0.01, 0.0, 1.0)
    ljc = N.NBodyLaw(1, 1, 1.0, 0.0, 332.0637, 4.0)
    # the batched entry point keeps j_stage 2 as its own symmetric tiles (every law with FP32 pair
    # arithmetic), in their fixed shape of 4 waves over 256-record blocks; so does the batched
    # backward for the laws it differentiates (gravity and LJC(linear))
    # the single-system tiles take the forces and leapfrog of every law and gravity's backward at
    # this size (2^20; LJC(linear)'s backward takes tiles of its own up to 2^17, and FP64 pair
    # arithmetic runs one-sided)
    ljc_const = N.NBodyLaw(2, 1, 1.0, 0.0, 332.0637, 4.0)
    ljc_sig = N.NBodyLaw(3, 2, 1.0, 0.0, 332.0637, 1.0)
    cases = [(0, grav(1), "sym"), (3, grav(2), "sym"), (0, grav(0), None), (0, grav(3), None),
             (0, ljc, "sym"), (3, ljc, "sym"), (0, ljc_const, "sym"), (3, ljc_const, "sym"),
             (0, ljc_sig, "sym"), (2, ljc_sig, None),
             (0, N.NBodyLaw(1, 0, 1.0, 0.0, 332.0637, 4.0), None),
             (1, ljc, "bsym"), (1, grav(1), "bsym"), (1, grav(0), None),
             (1, ljc_const, "bsym"), (1, ljc_sig, "bsym"), (2, grav(1), "sym"), (2, ljc, None), (2, ljc_const, None),
             (4, grav(1), None), (5, grav(2), None), (6, ljc, "bsym"), (6, grav(2), "bsym"),
             (6, ljc_const, None), (6, grav(0), None)]
    for api, law, kind in cases:
        c = N.NBodyConfig()
        try:
            assert lib.nbody_set_config(api, ctypes.byref(sym)) == 0
            assert lib.nbody_get_config(api, 1 << 20, 1, ctypes.byref(law), ctypes.byref(c)) == 0
        finally:
            lib.nbody_set_config(api, None)
        if kind == "sym":
            assert (c.block, c.i_per_lane, c.j_tile, c.j_stage) == (512, 2, 2048, 2), (api, law.kind)
        elif kind == "bsym":
            assert (c.block, c.i_per_lane, c.j_tile, c.j_stage) == (256, 4, 256, 2), (api, law.kind)
        else:
            assert 64 <= c.block <= 256 and c.j_stage in (0, 1), (api, law.kind, law.precision, c.block)
    # the rule takes the symmetric tiles for the forces of whole systems of every law from
    # 32,768 to 2,097,152 particles (four j parts below 65,536 where the shape takes them);
    # above that their O(n^2) partials (34 GB at 2^21) would outgrow the workspace, and a forced
    # symmetric configuration reads as one-sided there.  With the energies (nbody_get_config
    # assumes them) every LJC law takes the 8-wave shape.
    g1 = grav(2)
    for lw in (g1, ljc, ljc_const, ljc_sig):
        for n, want in [(32767, False), (32768, True), (1 << 21, True), ((1 << 21) + 1, False),
                        (1 << 22, False)]:
            c = N.NBodyConfig()
            assert lib.nbody_get_config(0, n, 1, ctypes.byref(lw), ctypes.byref(c)) == 0
            assert (c.j_stage == 2) == want, (lw.kind, n, c.j_stage)
            if want and lw.kind >= 1:
                assert (c.block, c.i_per_lane) == (512, 2), (lw.kind, n, c.block, c.i_per_lane)
            if want:
                parts = (4 if c.block == 256 else 2) if n < 1 << 16 else (2 if n <= 1 << 17 else 1)
                assert c.j_split == parts, (lw.kind, n, c.j_split)
            try:
                assert lib.nbody_set_config(0, ctypes.byref(sym)) == 0
                assert lib.nbody_get_config(0, n, 1, ctypes.byref(lw), ctypes.byref(c)) == 0
            finally:
                lib.nbody_set_config(0, None)
            assert (c.j_stage == 2) == (n <= 1 << 21), (lw.kind, n, c.j_stage)
    for lw in (g1, ljc):
        w_sym = lib.nbody_workspace_bytes(0, 1 << 21, 1, ctypes.byref(lw))
        w_one = lib.nbody_workspace_bytes(0, (1 << 21) + 64, 1, ctypes.byref(lw))
        assert w_sym >= 1024 * (1 << 21) * 16 and w_one < 4 << 30, (lw.kind, w_sym, w_one)


def test_flop_convention_and_version(N):
    lib = N.lib()
    # the Appendix convention: 19 flops per gravity interaction, 20 with the potential
    assert lib.nbody_flops_per_pair(0, 0, 0) == 19
    assert lib.nbody_flops_per_pair(0, 0, 1) == 20
    assert lib.nbody_flops_per_pair(0, 1, 0) == 30      # Table 1 lists 30 for LJC
    assert lib.nbody_flops_per_pair(2, 0, 0) == 41
    assert b"gfx950" in lib.nbody_version()
    # issue-rate probe: argument checks only (it launches kernels)
    assert lib.nbody_probe_workspace_bytes() > 0
    out = (ctypes.c_double * 9)()
    assert lib.nbody_probe_issue_rates(None, 9, None, 0, None) == N.NBODY_EINVAL
    assert lib.nbody_probe_issue_rates(out, 5, None, 0, None) == N.NBODY_EINVAL      # too few outputs
    assert lib.nbody_probe_issue_rates(out, 9, ctypes.c_void_p(4096), 16, None) == N.NBODY_EWORKSPACE


def test_python_binding_rejects_cpu_tensors(N):
    import torch
    from paper_0706_3060_amd import nbody as nb
    with pytest.raises(ValueError):
        nb.forces(torch.zeros(4, 3, dtype=torch.float64), torch.ones(4, dtype=torch.float64),
                  nb.gravity("fp64"))


def test_jerk_and_hermite_validation(N):
    lib = N.lib()
    g = law(N)
    lj = law(N, kind=1)
    plain = law(N, prec=3)

    def jerk(lw, n=10, ilist=None, ni=10, ws_bytes=1 << 30):
        return lib.nbody_forces_jerk(fake(), fake(), fake(), n, ilist, ni, ctypes.byref(lw), fake(),
                                     fake(), None, fake(), ws_bytes, None)

    assert jerk(lj) == N.NBODY_ENOTSUP
    assert b"gravity only" in lib.nbody_last_error()
    assert jerk(plain) == N.NBODY_ENOTSUP
    assert jerk(g, ni=5) == N.NBODY_EINVAL                 # no ilist: ni must equal n
    assert jerk(g, n=-1, ni=-1) == N.NBODY_EINVAL
    assert jerk(g, ws_bytes=64) == N.NBODY_EWORKSPACE
    assert jerk(g, n=0, ni=0) == 0
    assert lib.hermite_step(fake(), fake(), fake(), fake(), fake(), 10, ctypes.byref(g), 0.0, 1, fake(),
                            1 << 30, None) == N.NBODY_EINVAL
    assert lib.hermite_step(fake(), fake(), fake(), fake(), fake(), 10, ctypes.byref(g), float("nan"),
                            1, fake(), 1 << 30, None) == N.NBODY_EINVAL
    assert lib.hermite_step(fake(), fake(), fake(), fake(), fake(), 10, ctypes.byref(lj), 0.1, 1,
                            fake(), 1 << 30, None) == N.NBODY_ENOTSUP
    assert lib.hermite_step(None, None, None, None, None, 10, ctypes.byref(g), 0.1, 0, None, 0,
                            None) == 0
    assert lib.hermite_block_init(fake(), fake(), 10, 0.01, 0.1, fake(), fake(), None) == N.NBODY_EINVAL
    assert b"power of two" in lib.nbody_last_error()
    assert lib.hermite_block_init(fake(), fake(), 10, -1.0, 0.125, fake(), fake(), None) == N.NBODY_EINVAL
    assert lib.hermite_block_init(None, None, 0, 0.01, 0.125, None, None, None) == 0

    def block(eta=0.02, dt_max=0.125, nb=3, lw=g, ws_bytes=1 << 30, t_end=float("inf")):
        return lib.hermite_block_steps(fake(), fake(), fake(), fake(), fake(), fake(), fake(), 10,
                                       ctypes.byref(lw), eta, dt_max, t_end, nb, None, None, fake(),
                                       ws_bytes, None)

    assert block(eta=0.0) == N.NBODY_EINVAL
    assert block(dt_max=0.3) == N.NBODY_EINVAL
    assert block(nb=-1) == N.NBODY_EINVAL
    assert block(t_end=float("nan")) == N.NBODY_EINVAL
    assert block(lw=lj) == N.NBODY_ENOTSUP
    assert block(ws_bytes=1024) == N.NBODY_EWORKSPACE
    assert block(nb=0) == 0
    # workspaces: records, partials, and for the integrator the scheduling state
    assert lib.nbody_workspace_bytes(4, 4096, 1, ctypes.byref(g)) >= 4096 * 32
    assert lib.nbody_workspace_bytes(5, 4096, 1, ctypes.byref(g)) > \
        lib.nbody_workspace_bytes(4, 4096, 1, ctypes.byref(g)) + 4096 * 56
    assert lib.nbody_workspace_bytes(4, 4096, 1, ctypes.byref(lj)) == 0
    # Table 1 counts 42 flops for the acceleration-and-jerk kernel (with the potential here)
    assert lib.nbody_flops_per_pair(4, 0, 1) == 42
    assert lib.nbody_flops_per_pair(4, 0, 0) == 41
    assert lib.nbody_flops_per_pair(5, 1, 0) == 0
    good = N.NBodyConfig(256, 2, 256, 4, 1)
    assert lib.nbody_set_config(4, ctypes.byref(good)) == 0
    assert lib.nbody_set_config(5, ctypes.byref(good)) == 0
    assert lib.nbody_set_config(4, None) == 0 and lib.nbody_set_config(5, None) == 0
    assert lib.nbody_set_config(6, ctypes.byref(good)) == 0
    assert lib.nbody_set_config(6, None) == 0
    assert lib.nbody_set_config(7, ctypes.byref(good)) == N.NBODY_EINVAL


def test_jerk_tiles_rule(N):
    # the acceleration-and-jerk tiles (j_stage 2 of the jerk entry point): FP32 gravity, whole
    # systems of 32,768 to 524,288 particles by rule (two j parts up to 2^17), any size up to
    # 2^19 when forced, in their one shape (8 waves of 2 i chunks over 1024-record blocks);
    # FP64 pair arithmetic and larger systems run one-sided
    lib = N.lib()
    g = lambda prec: N.NBodyLaw(0, prec, 1.0, 0.01, 0.0, 1.0)

    def get(lw, n):
        c = N.NBodyConfig()
        assert lib.nbody_get_config(4, n, 1, ctypes.byref(lw), ctypes.byref(c)) == 0
        return c

    for prec in (1, 2):
        for n, split in [(32767, None), (32768, 2), (65536, 2), (1 << 17, 2), ((1 << 17) + 1, 1), (1 << 19, 1),
                         ((1 << 19) + 1, None)]:
            c = get(g(prec), n)
            assert (c.j_stage == 2) == (split is not None), (prec, n, c.j_stage)
            if split:
                assert (c.block, c.i_per_lane, c.j_tile, c.j_split) == (512, 2, 1024, split), (prec, n)
    assert get(g(0), 1 << 17).j_stage == 0
    forced = N.NBodyConfig(256, 4, 2048, 4, 2)
    try:
        assert lib.nbody_set_config(4, ctypes.byref(forced)) == 0
        for n in (1, 3001, 1 << 17, (1 << 17) + 1, 1 << 19):
            c = get(g(2), n)
            assert (c.block, c.i_per_lane, c.j_tile, c.j_split, c.j_stage) == \
                (512, 2, 1024, 2 if n <= 1 << 17 else 1, 2), n
        for lw, n in ((g(2), (1 << 19) + 1), (g(0), 4096)):
            c = get(lw, n)
            assert c.j_stage in (0, 1) and c.block <= 256, (lw.precision, n)
    finally:
        lib.nbody_set_config(4, None)
    # the workspace holds the tiles' block-padded records and their slot partials (32 bytes per
    # row, block and part), for the jerk entry point and for the shared Hermite step
    for api in (4, 5):
        for n in (1000, 1 << 17, 1 << 19):
            blocks = -(-n // 1024)
            parts = 2 if n <= 1 << 17 else 1
            w = lib.nbody_workspace_bytes(api, n, 1, ctypes.byref(g(2)))
            assert w >= parts * blocks * (blocks * 1024) * 32 + blocks * 1024 * 32, (api, n, w)


def test_ljc_adjoint_tiles_rule(N):
    # LJC(linear)'s single-system backward over unordered pairs (the batched adjoint's tiles over
    # one system, j_stage 2): FP32 pair arithmetic, whole systems of 16,384 to 262,144 atoms by
    # rule, any size up to 2^18 when forced, in the tiles' fixed shape; other laws' and FP64
    # backwards, and larger systems, stay as they were
    lib = N.lib()
    ljc = lambda prec: N.NBodyLaw(1, prec, 1.0, 0.0, 332.0637, 4.0)

    def get(lw, n):
        c = N.NBodyConfig()
        assert lib.nbody_get_config(2, n, 1, ctypes.byref(lw), ctypes.byref(c)) == 0
        return c

    for prec in (1, 2):
        for n, want in [(16383, False), (16384, True), (1 << 18, True), ((1 << 18) + 1, False)]:
            c = get(ljc(prec), n)
            assert (c.j_stage == 2) == want, (prec, n, c.j_stage)
            if want:
                assert (c.block, c.i_per_lane, c.j_tile, c.j_split) == (256, 4, 256, 1), (prec, n)
    assert get(ljc(0), 1 << 16).j_stage == 0
    forced = N.NBodyConfig(512, 2, 2048, 2, 2)
    try:
        assert lib.nbody_set_config(2, ctypes.byref(forced)) == 0
        for n in (1, 3001, 1 << 18):
            c = get(ljc(2), n)
            assert (c.block, c.i_per_lane, c.j_tile, c.j_split, c.j_stage) == (256, 4, 256, 1, 2), n
        c = get(ljc(2), (1 << 18) + 1)
        assert c.j_stage in (0, 1) and c.block <= 256
    finally:
        lib.nbody_set_config(2, None)
    # the workspace holds the records padded to whole 256-record blocks and 32 bytes of slot
    # partials per atom and block
    for n in (1000, 1 << 16, 1 << 18):
        blocks = -(-n // 256)
        w = lib.nbody_workspace_bytes(2, n, 1, ctypes.byref(ljc(2)))
        assert w >= blocks * (blocks * 256) * 32 + blocks * 256 * 64, (n, w)


def test_exclusions_and_batched_adjoint_validation(N):
    lib = N.lib()
    g = law(N)
    lj = law(N, kind=1)
    ljs = law(N, kind=3)
    plain = law(N, kind=1, prec=3)
    ex = N.NBodyExclusions(fake(), fake(), 4)

    def fx(lw, e=ex, n=10, ws_bytes=1 << 30):
        return lib.nbody_forces_excl(fake(), fake(), n, ctypes.byref(e) if e is not None else None,
                                     ctypes.byref(lw), fake(), None, fake(), ws_bytes, None)

    assert fx(g) == N.NBODY_ENOTSUP                        # exclusions are an LJC matter
    assert fx(plain) == N.NBODY_ENOTSUP
    assert fx(lj, e=None) == N.NBODY_EINVAL
    assert fx(lj, e=N.NBodyExclusions(None, fake(), 4)) == N.NBODY_EINVAL
    assert fx(lj, e=N.NBodyExclusions(fake(), None, 4)) == N.NBODY_EINVAL
    assert fx(lj, e=N.NBodyExclusions(fake(), fake(), -1)) == N.NBODY_EINVAL
    assert fx(lj, ws_bytes=64) == N.NBODY_EWORKSPACE
    assert fx(lj, n=0) == 0

    def off(vals):
        a = (ctypes.c_int64 * len(vals))(*vals)
        return ctypes.cast(a, ctypes.c_void_p), a

    p, keep = off([0, 5, 12])
    assert lib.nbody_forces_batched_excl(p, 2, fake(), fake(), ctypes.byref(ex), ctypes.byref(g), fake(),
                                         None, fake(), 1 << 30, None) == N.NBODY_ENOTSUP
    assert lib.nbody_forces_batched_excl(p, 2, fake(), fake(), None, ctypes.byref(lj), fake(), None,
                                         fake(), 1 << 30, None) == N.NBODY_EINVAL
    assert lib.nbody_forces_backward_excl(fake(), fake(), 10, ctypes.byref(ex), ctypes.byref(ljs), fake(),
                                          fake(), fake(), None, 0, None, fake(), 1 << 30,
                                          None) == N.NBODY_ENOTSUP

    def bb(lw, e=None, gp=True, gq=True, ws_bytes=1 << 30, o=p, S=2):
        return lib.nbody_forces_backward_batched(o, S, fake(), fake(),
                                                 ctypes.byref(e) if e is not None else None,
                                                 ctypes.byref(lw), fake(), fake() if gp else None,
                                                 fake() if gq else None, None, 0, None, fake(),
                                                 ws_bytes, None)

    assert bb(g) == N.NBODY_EINVAL                         # gravity: no parameter adjoint
    assert bb(g, e=ex, gq=False) == N.NBODY_ENOTSUP
    assert bb(ljs) == N.NBODY_ENOTSUP
    assert bb(lj, ws_bytes=64) == N.NBODY_EWORKSPACE
    assert bb(lj, gp=False, gq=False) == 0
    bad, keep2 = off([0, 7, 3])
    assert bb(lj, o=bad) == N.NBODY_EINVAL
    assert lib.nbody_workspace_bytes(6, 10000, 50, ctypes.byref(lj)) > 10000 * 64
    assert lib.nbody_flops_per_pair(6, 1, 0) == 68


def test_tuning_file_is_tied_to_its_device(N, tmp_path):
    """nbody_tune_load accepts a file written for this device (here: no GPU, so the
    architecture reads "unknown" and the CU count the 256 fallback) and rejects one
    written for another architecture or CU count, or naming no device."""
    lib = N.lib()
    entry = ('{"api": 0, "law": 3, "precision": 2, "potential": 0, "n_bucket": 5, "s_bucket": 5, '
             '"block": 256, "i_per_lane": 1, "j_tile": 256, "j_split": 2, "j_stage": 1, "ms": 1.0}')

    def write(name, head):
        p = tmp_path / name
        p.write_text('{%s"entries": [\n  %s\n]}\n' % (head, entry))
        return str(p).encode()

    assert lib.nbody_tune_load(write("ok.json", '"arch": "unknown", "device_cus": 256, ')) == 0
    assert lib.nbody_tune_load(write("arch.json", '"arch": "gfx942", "device_cus": 256, ')) == N.NBODY_EINVAL
    assert b"gfx942" in lib.nbody_last_error()
    assert lib.nbody_tune_load(write("cus.json", '"arch": "unknown", "device_cus": 304, ')) == N.NBODY_EINVAL
    assert lib.nbody_tune_load(write("none.json", "")) == N.NBODY_EINVAL
    out = tmp_path / "saved.json"
    assert lib.nbody_tune_save(str(out).encode()) == 0
    text = out.read_text()
    assert '"arch": "unknown"' in text and '"device_cus": 256' in text and '"j_split": 2' in text
    assert lib.nbody_tune_load(str(out).encode()) == 0


def test_tuning_file_parser_refuses_malformed_files(N, tmp_path):
    """Malformed tuning files (empty, truncated, binary, an over-long architecture
    name, entries with invalid launch shapes, a very long run of partial entries)
    are refused with NBODY_EINVAL; none of them may read or write out of bounds
    (this test also runs against the sanitizer build)."""
    lib = N.lib()
    head = '{"arch": "unknown", "device_cus": 256, "entries": [\n'
    good = ('{"api": 0, "law": 0, "precision": 2, "potential": 1, "n_bucket": 3, "s_bucket": 0, '
            '"block": 256, "i_per_lane": 1, "j_tile": 256, "j_split": 1, "j_stage": 1, "ms": 2.0}')
    cases = {
        "empty.json": b"",
        "truncated.json": (head + good[:60]).encode(),
        "binary.json": bytes(range(256)) * 64,
        "longarch.json": ('{"arch": "%s", "device_cus": 256, "entries": [%s]}' % ("g" * 5000, good)).encode(),
        "badshape.json": (head + good.replace('"block": 256', '"block": 7') + "]}").encode(),
        "badapi.json": (head + good.replace('"api": 0', '"api": 99') + "]}").encode(),
        "partial_run.json": (head + '{"api": 0, ' * 20000 + "]}").encode(),
        "noquote.json": b'{"arch": "unknown',
    }
    for name, data in cases.items():
        p = tmp_path / name
        p.write_bytes(data)
        assert lib.nbody_tune_load(str(p).encode()) == N.NBODY_EINVAL, name
        assert lib.nbody_last_error()
    assert lib.nbody_tune_load(str(tmp_path / "missing.json").encode()) == N.NBODY_EINVAL
    assert lib.nbody_tune_load(None) == N.NBODY_EINVAL
    ok = tmp_path / "ok.json"
    ok.write_text(head + good + "]}\n")
    assert lib.nbody_tune_load(str(ok).encode()) == 0


def test_tune_cache_environment_variable(N, tmp_path):
    """NBODY_TUNE_CACHE: a tuning file named there is read at the first configuration
    lookup of a process (checked in a child process, since the read happens once per
    process); without it the same lookup gives the built-in rule."""
    import subprocess
    import sys
    entry = ('{"api": 0, "law": 0, "precision": 2, "potential": 1, "n_bucket": 13, "s_bucket": 13, '
             '"block": 128, "i_per_lane": 2, "j_tile": 128, "j_split": 3, "j_stage": 1, "ms": 1.0}')
    cache = tmp_path / "cache.json"
    cache.write_text('{"arch": "unknown", "device_cus": 256, "entries": [\n  %s\n]}\n' % entry)
    code = (
        "import ctypes, sys\n"
        "sys.path.insert(0, %r)\n"
        "from paper_0706_3060_amd import _native as N\n"
        "import os\n"
        "if os.environ.get('NBODY_TEST_LIB'): N.LIB_PATH = os.environ['NBODY_TEST_LIB']\n"
        "law = N.NBodyLaw(0, 2, 1.0, 0.01, 0.0, 1.0)\n"
        "c = N.NBodyConfig()\n"
        "assert N.lib().nbody_get_config(0, 5000, 1, ctypes.byref(law), ctypes.byref(c)) == 0\n"
        "print(c.block, c.i_per_lane, c.j_tile, c.j_split, c.j_stage)\n" % ROOT)

    def lookup(env_value):
        env = dict(os.environ)
        env.pop("NBODY_TUNE_CACHE", None)
        if env_value is not None:
            env["NBODY_TUNE_CACHE"] = env_value
        r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env,
                           timeout=300)
        assert r.returncode == 0, r.stderr[-2000:]
        return r.stdout.split(), r.stderr

    tuned, _ = lookup(str(cache))
    assert tuned == ["128", "2", "128", "3", "1"]
    builtin, _ = lookup(None)
    assert builtin != tuned
    missing, err = lookup(str(tmp_path / "not_yet_written.json"))
    assert missing == builtin and "tuning cache" not in err
    other = tmp_path / "other.json"
    other.write_text(cache.read_text().replace('"arch": "unknown"', '"arch": "gfx942"'))
    refused, err = lookup(str(other))
    assert refused == builtin and "not used" in err


def test_tuning_file_save_is_atomic(N, tmp_path):
    """nbody_tune_save writes beside the target and renames over it: no temporary file is
    left behind, an existing file is replaced whole, and a path in a missing directory is
    refused with NBODY_EINVAL."""
    lib = N.lib()
    target = tmp_path / "cache.json"
    target.write_text("old contents")
    assert lib.nbody_tune_save(str(target).encode()) == 0
    assert target.read_text().startswith('{"arch": ')
    assert sorted(p.name for p in tmp_path.iterdir()) == ["cache.json"]
    assert lib.nbody_tune_save(str(tmp_path / "missing" / "cache.json").encode()) == N.NBODY_EINVAL
    assert sorted(p.name for p in tmp_path.iterdir()) == ["cache.json"]
