"""MI355X (gfx950) all-pairs N-body forces: softened gravity and LJ + Coulomb(4r).

The compute path is libnbody.so (hand-written HIP kernels behind the C ABI of
include/nbody.h); ``paper_0706_3060_amd.nbody`` is its torch binding and
``paper_0706_3060_amd.workloads`` draws seeded synthetic inputs.  The binding
is imported lazily so that the input generators work without a GPU stack.
"""
__all__ = ["nbody", "workloads"]


def __getattr__(name):
    if name in ("nbody", "workloads", "build"):
        import importlib
        return importlib.import_module("." + name, __name__)
    from . import nbody
    return getattr(nbody, name)
