"""The autograd Functions refuse parameter gradients that no adjoint provides (CPU only).

The hand-written parameter adjoint exists for LJC(linear) (per-atom q, sigma, epsilon).  Gravity
masses and the LJC(constant) / LJC(sigmoidal) parameters have none: a params tensor that
requires a gradient under those laws raises NotImplementedError when the forward is built,
before any work reaches a device, instead of leaving the gradient silently unset.
"""
import pytest
import torch


@pytest.fixture(scope="module")
def nb():
    from paper_0706_3060_amd import nbody
    return nbody


@pytest.mark.parametrize("kind", ["gravity", "ljc_constant", "ljc_sigmoidal"])
def test_unsupported_parameter_gradient_is_refused(nb, kind):
    pos = torch.zeros(4, 3, dtype=torch.float64, requires_grad=True)
    if kind == "gravity":
        law, par = nb.gravity("fp64", softening=0.1), torch.ones(4, dtype=torch.float64)
    elif kind == "ljc_constant":
        law, par = nb.ljc_constant("fp64"), torch.ones(4, 3, dtype=torch.float64)
    else:
        law, par = nb.ljc_sigmoidal((2e-4, -6e-3, 0.25, 0.4), "fp64"), torch.ones(4, 3, dtype=torch.float64)
    par.requires_grad_(True)
    with pytest.raises(NotImplementedError, match="no gradient with respect to"):
        nb.NBodyForcesFn.apply(pos, par, law)
    off = torch.tensor([0, 2, 4])
    with pytest.raises(NotImplementedError, match="no gradient with respect to"):
        nb.NBodyBatchedForcesFn.apply(pos, par, off, law)
