import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: longer CPU-only test")


@pytest.fixture(scope="session")
def oracle_mod():
    import oracle
    oracle.build(force=False)
    return oracle


# The full 256-system ensemble takes ~1 minute to draw serially; draw it once,
# in a fork pool, after collection and before any test touches the GPU.
_FULL_ENSEMBLE = {}


def pytest_collection_finish(session):
    wants = any(item.get_closest_marker("gpu") and "full_ensemble" in getattr(item, "fixturenames", ())
                for item in session.items)
    if not wants:
        return
    torch = sys.modules.get("torch")
    if torch is not None and torch.cuda.is_initialized():
        return
    from paper_0706_3060_amd import workloads as W
    _FULL_ENSEMBLE["data"] = W.batched_md(256, seed=4)


@pytest.fixture(scope="session")
def full_ensemble():
    if "data" not in _FULL_ENSEMBLE:
        from paper_0706_3060_amd import workloads as W
        _FULL_ENSEMBLE["data"] = W.batched_md(256, seed=4)
    return _FULL_ENSEMBLE["data"]
