import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long CPU test")
    # a GPU session computes its long oracle references in worker processes, started
    # here, before any test module touches the GPU
    if (getattr(config.option, "markexpr", "") or "").strip() == "gpu":
        tests_dir = os.path.dirname(os.path.abspath(__file__))
        if tests_dir not in sys.path:
            sys.path.insert(0, tests_dir)
        import gpu_common
        gpu_common.start_oracle_pool()


def pytest_unconfigure(config):
    mod = sys.modules.get("gpu_common")
    pool = getattr(mod, "_pool", None) if mod else None
    if pool is not None:
        pool.terminate()
        pool.join()
        mod._pool = None
