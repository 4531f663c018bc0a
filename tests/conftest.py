import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture
def sage_ctx_factory():
    """Open contexts on cuda:0 with config overrides; all closed at teardown."""
    from paper_2404_14691_amd import sage as S
    opened = []

    def make(**over):
        cfg = S.sage_config_default()
        cfg.pool_budget_bytes = 256 << 20
        for k, v in over.items():
            setattr(cfg, k, v)
        ctx = S.sage_open(0, cfg)
        opened.append(ctx)
        return ctx

    yield make
    for c in opened:
        S.sage_close(c)


@pytest.fixture
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch
