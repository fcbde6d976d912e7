"""Helpers shared by the GPU parity tests."""
import numpy as np
import pytest
import torch


def relerr(a, b) -> float:
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def to_dev(a: np.ndarray, dtype=torch.complex128) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a)).to(dtype).cuda()


def to_host(t: torch.Tensor) -> np.ndarray:
    torch.cuda.synchronize()
    return t.detach().cpu().to(torch.complex128).numpy()


@pytest.fixture(scope="session")
def ctx():
    from paper_2506_20350_amd.api import Context
    c = Context(0)
    yield c
    c.close()
