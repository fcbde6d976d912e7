"""Helpers shared by the GPU parity tests."""
import numpy as np
import pytest
import torch


def relerr(a, b) -> float:
    """Largest per-column relative error max_w ||a_w - b_w|| / ||b_w||.

    Arrays of two or more dimensions are columns along the first axis (the W
    right-hand sides of the vector layout, the images of a batch); a 1-D array
    is one column.  A zero reference column must be matched exactly (its error
    counts as infinite otherwise), so one wrong column, or a wrong ragged tail
    inside one, cannot hide behind the norm of the others.
    """
    a = np.asarray(a)
    b = np.asarray(b)
    assert a.shape == b.shape, (a.shape, b.shape)
    if a.ndim < 2:
        a, b = a.reshape(1, -1), b.reshape(1, -1)
    a = a.reshape(a.shape[0], -1)
    b = b.reshape(b.shape[0], -1)
    if a.shape[0] == 0:
        return 0.0
    num = np.linalg.norm(a - b, axis=1)
    den = np.linalg.norm(b, axis=1)
    err = np.where(den > 0, num / np.where(den > 0, den, 1.0), np.where(num > 0, np.inf, 0.0))
    return float(err.max())


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
