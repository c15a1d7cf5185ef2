"""Helpers shared by the GPU tests (device checks, host<->device copies)."""
import numpy as np
import pytest


def need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2310_03341_amd import api
    api.lib()  # raises loudly if the HIP library is missing
    return torch.device("cuda:0")


def to_dev_colmajor(M: np.ndarray, dev, ld=None):
    import torch
    from paper_2310_03341_amd import api
    n, m = M.shape
    out = api.colmajor(n, m, {np.complex128: torch.complex128, np.complex64: torch.complex64,
                              np.float64: torch.float64, np.float32: torch.float32}[M.dtype.type],
                       dev, ld)
    out.copy_(torch.from_numpy(np.ascontiguousarray(M)))
    return out
