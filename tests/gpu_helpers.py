"""Helpers for the GPU tests: moving seeded inputs to the device and comparing
the HIP path's results with the oracle's."""
import numpy as np
import pytest
import torch

import oracle as orc


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def to_dev(a: np.ndarray) -> torch.Tensor:
    """Column-major device copy of a NumPy matrix (same dtype)."""
    t = torch.from_numpy(np.ascontiguousarray(np.asarray(a).T)).cuda()
    return t.t()


def host(t: torch.Tensor) -> np.ndarray:
    return t.detach().cpu().numpy()


def gpu_id(A_np, **kw):
    """(perm, k, R, T) of the HIP path on host, for a NumPy input."""
    import paper_2012_00706_amd as mp
    A = to_dev(A_np)
    res = mp.column_id(A, **kw)
    torch.cuda.synchronize()
    return host(res.perm).astype(np.int64), res.k, host(res.R), host(res.T)


def rel_err(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    d = np.linalg.norm(a - b)
    s = np.linalg.norm(b)
    return d / s if s > 0 else d


def row_sign_align(R_gpu, R_ref):
    """Rows of R are unique up to sign; flip the GPU rows to match."""
    s = np.sign(np.diag(R_gpu) * np.diag(R_ref))
    s[s == 0] = 1.0
    return R_gpu * s[:, None]


def acceptance_bound(err_oracle, u_low, norm2_a):
    """err_mixed <= 1.1 err_oracle + 10 u_low ||A||_2."""
    return 1.1 * err_oracle + 10.0 * u_low * norm2_a


def spectral_error(A_np, perm, k, T):
    return orc.id_error(A_np, perm, k, T)[0]
