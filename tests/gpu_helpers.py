"""Helpers for the GPU tests: moving seeded inputs to the device and comparing
the HIP path's results with the oracle's."""
import numpy as np
import pytest
import torch

import oracle as orc

# Unit round-off of the split-BF16 update (ID_PREC_MIXED_BF16X3): each operand
# is x = hi + lo with hi, lo BF16 (8 significand bits each), and the product is
# hi*hi + hi*lo + lo*hi with FP32 accumulation.  The dropped lo*lo term and the
# remainder of the split are each below 2^-16 of the product, so the update is
# accurate to about 2^-16 of its size (the FP32 accumulation adds 2^-24).
U_BF16X3 = 2.0 ** -16

# Unit round-off per precision policy, for the acceptance rule
# err_mixed <= 1.1 err_oracle + 10 u_low ||A||_2.
U_LOW = {"mixed_bf16": orc.U_BF16, "mixed_bf16x3": U_BF16X3, "mixed_f16": orc.U_HALF,
         "mixed_f32": orc.U_SINGLE, "f64": orc.U_DOUBLE}


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


def assert_f64_parity(perm, k, R, T, ref, n, info=0):
    """Strict parity of an FP64 result with the oracle's CPQR ``ref`` (same k).

    The input must be gap-separated (every oracle pivot margin > 1e-8: the
    check fails otherwise, so no comparison is skipped).  Then the pivots are
    equal, R matches row by row up to row signs to 1e-12 max|R| element-wise,
    and T = R11^{-1} R12 matches element-wise to
    1e-12 max|T| max(1, kappa(R11) / 1e3) (the solve amplifies the rounding of
    R by up to kappa(R11)).  Returns the number of T entries compared."""
    assert k == ref.k
    if k:
        assert ref.margins.min() > 1e-8, "input not gap-separated"
    perm = np.asarray(perm).astype(np.int64)
    assert perm[:k].tolist() == ref.perm[:k].tolist()
    if k == 0:
        return 0
    np.testing.assert_allclose(row_sign_align(R[:k], ref.R), ref.R, rtol=0,
                               atol=1e-12 * np.abs(ref.R).max())
    if k == n:
        assert T.size == 0
        return 0
    assert info == 0
    Tref = orc.solve_T(ref.R, k)
    kappa = np.linalg.cond(ref.R[:, :k])
    tol = 1e-12 * np.abs(Tref).max() * max(1.0, kappa / 1e3)
    assert T.shape == Tref.shape
    dmax = np.abs(T - Tref).max()
    assert dmax <= tol, f"max |dT| {dmax:.3e} > {tol:.3e} (kappa {kappa:.2e})"
    return T.size
