"""The tall-skinny front end (ID_FLAG_GRAM: pivots and R from the FP64 Gram
matrix by pivoted Cholesky) against the oracle's column-pivoted Householder QR:
same pivots on gap-separated inputs, R up to row signs, T within the
kappa(R11)^2 u_64 error of the Gram route, the acceptance rule on a tall matrix,
and edge cases."""
import numpy as np
import pytest
import torch

import oracle as orc
import synth
from gpu_helpers import host, need_gpu, rel_err, row_sign_align, to_dev

pytestmark = pytest.mark.gpu


def _gram_id(A, **kw):
    import paper_2012_00706_amd as mp
    res = mp.column_id(to_dev(A), gram=True, **kw)
    torch.cuda.synchronize()
    return host(res.perm).astype(np.int64), res.k, host(res.R), host(res.T)


def _check(A, ref, perm, k, R, T):
    assert k == ref.k
    upto = int(np.argmax(ref.margins < 1e-7)) if np.any(ref.margins < 1e-7) else k
    assert perm[:upto].tolist() == ref.perm[:upto].tolist()
    if upto == k and k > 0:
        # row j of R from the Gram route is good to about u_64 ||A||^2 / |R_jj|
        Ra = row_sign_align(R, ref.R)
        nrm2 = np.linalg.norm(A, 2) ** 2
        tol_rows = 1e-13 * nrm2 / np.abs(np.diag(ref.R[:, :k])) + 1e-13 * np.abs(ref.R).max()
        assert np.all(np.abs(Ra - ref.R).max(axis=1) <= tol_rows)
        if T.size:
            kappa = np.linalg.cond(ref.R[:, :k])
            assert rel_err(T, orc.solve_T(ref.R, k)) <= 1e-14 * max(kappa, 1.0) ** 2 + 1e-13


@pytest.mark.parametrize("m,n,k", [(3000, 200, 60), (1000, 257, 70), (5000, 64, 64), (700, 130, 1)])
def test_gram_fixed_rank_matches_oracle(m, n, k):
    need_gpu()
    # sigma_k / sigma_1 >= 1e-4: within the front end's resolution (sqrt(u_64))
    A = synth.spectrum_matrix(m, n, synth.sigma_geom10(min(m, n), 20.0), m + 3, n + 3)
    ref = orc.cpqr(A, k=k)
    _check(A, ref, *_gram_id(A, k=k))


@pytest.mark.parametrize("m,n,k,dtype", [(3001, 150, 40, np.float32), (2999, 130, 30, np.float64)])
def test_gram_unaligned_columns(m, n, k, dtype):
    """Odd row counts: columns of A are not 16-byte aligned, so the Gram
    product takes its bounds-checked scalar loads."""
    need_gpu()
    A = synth.spectrum_matrix(m, n, synth.sigma_geom10(min(m, n), 20.0), m + 5, n + 5).astype(dtype)
    ref = orc.cpqr(A.astype(np.float64), k=k)
    _check(A.astype(np.float64), ref, *_gram_id(A, k=k))


@pytest.mark.parametrize("rule", ["pivot_rel", "frob_rel"])
def test_gram_adaptive_rank_matches_oracle(rule):
    need_gpu()
    A = synth.spectrum_matrix(4000, 300, synth.sigma_exp(300, 12.0), 31, 32)
    ref = orc.cpqr(A, tol=1e-3, rule=rule)
    _check(A, ref, *_gram_id(A, tol=1e-3, rule=rule))


def test_gram_fp32_storage():
    need_gpu()
    A = synth.spectrum_matrix(6000, 180, synth.sigma_geom10(180, 15.0), 41, 42).astype(np.float32)
    ref = orc.cpqr(A.astype(np.float64), k=50)
    _check(A, ref, *_gram_id(A, k=50))


def test_gram_tall_acceptance():
    """65536 x 256 fp32 with a snapshot-like spectrum: the error at the chosen
    rank is within the acceptance rule of the oracle's at the same rank."""
    need_gpu()
    s = synth.sigma_exp(256, 20.0)
    A = synth.spectrum_matrix(65536, 256, s, 51, 52).astype(np.float32)
    perm, k, R, T = _gram_id(A, tol=1e-3)
    assert k > 0
    e = orc.id_error(A, perm, k, T)[0]
    ref = orc.cpqr(A, k=k)
    e_ref = orc.id_error(A, ref.perm, k, orc.solve_T(ref.R, k))[0]
    assert e <= 1.1 * e_ref + 10 * orc.U_DOUBLE ** 0.5 * s[0]


def test_gram_matches_householder_path():
    need_gpu()
    import paper_2012_00706_amd as mp
    A = synth.spectrum_matrix(8000, 240, synth.sigma_exp(240, 15.0), 61, 62)
    At = to_dev(A)
    a = mp.column_id(At, tol=1e-4, gram=True)
    b = mp.column_id(At, tol=1e-4)
    assert a.k == b.k
    ref = orc.cpqr(A, tol=1e-4)
    upto = int(np.argmax(ref.margins < 1e-7)) if np.any(ref.margins < 1e-7) else ref.k
    assert host(a.perm)[:upto].tolist() == host(b.perm)[:upto].tolist()


def test_gram_edge_cases():
    need_gpu()
    import paper_2012_00706_amd as mp
    C = mp.C
    fr = mp.factor(torch.zeros((50, 20), dtype=torch.float64, device="cuda"), tol=1e-3, gram=True)
    assert fr.k == 0 and fr.info == 0
    assert host(fr.perm).tolist() == list(range(20))
    B = synth.gaussian(60, 10, seed=4)
    B[3, 7] = np.nan
    fr = mp.factor(to_dev(B), tol=1e-3, gram=True)
    assert fr.info == C["ID_INFO_NONFINITE"] and fr.k == 0
    one = synth.gaussian(40, 1, seed=5)
    perm, k, R, T = _gram_id(one, k=1)
    assert k == 1 and abs(abs(R[0, 0]) - np.linalg.norm(one)) <= 1e-13 * np.linalg.norm(one)
    full = synth.gaussian(300, 12, seed=6)
    # full rank through the fixed rank (an adaptive 1e-12 is below the
    # route's resolution and refused)
    res = mp.column_id(to_dev(full), k=12, gram=True)
    assert res.k == 12 and res.T.shape == (12, 0)
    with pytest.raises(mp.MpidError):
        mp.column_id(to_dev(full), tol=1e-12, gram=True)
    with pytest.raises(mp.MpidError):
        mp.factor(to_dev(full), k=3, gram=True, no_pivot=True)


def test_gram_guard_stops_at_resolution_floor():
    """sigma_i = 10^(-(i-1)/8), k = 60 (sigma_60 / sigma_1 = 4e-8): the Gram
    route resolves residual norms only down to about sqrt(8 n u_64) |R_00|
    (4.2e-7 at n = 200), so it stops there with ID_INFO_GRAM_LIMIT instead of
    returning pivots chosen by rounding noise.  The steps it made follow the
    oracle's pivots wherever the Gram rounding (relative perturbation of the
    residual norms about 64 u_64 |R_00|^2 / r_j^2) cannot reorder them."""
    need_gpu()
    import paper_2012_00706_amd as mp
    n = 200
    A = synth.spectrum_matrix(3000, n, synth.sigma_geom10(n, 8.0), 3003, 203)
    res = mp.column_id(to_dev(A), k=60, gram=True)
    assert res.info == mp.C["ID_INFO_GRAM_LIMIT"]
    k = res.k
    assert 0 < k < 60
    ref = orc.cpqr(A, k=60)
    r00 = ref.pivot_norms[0]
    floor = np.sqrt(8 * n * 2.0 ** -53) * r00
    # the stop sits at the floor (within the Gram route's own rounding)
    assert ref.pivot_norms[k] <= 1.5 * floor and ref.pivot_norms[k - 1] >= floor / 1.5
    delta = 64 * 2.0 ** -53 * r00 ** 2 / ref.pivot_norms ** 2
    bad = ref.margins[:k] <= delta[:k]
    upto = int(np.argmax(bad)) if np.any(bad) else k
    assert upto >= k // 2
    perm = host(res.perm).astype(np.int64)
    assert perm[:upto].tolist() == ref.perm[:upto].tolist()


def test_gram_refuses_tolerance_below_resolution():
    need_gpu()
    import paper_2012_00706_amd as mp
    A = synth.spectrum_matrix(2000, 100, synth.sigma_geom10(100, 8.0), 5, 6)
    with pytest.raises(mp.MpidError) as e:
        mp.column_id(to_dev(A), tol=1e-7, gram=True)
    assert e.value.code == mp.C["ID_ERR_UNSUPPORTED"]
    res = mp.column_id(to_dev(A), tol=1e-6, gram=True)  # at the limit: accepted
    assert res.k > 0
