"""The CholeskyQR tall front end (ID_FLAG_CHOLQR: the pivoted Householder
factorization of R0 = R2 R1 from CholeskyQR2, or R3 R2 R1 from three passes,
the first shifted when its plain Cholesky factorization fails)
against the oracle's column-pivoted Householder QR of A itself.  A = Q R0
with Q orthonormal, so both factorizations are the same one (Section 1.1):
same pivots on gap-separated inputs, R up to row signs to FP64 rounding, T to
kappa(R11) u_64 -- including ranks whose residual norms lie below the Gram
route's sqrt(u_64) floor.  Inputs beyond the route's reach (numerically
rank-deficient A) report ID_INFO_CHOLQR_BREAKDOWN."""
import numpy as np
import pytest
import torch

import oracle as orc
import synth
from gpu_helpers import assert_f64_parity, gpu_id, host, need_gpu, to_dev

pytestmark = pytest.mark.gpu


def _cq(A, **kw):
    import paper_2012_00706_amd as mp
    res = mp.column_id(to_dev(A), cholqr=True, **kw)
    torch.cuda.synchronize()
    return host(res.perm).astype(np.int64), res.k, host(res.R), host(res.T), res.info


@pytest.mark.parametrize("m,n,k,per_decade", [
    (3000, 200, 60, 20.0),   # kappa(A) = 1e10: shifted CholeskyQR3
    (3000, 100, 60, 8.0),    # sigma_60 / sigma_1 = 4e-8: below the Gram route's floor
    (5000, 64, 64, 10.0),    # full rank, T empty; CholeskyQR2
    (700, 130, 1, 20.0),
    (1001, 257, 70, 25.0),   # ragged: odd rows, a 257th column past the 64-wide panels
    (3000, 150, 60, 18.0),   # kappa(A) = 2e8: ||R2 - I||_F near the two-pass bound
    (300, 300, 100, 30.0),   # square (m = n), kappa(A) = 1e10
])
def test_cholqr_fixed_rank_matches_oracle(m, n, k, per_decade):
    need_gpu()
    A = synth.spectrum_matrix(m, n, synth.sigma_geom10(n, per_decade), m + 7, n + 7)
    ref = orc.cpqr(A, k=k)
    perm, kk, R, T, info = _cq(A, k=k)
    assert_f64_parity(perm, kk, R, T, ref, n, info=info)


def test_cholqr_fp32_storage_unaligned():
    """fp32 storage with an odd row count: the Gram products and A R^{-1}
    take their bounds-checked scalar loads of the fp32 columns."""
    need_gpu()
    A = synth.spectrum_matrix(2999, 130, synth.sigma_geom10(130, 20.0), 81, 82).astype(np.float32)
    ref = orc.cpqr(A.astype(np.float64), k=30)
    perm, k, R, T, info = _cq(A, k=30)
    assert_f64_parity(perm, k, R, T, ref, 130, info=info)


@pytest.mark.parametrize("rule", ["pivot_rel", "frob_rel"])
def test_cholqr_adaptive_rank_below_gram_floor(rule):
    """tol = 1e-8 (the Gram route refuses adaptive tolerances below 1e-6):
    the rank and every pivot are the oracle's."""
    need_gpu()
    A = synth.spectrum_matrix(4000, 150, synth.sigma_geom10(150, 15.0), 91, 92)
    ref = orc.cpqr(A, tol=1e-8, rule=rule)
    assert 80 < ref.k < 150
    perm, k, R, T, info = _cq(A, tol=1e-8, rule=rule)
    assert_f64_parity(perm, k, R, T, ref, 150, info=info)


def test_cholqr_tall_fp32_snapshot_like():
    """65536 x 256 fp32 with a snapshot-like spectrum, tol 1e-3: the oracle's
    rank and pivots, and the Householder FP64 path's."""
    need_gpu()
    A = synth.spectrum_matrix(65536, 256, synth.sigma_exp(256, 20.0), 51, 52).astype(np.float32)
    perm, k, R, T, info = _cq(A, tol=1e-3)
    ref = orc.cpqr(A.astype(np.float64), k=k)
    assert k == orc.cpqr(A.astype(np.float64), tol=1e-3).k
    assert_f64_parity(perm, k, R, T, ref, 256, info=info)
    hperm, hk, _, _ = gpu_id(A, tol=1e-3)
    assert hk == k and hperm[:k].tolist() == perm[:k].tolist()


def test_cholqr_breakdown_reported():
    """sigma_i = 10^(-(i-1)/8), n = 200: kappa(A) = 1e25, beyond what the
    shifted first pass can bring within reach of the plain ones; the call
    reports ID_INFO_CHOLQR_BREAKDOWN and factors nothing."""
    need_gpu()
    import paper_2012_00706_amd as mp
    A = synth.spectrum_matrix(3000, 200, synth.sigma_geom10(200, 8.0), 3003, 203)
    fr = mp.factor(to_dev(A), k=60, cholqr=True)
    assert fr.info == mp.C["ID_INFO_CHOLQR_BREAKDOWN"] and fr.k == 0
    assert host(fr.perm).tolist() == list(range(200))
    # the same input through the Householder path is fine
    res = mp.column_id(to_dev(A), k=60)
    assert res.k == 60 and res.info == 0


def test_cholqr_edge_cases():
    need_gpu()
    import paper_2012_00706_amd as mp
    C = mp.C
    fr = mp.factor(torch.zeros((50, 20), dtype=torch.float64, device="cuda"), tol=1e-3, cholqr=True)
    assert fr.k == 0 and fr.info == 0
    assert host(fr.perm).tolist() == list(range(20))
    B = synth.gaussian(60, 10, seed=4)
    B[3, 7] = np.nan
    fr = mp.factor(to_dev(B), tol=1e-3, cholqr=True)
    assert fr.info == C["ID_INFO_NONFINITE"] and fr.k == 0
    one = synth.gaussian(40, 1, seed=5)
    perm, k, R, T, info = _cq(one, k=1)
    assert k == 1 and abs(abs(R[0, 0]) - np.linalg.norm(one)) <= 1e-14 * np.linalg.norm(one)
    full = synth.gaussian(300, 12, seed=6)
    perm, k, R, T, info = _cq(full, tol=1e-12)
    assert k == 12 and T.shape == (12, 0)
    ref = orc.cpqr(full, k=12)
    assert perm.tolist() == ref.perm.tolist()
    with pytest.raises(mp.MpidError) as e:
        mp.factor(to_dev(synth.gaussian(10, 20, seed=7)), k=3, cholqr=True)  # m < n
    assert e.value.code == C["ID_ERR_UNSUPPORTED"]
    for kw in (dict(no_pivot=True), dict(round_to="f32"), dict(profile=True)):
        with pytest.raises(mp.MpidError):
            mp.factor(to_dev(full), k=3, cholqr=True, **kw)
    with pytest.raises((mp.MpidError, ValueError)):
        mp.factor(to_dev(full), k=3, cholqr=True, gram=True)


def test_cholqr_repeated_calls_share_nothing():
    """Two calls in a row with one workspace, the second on a smaller input:
    the flags and buffers are reset per call."""
    need_gpu()
    import paper_2012_00706_amd as mp
    A1 = synth.spectrum_matrix(3000, 200, synth.sigma_geom10(200, 8.0), 3003, 203)  # breaks down
    A2 = synth.spectrum_matrix(2000, 120, synth.sigma_geom10(120, 20.0), 5, 6)
    o = mp.make_opts(60, None, "f64", "pivot_rel", 0, 0, False, False, False, None, True)
    ws = mp.workspace_size(3000, 200, torch.float64, o)
    work = torch.empty(ws, dtype=torch.uint8, device="cuda")
    fr = mp.factor(to_dev(A1), k=60, cholqr=True, work=work)
    assert fr.info == mp.C["ID_INFO_CHOLQR_BREAKDOWN"]
    fr = mp.factor(to_dev(A2), k=40, cholqr=True, work=work)
    ref = orc.cpqr(A2, k=40)
    assert fr.info == 0 and fr.k == 40
    assert host(fr.perm)[:40].tolist() == ref.perm[:40].tolist()
