"""id_factor_noalloc (the allocation-free factorization) against id_factor,
through the C ABI: identical pivots, rank, info and R bit for bit, on two
calls in a row (the second smaller, so stale scratch from the first is
present), plus the pivots of the FP64 case against the oracle."""
import ctypes

import numpy as np
import pytest
import torch

import oracle as orc
import synth
from gpu_helpers import host, need_gpu, to_dev

pytestmark = pytest.mark.gpu


def _noalloc(A, k=None, tol=None, prec="f64"):
    """One id_factor_noalloc call through ctypes; returns (perm, k, R, info)."""
    import paper_2012_00706_amd as mp
    from paper_2012_00706_amd.api import DTYPE, _stream
    lib = mp.load()
    A, lda = mp.colmajor(A)
    m, n = A.shape
    o = mp.make_opts(k=k, tol=tol, prec=prec)
    kc = mp.kcap_of(m, n, o)
    R = torch.full((n, max(kc, 1)), float("nan"), dtype=torch.float64, device=A.device).t()
    perm = torch.full((n,), -1, dtype=torch.int32, device=A.device)
    k_out = ctypes.c_int64(-1)
    info = ctypes.c_int32(-1)
    rc = lib.id_factor_noalloc(A.data_ptr(), DTYPE[A.dtype], m, n, lda, ctypes.byref(o),
                               perm.data_ptr(), R.data_ptr(), R.stride(1), ctypes.byref(k_out),
                               ctypes.byref(info), _stream(A.device))
    assert rc == 0, lib.id_status_string(rc).decode()
    torch.cuda.synchronize()
    kk = int(k_out.value)
    return host(perm).astype(np.int64), kk, host(R[:kk]), int(info.value)


def _factor(A, k=None, tol=None, prec="f64"):
    import paper_2012_00706_amd as mp
    fr = mp.factor(A, k=k, tol=tol, prec=prec)
    torch.cuda.synchronize()
    return host(fr.perm).astype(np.int64), fr.k, host(fr.R), fr.info


def test_noalloc_matches_id_factor_two_calls():
    need_gpu()
    import paper_2012_00706_amd as mp
    assert mp.load().id_noalloc_scratch_bytes() == mp.C["ID_NOALLOC_SCRATCH_MB"] << 20
    # call 1: the FP64 parity matrix (1000 x 500, fixed k = 50)
    A1 = synth.config1()
    d1 = to_dev(A1)
    p, k, R, info = _noalloc(d1, k=50, prec="f64")
    q, kq, Rq, infoq = _factor(d1, k=50, prec="f64")
    assert (k, info) == (kq, infoq) == (50, 0)
    assert np.array_equal(p, q)
    assert np.array_equal(R, Rq)
    ref = orc.cpqr(A1, k=50)
    assert p[:50].tolist() == ref.perm[:50].tolist()
    # call 2, smaller: fp32 storage, split-BF16 update, adaptive rank
    A2 = synth.spectrum_matrix(600, 160, synth.sigma_exp(160, 12.0), 91, 92).astype(np.float32)
    d2 = to_dev(A2)
    p, k, R, info = _noalloc(d2, tol=1e-3, prec="mixed_bf16x3")
    q, kq, Rq, infoq = _factor(d2, tol=1e-3, prec="mixed_bf16x3")
    assert 0 < k < 160 and (k, info) == (kq, infoq)
    assert np.array_equal(p, q)
    assert np.array_equal(R, Rq)


def test_noalloc_refuses_what_does_not_fit():
    need_gpu()
    import paper_2012_00706_amd as mp
    A = torch.zeros((20000, 2000), dtype=torch.float32, device="cuda")
    with pytest.raises(mp.MpidError) as e:
        mp.factor_noalloc(A, tol=1e-3, prec="mixed_bf16x3")
    assert e.value.code == mp.C["ID_ERR_SCRATCH"]
