"""id_solve_T (T = R11^-1 R12, FP64) against a library triangular solve, at
sizes around the 64-row and 16-column tile edges, plus the singular case."""
import numpy as np
import pytest
import scipy.linalg
import torch

from gpu_helpers import host, need_gpu, rel_err, to_dev

pytestmark = pytest.mark.gpu


def _upper(k, n, seed):
    rng = np.random.default_rng(seed)
    R = np.triu(rng.standard_normal((k, n)))
    d = np.abs(np.diag(R[:, :k])) + 1.0
    R[np.arange(k), np.arange(k)] = d * np.sign(rng.standard_normal(k))
    return R


@pytest.mark.parametrize("k,extra", [(1, 1), (1, 0), (16, 15), (63, 17), (64, 16), (65, 33),
                                     (130, 100), (300, 257)])
def test_solve_T_matches_library(k, extra):
    need_gpu()
    import paper_2012_00706_amd as mp
    n = k + extra
    R = _upper(k, n, seed=k * 1000 + extra)
    T, info = mp.solve_T(to_dev(R), k, n)
    torch.cuda.synchronize()
    if extra == 0:
        assert int(info.item()) == mp.C["ID_INFO_RANK_FULL"]
        return
    assert int(info.item()) == 0
    ref = scipy.linalg.solve_triangular(R[:, :k], R[:, k:], lower=False)
    cond = np.linalg.cond(R[:, :k])
    assert rel_err(host(T), ref) <= 1e-13 * cond
    # element by element, relative to the largest entry
    assert np.abs(host(T) - ref).max() <= 1e-13 * cond * np.abs(ref).max()


def test_solve_T_singular_reported():
    need_gpu()
    import paper_2012_00706_amd as mp
    R = _upper(10, 30, seed=3)
    R[6, 6] = 0.0
    T, info = mp.solve_T(to_dev(R), 10, 30, check=False)
    torch.cuda.synchronize()
    assert int(info.item()) == mp.C["ID_INFO_SINGULAR"]
