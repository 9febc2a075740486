"""Sketching front end (id_sketch, then the FP64 factorization of the sketch)
against the oracle's randomized ID on the same seeded test matrix: the sketch
Y = Omega A entry by entry within the FP64 summation bound, the same pivots and
T on gap-separated inputs, exactness at exact rank, edge cases, and sampled
entries of the sketch at the benchmark and snapshot sizes."""
import math

import numpy as np
import pytest
import torch

import oracle as orc
import synth
from gpu_helpers import host, need_gpu, rel_err, to_dev

pytestmark = pytest.mark.gpu


def _omega_dev(Om: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(Om)).cuda()


def _y_bound(Om, A):
    """|Y_gpu - Y| <= gamma_m (|Omega| |A|) for any summation order (gamma_m ~ m u_64)."""
    m = A.shape[0]
    return 1.01 * m * orc.U_DOUBLE * (np.abs(Om) @ np.abs(A.astype(np.float64))) + 1e-300


@pytest.mark.parametrize("l,m,n,dtype", [(70, 2017, 130, np.float64), (64, 4096, 64, np.float32),
                                         (1, 300, 5, np.float64), (130, 50, 200, np.float32),
                                         (20, 70000, 33, np.float32)])
def test_sketch_matches_oracle_entrywise(l, m, n, dtype):
    need_gpu()
    import paper_2012_00706_amd as mp
    A = synth.gaussian(m, n, seed=l + n, dtype=dtype)
    Om = synth.sketch_matrix(l, m, seed=m)
    Y = host(mp.sketch(to_dev(A), _omega_dev(Om)))
    ref = Om @ A.astype(np.float64)
    assert Y.shape == (l, n)
    assert np.all(np.abs(Y - ref) <= _y_bound(Om, A))


@pytest.mark.parametrize("rule,tol,k", [("pivot_rel", 1e-3, None), ("frob_rel", 1e-4, None),
                                        ("pivot_rel", None, 25)])
def test_sketch_id_matches_oracle(rule, tol, k):
    need_gpu()
    import paper_2012_00706_amd as mp
    A = synth.spectrum_matrix(3000, 260, synth.sigma_exp(260, 9.0), 71, 72).astype(np.float32)
    Om = synth.sketch_matrix(96, 3000, seed=73)
    ref = orc.sketch_id(A, Om, k=k, tol=tol, rule=rule)
    res = mp.sketch_id(to_dev(A), _omega_dev(Om), k=k, tol=tol, rule=rule)
    torch.cuda.synchronize()
    assert res.k == ref.k
    perm = host(res.perm).astype(np.int64)
    upto = int(np.argmax(ref.margins < 1e-9)) if np.any(ref.margins < 1e-9) else ref.k
    assert perm[:upto].tolist() == ref.perm[:upto].tolist()
    if upto == ref.k and ref.T.size:
        # Y differs from the oracle's by summation order (~sqrt(m) u_64
        # relative); T = R11^{-1} R12 amplifies that by up to kappa(R11)
        kappa = np.linalg.cond(ref.R[:, :ref.k])
        assert rel_err(host(res.T), ref.T) <= 10 * math.sqrt(3000) * orc.U_DOUBLE * kappa + 1e-12
    assert np.all(np.abs(host(res.Y) - ref.Y) <= _y_bound(Om, A))


def test_sketch_id_exact_rank():
    """A of exact rank 12, l = 40: A(:, J) T reproduces A (float64)."""
    need_gpu()
    import paper_2012_00706_amd as mp
    A = synth.low_rank(5000, 300, 12, seed=81)
    Om = synth.sketch_matrix(40, 5000, seed=82)
    res = mp.sketch_id(to_dev(A), _omega_dev(Om), tol=1e-10)
    assert res.k == 12
    perm = host(res.perm).astype(np.int64)
    E = A[:, perm[12:]] - A[:, perm[:12]] @ host(res.T)
    assert np.linalg.norm(E) <= 1e-11 * np.linalg.norm(A)


def test_sketch_error_close_to_deterministic():
    """Oversampled Gaussian sketch: the error at the sketch's rank stays within
    a small factor of the deterministic ID's error at the same rank."""
    need_gpu()
    import paper_2012_00706_amd as mp
    A = synth.spectrum_matrix(4000, 300, synth.sigma_exp(300, 12.0), 91, 92).astype(np.float32)
    Om = synth.sketch_matrix(120, 4000, seed=93)
    res = mp.sketch_id(to_dev(A), _omega_dev(Om), tol=1e-3)
    k = res.k
    assert 0 < k < 120
    e = orc.id_error(A, host(res.perm).astype(np.int64), k, host(res.T))[0]
    ref = orc.cpqr(A, k=k)
    e_det = orc.id_error(A, ref.perm, k, orc.solve_T(ref.R, k))[0]
    assert e <= 10.0 * e_det


def test_sketch_edge_cases():
    need_gpu()
    import paper_2012_00706_amd as mp
    C = mp.C
    # no rows: Y = 0
    A0 = torch.zeros((0, 7), dtype=torch.float64, device="cuda")
    Y = mp.sketch(A0, torch.zeros((5, 0), dtype=torch.float64, device="cuda"))
    assert Y.shape == (5, 7) and float(Y.abs().max()) == 0.0
    # one column, one sketch row
    a = synth.gaussian(999, 1, seed=3)
    om = synth.sketch_matrix(1, 999, seed=4)
    y = host(mp.sketch(to_dev(a), _omega_dev(om)))
    assert abs(y[0, 0] - math.fsum(om[0] * a[:, 0])) <= _y_bound(om, a)[0, 0]
    # a non-finite entry reaches Y and the factorization of Y reports it
    B = synth.gaussian(200, 9, seed=5)
    B[17, 4] = np.inf
    Yb = mp.sketch(to_dev(B), _omega_dev(synth.sketch_matrix(6, 200, seed=6)))
    assert not torch.isfinite(Yb[:, 4]).any() and torch.isfinite(Yb[:, 3]).all()
    fr = mp.factor(Yb, tol=1e-3)
    assert fr.info == C["ID_INFO_NONFINITE"]
    # shape errors are caught before any launch
    with pytest.raises(ValueError):
        mp.sketch(to_dev(B), torch.zeros((6, 199), dtype=torch.float64, device="cuda"))
    with pytest.raises(ValueError):
        mp.sketch(to_dev(B), torch.zeros((6, 200), dtype=torch.float32, device="cuda"))
    # a transposed (column-major) Omega view is accepted and copied
    Om = synth.sketch_matrix(8, 200, seed=7)
    Omt = torch.from_numpy(np.asfortranarray(Om)).cuda()
    Omt = Omt.t().contiguous().t()
    assert Omt.stride(1) != 1
    np.testing.assert_array_equal(host(mp.sketch(to_dev(B[:, :4]), Omt)),
                                  host(mp.sketch(to_dev(B[:, :4]), _omega_dev(Om))))


def test_sketch_deterministic():
    """Fixed chunk order: two calls give bitwise equal sketches."""
    need_gpu()
    import paper_2012_00706_amd as mp
    A = to_dev(synth.gaussian(30000, 100, seed=11, dtype=np.float32))
    Om = _omega_dev(synth.sketch_matrix(50, 30000, seed=12))
    assert torch.equal(mp.sketch(A, Om), mp.sketch(A, Om))


@pytest.mark.parametrize("case", ["benchmark", "snapshot"])
def test_sketch_full_size_sampled(case):
    """At the benchmark (20000 x 2000, l = 400) and snapshot (1,048,576 x 512,
    l = 320) sizes: 48 sampled entries of Y against FP64 dot products, and the
    randomized ID's error within a factor of the deterministic error bound."""
    need_gpu()
    import paper_2012_00706_amd as mp
    if case == "benchmark":
        A = synth.config2()
        l = 400
    else:
        A = synth.config3()
        l = 320
    m, n = A.shape
    Om = synth.sketch_matrix(l, m, seed=2024)
    Ad, Omd = to_dev(A), _omega_dev(Om)
    Y = host(mp.sketch(Ad, Omd))
    rng = np.random.default_rng(5)
    for r, c in zip(rng.integers(0, l, 48), rng.integers(0, n, 48)):
        ref = math.fsum(Om[r] * A[:, c].astype(np.float64))
        bound = 1.01 * m * orc.U_DOUBLE * float(np.abs(Om[r]) @ np.abs(A[:, c].astype(np.float64)))
        assert abs(Y[r, c] - ref) <= bound
    res = mp.sketch_id(Ad, Omd, tol=1e-3)
    assert 0 < res.k < l
    del Omd
    E = mp.reconstruct(Ad, res.perm, res.k, res.T, residual=True)
    Et = E.t()
    err = math.sqrt(max(float(torch.linalg.eigvalsh(torch.mm(Et, Et.t()))[-1]), 0.0))
    fro = float(torch.linalg.norm(Ad.double()))
    # the error sits at the level the rank rule asked for (tol times the
    # largest column norm, within the usual sqrt(k (n - k)) growth)
    assert err <= 1e-3 * fro * math.sqrt(1 + res.k * (n - res.k))
    if case == "benchmark":
        # known spectrum: within the column-ID growth factor of sigma_{k+1}
        sig = synth.sigma_exp(min(m, n), 40.0)
        assert err <= 10.0 * math.sqrt(1 + res.k * (n - res.k)) * sig[res.k]
