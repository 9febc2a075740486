"""The lock-step batched path (id_factor_lockstep through the C ABI): every
item against the oracle (pivots, R and T element-wise on gap-separated FP64
inputs), panel widths, row-tile and column-chunk shapes, mixed-precision
acceptance, per-item conditions, agreement with the single-matrix path, and
members of the batched workload at full size checked through properties that
hold at any size."""
import numpy as np
import pytest
import torch

import oracle as orc
import synth
from gpu_helpers import U_LOW, host, need_gpu, to_dev
from test_gpu_batched import SHAPES, _check_item_f64, _inputs

pytestmark = pytest.mark.gpu


def test_lockstep_fixed_rank_matches_oracle():
    need_gpu()
    import paper_2012_00706_amd as mp
    As = _inputs(SHAPES)
    res = mp.factor_lockstep([to_dev(A) for A in As], k=40, prec="f64")
    for A, r in zip(As, res):
        _check_item_f64(A, r, k_req=40)


@pytest.mark.parametrize("rule", ["pivot_rel", "frob_rel"])
def test_lockstep_adaptive_rank_matches_oracle(rule):
    """Items that stop at very different ranks (a few steps to several
    panels): each one leaves the step launches when it is done."""
    need_gpu()
    import paper_2012_00706_amd as mp
    shapes = [(800, 200), (450, 130), (1200, 96), (333, 300), (600, 40), (2500, 180)]
    decays = [10.0, 4.0, 30.0, 10.0, 2.0, 60.0]
    As = [synth.spectrum_matrix(m, n, synth.sigma_exp(min(m, n), d), 41 + i, 42 + i)
          for i, ((m, n), d) in enumerate(zip(shapes, decays))]
    res = mp.factor_lockstep([to_dev(A) for A in As], tol=1e-3, rule=rule, prec="f64")
    ks = [r.k for r in res]
    assert max(ks) > 2 * min(ks)
    for A, r in zip(As, res):
        _check_item_f64(A, r, tol=1e-3, rule=rule)


@pytest.mark.parametrize("nb", [1, 7, 32])
def test_lockstep_panel_width(nb):
    need_gpu()
    import paper_2012_00706_amd as mp
    As = _inputs([(500, 120), (700, 64), (260, 200), (1500, 300)], decay=15.0, seed0=500)
    res = mp.factor_lockstep([to_dev(A) for A in As], k=45, prec="f64", nb=nb)
    for A, r in zip(As, res):
        _check_item_f64(A, r, k_req=45)


@pytest.mark.parametrize("rt,cw", [(64, 0), (256, 0), (128, 128), (128, 512)])
def test_lockstep_tile_shapes(monkeypatch, rt, cw):
    """Row tiles of 64 / 128 / 256 rows and FP64 column chunks of 128 / 256 /
    512 positions give the oracle's pivots, R and T (several tiles and chunks
    with ragged tails)."""
    need_gpu()
    import paper_2012_00706_amd as mp
    monkeypatch.setenv("MPID_LOCKSTEP_RT", str(rt))
    if cw:
        monkeypatch.setenv("MPID_LOCKSTEP_CW", str(cw))
    As = _inputs([(3000, 700), (1000, 257), (129, 33), (5000, 90)], seed0=610)
    res = mp.factor_lockstep([to_dev(A) for A in As], k=50, prec="f64")
    for A, r in zip(As, res):
        _check_item_f64(A, r, k_req=50)


def test_lockstep_f32_storage_f64_path():
    need_gpu()
    import paper_2012_00706_amd as mp
    As = _inputs([(700, 130), (300, 80)], dtype=np.float32, decay=10.0, seed0=700)
    res = mp.factor_lockstep([to_dev(A) for A in As], k=33, prec="f64")
    for A, r in zip(As, res):
        _check_item_f64(A.astype(np.float64), r, k_req=33)


@pytest.mark.parametrize("prec", ["mixed_bf16x3", "mixed_bf16", "mixed_f16", "mixed_f32"])
def test_lockstep_mixed_acceptance(prec):
    """Mixed precision is accepted on error: at the rank it chose, each item's
    spectral error is within 1.1x the oracle's at the same rank plus
    10 u_low ||A||_2."""
    need_gpu()
    import paper_2012_00706_amd as mp
    u_low = U_LOW[prec]
    shapes = [(3000, 400), (1500, 250), (800, 600), (2000, 97)]
    As, norms = [], []
    for i, (m, n) in enumerate(shapes):
        s = synth.sigma_exp(min(m, n), 40.0)
        As.append(synth.spectrum_matrix(m, n, s, 51 + 2 * i, 52 + 2 * i).astype(np.float32))
        norms.append(s[0])
    res = mp.factor_lockstep([to_dev(A) for A in As], tol=1e-3, prec=prec)
    for A, r, nrm in zip(As, res, norms):
        assert r.k > 0 and r.info in (0, mp.C["ID_INFO_RANK_FULL"])
        perm = host(r.perm).astype(np.int64)
        e = orc.id_error(A, perm, r.k, host(r.T))[0]
        ref = orc.cpqr(A, k=r.k)
        e_ref = orc.id_error(A, ref.perm, r.k, orc.solve_T(ref.R, r.k))[0]
        assert e <= 1.1 * e_ref + 10 * u_low * nrm


def test_lockstep_matches_single_path():
    """Every item gets the rank, pivots and (to rounding) R and T of
    id_factor with the same options, FP64 and the benchmark's mixed BF16x3."""
    need_gpu()
    import paper_2012_00706_amd as mp
    As = _inputs([(1000, 257), (2100, 100), (300, 150), (4000, 600)], seed0=900)
    # the two paths sum in different orders (other sweep tiles): R to rounding
    # of the working copy (FP64, or FP32 for the mixed path), T through R11^-1
    for prec, tol, rtol_r, rtol_t in (("f64", 1e-9, 1e-12, 1e-8),
                                      ("mixed_bf16x3", 1e-3, 1e-5, 1e-2)):
        Ad = [to_dev(A.astype(np.float32)) for A in As]
        res = mp.factor_lockstep(Ad, tol=tol, prec=prec)
        for A, r in zip(Ad, res):
            one = mp.column_id(A, tol=tol, prec=prec)
            # the lock-step info also carries id_solve_T's conditions
            want = one.info or (mp.C["ID_INFO_RANK_FULL"] if one.k == A.shape[1] else 0)
            assert r.k == one.k and r.info == want, (prec, r.k, r.info, one.k, one.info)
            assert np.array_equal(host(r.perm), host(one.perm)), prec
            R1 = np.asarray(host(one.R))[:, :one.k]
            dR = np.max(np.abs(np.asarray(host(r.R))[:, :r.k] - R1))
            assert dR <= rtol_r * np.max(np.abs(R1)), (prec, dR)
            T1 = np.asarray(host(one.T))
            dT = np.max(np.abs(np.asarray(host(r.T)) - T1)) if T1.size else 0.0
            assert dT <= rtol_t * max(np.max(np.abs(T1)) if T1.size else 0.0, 1.0), (prec, dT)


def test_lockstep_item_conditions():
    """NaN in one item, an all-zero item, a full-rank item and a numerically
    singular fixed-rank item each get their own info; the others are unaffected."""
    need_gpu()
    import paper_2012_00706_amd as mp
    C = mp.C
    good = synth.spectrum_matrix(200, 60, synth.sigma_geom10(60, 12.0), 1, 2)
    bad = synth.gaussian(80, 20, seed=3)
    bad[5, 7] = np.inf
    zero = np.zeros((50, 20))
    res = mp.factor_lockstep([to_dev(x) for x in (good, bad, zero)], tol=1e-3, prec="f64")
    _check_item_f64(good, res[0], tol=1e-3)
    assert res[1].info == C["ID_INFO_NONFINITE"] and res[1].k == 0
    assert res[2].k == 0 and res[2].info == 0
    assert sorted(host(res[2].perm).tolist()) == list(range(20))
    full = synth.gaussian(40, 12, seed=2)
    low = synth.low_rank(60, 20, 4, seed=3)
    res = mp.factor_lockstep([to_dev(full), to_dev(low)], k=8, prec="f64")
    assert res[0].k == 8 and res[0].info == 0
    assert res[1].k == 8 and res[1].info == C["ID_INFO_SINGULAR"]
    res = mp.factor_lockstep([to_dev(full)], tol=1e-14, prec="f64")
    assert res[0].k == 12 and res[0].info == C["ID_INFO_RANK_FULL"] and res[0].T.shape == (12, 0)


def test_lockstep_repeat_calls_and_plans():
    """A plan runs twice with the same results; two plans in a row (the
    second smaller) do not disturb each other's state."""
    need_gpu()
    import paper_2012_00706_amd as mp
    As = _inputs([(1000, 257), (300, 150), (2100, 100)], seed0=960)
    plan = mp.LockstepID([to_dev(A) for A in As], k=30, prec="f64")
    plan.run()
    first = [(r.k, host(r.perm).copy(), host(r.R).copy(), host(r.T).copy()) for r in plan.results()]
    small = mp.factor_lockstep([to_dev(As[1])], k=12, prec="f64")
    _check_item_f64(As[1], small[0], k_req=12)
    plan.run()
    for a, r in zip(first, plan.results()):
        assert a[0] == r.k
        assert np.array_equal(a[1], host(r.perm))
        assert np.array_equal(a[2], host(r.R)) and np.array_equal(a[3], host(r.T))


def test_lockstep_rejects_tall_items():
    need_gpu()
    import paper_2012_00706_amd as mp
    with pytest.raises(ValueError):
        mp.LockstepID([torch.zeros((3, 49153), device="cuda").t()], k=2)


def test_lockstep_workload_full_size_properties():
    """Sixteen members of the batched workload (m up to 20000, n up to 800,
    sigma_j = j^-2, fp32, tol 1e-4, mixed BF16x3) at full size, checked through
    properties that hold at any size: the rank rule at the chosen k (from the
    FP64 residual A - A_J T) and pivot dominance of R; the three smallest
    members against the oracle's error at the same k."""
    need_gpu()
    import paper_2012_00706_amd as mp
    mats = synth.config4(batch=16)
    As = [to_dev(A) for A in mats]
    tol = 1e-4
    res = mp.factor_lockstep(As, tol=tol, prec="mixed_bf16x3")
    for A, r in zip(As, res):
        m, n = A.shape
        k = r.k
        assert 0 < k <= min(m, n)
        d = r.R.diagonal()[:k].abs()
        r00 = float(d[0])
        if k < n:
            assert float(d[-1]) > tol * r00 * (1 - 1e-2)
            E = mp.reconstruct(A, r.perm, k, r.T, residual=True)
            assert float(E.norm(dim=0).max()) <= tol * r00 * (1 + 1e-2)
        Rh = host(r.R)
        for j in range(0, k, max(1, k // 16)):
            tail = np.sqrt((Rh[j:, j + 1:] ** 2).sum(axis=0))
            assert np.all(abs(Rh[j, j]) >= tail * (1 - 1e-2) - 1e-6)
    for i in np.argsort([a.shape[0] * a.shape[1] for a in mats])[:3]:
        A, r = mats[i], res[i]
        perm = host(r.perm).astype(np.int64)
        e = orc.id_error(A, perm, r.k, host(r.T))[0]
        ref = orc.cpqr(A, k=r.k)
        e_ref = orc.id_error(A, ref.perm, r.k, orc.solve_T(ref.R, r.k))[0]
        assert e <= 1.1 * e_ref + 10 * U_LOW["mixed_bf16x3"] * 1.0  # sigma_1 = 1


def test_lockstep_simulated_single_matches_single_path():
    """The simulated single precision ID (every kept value rounded to binary32,
    the FP32 update) in lock step gives each item the rank, pivots and
    (rounded) T of column_id with the same options."""
    need_gpu()
    import paper_2012_00706_amd as mp
    As = [to_dev(A.astype(np.float32)) for A in _inputs([(1500, 300), (800, 120)], seed0=980)]
    res = mp.factor_lockstep(As, tol=1e-4, prec="mixed_f32", round_to="f32")
    for A, r in zip(As, res):
        one = mp.column_id(A, tol=1e-4, prec="mixed_f32", round_to="f32")
        assert r.k == one.k
        assert np.array_equal(host(r.perm), host(one.perm))
        T1 = np.asarray(host(one.T))
        Tl = np.asarray(host(r.T))
        # T rounded to binary32 on both sides
        assert np.array_equal(Tl.astype(np.float32).astype(np.float64), Tl)
        assert np.max(np.abs(Tl - T1)) <= 1e-5 * max(np.max(np.abs(T1)), 1.0)


def test_concurrent_calls_from_two_threads():
    """Two host threads factoring on their own streams at the same time (each
    with its own pinned panel-end slots) get the results of sequential calls."""
    need_gpu()
    import threading
    import paper_2012_00706_amd as mp
    As = [to_dev(A) for A in _inputs([(3000, 400), (2500, 350)], seed0=990)]
    ref = [mp.column_id(A, tol=1e-8, prec="f64") for A in As]
    torch.cuda.synchronize()
    out = [None, None]
    errs = []

    def work(idx):
        try:
            s = torch.cuda.Stream()
            with torch.cuda.stream(s):
                for _ in range(3):
                    r = mp.column_id(As[idx], tol=1e-8, prec="f64")
                s.synchronize()
                out[idx] = r
        except Exception as e:  # noqa: BLE001 -- reported below
            errs.append(e)

    ts = [threading.Thread(target=work, args=(i,)) for i in range(2)]
    for t in ts:
        t.start()
    for t in ts:
        t.join()
    assert not errs, errs
    for r, q in zip(out, ref):
        assert r.k == q.k
        assert np.array_equal(host(r.perm), host(q.perm))
        assert np.array_equal(host(r.R), host(q.R))
        assert np.array_equal(host(r.T), host(q.T))
