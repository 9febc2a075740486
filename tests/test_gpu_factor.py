"""Parity of the HIP factorization + solve (through the C ABI) with the CPU
oracle: FP64 pivots exactly and T to 1e-12 on gap-separated inputs, at sizes
that span several tiles with ragged tails; edge cases; determinism."""
import numpy as np
import pytest
import torch

import oracle as orc
import synth
from gpu_helpers import (U_LOW, assert_f64_parity, gpu_id, host, need_gpu, rel_err,
                         row_sign_align, to_dev)

pytestmark = pytest.mark.gpu


def _check_f64_parity(A, k):
    """FP64 path vs the oracle: strict parity (gap-separated input; pivots,
    R and T element-wise) and the same spectral error."""
    perm, kk, R, T = gpu_id(A, k=k, prec="f64")
    ref = orc.cpqr(A, k=k)
    assert_f64_parity(perm, kk, R, T, ref, A.shape[1])
    if 0 < kk < A.shape[1]:
        e = orc.id_error(A, perm, kk, T)[0]
        e_ref = orc.id_error(A, ref.perm, kk, orc.solve_T(ref.R, kk))[0]
        assert abs(e - e_ref) <= 1e-10 * max(e_ref, 1e-300) + 1e-14 * np.linalg.norm(A, 2)


def test_config1_f64_parity():
    need_gpu()
    A = synth.config1()
    _check_f64_parity(A, 50)


@pytest.mark.parametrize("m,n,k", [
    (300, 150, 40),     # several sweep tiles, one panel + part
    (1000, 257, 70),    # ragged column tail, three panels
    (2100, 100, 33),    # many row tiles, panel boundary + 1
    (65, 64, 64),       # full rank square-ish, m = 65
    (129, 33, 33),      # k = n
    (40, 90, 40),       # wide: k = m
])
def test_f64_parity_shapes(m, n, k):
    """Every input here is gap-separated (smallest oracle margin >= 1.3e-4), so
    pivots, R and T are compared in full."""
    need_gpu()
    r = min(m, n)
    A = synth.spectrum_matrix(m, n, synth.sigma_geom10(r, 12.0), 100 + m, 200 + n)
    _check_f64_parity(A, k)


@pytest.mark.parametrize("nb", [1, 7, 32])
def test_panel_width_does_not_change_result(nb):
    need_gpu()
    A = synth.spectrum_matrix(500, 120, synth.sigma_geom10(120, 15.0), 5, 6)
    ref = orc.cpqr(A, k=45)
    perm, kk, R, T = gpu_id(A, k=45, prec="f64", nb=nb)
    assert assert_f64_parity(perm, kk, R, T, ref, 120) > 0


@pytest.mark.parametrize("rule", ["pivot_rel", "frob_rel"])
def test_adaptive_rank_matches_oracle(rule):
    need_gpu()
    A = synth.spectrum_matrix(800, 200, synth.sigma_exp(200, 10.0), 41, 42)
    tol = 1e-3
    ref = orc.cpqr(A, tol=tol, rule=rule)
    perm, kk, R, T = gpu_id(A, tol=tol, rule=rule, prec="f64")
    assert assert_f64_parity(perm, kk, R, T, ref, 200) > 0


def test_exact_low_rank_recovered():
    need_gpu()
    A = synth.low_rank(700, 130, 23, seed=3)
    perm, kk, R, T = gpu_id(A, tol=1e-10, prec="f64")
    assert kk == 23
    _, ef = orc.id_error(A, perm, kk, T)
    assert ef <= 1e-12 * np.linalg.norm(A)


@pytest.mark.parametrize("prec", ["mixed_bf16", "mixed_f16", "mixed_bf16x3", "mixed_f32"])
def test_mixed_acceptance_bound(prec):
    """err_mixed <= 1.1 err_oracle(same k) + 10 u_low ||A||_2 with the unit
    round-off of each policy's update (BF16 2^-8, FP16 2^-11, split BF16
    2^-16, FP32 2^-24)."""
    need_gpu()
    u_low = U_LOW[prec]
    A = synth.spectrum_matrix(3000, 400, synth.sigma_exp(400, 40.0), 51, 52).astype(np.float32)
    perm, kk, R, T = gpu_id(A, tol=1e-3, prec=prec)
    assert kk > 0
    e_mixed = orc.id_error(A, perm, kk, T)[0]
    ref = orc.cpqr(A, k=kk)
    e_ref = orc.id_error(A, ref.perm, kk, orc.solve_T(ref.R, kk))[0]
    norm2 = synth.sigma_exp(400, 40.0)[0]
    assert e_mixed <= 1.1 * e_ref + 10 * u_low * norm2


def test_mixed_fp16_tiny_values_scaled():
    """The FP16 path scales its operands by powers of two, so a matrix whose
    entries sit far below FP16's normal range still factors accurately."""
    need_gpu()
    A = (synth.spectrum_matrix(1500, 200, synth.sigma_pow(200, 2.0), 61, 62) * 1e-9).astype(np.float32)
    perm, kk, R, T = gpu_id(A, k=40, prec="mixed_f16")
    e = orc.id_error(A, perm, kk, T)[0]
    ref = orc.cpqr(A, k=40)
    e_ref = orc.id_error(A, ref.perm, 40, orc.solve_T(ref.R, 40))[0]
    assert e <= 1.1 * e_ref + 10 * orc.U_HALF * 1e-9


def test_identity_block_and_reconstruction():
    need_gpu()
    import paper_2012_00706_amd as mp
    A = synth.spectrum_matrix(400, 90, synth.sigma_exp(90, 8.0), 71, 72)
    At = to_dev(A)
    res = mp.column_id(At, k=30)
    Y = host(mp.reconstruct(At, res.perm, res.k, res.T))
    perm = host(res.perm).astype(np.int64)
    J = perm[:30]
    assert np.array_equal(Y[:, J], A[:, J])
    Yref = orc.reconstruct(A, perm, 30, host(res.T))
    assert rel_err(Y, Yref) <= 1e-14
    E = host(mp.reconstruct(At, res.perm, res.k, res.T, residual=True))
    assert rel_err(E, A - Yref) <= 1e-10


def test_determinism_bitwise():
    need_gpu()
    A = synth.spectrum_matrix(2000, 300, synth.sigma_exp(300, 30.0), 81, 82).astype(np.float32)
    p1, k1, R1, T1 = gpu_id(A, tol=1e-3, prec="mixed_bf16")
    p2, k2, R2, T2 = gpu_id(A, tol=1e-3, prec="mixed_bf16")
    assert k1 == k2 and np.array_equal(p1, p2)
    assert np.array_equal(R1, R2) and np.array_equal(T1, T2)


# ---------------------------------------------------------------- edge cases

def test_zero_matrix_gives_rank_zero():
    need_gpu()
    import paper_2012_00706_amd as mp
    A = torch.zeros((50, 20), dtype=torch.float64, device="cuda")
    fr = mp.factor(A, tol=1e-3)
    assert fr.k == 0


def test_nonfinite_input_reported():
    need_gpu()
    import paper_2012_00706_amd as mp
    A = synth.gaussian(60, 10, seed=1)
    A[7, 3] = np.nan
    fr = mp.factor(to_dev(A), tol=1e-3)
    assert fr.info == mp.C["ID_INFO_NONFINITE"] and fr.k == 0


def test_full_rank_and_singular_fixed_rank():
    need_gpu()
    import paper_2012_00706_amd as mp
    A = synth.gaussian(40, 12, seed=2)
    res = mp.column_id(to_dev(A), tol=1e-14)
    assert res.k == 12 and res.T.shape == (12, 0)
    L = synth.low_rank(60, 20, 4, seed=3)
    fr = mp.factor(to_dev(L), k=8)
    with pytest.raises(mp.MpidError):
        mp.solve_T(fr.R, fr.k, 20)


@pytest.mark.parametrize("m,n", [(1, 1), (1, 7), (9, 1), (2, 3)])
def test_degenerate_shapes(m, n):
    need_gpu()
    A = synth.gaussian(m, n, seed=m * 10 + n)
    k = min(m, n)
    perm, kk, R, T = gpu_id(A, k=k, prec="f64")
    ref = orc.cpqr(A, k=k)
    assert perm[:k].tolist() == ref.perm[:k].tolist()
    np.testing.assert_allclose(np.abs(R), np.abs(ref.R), rtol=1e-13, atol=1e-14)


@pytest.mark.parametrize("m,n,k", [(2000, 200, 120), (3000, 150, 70), (700, 300, 97)])
def test_fixed_rank_below_n_multi_panel(m, n, k):
    """Fixed k < n over several panels: the last rows of R (and so T) match the
    oracle; steps enqueued after the last one must leave them alone."""
    need_gpu()
    A = synth.spectrum_matrix(m, n, synth.sigma_geom10(min(m, n), 40.0), m + 1, n + 1)
    perm, kk, R, T = gpu_id(A, k=k, prec="f64")
    ref = orc.cpqr(A, k=k)
    assert kk == k
    assert assert_f64_parity(perm, kk, R, T, ref, n) > 0


def test_mixed_f32_matches_fp64_pivots():
    """The FP32 matrix-core update keeps the FP32 working copy accurate to
    about u_32: on a gap-separated input the pivots equal the oracle's and T
    agrees to the FP32 level."""
    need_gpu()
    A = synth.spectrum_matrix(2000, 300, synth.sigma_geom10(300, 30.0), 91, 92).astype(np.float32)
    perm, kk, R, T = gpu_id(A, k=60, prec="mixed_f32")
    ref = orc.cpqr(A, k=60)
    assert ref.margins.min() > 1e-4  # gap-separated: every pivot and T compared
    assert perm[:60].tolist() == ref.perm[:60].tolist()
    kappa = np.linalg.cond(ref.R[:, :60])
    assert rel_err(T, orc.solve_T(ref.R, 60)) <= 1e-5 * kappa


@pytest.mark.parametrize("path", ["f64", "mixed_bf16x3", "gram", "batched"])
def test_exact_ties_follow_swap_order(path):
    """Exact norm ties at every step, across panel boundaries (n = 90, k = 70,
    panels of 32): the pivot order equals the oracle's (first maximum in the
    current swap order), for the FP64 and mixed paths, the Gram front end and
    the batched kernel."""
    need_gpu()
    import paper_2012_00706_amd as mp
    A = synth.tie_matrix(90, seed=5)
    ref = orc.cpqr(A, k=70)
    Ad = to_dev(A.astype(np.float32) if path == "mixed_bf16x3" else A)
    if path == "batched":
        r = mp.factor_batched([Ad], k=70, prec="f64")[0]
        perm, k = host(r.perm), r.k
    else:
        res = mp.column_id(Ad, k=70, prec="f64" if path == "gram" else path, gram=path == "gram")
        perm, k = host(res.perm), res.k
    assert k == 70
    assert perm[:70].tolist() == ref.perm[:70].tolist()


@pytest.mark.parametrize("prec", ["f64", "mixed_bf16x3"])
def test_stale_workspace_does_not_leak(prec):
    """Regression: the step finalization loads per-position data for every
    position up to the host's (lagged) column bound, past the live columns,
    where the workspace holds stale or never-written entries.  Results with a
    workspace filled with 0xFF bytes (NaN doubles, -1 integers) or random
    bytes equal, bitwise, those with a zeroed one (several panels, adaptive
    rank)."""
    need_gpu()
    import paper_2012_00706_amd as mp
    A = synth.spectrum_matrix(3000, 300, synth.sigma_exp(300, 12.0), 97, 98)
    if prec != "f64":
        A = A.astype(np.float32)
    Ad = to_dev(A)
    o = mp.make_opts(tol=1e-4, prec=prec)
    ws = mp.workspace_size(3000, 300, Ad.dtype, o)
    outs = []
    gen = torch.Generator(device="cuda").manual_seed(3)
    for fill in ("zero", "ones", "random"):
        if fill == "zero":
            work = torch.zeros(ws, dtype=torch.uint8, device="cuda")
        elif fill == "ones":
            work = torch.full((ws,), 255, dtype=torch.uint8, device="cuda")
        else:
            work = torch.randint(0, 256, (ws,), dtype=torch.uint8, device="cuda", generator=gen)
        fr = mp.factor(Ad, tol=1e-4, prec=prec, work=work)
        torch.cuda.synchronize()
        outs.append((fr.k, host(fr.perm).copy(), host(fr.R).copy()))
    assert outs[0][0] > 64  # more than two panels
    for k, perm, R in outs[1:]:
        assert k == outs[0][0]
        assert np.array_equal(perm, outs[0][1])
        assert np.array_equal(R, outs[0][2])


@pytest.mark.parametrize("prec", ["f64", "mixed_bf16x3"])
def test_tall_input_folded_partials(prec):
    """30000 x 100 (469 row tiles of 64 rows: the step finalization reads
    partials folded over groups of row tiles): FP64 pivots and T equal the
    oracle's; the mixed path's pivots too on this gap-separated input."""
    need_gpu()
    A = synth.spectrum_matrix(30000, 100, synth.sigma_geom10(100, 15.0), 101, 102)
    if prec == "f64":
        _check_f64_parity(A, 40)
    else:
        A32 = A.astype(np.float32)
        perm, k, R, T = gpu_id(A32, k=40, prec=prec)
        ref = orc.cpqr(A32.astype(np.float64), k=40)
        assert k == 40 and perm[:40].tolist() == ref.perm[:40].tolist()
        assert rel_err(T, orc.solve_T(ref.R, 40)) <= 1e-4


# ---------------------------------------------------------------- metamorphic invariances

@pytest.mark.parametrize("prec", ["f64", "mixed_bf16x3", "mixed_f32"])
def test_power_of_two_scaling_is_exact(prec):
    """Scaling A by 2^s scales every floating-point value the factorization
    forms by exactly 2^s (no rounding changes; no value reaches the FP16
    scaling's range limits here), so pivots, k and T are bitwise unchanged and
    R is exactly 2^s times R."""
    need_gpu()
    A = synth.spectrum_matrix(1500, 260, synth.sigma_exp(260, 30.0), 61, 62).astype(np.float32)
    p1, k1, R1, T1 = gpu_id(A, tol=1e-4, prec=prec)
    for s in (-7, 5):
        As = (A * np.float32(2.0 ** s)).astype(np.float32)
        p2, k2, R2, T2 = gpu_id(As, tol=1e-4, prec=prec)
        assert k1 == k2 and np.array_equal(p1, p2), (prec, s)
        assert np.array_equal(R1 * 2.0 ** s, R2), (prec, s)
        assert np.array_equal(T1, T2), (prec, s)


def test_row_and_column_permutations():
    """FP64 path: permuting the rows of A leaves the pivots, |R| and T
    unchanged (to rounding); permuting its columns permutes the pivots the
    same way (gap-separated input: no near-ties)."""
    need_gpu()
    rng = np.random.default_rng(63)
    A = synth.spectrum_matrix(900, 180, synth.sigma_geom10(180, 10.0), 63, 64)
    k = 40
    p1, _, R1, T1 = gpu_id(A, k=k, prec="f64")
    rows = rng.permutation(A.shape[0])
    p2, _, R2, T2 = gpu_id(np.asfortranarray(A[rows]), k=k, prec="f64")
    assert np.array_equal(p1, p2)
    assert np.max(np.abs(np.abs(R2) - np.abs(R1))) <= 1e-12 * np.max(np.abs(R1))
    assert np.max(np.abs(T2 - T1)) <= 1e-10 * max(np.max(np.abs(T1)), 1.0)
    cols = rng.permutation(A.shape[1])
    p3, _, R3, _ = gpu_id(np.asfortranarray(A[:, cols]), k=k, prec="f64")
    assert np.array_equal(cols[p3[:k]], p1[:k])
    assert np.max(np.abs(np.abs(np.diag(R3[:, :k])) - np.abs(np.diag(R1[:, :k])))) <= \
        1e-12 * abs(R1[0, 0])


@pytest.mark.parametrize("prec", ["f64", "mixed_bf16x3", "mixed_f32"])
def test_fixed_rank_after_early_panel_end(prec):
    """sigma_j = j^-2, k = 40: the FP32 working copy's downdated norms cancel
    within the first panel, which ends after a few steps; the panel enqueued
    behind it assumes that it ran all its steps (at most kcap minus that
    optimistic start), so a later panel takes the rest.  The rank is exactly
    k; FP64: the oracle's pivots, R and T; mixed: the acceptance rule and the
    oracle's pivots up to the first margin below 1e-3."""
    need_gpu()
    s = np.arange(1, 201, dtype=np.float64) ** -2.0
    A = synth.spectrum_matrix(3000, 200, s, 501, 502)
    if prec != "f64":
        A = A.astype(np.float32)
    perm, kk, R, T = gpu_id(A, k=40, prec=prec)
    assert kk == 40
    ref = orc.cpqr(A.astype(np.float64), k=40)
    if prec == "f64":
        assert_f64_parity(perm, kk, R, T, ref, 200)
        return
    upto = int(np.argmax(ref.margins < 1e-3)) if np.any(ref.margins < 1e-3) else 40
    assert upto >= 10
    assert perm[:upto].tolist() == ref.perm[:upto].tolist()
    e = orc.id_error(A, perm, 40, T)[0]
    e_ref = orc.id_error(A, ref.perm, 40, orc.solve_T(ref.R, 40))[0]
    assert e <= 1.1 * e_ref + 10 * U_LOW[prec] * s[0]


def test_back_to_back_calls_share_a_workspace():
    """id_factor returns once k is known, with its final gather of R and perm
    still in flight on the stream: a second call on the same stream and the
    same workspace (no synchronization in between) must not disturb the
    first call's outputs, and both equal the results of separate calls."""
    need_gpu()
    import paper_2012_00706_amd as mp
    A1 = synth.spectrum_matrix(2000, 300, synth.sigma_exp(300, 12.0), 71, 72)
    A2 = synth.spectrum_matrix(2500, 280, synth.sigma_exp(280, 10.0), 73, 74)
    d1, d2 = to_dev(A1), to_dev(A2)
    ref = []
    for d in (d1, d2):
        fr = mp.factor(d, tol=1e-4, prec="f64")
        torch.cuda.synchronize()
        ref.append((fr.k, host(fr.perm).copy(), host(fr.R).copy()))
    o = mp.make_opts(tol=1e-4, prec="f64")
    work = torch.empty(mp.workspace_size(2500, 300, torch.float64, o), dtype=torch.uint8,
                       device="cuda")
    f1 = mp.factor(d1, tol=1e-4, prec="f64", work=work)
    f2 = mp.factor(d2, tol=1e-4, prec="f64", work=work)
    torch.cuda.synchronize()
    for fr, (k, perm, R) in zip((f1, f2), ref):
        assert fr.k == k
        assert np.array_equal(host(fr.perm), perm)
        assert np.array_equal(host(fr.R), R)
