"""Adjoint of the ID with the skeleton held fixed (id_backward through the C ABI
and the autograd Function) against the oracle's FP64 adjoint and against FP64
central differences."""
import numpy as np
import pytest
import torch

import oracle as orc
import synth
from gpu_helpers import host, need_gpu, rel_err, to_dev

pytestmark = pytest.mark.gpu


def _gpu_T_frozen(A64_dev, perm_dev, k):
    """T of a float64 device matrix with the column order held fixed: unpivoted
    QR of A(:, perm) on the GPU, then the triangular solve."""
    import paper_2012_00706_amd as mp
    Ap = A64_dev[:, perm_dev.long()]
    fr = mp.factor(Ap, k=k, prec="f64", no_pivot=True)
    T, _ = mp.solve_T(fr.R, k, A64_dev.shape[1])
    return T


@pytest.mark.parametrize("m,n,k,dtype", [(300, 80, 20, np.float64), (700, 130, 33, np.float32),
                                         (90, 40, 40, np.float64), (257, 65, 1, np.float64)])
def test_backward_matches_oracle_adjoint(m, n, k, dtype):
    need_gpu()
    import paper_2012_00706_amd as mp
    rng = np.random.default_rng(m + n + k)
    A = synth.spectrum_matrix(m, n, synth.sigma_exp(min(m, n), 10.0), m, n).astype(dtype)
    res = mp.column_id(to_dev(A), k=k)
    perm = host(res.perm).astype(np.int64)
    T = host(res.T)
    gT = rng.standard_normal(T.shape)
    gY = rng.standard_normal((m, n))
    gA = host(mp.backward(to_dev(A), res.perm, k, res.T, gT=to_dev(gT), gY=to_dev(gY)))
    ref = orc.adjoint(A, perm, k, T, gT=gT, gY=gY)
    assert rel_err(gA, ref) <= 1e-10
    # each cotangent alone
    g1 = host(mp.backward(to_dev(A), res.perm, k, res.T, gT=to_dev(gT)))
    assert rel_err(g1, orc.adjoint(A, perm, k, T, gT=gT)) <= 1e-10
    g2 = host(mp.backward(to_dev(A), res.perm, k, res.T, gY=to_dev(gY)))
    assert rel_err(g2, orc.adjoint(A, perm, k, T, gY=gY)) <= 1e-10


def test_autograd_loss_gradient_envelope():
    need_gpu()
    import paper_2012_00706_amd as mp
    A = synth.spectrum_matrix(400, 120, synth.sigma_exp(120, 12.0), 91, 92)
    At = to_dev(A).clone().requires_grad_(True)
    T, Y = mp.ColumnID.apply(At, 25)
    L = ((At.double() - Y) ** 2).sum()
    L.backward()
    res = mp.ColumnID.last
    perm = host(res.perm).astype(np.int64)
    ref = orc.loss_gradient(A, perm, 25, host(res.T))
    assert rel_err(host(At.grad), ref) <= 1e-9


def test_config5_adjoint_central_differences():
    """8192 x 1024 fp32, sigma_i = exp(-i/64), k = 128, J frozen from the
    forward pass: the directional derivatives of L = ||A - A(:,J) T||_F^2 and of
    <G, T> match FP64 central differences (h = 1e-6) on 64 seeded directions,
    and the gradient matches the oracle's FP64 adjoint."""
    need_gpu()
    import paper_2012_00706_amd as mp
    A32 = synth.config5()
    m, n = A32.shape
    k = 128
    A64 = A32.astype(np.float64)
    A_dev = to_dev(A64)
    res = mp.column_id(to_dev(A32), k=k, prec="mixed_bf16x3")
    perm_dev = res.perm
    perm = host(perm_dev).astype(np.int64)
    # T of the stored matrix with J frozen (FP64 path) and the loss gradient
    T0 = _gpu_T_frozen(A_dev, perm_dev, k)
    E0 = mp.reconstruct(A_dev, perm_dev, k, T0, residual=True)
    gA_loss = host(2.0 * E0 + mp.backward(A_dev, perm_dev, k, T0, gY=-2.0 * E0))
    ref = orc.loss_gradient(A64, perm, k, host(T0))
    assert rel_err(gA_loss, ref) <= 1e-9
    rng = np.random.default_rng(19)
    G = rng.standard_normal((k, n - k))
    gA_T = host(mp.backward(A_dev, perm_dev, k, T0, gT=to_dev(G)))
    G_dev = to_dev(G)
    h = 1e-6
    worst_L = worst_T = 0.0
    for D in synth.config5_directions(m, n, count=64):
        D_dev = to_dev(D)
        vals_L, vals_T = [], []
        for sgn in (1.0, -1.0):
            Ap = A_dev + sgn * h * D_dev
            Tp = _gpu_T_frozen(Ap, perm_dev, k)
            Ep = mp.reconstruct(Ap, perm_dev, k, Tp, residual=True)
            vals_L.append(float((Ep ** 2).sum()))
            vals_T.append(float((G_dev * Tp).sum()))
        fd_L = (vals_L[0] - vals_L[1]) / (2 * h)
        fd_T = (vals_T[0] - vals_T[1]) / (2 * h)
        an_L = float(np.sum(gA_loss * D))
        an_T = float(np.sum(gA_T * D))
        worst_L = max(worst_L, abs(fd_L - an_L) / max(abs(an_L), 1e-3))
        worst_T = max(worst_T, abs(fd_T - an_T) / max(abs(an_T), 1e-3))
    assert worst_L <= 1e-6, worst_L
    assert worst_T <= 1e-6, worst_T


def test_backward_with_forward_R_factor():
    """Passing R11 of the FP64 forward factorization (the skeleton's R factor)
    gives the same adjoint as recomputing it, to rounding."""
    need_gpu()
    import paper_2012_00706_amd as mp
    rng = np.random.default_rng(5)
    A = synth.spectrum_matrix(900, 150, synth.sigma_exp(150, 12.0), 21, 22)
    At = to_dev(A)
    res = mp.column_id(At, k=40, prec="f64")
    gT = to_dev(rng.standard_normal((40, 110)))
    gY = to_dev(rng.standard_normal((900, 150)))
    g0 = host(mp.backward(At, res.perm, 40, res.T, gT=gT, gY=gY))
    g1 = host(mp.backward(At, res.perm, 40, res.T, gT=gT, gY=gY, R11=res.R[:, :40]))
    assert rel_err(g1, g0) <= 1e-12
    ref = orc.adjoint(A, host(res.perm).astype(np.int64), 40, host(res.T), gT=host(gT), gY=host(gY))
    assert rel_err(g1, ref) <= 1e-10


@pytest.mark.parametrize("m,n,k,fused", [(600, 300, 200, "1"), (531, 190, 129, "1"),
                                         (300, 80, 20, "0"), (700, 330, 270, "1"),
                                         (1000, 400, 150, "0")])
def test_backward_product_paths(monkeypatch, m, n, k, fused):
    """Both product paths of id_backward against the oracle's adjoint: the
    fused pass over 16-row strips (skeletons up to 256 columns; 129..256 use
    four column blocks per wave) and the separate large-tile launches (forced,
    or k > 256), with ragged strips and coefficient chunks."""
    need_gpu()
    import paper_2012_00706_amd as mp
    monkeypatch.setenv("MPID_ADJ_FUSED", fused)
    rng = np.random.default_rng(m + 7 * k)
    A = synth.spectrum_matrix(m, n, synth.sigma_exp(min(m, n), 40.0), m + 1, n + 1)
    res = mp.column_id(to_dev(A), k=k)
    perm = host(res.perm).astype(np.int64)
    T = host(res.T)
    gT = rng.standard_normal(T.shape)
    gY = rng.standard_normal((m, n))
    gA = host(mp.backward(to_dev(A), res.perm, k, res.T, gT=to_dev(gT), gY=to_dev(gY),
                          R11=res.R[:, :k]))
    ref = orc.adjoint(A, perm, k, T, gT=gT, gY=gY)
    assert rel_err(gA, ref) <= 1e-10


@pytest.mark.parametrize("k,dtype", [(100, np.float64), (200, np.float64), (90, np.float32)])
def test_backward_tall_strips(monkeypatch, k, dtype):
    """Tall inputs take the fused pass over 32-row strips (two matrix-core row
    blocks per strip, chosen while the strips still give every compute unit a
    block): against the oracle's adjoint, and against the 16-row strips
    (MPID_ADJ_RB2=0), with a ragged last strip; k up to 128 and 129..256."""
    need_gpu()
    import paper_2012_00706_amd as mp
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    m, n = 32 * cus + 8, 300
    rng = np.random.default_rng(k)
    A = synth.spectrum_matrix(m, n, synth.sigma_exp(n, 40.0), m + 3, n + 3).astype(dtype)
    res = mp.column_id(to_dev(A), k=k)
    perm = host(res.perm).astype(np.int64)
    T = host(res.T)
    gT = rng.standard_normal(T.shape)
    gY = rng.standard_normal((m, n))
    args = (to_dev(A), res.perm, k, res.T)
    kw = dict(gT=to_dev(gT), gY=to_dev(gY), R11=res.R[:, :k])
    g2 = host(mp.backward(*args, **kw))
    monkeypatch.setenv("MPID_ADJ_RB2", "0")
    g1 = host(mp.backward(*args, **kw))
    assert rel_err(g2, g1) <= 1e-12
    ref = orc.adjoint(A.astype(np.float64), perm, k, T, gT=gT, gY=gY)
    assert rel_err(g2, ref) <= 1e-10


def test_backward_singular_skeleton_reported():
    """A singular R factor of the skeleton is reported (ID_INFO_SINGULAR, as
    MpidError) instead of a gradient, with the caller's R11 and with the QR
    computed inside; a regular call on the same thread afterwards still
    matches the oracle's adjoint."""
    need_gpu()
    import paper_2012_00706_amd as mp
    A = synth.spectrum_matrix(500, 40, synth.sigma_exp(40, 20.0), 501, 41)
    k = 10
    res = mp.column_id(to_dev(A), k=k)
    rng = np.random.default_rng(3)
    gT = rng.standard_normal((k, 40 - k))
    gY = rng.standard_normal((500, 40))
    R11 = res.R[:, :k].clone()
    R11[4, 4] = 0.0
    with pytest.raises(mp.MpidError) as e:
        mp.backward(to_dev(A), res.perm, k, res.T, gT=to_dev(gT), gY=to_dev(gY), R11=R11)
    assert e.value.code == mp.C["ID_INFO_SINGULAR"]
    perm = host(res.perm).astype(np.int64)
    A2 = A.copy()
    A2[:, perm[1]] = A2[:, perm[0]]  # two equal skeleton columns
    with pytest.raises(mp.MpidError) as e:
        mp.backward(to_dev(A2), res.perm, k, res.T, gT=to_dev(gT), gY=to_dev(gY))
    assert e.value.code == mp.C["ID_INFO_SINGULAR"]
    gA = host(mp.backward(to_dev(A), res.perm, k, res.T, gT=to_dev(gT), gY=to_dev(gY),
                          R11=res.R[:, :k]))
    ref = orc.adjoint(A, perm, k, host(res.T), gT=gT, gY=gY)
    assert rel_err(gA, ref) <= 1e-10
