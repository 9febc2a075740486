"""The paper's accuracy study (Section 3.1 and 3.2, Table 3 datasets) as
assertions: 1000 x 1000 matrices with sigma_i = i^-1 (Slow), i^-2 (Medium),
i^-4 (Fast); relative spectral errors of the low-precision IDs against the
oracle's double-precision ID, ||A_D - A_X||_2 / ||A_D||_2, and against the
matrix.

Variants (Section 2's three approximations):
  mixed single  A cast to binary32, the factorization's working copy and
                update in FP32 (ID_PREC_MIXED_F32), skeleton from A_D
  single        the literal simulated single precision ID: every value the
                factorization keeps (and T) rounded to binary32
                (ID_FLAG_ROUND_F32), skeleton from A_L = fl32(A_D)
  mixed half    A cast to binary16, every kept value rounded to binary16, the
                FP16 update without operand scaling (ID_FLAG_ROUND_F16),
                skeleton from A_D
  half          the same, skeleton from A_L = fl16(A_D)
The paper's figures are lost; its prose statements are asserted where they
hold here, with the measured margins noted."""
import numpy as np
import pytest
import torch

import oracle as orc
import synth
from gpu_helpers import host, need_gpu, to_dev

pytestmark = pytest.mark.gpu

KINDS = ("slow", "medium", "fast")
KMAX = 50

_cache = {}


def _dataset(kind):
    """(A_D, oracle double ID to rank KMAX) of a Table 3 dataset, cached."""
    if kind not in _cache:
        A = synth.paper_dataset(kind)
        _cache[kind] = (A, orc.cpqr(A, k=KMAX))
    return _cache[kind]


def _oracle_recon(A, ref, k):
    """A_D's rank-k ID from the oracle (its first k steps are the rank-k CPQR)."""
    return orc.reconstruct(A, ref.perm, k, orc.solve_T(ref.R[:k], k))


def _gpu_variant(A, k, store, prec, round_to, low_skeleton):
    """(reconstruction, info, T finite) of one low-precision ID on the GPU."""
    import paper_2012_00706_amd as mp
    AL = np.asarray(A.astype(store), dtype=np.float32)
    ALd = to_dev(AL)
    res = mp.column_id(ALd, k=k, prec=prec, round_to=round_to)
    _, info = mp.solve_T(res.R, res.k, A.shape[1])
    Y = mp.reconstruct(ALd if low_skeleton else to_dev(A), res.perm, res.k, res.T)
    torch.cuda.synchronize()
    T = host(res.T)
    return host(Y), int(info.item()), bool(np.all(np.isfinite(T))), res


def _rel(X, Y):
    return orc.spectral_norm(X - Y) / orc.spectral_norm(X)


@pytest.mark.parametrize("kind", KINDS)
def test_mixed_single_within_single_roundoff(kind):
    """Section 3.1: the mixed single precision ID is as close to the double
    precision ID as single precision allows -- below single-precision unit
    round-off (2^-24 = 6e-8), over the target rank at n = 1000 and over the
    column count at k = 20 (the paper: almost all points below it for Fast
    and Medium, and about 1e-8 over the column count; measured here: at most
    1.2e-8 on all three datasets)."""
    need_gpu()
    A, ref = _dataset(kind)
    for k in (10, 20, 30, 40, 50):
        Y, info, finite, _ = _gpu_variant(A, k, np.float32, "mixed_f32", None, False)
        assert info == 0 and finite
        e = _rel(_oracle_recon(A, ref, k), Y)
        assert e <= orc.U_SINGLE, (kind, k, e)
    for n in (100, 400, 1000):
        An = np.asfortranarray(A[:, :n])
        refn = orc.cpqr(An, k=20)
        Y, info, finite, _ = _gpu_variant(An, 20, np.float32, "mixed_f32", None, False)
        e = _rel(_oracle_recon(An, refn, 20), Y)
        assert info == 0 and finite and e <= orc.U_SINGLE, (kind, n, e)


@pytest.mark.parametrize("kind", KINDS)
def test_single_id_within_1e6_of_double(kind):
    """Section 3.1: the (literal) single precision ID -- skeleton columns and
    coefficients in single precision -- stays within 1e-6 of the double ID
    (the paper states it for the hardest, Slow, dataset; measured here: at
    most 3.0e-7), and its error against the matrix equals the double ID's to
    within that (Section 3.2: single ID performs almost exactly as well)."""
    need_gpu()
    A, ref = _dataset(kind)
    for k in (10, 20, 30, 40, 50):
        Y, info, finite, _ = _gpu_variant(A, k, np.float32, "mixed_f32", "f32", True)
        assert info == 0 and finite
        YD = _oracle_recon(A, ref, k)
        e = _rel(YD, Y)
        assert e <= 1e-6, (kind, k, e)
        e_truth_d = _rel(A, YD)
        e_truth = _rel(A, Y)
        assert abs(e_truth - e_truth_d) <= 1e-6 + 1e-3 * e_truth_d, (kind, k, e_truth, e_truth_d)


def test_single_id_pivots_follow_oracle_on_fl32():
    """The single ID chooses the pivots the oracle's CPQR chooses on
    fl32(A) (the matrix it factors), up to the first step whose pivot margin
    is within the reach of single-precision rounding: the working copy and
    the norms carry errors of about u_32 |R_00|, which relative to a residual
    norm r_j is u_32 |R_00| / r_j (8 times that is taken as the reach; on
    the Fast matrix it covers the first steps only)."""
    need_gpu()
    for kind in ("slow", "medium", "fast"):
        A, _ = _dataset(kind)
        AL = A.astype(np.float32).astype(np.float64)
        ref = orc.cpqr(AL, k=KMAX)
        _, _, _, res = _gpu_variant(A, KMAX, np.float32, "mixed_f32", "f32", True)
        perm = host(res.perm).astype(np.int64)
        reach = 8 * orc.U_SINGLE * ref.pivot_norms[0] / ref.pivot_norms[:KMAX]
        close = ref.margins[:KMAX] <= reach
        upto = int(np.argmax(close)) if np.any(close) else KMAX
        assert upto >= 5, (kind, upto)
        assert perm[:upto].tolist() == ref.perm[:upto].tolist(), kind


@pytest.mark.parametrize("kind", KINDS)
def test_mixed_half_within_two_digits(kind):
    """Section 3.1: the mixed half precision ID stays within 1-2 digits of
    the double ID (relative spectral error <= 1e-2; measured here: 3.4e-4 to
    1.6e-3) at low target ranks, where it does not break down."""
    need_gpu()
    A, ref = _dataset(kind)
    for k in (5, 10, 20):
        Y, info, finite, _ = _gpu_variant(A, k, np.float16, "mixed_f16", "f16", False)
        assert info == 0 and finite
        e = _rel(_oracle_recon(A, ref, k), Y)
        assert e <= 1e-2, (kind, k, e)


def test_half_breaks_down_on_fast_decay():
    """Sections 3.1-3.2: on the Fast matrix the half precision IDs stop
    approximating as the rank grows.  Their error against the matrix stalls
    near half-precision round-off (>= 1e-4) from k = 10 on, while the double
    ID's keeps falling (1.1e-4 at k = 10 down to 3.4e-7 at k = 50), and
    for the larger ranks the factorization breaks down (non-finite
    coefficients or a singular R11) as binary16 values run out of range.
    The paper sees the breakdown beyond k = 21 in its own emulation (modified
    Gram-Schmidt, every operation in single precision on half-precision
    values); here, with Householder reflectors and FP64 arithmetic on binary16
    values, it comes later (measured between k = 35 and 40) -- but it comes,
    and nothing at k <= 21 breaks."""
    need_gpu()
    import paper_2012_00706_amd as mp
    A, ref = _dataset("fast")
    for k in (10, 15, 21):
        Y, info, finite, _ = _gpu_variant(A, k, np.float16, "mixed_f16", "f16", False)
        assert info == 0 and finite, k
        e_d = _rel(A, _oracle_recon(A, ref, k))
        e = _rel(A, Y)
        assert e >= 1e-4 and e > 3 * e_d, (k, e, e_d)
    broke = []
    for k in range(22, KMAX + 1, 4):
        try:
            Y, info, finite, _ = _gpu_variant(A, k, np.float16, "mixed_f16", "f16", True)
            bad = info == mp.C["ID_INFO_SINGULAR"] or not finite or not np.all(np.isfinite(Y))
        except mp.MpidError:
            bad = True
        broke.append(bad)
    assert any(broke), "no breakdown up to k = 50"
