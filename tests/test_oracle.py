"""Pins of the CPU FP64 oracle against values and facts that do not come from
the oracle itself: numbers printed in the paper, closed forms, LAPACK's pivoted
QR, least squares, invariants, brute force and finite differences."""
import math

import numpy as np
import pytest
import scipy.linalg

import oracle as orc
import synth
from conftest import read_golden


# ---------------------------------------------------------------- paper values

def test_table1_unit_roundoff_matches_formats():
    """Table 1: unit round-off of half/single/double to two significant digits
    equals 2^-11, 2^-24, 2^-53."""
    rows = {r[0]: (int(r[1]), int(r[2]), float(r[3]))
            for r in read_golden("table1_unit_roundoff.txt")}
    mine = {"half": orc.U_HALF, "single": orc.U_SINGLE, "double": orc.U_DOUBLE}
    for name, (ebits, mbits, u) in rows.items():
        assert mine[name] == 2.0 ** -(mbits + 1)
        assert float(f"{mine[name]:.1e}") == u


def test_table3_dataset_statistics():
    """Table 3: sigma_50/sigma_1 and sigma_n/sigma_1 of the three synthetic
    datasets, from the decay laws i^-1, i^-2, i^-4 at n = 1000."""
    for name, p, m, n, s50, sn in read_golden("table3_datasets.txt"):
        sig = synth.sigma_pow(int(n), float(p))
        assert float(f"{sig[49] / sig[0]:.1e}") == float(s50)
        assert math.isclose(sig[-1] / sig[0], float(sn), rel_tol=1e-12)


def test_table3_statistics_of_generated_medium_dataset():
    """The generated Medium matrix carries the Table 3 spectrum (pins the
    generator, which both sides share)."""
    a = synth.paper_dataset("medium", n=1000)
    s = np.linalg.svd(a, compute_uv=False)
    assert float(f"{s[49] / s[0]:.1e}") == 4.0e-4
    assert math.isclose(s[-1] / s[0], 1e-6, rel_tol=1e-8)


def test_optimal_rank20_errors_and_eckart_young():
    """Section 3.1: the optimal rank-20 errors are sigma_21 = 1/21, 1/441 and
    about 5e-6; every rank-20 ID error is at least sigma_21 (Eckart-Young) and
    at most Lemma 1's factor times it, in practice."""
    vals = {r[0]: float(r[1]) for r in read_golden("section3_error_values.txt")}
    assert math.isclose(vals["sigma21_slow"], 1.0 / 21, rel_tol=1e-15)
    assert math.isclose(vals["sigma21_medium"], 1.0 / 441, rel_tol=1e-15)
    assert float(f"{21.0 ** -4:.0e}") == vals["sigma21_fast_approx"]
    for kind, key in (("slow", "sigma21_slow"), ("medium", "sigma21_medium")):
        a = synth.paper_dataset(kind, n=300)
        s = np.linalg.svd(a, compute_uv=False)
        J, T, perm, k = orc.column_id(a, k=20)
        e2, _ = orc.id_error(a, perm, k, T)
        assert e2 >= s[20] * (1 - 1e-10)
        assert e2 <= math.sqrt(1 + 20 * (300 - 20)) * s[20]


def test_lemma1_number_printed_for_fast_k51():
    """Section 3.1 quotes 3.3e-5 for sqrt(1+k(n-k)) sigma at k=51, n=1000 on the
    Fast dataset; the printed value uses sigma_k (off-by-one reading)."""
    vals = {r[0]: float(r[1]) for r in read_golden("section3_error_values.txt")}
    k, n = 51, 1000
    factor = math.sqrt(1 + k * (n - k))
    assert float(f"{factor * k ** -4.0:.1e}") == vals["lemma1_fast_k51_printed"]
    assert float(f"{factor * (k + 1) ** -4.0:.1e}") != vals["lemma1_fast_k51_printed"]


# ---------------------------------------------------------------- closed forms

def test_rank_one_closed_form():
    """k = 1: the skeleton is the column of largest norm and T_l is the
    least-squares coefficient a_J^T a_l / ||a_J||^2."""
    a = synth.gaussian(40, 9, seed=21)
    a[:, 5] *= 3.0
    J, T, perm, k = orc.column_id(a, k=1)
    assert J.tolist() == [5]
    aj = a[:, 5]
    want = np.array([aj @ a[:, l] / (aj @ aj) for l in perm[1:]])
    np.testing.assert_allclose(T[0], want, rtol=1e-13, atol=1e-15)


def test_orthogonal_columns_closed_form_and_rank_rules():
    """A = Q diag(d) with orthonormal Q: the pivots come in decreasing d,
    |R_jj| = d_(j), T = 0, and both rank rules stop where the closed forms say."""
    rng = np.random.default_rng(5)
    n = 12
    q = synth.haar(50, n, seed=77)
    d = rng.permutation(np.geomspace(1.0, 1e-6, n))
    a = q * d[None, :]
    order = np.argsort(-d, kind="stable")
    res = orc.cpqr(a, k=n)
    assert res.perm.tolist() == order.tolist()
    np.testing.assert_allclose(np.abs(np.diag(res.R)), d[order], rtol=1e-12)
    T = orc.solve_T(res.R, 6)
    assert np.max(np.abs(T)) < 1e-10
    tol = 3e-4
    ds = d[order]
    r = orc.cpqr(a, tol=tol, rule="pivot_rel")
    assert r.k == int(np.sum(ds > tol * ds[0]))
    rf = orc.cpqr(a, tol=tol, rule="frob_rel")
    tails = np.sqrt(np.cumsum((ds ** 2)[::-1])[::-1])
    assert rf.k == int(np.argmax(tails <= tol * np.linalg.norm(ds)))


def test_exact_low_rank_recovered():
    """An exactly rank-r input is recovered to 1e-12 and the adaptive rank is r."""
    for (m, n, r, seed) in ((60, 40, 7, 1), (200, 90, 25, 2), (35, 35, 34, 3)):
        a = synth.low_rank(m, n, r, seed)
        res = orc.cpqr(a, tol=1e-10)
        assert res.k == r
        T = orc.solve_T(res.R, res.k)
        e2, ef = orc.id_error(a, res.perm, res.k, T)
        assert ef <= 1e-12 * np.linalg.norm(a)


def test_tiny_hand_example():
    """3 x 3 example worked by hand: columns (3,0,0), (1,1,0), (2,2,1).
    Norms 3, sqrt2, 3: tie -> first column.  After removing e_1 the residual
    norms are 1 and sqrt5 -> column 2 next; T solves [3 2; 0 -sqrt5]."""
    a = np.array([[3.0, 1.0, 2.0], [0.0, 1.0, 2.0], [0.0, 0.0, 1.0]])
    res = orc.cpqr(a, k=2)
    assert res.perm.tolist() == [0, 2, 1]
    np.testing.assert_allclose(np.abs(res.R[0]), [3.0, 2.0, 1.0], rtol=1e-15)
    np.testing.assert_allclose(abs(res.R[1, 1]), math.sqrt(5.0), rtol=1e-15)
    T = orc.solve_T(res.R, 2)
    # column 1 = x * col0 + y * col2 in the least-squares sense restricted to
    # span{e1, (2,2,1)}: col1 = (1,1,0); projection coefficients by hand:
    # minimise |(1,1,0) - x(3,0,0) - y(2,2,1)|: y = 2/5, x = (1 - 4/5)/3 = 1/15
    np.testing.assert_allclose(T[:, 0], [1.0 / 15.0, 2.0 / 5.0], rtol=1e-14)


# ---------------------------------------------------------------- invariants

@pytest.fixture(scope="module")
def c1_small():
    """Config-1 shape scaled down: 300 x 150, sigma_i = 10^-((i-1)/25)."""
    return synth.spectrum_matrix(300, 150, synth.sigma_geom10(150, 25.0), 31, 32)


def test_diag_nonincreasing_and_dominance(c1_small):
    res = orc.cpqr(c1_small, k=40)
    d = np.abs(np.diag(res.R))
    assert np.all(d[1:] <= d[:-1] * (1 + 10 * orc.U_DOUBLE))
    # CPQR dominance: R_jj^2 >= sum_{i=j}^{k-1} R_il^2 for every l > j
    R = res.R
    for j in range(res.k):
        tail = np.sum(R[j:, j + 1:] ** 2, axis=0)
        assert np.all(R[j, j] ** 2 >= tail * (1 - 1e-12))


def test_q_orthogonal_and_factorisation(c1_small):
    a = c1_small
    m = a.shape[0]
    res = orc.cpqr(a, k=40)
    Q = orc.form_q(res.V, res.tau)
    assert np.linalg.norm(Q.T @ Q - np.eye(res.k)) <= 10 * m * orc.U_DOUBLE
    az = a[:, res.perm]
    # first k columns are reproduced exactly by Q R11
    err = np.linalg.norm(az[:, :res.k] - Q @ res.R[:, :res.k]) / np.linalg.norm(a)
    assert err <= 10 * m * orc.U_DOUBLE
    # what Q R misses of the rest is exactly the residual block
    miss = np.linalg.norm(az - Q @ res.R)
    assert math.isclose(miss, np.linalg.norm(res.residual), rel_tol=1e-10)


def test_error_equals_norm_of_R22(c1_small):
    """||A - A_J P||_2 = ||R22||_2 (A Z = Q R with T = R11^-1 R12)."""
    res = orc.cpqr(c1_small, k=30)
    T = orc.solve_T(res.R, res.k)
    e2, _ = orc.id_error(c1_small, res.perm, res.k, T)
    assert math.isclose(e2, np.linalg.norm(res.residual, 2), rel_tol=1e-9)


def test_matches_lapack_dgeqp3_on_gap_separated_input():
    """Pivots equal LAPACK's dgeqp3 and |R| rows agree on config 1 (1000 x 500,
    k = 50), whose per-step pivot margins are far above rounding."""
    a = synth.config1()
    res = orc.cpqr(a, k=50)
    assert res.margins.min() > 1e-4
    r_l, p_l = scipy.linalg.qr(a, pivoting=True, mode="r")
    assert res.perm[:50].tolist() == p_l[:50].tolist()
    np.testing.assert_allclose(np.abs(res.R[:, :50]), np.abs(r_l[:50, :50]), rtol=1e-10,
                               atol=1e-13)


def test_T_equals_least_squares_and_pinv(c1_small):
    res = orc.cpqr(c1_small, k=35)
    T = orc.solve_T(res.R, res.k)
    J, Jc = res.perm[:35], res.perm[35:]
    ls = np.linalg.lstsq(c1_small[:, J], c1_small[:, Jc], rcond=None)[0]
    kappa = np.linalg.cond(res.R[:, :35])
    assert np.max(np.abs(T - ls)) <= kappa * 1e-13 * max(1.0, np.max(np.abs(ls)))
    Tp = orc.solve_T_pinv(res.R, res.k)
    np.testing.assert_allclose(T, Tp, rtol=0, atol=kappa * 1e-13 * np.max(np.abs(T)))


def test_identity_block_exact(c1_small):
    J, T, perm, k = orc.column_id(c1_small, k=20)
    P = orc.coefficient_matrix(perm, k, T)
    assert np.array_equal(P[:, J], np.eye(k))
    Y = orc.reconstruct(c1_small, perm, k, T)
    assert np.array_equal(Y[:, J], c1_small[:, J])


def test_brute_force_subsets_bound_lemma1():
    """Lemma 1: the best k-subset satisfies ||A - A_S A_S^+ A||_2 <=
    sqrt(1 + k(n-k)) sigma_{k+1}; the greedy CPQR skeleton is never better
    than the best subset, and its ID error equals its projection error."""
    for seed in range(4):
        a = synth.spectrum_matrix(14, 8, synth.sigma_pow(8, 1.5), 100 + seed, 200 + seed)
        s = np.linalg.svd(a, compute_uv=False)
        for k in (2, 3):
            best, S = orc.brute_force_best_subset(a, k)
            assert best <= math.sqrt(1 + k * (8 - k)) * s[k]
            assert best >= s[k] * (1 - 1e-12)
            J, T, perm, kk = orc.column_id(a, k=k)
            e2, _ = orc.id_error(a, perm, kk, T)
            assert e2 >= best * (1 - 1e-12)
            AS = a[:, J]
            proj = orc.spectral_norm(a - AS @ np.linalg.pinv(AS) @ a)
            assert math.isclose(e2, proj, rel_tol=1e-9)


def test_tie_break_first_in_order():
    """Duplicated columns tie exactly: the first in current order is chosen
    (LAPACK idamax semantics), here matching dgeqp3."""
    a = synth.gaussian(30, 6, seed=9)
    a[:, 4] = a[:, 1] * 2.0
    a[:, 2] = a[:, 1] * 2.0
    res = orc.cpqr(a, k=3)
    assert res.perm[0] == 2
    _, p_l = scipy.linalg.qr(a, pivoting=True, mode="r")
    assert res.perm[0] == p_l[0]


def test_tie_break_follows_swap_order_like_dgeqp3():
    """Exact ties at every step (orthogonal disjoint-support columns with
    repeated integer norms): the whole pivot order equals LAPACK's dgeqp3,
    including ties between columns whose order earlier swaps changed."""
    a = synth.tie_matrix(70, seed=3)
    res = orc.cpqr(a, k=40)
    _, p_l = scipy.linalg.qr(a, pivoting=True, mode="r")
    assert res.perm[:40].tolist() == p_l[:40].tolist()
    # the swap order differs from "smallest original index first" somewhere
    lev = np.abs(a).max(axis=0)
    naive = sorted(range(70), key=lambda c: (-lev[c], c))
    assert res.perm[:40].tolist() != naive[:40]


# ---------------------------------------------------------------- metamorphic

def test_metamorphic_invariances(c1_small):
    a = c1_small
    base = orc.cpqr(a, k=25)
    T0 = orc.solve_T(base.R, 25)
    m = a.shape[0]
    # orthogonal left factor
    Wq = synth.haar(m, m, seed=55)
    r1 = orc.cpqr(Wq @ a, k=25)
    assert r1.perm.tolist() == base.perm.tolist()
    np.testing.assert_allclose(orc.solve_T(r1.R, 25), T0, atol=1e-10)
    # row permutation
    rp = np.random.default_rng(3).permutation(m)
    r2 = orc.cpqr(a[rp], k=25)
    assert r2.perm.tolist() == base.perm.tolist()
    np.testing.assert_allclose(orc.solve_T(r2.R, 25), T0, atol=1e-10)
    # power-of-two scaling is exact
    r3 = orc.cpqr(a * 2.0 ** 7, k=25)
    assert r3.perm.tolist() == base.perm.tolist()
    assert np.array_equal(orc.solve_T(r3.R, 25), T0)


# ---------------------------------------------------------------- edge cases

def test_singular_fixed_rank_raises():
    a = synth.low_rank(30, 10, 3, seed=4)
    res = orc.cpqr(a, k=5)
    with pytest.raises(orc.SingularR11):
        orc.solve_T(res.R, 5)


def test_zero_matrix_adaptive_rank_zero():
    a = np.zeros((20, 6))
    res = orc.cpqr(a, tol=1e-3)
    assert res.k == 0
    assert orc.solve_T(res.R, 0).shape == (0, 6)


def test_full_rank_k_equals_n():
    a = synth.gaussian(20, 6, seed=8)
    res = orc.cpqr(a, tol=1e-14)
    assert res.k == 6
    T = orc.solve_T(res.R, 6)
    assert T.shape == (6, 0)
    e2, ef = orc.id_error(a, res.perm, 6, T)
    assert ef == 0.0


def test_unpivoted_matches_numpy_qr():
    a = synth.gaussian(40, 12, seed=10)
    res = orc.cpqr(a, k=12, pivoting=False)
    assert res.perm.tolist() == list(range(12))
    r = np.linalg.qr(a, mode="r")
    np.testing.assert_allclose(np.abs(res.R), np.abs(r), rtol=1e-12, atol=1e-13)


# ---------------------------------------------------------------- adjoint

def _T_frozen(a, perm, k):
    """T with the skeleton held fixed, by least squares (independent of the
    closed-form adjoint)."""
    J, Jc = perm[:k], perm[k:]
    return np.linalg.lstsq(a[:, J], a[:, Jc], rcond=None)[0]


def test_adjoint_matches_central_differences():
    rng = np.random.default_rng(12)
    a = synth.spectrum_matrix(30, 12, synth.sigma_exp(12, 4.0), 61, 62)
    res = orc.cpqr(a, k=4)
    perm, k = res.perm, 4
    T = orc.solve_T(res.R, k)
    gT = rng.standard_normal(T.shape)
    gY = rng.standard_normal(a.shape)

    def ell(x):
        t = _T_frozen(x, perm, k)
        y = orc.reconstruct(x, perm, k, t)
        return float(np.sum(gT * t) + np.sum(gY * y))

    g = orc.adjoint(a, perm, k, T, gT=gT, gY=gY)
    h = 1e-6
    for _ in range(6):
        d = rng.standard_normal(a.shape)
        d /= np.linalg.norm(d)
        fd = (ell(a + h * d) - ell(a - h * d)) / (2 * h)
        an = float(np.sum(g * d))
        assert abs(fd - an) <= 1e-7 * max(1.0, abs(an))


def test_loss_gradient_envelope_and_consistency():
    rng = np.random.default_rng(13)
    a = synth.spectrum_matrix(25, 10, synth.sigma_exp(10, 3.0), 63, 64)
    res = orc.cpqr(a, k=3)
    perm, k = res.perm, 3
    T = orc.solve_T(res.R, k)

    def L(x):
        t = _T_frozen(x, perm, k)
        return float(np.sum((x - orc.reconstruct(x, perm, k, t)) ** 2))

    g = orc.loss_gradient(a, perm, k, T)
    h = 1e-6
    for _ in range(6):
        d = rng.standard_normal(a.shape)
        d /= np.linalg.norm(d)
        fd = (L(a + h * d) - L(a - h * d)) / (2 * h)
        assert abs(fd - float(np.sum(g * d))) <= 1e-7 * max(1.0, abs(fd))
    # the same gradient through the reconstruction adjoint: L = ||A - Y||^2
    E = a - orc.reconstruct(a, perm, k, T)
    g2 = 2.0 * E + orc.adjoint(a, perm, k, T, gY=-2.0 * E)
    np.testing.assert_allclose(g2, g, atol=1e-10)


# ---------------------------------------------------------------- planted mistakes

def test_pins_catch_planted_reflector_sign_error(monkeypatch):
    """A wrong sign planted in the oracle's reflector is caught by the exact
    low-rank recovery pin."""
    good = orc.id_oracle._reflector

    def bad(x):
        v, tau, beta = good(x)
        v = v.copy()
        v[1:] = -v[1:]
        return v, tau, beta

    monkeypatch.setattr(orc.id_oracle, "_reflector", bad)
    a = synth.low_rank(60, 40, 7, 1)
    res = orc.cpqr(a, k=7)
    T = orc.solve_T(res.R, 7)
    _, ef = orc.id_error(a, res.perm, 7, T)
    assert ef > 1e-6 * np.linalg.norm(a)


def test_pins_catch_planted_transposed_solve():
    """Using R11^T instead of R11 in the solve is caught by least squares."""
    a = synth.spectrum_matrix(80, 30, synth.sigma_exp(30, 5.0), 71, 72)
    res = orc.cpqr(a, k=10)
    R = res.R.copy()
    bad = R.copy()
    bad[:, :10] = R[:, :10].T
    Tb = np.linalg.solve(bad[:, :10], R[:, 10:])
    ls = _T_frozen(a, res.perm, 10)
    assert np.max(np.abs(Tb - ls)) > 1e-3


# ---------------------------------------------------------------- sketching front end

def test_sketch_identity_reduces_to_deterministic_id():
    """Omega = I: the sketch is A itself, so the randomized ID is the ID."""
    A = synth.spectrum_matrix(60, 25, synth.sigma_geom10(25, 6.0), 3, 4)
    sk = orc.sketch_id(A, np.eye(60), tol=1e-4)
    ref = orc.cpqr(A, tol=1e-4)
    assert sk.k == ref.k and sk.perm.tolist() == ref.perm.tolist()
    np.testing.assert_array_equal(sk.T, orc.solve_T(ref.R, ref.k))


def test_sketch_exact_rank_recovered():
    """Exact rank r, l > r Gaussian rows: Y has the row space of A, so the
    ID read off Y reproduces A exactly at k = r."""
    A = synth.low_rank(300, 70, 9, seed=12)
    Om = synth.sketch_matrix(20, 300, seed=13)
    sk = orc.sketch_id(A, Om, k=9)
    J = sk.perm[:9]
    E = A[:, sk.perm[9:]] - A[:, J] @ sk.T
    assert np.linalg.norm(E) <= 1e-12 * np.linalg.norm(A)
    # the adaptive rule stops at the exact rank too
    assert orc.sketch_id(A, Om, tol=1e-10).k == 9


def test_sketch_left_orthogonal_invariance():
    """Replacing Omega by Q Omega (Q orthogonal l x l) leaves every residual
    column norm and R up to row signs unchanged: same pivots, same T."""
    A = synth.spectrum_matrix(200, 40, synth.sigma_exp(40, 5.0), 5, 6)
    Om = synth.sketch_matrix(24, 200, seed=7)
    Q = synth.haar(24, 24, seed=8)
    a = orc.sketch_id(A, Om, tol=1e-3)
    b = orc.sketch_id(A, Q @ Om, tol=1e-3)
    upto = int(np.argmax(a.margins < 1e-8)) if np.any(a.margins < 1e-8) else a.k
    assert a.k == b.k and a.perm[:upto].tolist() == b.perm[:upto].tolist()
    if upto == a.k:
        np.testing.assert_allclose(b.T, a.T, rtol=0, atol=1e-10 * max(1.0, np.abs(a.T).max()))
    # and a scaled sketch gives the same coefficients
    c = orc.sketch_id(A, 3.0 * Om, tol=1e-3)
    assert c.perm.tolist() == a.perm.tolist()
    np.testing.assert_allclose(c.T, a.T, rtol=0, atol=1e-12 * max(1.0, np.abs(a.T).max()))


def test_sketch_Y_is_the_left_product():
    """Y(r, l) is the dot product of row r of Omega with column l of A (brute
    force, entry by entry)."""
    A = synth.gaussian(17, 5, seed=21)
    Om = synth.sketch_matrix(3, 17, seed=22)
    sk = orc.sketch_id(A, Om, k=2)
    for r in range(3):
        for l in range(5):
            assert abs(sk.Y[r, l] - math.fsum(Om[r, i] * A[i, l] for i in range(17))) <= 1e-13
    with pytest.raises(ValueError):
        orc.sketch_id(A, Om.T, k=2)


def test_sketch_error_near_best_subset():
    """On a tiny matrix the randomized ID with oversampling stays within a
    modest factor of the best k-column subset (brute force) and of sigma_{k+1}."""
    A = synth.spectrum_matrix(40, 10, synth.sigma_geom10(10, 3.0), 31, 32)
    k = 3
    best, _ = orc.brute_force_best_subset(A, k)
    sig = np.linalg.svd(A, compute_uv=False)
    worst = 0.0
    for seed in range(5):
        sk = orc.sketch_id(A, synth.sketch_matrix(k + 8, 40, seed=100 + seed), k=k)
        e = orc.id_error(A, sk.perm, k, sk.T)[0]
        assert e >= best * (1 - 1e-12)
        worst = max(worst, e / sig[k])
    assert worst <= 10.0 * math.sqrt(1 + k * (10 - k))
