"""Plain, slow, FP64 reference implementation of the column interpolative
decomposition (ID) of Dunton & Fox, "Mixed precision matrix interpolative
decompositions for model reduction" (arXiv 2012.00706).

TEST INFRASTRUCTURE ONLY -- used by ``tests/``, ``smoke()`` and the CPU
baseline of ``bench.py``; never by the product path.

What is computed (paper references are to sections / equations / algorithms):

* ``cpqr``       -- column-pivoted Householder QR truncated after k steps:
                    A Z = Q R (Section 1.1, eq. (6)), the pivot being the
                    remaining column of largest residual 2-norm, recomputed
                    from scratch at every step (the plain definition; no norm
                    downdating, no blocking).  The paper names a modified
                    Gram-Schmidt scheme; Householder reflectors give the same
                    pivots and the same R up to row signs in exact arithmetic.
* ``solve_T``    -- T = R11^{-1} R12 by explicit back-substitution (eq. (8),
                    Algorithm 1, coefficient step).  ``solve_T_pinv`` is the
                    paper's literal pseudo-inverse form (Remark 1.1).
* ``coefficient_matrix`` -- P with P(:, perm) = [I_k  T] (eq. (8)).
* ``reconstruct`` / ``id_error`` -- A(:, J) P and ||A - A(:, J) P||, all in
                    double precision (the remark after Lemma 1).
* ``adjoint``    -- gradient of a scalar loss through T (and through the
                    reconstruction) with respect to A, the skeleton J held
                    fixed.  Not in the paper: derived from T = A_J^+ A_Jc.
* ``brute_force_best_subset`` -- exhaustive best k-column subset on tiny
                    inputs (the existence statement of Lemma 1).
* ``sketch_id``  -- randomized ID through a sketch Y = Omega A (named as
                    future work in Section 5, without an algorithm): the
                    skeleton and T come from the column-pivoted QR of Y.

Every function here is pinned by tests under ``tests/`` against something
other than itself: closed forms, LAPACK's pivoted QR, least squares,
invariants, brute force and finite differences.  Parity status: pinned.
"""
from __future__ import annotations

import itertools
import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "U_HALF",
    "U_SINGLE",
    "U_DOUBLE",
    "U_BF16",
    "CPQRResult",
    "SingularR11",
    "cpqr",
    "solve_T",
    "solve_T_pinv",
    "coefficient_matrix",
    "reconstruct",
    "spectral_norm",
    "id_error",
    "form_q",
    "adjoint",
    "loss_gradient",
    "brute_force_best_subset",
    "column_id",
    "SketchIDResult",
    "sketch_id",
]

# Unit round-off u = 2^-t of the formats of Table 1 (IEEE half, single,
# double); BF16 (8 significand bits) is not in the paper.
U_HALF = 2.0 ** -11
U_SINGLE = 2.0 ** -24
U_DOUBLE = 2.0 ** -53
U_BF16 = 2.0 ** -8


class SingularR11(ArithmeticError):
    """R11 has a diagonal entry that is zero relative to |R_00|."""


@dataclass
class CPQRResult:
    perm: np.ndarray        # (n,) int64; A[:, perm] = Q R
    k: int                  # number of completed pivot steps
    R: np.ndarray           # (k, n) float64, upper trapezoidal in pivot order
    tau: np.ndarray         # (k,) Householder scalars
    V: np.ndarray           # (m, k) reflectors, unit entry at row j of column j
    residual: np.ndarray    # (m-k, n-k) trailing block R22 after k steps
    margins: np.ndarray     # (k,) (r_1 - r_2) / r_1 of the residual norms per step
    pivot_norms: np.ndarray  # (k,) residual norm of the chosen column per step


def _reflector(x: np.ndarray):
    """Householder reflector H = I - tau v v^T with H x = beta e_1, v_0 = 1.

    Conventions of LAPACK's dlarfg: beta = -sgn(alpha) * ||x||, sgn(0) = +1;
    when the tail of x is zero, tau = 0 and beta = alpha.
    """
    alpha = x[0]
    sigma = math.sqrt(float(np.dot(x[1:], x[1:]))) if x.shape[0] > 1 else 0.0
    v = np.zeros_like(x)
    v[0] = 1.0
    if sigma == 0.0:
        return v, 0.0, float(alpha)
    h = math.hypot(alpha, sigma)
    beta = -h if alpha >= 0.0 else h
    tau = (beta - alpha) / beta
    v[1:] = x[1:] / (alpha - beta)
    return v, tau, beta


def cpqr(A, k: int | None = None, tol: float | None = None, rule: str = "pivot_rel",
         kmax: int | None = None, pivoting: bool = True) -> CPQRResult:
    """Rank-k column-pivoted Householder QR of A (Section 1.1, eq. (6)-(7)).

    At step j every remaining column's residual norm ||W[j:, l]|| is
    recomputed; the pivot is the first column (in current order) attaining the
    maximum.  The chosen column is swapped to position j, a reflector is built
    from its tail and applied to the remaining columns.

    Rank selection:
      * ``k`` given: exactly k steps (Algorithm 1, "k <- target rank").
      * ``tol`` given, ``rule="pivot_rel"``: stop before step j >= 1 when the
        largest residual column norm is <= tol * |R_00|; always stop when it
        is zero.
      * ``tol`` given, ``rule="frob_rel"``: stop when the Frobenius norm of
        the whole residual block is <= tol * ||A||_F.
    ``kmax`` caps the number of steps (default min(m, n)).
    ``pivoting=False`` gives the unpivoted Householder QR.
    """
    W = np.array(A, dtype=np.float64, order="F", copy=True)
    if W.ndim != 2:
        raise ValueError("cpqr: A must be a matrix")
    m, n = W.shape
    cap = min(m, n) if kmax is None else min(int(kmax), m, n)
    if k is not None:
        if k < 0 or k > min(m, n):
            raise ValueError("cpqr: k out of range")
        cap = min(cap, int(k))
    elif tol is None:
        raise ValueError("cpqr: give k or tol")
    if rule not in ("pivot_rel", "frob_rel"):
        raise ValueError("cpqr: unknown rank rule")
    fro_a = float(np.linalg.norm(W)) if rule == "frob_rel" else 0.0

    perm = np.arange(n, dtype=np.int64)
    taus, vs, margins, pnorms = [], [], [], []
    r00 = 0.0
    j = 0
    while j < cap:
        r = np.sqrt(np.sum(W[j:, j:] ** 2, axis=0))
        q = int(np.argmax(r)) if pivoting else 0
        rp = float(r[q])
        if k is None:
            if rp == 0.0:
                break
            if rule == "pivot_rel" and j > 0 and rp <= tol * r00:
                break
            if rule == "frob_rel" and math.sqrt(float(np.sum(r * r))) <= tol * fro_a:
                break
        if r.shape[0] > 1:
            top2 = np.sort(r)[-2:]
            margins.append((top2[1] - top2[0]) / top2[1] if top2[1] > 0 else 0.0)
        else:
            margins.append(1.0)
        pnorms.append(rp)
        p = j + q
        if p != j:
            W[:, [j, p]] = W[:, [p, j]]
            perm[[j, p]] = perm[[p, j]]
        v, tau, beta = _reflector(W[j:, j].copy())
        if tau != 0.0:
            block = W[j:, j + 1:]
            block -= np.outer(tau * v, v @ block)
        W[j, j] = beta
        W[j + 1:, j] = 0.0
        if j == 0:
            r00 = abs(beta)
        full_v = np.zeros(m)
        full_v[j:] = v
        vs.append(full_v)
        taus.append(tau)
        j += 1

    kk = j
    R = np.triu(W[:kk, :]).copy()
    V = np.array(vs).T.reshape(m, kk) if kk else np.zeros((m, 0))
    return CPQRResult(perm=perm, k=kk, R=R, tau=np.array(taus, dtype=np.float64), V=V,
                      residual=W[kk:, kk:].copy(), margins=np.array(margins),
                      pivot_norms=np.array(pnorms))


def solve_T(R: np.ndarray, k: int | None = None) -> np.ndarray:
    """T = R11^{-1} R12 by back-substitution (eq. (8); Algorithm 1).

    R is k x n in pivot order.  Row i of T, from the last row up:
    T_i = (R12_i - sum_{l > i} R11_il T_l) / R11_ii.
    Raises ``SingularR11`` when some |R_ii| <= n * u_double * |R_00|.
    """
    R = np.asarray(R, dtype=np.float64)
    kk = R.shape[0] if k is None else int(k)
    n = R.shape[1]
    R11 = R[:kk, :kk]
    R12 = R[:kk, kk:]
    if kk == 0:
        return np.zeros((0, n))
    d = np.abs(np.diag(R11))
    if np.any(d <= n * U_DOUBLE * d[0]) or d[0] == 0.0:
        raise SingularR11("R11 is numerically singular")
    T = np.zeros((kk, n - kk))
    for i in range(kk - 1, -1, -1):
        T[i, :] = (R12[i, :] - R11[i, i + 1:] @ T[i + 1:, :]) / R11[i, i]
    return T


def solve_T_pinv(R: np.ndarray, k: int | None = None) -> np.ndarray:
    """The paper's literal form T = R11^+ R12 with the SVD pseudo-inverse
    (Remark 1.1, Algorithm 1)."""
    R = np.asarray(R, dtype=np.float64)
    kk = R.shape[0] if k is None else int(k)
    return np.linalg.pinv(R[:kk, :kk]) @ R[:kk, kk:]


def coefficient_matrix(perm: np.ndarray, k: int, T: np.ndarray) -> np.ndarray:
    """P (k x n) with P(:, perm) = [I_k  T], i.e. P = [I T] Z^T (eq. (8))."""
    perm = np.asarray(perm)
    n = perm.shape[0]
    P = np.zeros((k, n))
    P[:, perm[:k]] = np.eye(k)
    P[:, perm[k:]] = T
    return P


def reconstruct(A, perm: np.ndarray, k: int, T: np.ndarray) -> np.ndarray:
    """A(:, J) P evaluated in double precision, J = perm[:k] (eq. (4)-(5) and the
    remark after Lemma 1)."""
    A64 = np.asarray(A, dtype=np.float64)
    J = np.asarray(perm)[:k]
    return A64[:, J] @ coefficient_matrix(perm, k, T)


def spectral_norm(E: np.ndarray) -> float:
    """||E||_2 = sqrt(lambda_max(E^T E)), Gram matrix and eigenvalue in FP64."""
    E = np.asarray(E, dtype=np.float64)
    if E.size == 0:
        return 0.0
    G = E.T @ E if E.shape[0] >= E.shape[1] else E @ E.T
    return math.sqrt(max(float(np.linalg.eigvalsh(G)[-1]), 0.0))


def id_error(A, perm: np.ndarray, k: int, T: np.ndarray):
    """(||A - A(:,J)P||_2, ||A - A(:,J)P||_F), all in FP64."""
    E = np.asarray(A, dtype=np.float64) - reconstruct(A, perm, k, T)
    return spectral_norm(E), float(np.linalg.norm(E))


def form_q(V: np.ndarray, tau: np.ndarray) -> np.ndarray:
    """Thin Q = H_0 H_1 ... H_{k-1} [I_k; 0] from the reflectors of ``cpqr``."""
    m, k = V.shape
    Q = np.zeros((m, k))
    Q[:k, :k] = np.eye(k)
    for j in range(k - 1, -1, -1):
        v = V[:, j]
        Q -= np.outer(tau[j] * v, v @ Q)
    return Q


def column_id(A, k: int | None = None, tol: float | None = None, rule: str = "pivot_rel"):
    """Algorithm 1 end to end: returns (J, T, perm, k)."""
    res = cpqr(A, k=k, tol=tol, rule=rule)
    T = solve_T(res.R, res.k)
    return res.perm[:res.k].copy(), T, res.perm, res.k


def adjoint(A, perm: np.ndarray, k: int, T: np.ndarray, gT=None, gY=None) -> np.ndarray:
    """Gradient with respect to A of a loss that depends on T and/or on the
    reconstruction Y = A(:,J) P, with the skeleton J = perm[:k] held fixed.

    With B = A(:,J), C = A(:,Jc) the coefficients are the least-squares
    solution T = B^+ C = (B^T B)^{-1} B^T C (equal to R11^{-1} R12 by eq. (6)-(8)).
    Writing G = (B^T B)^{-1} and Rres = C - B T, a cotangent Tbar of T gives
        Cbar = B G Tbar,    Bbar = Rres Tbar^T G - B G Tbar T^T,
    and a cotangent Ybar of Y = [B, B T] adds Ybar_J + Ybar_Jc T^T to Bbar and
    B^T Ybar_Jc to Tbar.  G is applied through the R factor of an FP64 QR of B.
    Returns gA (m x n, float64).
    """
    A64 = np.asarray(A, dtype=np.float64)
    m, n = A64.shape
    perm = np.asarray(perm)
    J, Jc = perm[:k], perm[k:]
    B, C = A64[:, J], A64[:, Jc]
    T = np.asarray(T, dtype=np.float64).reshape(k, n - k)
    Tbar = np.zeros((k, n - k)) if gT is None else np.array(gT, dtype=np.float64)
    Bbar = np.zeros((m, k))
    if gY is not None:
        gY = np.asarray(gY, dtype=np.float64)
        Bbar += gY[:, J] + gY[:, Jc] @ T.T
        Tbar = Tbar + B.T @ gY[:, Jc]
    Rb = np.linalg.qr(B, mode="r")
    # X = G Tbar = R^{-1} R^{-T} Tbar
    X = np.linalg.solve(Rb, np.linalg.solve(Rb.T, Tbar))
    Wt = B @ X
    Rres = C - B @ T
    Bbar += Rres @ X.T - Wt @ T.T
    gA = np.zeros((m, n))
    gA[:, J] = Bbar
    gA[:, Jc] = Wt
    return gA


def loss_gradient(A, perm: np.ndarray, k: int, T: np.ndarray) -> np.ndarray:
    """Gradient of L = ||A - A(:,J) P||_F^2 with J fixed and T = B^+ C.

    Since B^T Rres = 0 at the least-squares T, the dependence through T drops
    out: dL/dC = 2 Rres, dL/dB = -2 Rres T^T.
    """
    A64 = np.asarray(A, dtype=np.float64)
    perm = np.asarray(perm)
    J, Jc = perm[:k], perm[k:]
    Rres = A64[:, Jc] - A64[:, J] @ T
    gA = np.zeros_like(A64)
    gA[:, Jc] = 2.0 * Rres
    gA[:, J] = -2.0 * Rres @ np.asarray(T).T
    return gA


def brute_force_best_subset(A, k: int):
    """Exhaustive search over all k-column subsets S of the error
    ||A - A_S A_S^+ A||_2 (tiny inputs only).  Returns (best_error, best_S)."""
    A64 = np.asarray(A, dtype=np.float64)
    n = A64.shape[1]
    best, best_s = math.inf, None
    for S in itertools.combinations(range(n), k):
        AS = A64[:, list(S)]
        E = A64 - AS @ (np.linalg.pinv(AS) @ A64)
        e = spectral_norm(E)
        if e < best:
            best, best_s = e, S
    return best, best_s



@dataclass
class SketchIDResult:
    perm: np.ndarray     # (n,) int64 pivot order of Y's factorization
    k: int               # rank reached on Y
    T: np.ndarray        # (k, n-k) interpolation coefficients, A ~ A(:, perm[:k]) T
    Y: np.ndarray        # (l, n) the sketch Omega A
    R: np.ndarray        # (k, n) R factor of Y in pivot order
    margins: np.ndarray  # pivot margins of Y's factorization (see CPQRResult)


def sketch_id(A, Omega, k: int | None = None, tol: float | None = None,
              rule: str = "pivot_rel") -> SketchIDResult:
    """Column ID of A from a sketch of its columns.

    Section 5 names sketching as a way to cut the cost of the ID but gives no
    algorithm; this is the usual randomized column ID.  A random test matrix
    Omega (l x m, l << m, drawn by the caller) compresses every column of A to
    l entries, Y = Omega A.  Since Omega is close to an isometry on the range
    of A, the column-pivoted QR of Y (same rank rules as ``cpqr``, tolerances
    applied to Y's residual norms) chooses the skeleton J, and the
    coefficients solve Y(:, J) T = Y(:, Jc) through Y's R factor (eq. (8) on
    Y): T = R_Y11^{-1} R_Y12.  When A has exact rank r <= l and Omega is
    injective on its range, A(:, Jc) = A(:, J) T exactly for k = r.
    """
    A64 = np.asarray(A, dtype=np.float64)
    Om = np.asarray(Omega, dtype=np.float64)
    if A64.ndim != 2 or Om.ndim != 2 or Om.shape[1] != A64.shape[0]:
        raise ValueError("sketch_id: Omega must be l x m for an m x n matrix A")
    Y = Om @ A64
    res = cpqr(Y, k=k, tol=tol, rule=rule)
    T = solve_T(res.R, res.k)
    return SketchIDResult(perm=res.perm, k=res.k, T=T, Y=Y, R=res.R, margins=res.margins)
