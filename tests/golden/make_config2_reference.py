"""Writes tests/golden/config2_reference.txt: the oracle's column ID of the
20000 x 2000 benchmark matrix (stored fp32, A = U diag(exp(-i/40)) V^T with
Haar U, V; synth.config2), so that the full-size GPU parity test does not
re-run the ~2-minute CPU oracle.

Everything written comes from ``oracle`` (the FP64 column-pivoted Householder
QR of Section 1.1, eq. (6)-(7), back-substitution for T = R11^{-1} R12,
eq. (8), and FP64 errors as in the remark after Lemma 1) on the exact FP64
promotion of the stored matrix:

* the rank the pivot-relative rule gives at tolerance 1e-3 (stop before step
  j >= 1 when the largest residual column norm is <= 1e-3 |R_00|), the pivot
  order of its first k steps, the smallest pivot margin, |R_00|, kappa(R11)
  and max |T|;
* ||A - A(:, J) P||_2 at every rank k - 12 .. k + 12 (prefixes of one
  factorization truncated at k + 12 steps);
* 600 seeded entries of R (rows scaled so that diag(R) > 0) and 600 of T.

Run from the repository root:  python tests/golden/make_config2_reference.py
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as orc  # noqa: E402
import synth  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "config2_reference.txt")
TOL = 1e-3
SPAN = 12
NSAMPLE = 600


def main():
    t0 = time.perf_counter()
    A64 = synth.config2().astype(np.float64)
    m, n = A64.shape
    ad = orc.cpqr(A64, tol=TOL)
    k = ad.k
    # one longer factorization: its first j steps are the rank-j CPQR
    ref = orc.cpqr(A64, k=k + SPAN)
    assert ref.perm[:k].tolist() == ad.perm[:k].tolist()
    errs = {}
    for kk in range(k - SPAN, k + SPAN + 1):
        T = orc.solve_T(ref.R[:kk], kk)
        errs[kk] = orc.id_error(A64, ref.perm, kk, T)[0]
    R = ad.R.copy()
    R *= np.sign(np.diag(R[:, :k]))[:, None]
    T = orc.solve_T(ad.R, k)
    kappa = np.linalg.cond(ad.R[:, :k])
    rng = np.random.default_rng(20000)
    ri = rng.integers(0, k, NSAMPLE)
    rc = np.array([rng.integers(i, n) for i in ri])  # upper trapezoid
    ti = rng.integers(0, k, NSAMPLE)
    tc = rng.integers(0, n - k, NSAMPLE)
    with open(OUT, "w") as f:
        f.write("# Oracle column ID of the 20000 x 2000 benchmark matrix (synth.config2, fp32\n")
        f.write("# storage promoted to FP64); written by make_config2_reference.py, which\n")
        f.write("# calls only oracle/ and synth/.  Pivot-relative rank rule at tol 1e-3.\n")
        f.write(f"k {k}\n")
        f.write(f"r00 {abs(ad.R[0, 0]):.17e}\n")
        f.write(f"min_margin {ad.margins.min():.6e}\n")
        f.write(f"kappa_R11 {kappa:.6e}\n")
        f.write(f"max_abs_T {np.abs(T).max():.17e}\n")
        f.write("perm " + " ".join(str(int(p)) for p in ad.perm[:k]) + "\n")
        for kk, e in errs.items():
            f.write(f"err2 {kk} {e:.17e}\n")
        for i, c in zip(ri, rc):
            f.write(f"R {i} {c} {R[i, c]:.17e}\n")
        for i, c in zip(ti, tc):
            f.write(f"T {i} {c} {T[i, c]:.17e}\n")
    print(f"wrote {OUT}: k = {k}, {time.perf_counter() - t0:.0f} s")


if __name__ == "__main__":
    main()
