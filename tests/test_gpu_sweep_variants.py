"""Parity of every reflector-sweep variant with the oracle.

The sweep kernel comes in three row tiles -- 64, 128 and 256 rows per
workgroup -- and the tile is picked at every pivot step from the number of
live blocks (more than 1024 blocks of 64-row tiles take 128-row tiles, more
than 1024 of those take 256-row tiles; the environment variable
MPID_SWEEP_RT forces one).  Because the live row count m - j shrinks as the
factorization proceeds, the tile can change in the middle of one
factorization.  These tests run:

* each tile forced, on the FP64 path (strict parity: pivots, R and T
  element-wise) and on the split-BF16 mixed path;
* a natural 65600 x 300 input whose tile changes at step 64 (FP64 path:
  256 -> 128 rows; mixed path: 128 -> 64 rows);
* the full-size 20000 x 2000 benchmark matrix (the 128-row-tile variant),
  FP64 and mixed, at tolerance 1e-3, against the oracle's rank-k CPQR
  (Section 1.1, eq. (6)-(8); Algorithms 1 and 2).
"""
import os

import numpy as np
import pytest

import oracle as orc
import synth
from gpu_helpers import (U_LOW, acceptance_bound, assert_f64_parity, gpu_id, need_gpu,
                         row_sign_align)

pytestmark = pytest.mark.gpu

_CACHE = {}


def _case(name):
    """(A, k, oracle CPQR) of a named input, computed once per session."""
    if name not in _CACHE:
        if name == "config1":
            A, k = synth.config1(), 50
        elif name == "3000x700":
            A, k = synth.spectrum_matrix(3000, 700, synth.sigma_geom10(700, 40.0), 31, 32), 150
        elif name == "3000x700_f32":
            A = synth.spectrum_matrix(3000, 700, synth.sigma_geom10(700, 40.0), 31,
                                      32).astype(np.float32)
            k = 150
        elif name == "65600x300_f32":
            A = synth.spectrum_matrix(65600, 300, synth.sigma_geom10(300, 30.0), 111,
                                      112).astype(np.float32)
            k = 80
        else:
            raise KeyError(name)
        _CACHE[name] = (A, k, orc.cpqr(A.astype(np.float64), k=k))
    return _CACHE[name]


def resolved_steps(ref, u_low, c=10.0):
    """Leading pivot steps a low-precision update cannot reorder.

    The blocked update rounds every updated entry to about u_low of the
    update's size, which is at most |R_00|; at step j the residual norms are
    about the pivot norm r_j, so they are perturbed by up to ~ u_low |R_00| /
    r_j relative.  Steps are counted until the first whose oracle margin is
    below c times that."""
    r00 = ref.pivot_norms[0] if ref.k else 1.0
    delta = c * u_low * r00 / np.maximum(ref.pivot_norms, 1e-300)
    bad = ref.margins <= delta
    return int(np.argmax(bad)) if np.any(bad) else ref.k


def _mixed_checks(A, k, ref, perm, kk, R, T, prec):
    """Mixed path against the oracle at the same rank: the acceptance rule
    err_mixed <= 1.1 err_oracle + 10 u_low ||A||_2 (the criterion for the
    mixed path; Algorithm 2), and the pivots of every step the update's
    rounding cannot reorder equal the oracle's.  Returns that step count."""
    assert kk == k
    upto = resolved_steps(ref, U_LOW[prec])
    assert upto >= 1
    assert perm[:upto].tolist() == ref.perm[:upto].tolist()
    e_m = orc.id_error(A, perm, kk, T)[0]
    e_o = orc.id_error(A, ref.perm, k, orc.solve_T(ref.R, k))[0]
    norm2 = orc.spectral_norm(A)
    assert e_m <= acceptance_bound(e_o, U_LOW[prec], norm2), (e_m, e_o)
    return upto


@pytest.mark.parametrize("rt", [64, 128, 256])
@pytest.mark.parametrize("case", ["config1", "3000x700"])
def test_forced_row_tile_f64(rt, case, monkeypatch):
    """FP64 path with the sweep's row tile forced: pivots, R and T equal the
    oracle's element-wise (inputs gap-separated)."""
    need_gpu()
    A, k, ref = _case(case)
    monkeypatch.setenv("MPID_SWEEP_RT", str(rt))
    perm, kk, R, T = gpu_id(A, k=k, prec="f64")
    assert assert_f64_parity(perm, kk, R, T, ref, A.shape[1]) > 0


@pytest.mark.parametrize("rt", [64, 128, 256])
def test_forced_row_tile_f64_from_fp32_storage(rt, monkeypatch):
    """FP64 path on an fp32-stored input (the working copy is the exact FP64
    promotion), tile forced: strict parity with the oracle on the promoted
    matrix."""
    need_gpu()
    A, k, ref = _case("3000x700_f32")
    monkeypatch.setenv("MPID_SWEEP_RT", str(rt))
    perm, kk, R, T = gpu_id(A, k=k, prec="f64")
    assert assert_f64_parity(perm, kk, R, T, ref, A.shape[1]) > 0


@pytest.mark.parametrize("rt", [64, 128, 256])
@pytest.mark.parametrize("prec", ["mixed_bf16x3", "mixed_f32"])
def test_forced_row_tile_mixed(rt, prec, monkeypatch):
    """Mixed paths with the tile forced: acceptance rule and pivot agreement
    (see _mixed_checks), and the rows of R of the agreeing steps element-wise
    within what the working precision allows: the FP32 working copy and the
    update's rounding (about u_low |R_00| per panel, five panels here) move R
    by at most 10 * 5 * u |R_00|, u = max(u_low, 2^-24)."""
    need_gpu()
    A, k, ref = _case("3000x700_f32")
    monkeypatch.setenv("MPID_SWEEP_RT", str(rt))
    perm, kk, R, T = gpu_id(A, k=k, prec=prec)
    upto = _mixed_checks(A, k, ref, perm, kk, R, T, prec)
    u = max(U_LOW[prec], orc.U_SINGLE)
    # rows and columns in pivot order agree only up to the agreeing steps
    Ra = row_sign_align(R[:upto, :upto], ref.R[:upto, :upto])
    np.testing.assert_allclose(Ra, ref.R[:upto, :upto], rtol=0,
                               atol=50 * u * abs(ref.R[0, 0]))


def test_tile_switch_mid_factorization_f64():
    """65600 x 300 (fp32 storage) on the FP64 path: 2 column chunks of 256
    positions; 1026 blocks of 128-row tiles at step 0 (-> 256-row tiles) and
    1024 once j >= 64 (-> 128-row tiles), so the tile changes inside the
    factorization.  Strict parity with the oracle over k = 80 steps."""
    need_gpu()
    A, k, ref = _case("65600x300_f32")
    perm, kk, R, T = gpu_id(A, k=k, prec="f64")
    assert assert_f64_parity(perm, kk, R, T, ref, A.shape[1]) > 0


@pytest.mark.parametrize("prec", ["mixed_bf16x3", "mixed_f32"])
def test_tile_switch_mid_factorization_mixed(prec):
    """The same input on the mixed paths (one column chunk of 512 positions):
    1025 blocks of 64-row tiles at step 0 (-> 128-row tiles), 1024 once
    j >= 64 (-> 64-row tiles)."""
    need_gpu()
    A, k, ref = _case("65600x300_f32")
    perm, kk, R, T = gpu_id(A, k=k, prec=prec)
    _mixed_checks(A, k, ref, perm, kk, R, T, prec)



# ---------------------------------------------------------------- full size

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                      "config2_reference.txt")


def _read_config2_reference():
    """The oracle's ID of the benchmark matrix (see make_config2_reference.py)."""
    ref = {"err2": {}, "R": [], "T": []}
    with open(GOLDEN) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            w = line.split()
            if w[0] == "perm":
                ref["perm"] = [int(x) for x in w[1:]]
            elif w[0] == "err2":
                ref["err2"][int(w[1])] = float(w[2])
            elif w[0] in ("R", "T"):
                ref[w[0]].append((int(w[1]), int(w[2]), float(w[3])))
            elif w[0] == "k":
                ref["k"] = int(w[1])
            else:
                ref[w[0]] = float(w[1])
    return ref


@pytest.fixture(scope="module")
def config2():
    need_gpu()
    return synth.config2(), _read_config2_reference()


def test_config2_full_size_f64(config2):
    """Full size (20000 x 2000, tol 1e-3, 128-row sweep tiles), FP64 path:
    the rank and all k pivots equal the oracle's (every step is
    gap-separated: smallest margin 1.7e-5), R and T on 600 seeded entries
    each within 1e-12 max|R| and 1e-12 max|T| max(1, kappa(R11)/1e3), and the
    error equals the oracle's."""
    A, ref = config2
    perm, k, R, T = gpu_id(A, tol=1e-3, prec="f64")
    assert ref["min_margin"] > 1e-8
    assert k == ref["k"]
    assert perm[:k].tolist() == ref["perm"]
    Rs = R * np.sign(np.diag(R[:, :k]))[:, None]
    r_tol = 1e-12 * ref["r00"]
    for i, c, v in ref["R"]:
        assert abs(Rs[i, c] - v) <= r_tol, (i, c, Rs[i, c], v)
    t_tol = 1e-12 * ref["max_abs_T"] * max(1.0, ref["kappa_R11"] / 1e3)
    for i, c, v in ref["T"]:
        assert abs(T[i, c] - v) <= t_tol, (i, c, T[i, c], v)
    e = orc.id_error(A.astype(np.float64), perm, k, T)[0]
    assert abs(e - ref["err2"][k]) <= 1e-10 * ref["err2"][k]


def test_config2_full_size_mixed(config2):
    """Full size, split-BF16 mixed path (the benchmark's precision): its error
    at the rank it chose is within 1.1x the oracle's at that rank plus
    10 u_low ||A||_2 with u_low = 2^-16 (||A||_2 = sigma_1 = exp(-1/40))."""
    A, ref = config2
    perm, km, R, T = gpu_id(A, tol=1e-3, prec="mixed_bf16x3")
    assert km in ref["err2"], "rank outside the stored range"
    e_m = orc.id_error(A.astype(np.float64), perm, km, T)[0]
    sigma1 = float(synth.sigma_exp(2000, 40.0)[0])
    assert e_m <= acceptance_bound(ref["err2"][km], U_LOW["mixed_bf16x3"], sigma1), (
        e_m, ref["err2"][km])
