"""Seeded synthetic matrices for the column-ID workloads.

Every generator is deterministic in its seed (NumPy PCG64 streams) and returns
a column-major (Fortran-ordered) NumPy array, built in float64 and cast to the
storage dtype last.

Workloads (restated from the paper's experimental setup, Section 3 and Table 3,
and the benchmark configurations of this project):

* ``spectrum_matrix`` -- A = U diag(sigma) V^T with Haar-distributed orthonormal
  factors (QR of a Gaussian matrix with the signs of diag(R) folded into Q,
  Mezzadri's recipe).
* ``paper_dataset`` -- the paper's Slow / Medium / Fast test matrices: 1000 x
  1000 with sigma_i = i^-1, i^-2, i^-4 (Section 3, Table 3).  The paper does not
  say how U and V were drawn; Haar factors are used here.
* ``config1`` .. ``config5`` -- the five benchmark workloads (parity, mixed
  20000 x 2000, snapshot stand-in, batched, adjoint).
* ``snapshot_matrix`` -- a flow-snapshot-shaped stand-in for the particle data
  of Section 4, which is not available: random Fourier velocity modes with a
  k^(-5/3) shell spectrum plus a positive concentration field, slowly drifting
  phases across snapshots.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "haar",
    "spectrum_matrix",
    "sigma_exp",
    "sigma_pow",
    "sigma_geom10",
    "paper_dataset",
    "PAPER_DECAY",
    "config1",
    "config2",
    "config3",
    "config4",
    "config5",
    "config5_directions",
    "snapshot_matrix",
    "gaussian",
    "low_rank",
    "sketch_matrix",
    "tie_matrix",
    "CONFIG_SEEDS",
]

# Seeds of the five benchmark workloads (U seed, V seed, ...).
CONFIG_SEEDS = {
    "config1": (1, 2),
    "config2": (3, 4),
    "config3": (5,),
    "config4": (6,),  # sizes; member i uses seed 1000 + i
    "config5": (7, 8, 9),
}

# Singular-value decay exponents of the paper's three datasets (Section 3).
PAPER_DECAY = {"slow": 1.0, "medium": 2.0, "fast": 4.0}


def haar(m: int, n: int, seed: int) -> np.ndarray:
    """m x n matrix with orthonormal columns drawn from the Haar measure.

    QR of an m x n standard Gaussian matrix, with column signs fixed so that
    diag(R) > 0 (Mezzadri 2007).  The QR here is LAPACK's, used only to draw
    the random factor.
    """
    if n > m:
        raise ValueError("haar: need n <= m")
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((m, n))
    q, r = np.linalg.qr(g, mode="reduced")
    d = np.sign(np.diag(r))
    d[d == 0] = 1.0
    return q * d[None, :]


def sigma_exp(n: int, scale: float) -> np.ndarray:
    """sigma_i = exp(-i/scale), i = 1..n."""
    i = np.arange(1, n + 1, dtype=np.float64)
    return np.exp(-i / scale)


def sigma_pow(n: int, p: float) -> np.ndarray:
    """sigma_i = i^-p, i = 1..n."""
    i = np.arange(1, n + 1, dtype=np.float64)
    return i ** (-p)


def sigma_geom10(n: int, per_decade: float) -> np.ndarray:
    """sigma_i = 10^(-(i-1)/per_decade), i = 1..n."""
    i = np.arange(1, n + 1, dtype=np.float64)
    return 10.0 ** (-(i - 1) / per_decade)


def spectrum_matrix(m: int, n: int, sigma: np.ndarray, seed_u: int, seed_v: int,
                    dtype=np.float64) -> np.ndarray:
    """A = U diag(sigma) V^T (m x n), U m x r and V n x r Haar, r = min(m, n).

    Built in float64, cast to ``dtype`` last, returned column-major.
    """
    r = min(m, n)
    sigma = np.asarray(sigma, dtype=np.float64)
    if sigma.shape != (r,):
        raise ValueError("spectrum_matrix: sigma must have min(m, n) entries")
    u = haar(m, r, seed_u)
    v = haar(n, r, seed_v)
    a = (u * sigma[None, :]) @ v.T
    return np.asfortranarray(a.astype(dtype))


def paper_dataset(kind: str, n: int = 1000, m: int = 1000, seed: int = 11) -> np.ndarray:
    """The paper's synthetic datasets (Section 3, Table 3): 1000 x 1000 with
    sigma_i = i^-1 (Slow), i^-2 (Medium) or i^-4 (Fast), float64.

    When fewer columns are wanted the paper takes the first n columns of the
    1000-column matrix, which is what ``n`` does here.
    """
    p = PAPER_DECAY[kind]
    full = spectrum_matrix(m, 1000, sigma_pow(min(m, 1000), p), seed, seed + 1)
    return np.asfortranarray(full[:, :n])


def config1() -> np.ndarray:
    """Plain FP64 parity workload: 1000 x 500, sigma_i = 10^-((i-1)/25), fp64."""
    su, sv = CONFIG_SEEDS["config1"]
    return spectrum_matrix(1000, 500, sigma_geom10(500, 25.0), su, sv, np.float64)


def config2(m: int = 20000, n: int = 2000) -> np.ndarray:
    """Mixed-precision workload: 20000 x 2000, sigma_i = exp(-i/40), stored fp32."""
    su, sv = CONFIG_SEEDS["config2"]
    return spectrum_matrix(m, n, sigma_exp(min(m, n), 40.0), su, sv, np.float32)


def config4(batch: int = 256, seed: int | None = None, m_range=(2000, 20000),
            n_range=(100, 800)):
    """Batched workload: ``batch`` matrices, m_i ~ U{m_range}, n_i ~ U{n_range},
    sigma_j = j^-2, Haar factors seeded 1000 + i, stored fp32.

    Returns a list of column-major float32 arrays.
    """
    (s,) = CONFIG_SEEDS["config4"] if seed is None else (seed,)
    rng = np.random.default_rng(s)
    ms = rng.integers(m_range[0], m_range[1] + 1, size=batch)
    ns = rng.integers(n_range[0], n_range[1] + 1, size=batch)
    out = []
    for i in range(batch):
        m, n = int(ms[i]), int(ns[i])
        r = min(m, n)
        out.append(spectrum_matrix(m, n, sigma_pow(r, 2.0), 1000 + 2 * i, 1001 + 2 * i,
                                   np.float32))
    return out


def config5(m: int = 8192, n: int = 1024) -> np.ndarray:
    """Adjoint workload: 8192 x 1024, sigma_i = exp(-i/64), stored fp32."""
    su, sv, _ = CONFIG_SEEDS["config5"]
    return spectrum_matrix(m, n, sigma_exp(min(m, n), 64.0), su, sv, np.float32)


def config5_directions(m: int, n: int, count: int = 64, seed: int | None = None):
    """``count`` Gaussian directions D_r (m x n, float64) with ||D_r||_F = 1."""
    s = CONFIG_SEEDS["config5"][2] if seed is None else seed
    rng = np.random.default_rng(s)
    for _ in range(count):
        d = rng.standard_normal((m, n))
        yield np.asfortranarray(d / np.linalg.norm(d))


def _random_modes(rng, count: int, kmax: float):
    """``count`` distinct integer wavevectors with 0 < |k| <= kmax."""
    r = int(np.floor(kmax))
    ax = np.arange(-r, r + 1)
    kx, ky, kz = np.meshgrid(ax, ax, ax, indexing="ij")
    kk = np.stack([kx.ravel(), ky.ravel(), kz.ravel()], axis=1)
    norm = np.sqrt((kk.astype(np.float64) ** 2).sum(axis=1))
    kk = kk[(norm > 0) & (norm <= kmax)]
    idx = rng.choice(len(kk), size=count, replace=False)
    return kk[idx].astype(np.float64)


def _mode_field(grid: int, modes: np.ndarray, coeff: np.ndarray, phase: np.ndarray):
    """Real field sum_m coeff_m cos(k_m . x + phase_m(t)) on a grid^3 periodic box,
    for every snapshot t.  coeff: (M,), phase: (M, T).  Returns (grid^3, T),
    rows in C order (i_x, i_y, i_z) with i_z fastest.

    Uses cos(k.x + phi) = Re(exp(i k.x) exp(i phi)), so the field is the real
    part of a (grid^3 x M) by (M x T) complex product.
    """
    x = np.arange(grid) * (2.0 * np.pi / grid)
    # separable exponentials per axis
    ex = np.exp(1j * np.outer(x, modes[:, 0]))  # (grid, M)
    ey = np.exp(1j * np.outer(x, modes[:, 1]))
    ez = np.exp(1j * np.outer(x, modes[:, 2]))
    basis = (ex[:, None, None, :] * ey[None, :, None, :] * ez[None, None, :, :])
    basis = basis.reshape(grid ** 3, -1)  # (grid^3, M)
    right = coeff[:, None] * np.exp(1j * phase)  # (M, T)
    return (basis @ right).real


def snapshot_matrix(grid: int = 64, snapshots: int = 512, n_vel_modes: int = 128,
                    n_conc_modes: int = 64, kmax: float = 16.0, drift: float = 0.01,
                    seed: int | None = None, dtype=np.float32) -> np.ndarray:
    """Flow-snapshot stand-in: rows = 4 fields (u_x, u_y, u_z, c) x grid^3 points,
    columns = snapshots.

    Velocity: ``n_vel_modes`` wavevectors with amplitude |k|^(-11/6) (shell
    energy ~ k^(-5/3)), random directions projected perpendicular to k,
    phases phi_m(t) = U[0, 2 pi) + a Gaussian random walk of step ``drift``;
    rescaled to unit rms.  Concentration: a scalar field from
    ``n_conc_modes`` modes with the same recipe, standardised, then
    c = exp(0.5 s) / mean(exp(0.5 s)) (positive).
    """
    s = CONFIG_SEEDS["config3"][0] if seed is None else seed
    rng = np.random.default_rng(s)
    t = snapshots

    def phases(count):
        p0 = rng.uniform(0.0, 2.0 * np.pi, size=(count, 1))
        steps = rng.normal(0.0, drift, size=(count, t))
        steps[:, 0] = 0.0
        return p0 + np.cumsum(steps, axis=1)

    km = _random_modes(rng, n_vel_modes, kmax)
    kn = np.linalg.norm(km, axis=1)
    amp = kn ** (-11.0 / 6.0)
    d = rng.standard_normal((n_vel_modes, 3))
    khat = km / kn[:, None]
    d = d - (d * khat).sum(axis=1, keepdims=True) * khat
    d = d / np.linalg.norm(d, axis=1, keepdims=True)
    ph = phases(n_vel_modes)

    npts = grid ** 3
    out = np.empty((4 * npts, t), dtype=np.float64, order="F")
    vel = []
    for c in range(3):
        vel.append(_mode_field(grid, km, amp * d[:, c], ph))
    rms = np.sqrt(np.mean([np.mean(v ** 2) for v in vel]))
    for c in range(3):
        out[c * npts:(c + 1) * npts, :] = vel[c] / rms
    del vel

    kc = _random_modes(rng, n_conc_modes, kmax)
    ampc = np.linalg.norm(kc, axis=1) ** (-11.0 / 6.0)
    phc = phases(n_conc_modes)
    sfield = _mode_field(grid, kc, ampc, phc)
    sfield = (sfield - sfield.mean()) / sfield.std()
    cfield = np.exp(0.5 * sfield)
    out[3 * npts:, :] = cfield / cfield.mean()
    return np.asfortranarray(out.astype(dtype))


def config3(grid: int = 64, snapshots: int = 512) -> np.ndarray:
    """Snapshot workload: 1,048,576 x 512 (64^3 x 4 fields), stored fp32."""
    return snapshot_matrix(grid=grid, snapshots=snapshots)


def gaussian(m: int, n: int, seed: int, dtype=np.float64) -> np.ndarray:
    """Standard Gaussian m x n matrix, column-major."""
    rng = np.random.default_rng(seed)
    return np.asfortranarray(rng.standard_normal((m, n)).astype(dtype))


def low_rank(m: int, n: int, r: int, seed: int, dtype=np.float64) -> np.ndarray:
    """Exactly rank-r matrix B C with B (m x r), C (r x n) standard Gaussian."""
    rng = np.random.default_rng(seed)
    b = rng.standard_normal((m, r))
    c = rng.standard_normal((r, n))
    return np.asfortranarray((b @ c).astype(dtype))


def sketch_matrix(l: int, m: int, seed: int) -> np.ndarray:
    """Gaussian test matrix Omega (l x m, standard normal entries) for a sketch
    Y = Omega A, row-major: Omega[r, i] is element r * m + i."""
    rng = np.random.default_rng(seed)
    return np.ascontiguousarray(rng.standard_normal((l, m)))


def tie_matrix(n: int, seed: int, levels: int = 6, rows_per_col: int = 4, top: int = 40,
               dtype=np.float64) -> np.ndarray:
    """Columns with disjoint row supports below the first ``top`` rows, each
    holding ``rows_per_col`` equal small-integer entries drawn from ``levels``
    values: the columns are exactly orthogonal, every squared norm is an exact
    integer, and many norms tie exactly (before and after any number of
    Householder steps, which leave disjoint columns untouched)."""
    rng = np.random.default_rng(seed)
    m = top + rows_per_col * n
    a = np.zeros((m, n))
    lev = rng.integers(1, levels + 1, n)
    sign = rng.choice([-1.0, 1.0], (rows_per_col, n))
    for col in range(n):
        r0 = top + rows_per_col * col
        a[r0:r0 + rows_per_col, col] = lev[col] * sign[:, col]
    return np.asfortranarray(a.astype(dtype))
