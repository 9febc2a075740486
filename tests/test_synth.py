"""The seeded input generators: same seed, same matrix (bitwise, within one
process); the prescribed spectra are the matrices' singular values; the
batched workload's shapes follow its recipe."""
import numpy as np

import synth
from synth import inputs


def test_generators_are_deterministic():
    a = synth.spectrum_matrix(300, 120, synth.sigma_exp(120, 10.0), 3, 4)
    b = synth.spectrum_matrix(300, 120, synth.sigma_exp(120, 10.0), 3, 4)
    c = synth.spectrum_matrix(300, 120, synth.sigma_exp(120, 10.0), 3, 5)
    assert np.array_equal(a, b)
    assert not np.array_equal(a, c)
    assert np.array_equal(synth.gaussian(50, 20, seed=9), synth.gaussian(50, 20, seed=9))


def test_prescribed_spectrum_is_exact():
    """A = U diag(sigma) V^T with Haar U (m x n, orthonormal columns) and V:
    the singular values are sigma to rounding, for every spectrum family."""
    for sig in (synth.sigma_exp(150, 10.0), synth.sigma_pow(150, 2.0),
                synth.sigma_geom10(150, 12.0)):
        A = synth.spectrum_matrix(400, 150, sig, 21, 22)
        s = np.linalg.svd(A, compute_uv=False)
        assert np.max(np.abs(s - np.sort(sig)[::-1])) <= 1e-13 * sig.max()


def test_haar_factors_are_orthonormal():
    U = synth.haar(500, 80, 31)
    assert np.max(np.abs(U.T @ U - np.eye(80))) <= 1e-13


def test_config1_recipe():
    """Config 1: 1000 x 500 fp64, sigma_i = 10^{-(i-1)/25}."""
    A = synth.config1()
    assert A.shape == (1000, 500) and A.dtype == np.float64
    s = np.linalg.svd(A, compute_uv=False)
    want = 10.0 ** (-np.arange(500) / 25.0)
    assert np.max(np.abs(s - want)) <= 1e-13


def test_batched_workload_shapes():
    """Config 4 draws m ~ U{2000..20000}, n ~ U{100..800} from its own seed
    (the shapes alone, without generating the matrices)."""
    (seed,) = inputs.CONFIG_SEEDS["config4"]
    rng = np.random.default_rng(seed)
    ms = rng.integers(2000, 20001, size=256)
    ns = rng.integers(100, 801, size=256)
    assert ms.min() >= 2000 and ms.max() <= 20000 and ns.min() >= 100 and ns.max() <= 800
    rng2 = np.random.default_rng(seed)
    assert np.array_equal(ms, rng2.integers(2000, 20001, size=256))
