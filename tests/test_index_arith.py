"""Index arithmetic of the device kernels, checked on the host in IEEE FP64.

The kernels split cell indices by the grid sizes without integer division: for
0 <= n < 2^51 and inv = 1/d rounded to FP64, truncating the FP64 product
(n + 1/2) * inv gives n // d, because (n + 1/2) / d lies at least 1/(2d) from an
integer while the product is within (n + 1/2) 2^-52 / d of it.  These tests run the
same two FP64 operations (numpy float64 is IEEE round-to-nearest) against Python's
integer division, exhaustively where the divisor is small and at the quotient
boundaries where it is large.
"""
import numpy as np
import pytest


def qdiv(n: np.ndarray, d: int) -> np.ndarray:
    inv = np.float64(1.0) / np.float64(d)
    return ((n.astype(np.float64) + 0.5) * inv).astype(np.int64)


@pytest.mark.parametrize("d", list(range(1, 130)) + [255, 256, 257, 1000, 4761, 4096])
def test_quotient_is_exact_for_every_small_numerator(d):
    n = np.arange(0, 200 * d + 7, dtype=np.int64)
    np.testing.assert_array_equal(qdiv(n, d), n // d)


@pytest.mark.parametrize("d", [3, 7, 69, 512, 4761, 65536, 328509, (1 << 20) - 1])
def test_quotient_is_exact_at_the_boundaries_up_to_2_pow_40(d):
    k = np.unique(np.concatenate([np.arange(0, 4096), np.geomspace(1, (1 << 40) // d, 4000).astype(np.int64)]))
    n = np.concatenate([k * d - 1, k * d, k * d + d - 1])
    n = n[n >= 0]
    np.testing.assert_array_equal(qdiv(n, d), n // d)


def test_quotient_is_exact_on_random_cell_indices():
    # cell counts go up to 2^26; cells per slice and layers per slice are divisors
    rng = np.random.default_rng(20250715)
    for d in rng.integers(1, 1 << 22, size=200):
        n = rng.integers(0, 1 << 26, size=2000)
        np.testing.assert_array_equal(qdiv(n, int(d)), n // int(d))
