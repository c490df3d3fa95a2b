"""Pins of the oracle's implicit response (oracle/response.py)."""

import numpy as np
import pytest
from scipy import stats

from oracle.kron import kron_explicit
from oracle.response import box_muller, implicit_response, noise


def _words(u1_bits, u2_bits):
    return np.uint64(u1_bits << 11), np.uint64(u2_bits << 11)


def test_box_muller_closed_forms():
    top = (1 << 53) - 1
    # u1 = 1: radius 0 whatever the angle
    assert box_muller(*_words(top, 12345)) == 0.0
    # u2 = 0: the angle's cosine is 1; smallest u1 = 2^-53 gives sqrt(106 ln 2)
    assert box_muller(*_words(0, 0)) == pytest.approx(np.sqrt(106.0 * np.log(2.0)), rel=1e-15)
    # u2 = 1/2: cosine -1
    z = box_muller(*_words((1 << 52) - 1, 1 << 52))
    assert z == pytest.approx(-np.sqrt(-2.0 * np.log(0.5)), rel=1e-15)
    # the low 11 bits of each word are ignored
    assert box_muller(np.uint64(7 << 11 | 2047), np.uint64(5 << 11 | 1)) == box_muller(*_words(7, 5))


def test_noise_is_standard_normal():
    n = 1 << 18
    z = noise(np.arange(n // 4), 4, seed=11, stream=3).ravel()
    assert abs(z.mean()) < 5.0 / np.sqrt(n)
    assert abs(z.var() - 1.0) < 5.0 * np.sqrt(2.0 / n)
    assert stats.kstest(z, "norm").pvalue > 1e-3


def test_noise_depends_on_row_rhs_and_key():
    a = noise([5, 6], 2, seed=1, stream=2)
    assert a.shape == (2, 2)
    assert len(np.unique(a)) == 4
    assert not np.array_equal(a, noise([5, 6], 2, seed=1, stream=3))
    assert not np.array_equal(a, noise([5, 6], 2, seed=2, stream=2))
    # row 6 of a two-row request is row 6 of any request
    assert np.array_equal(a[1], noise([6], 2, seed=1, stream=2)[0])


def test_implicit_response_equals_explicit_product():
    rng = np.random.default_rng(4)
    As = [rng.standard_normal((4, 2)), rng.standard_normal((3, 3)), rng.standard_normal((5, 2))]
    X = rng.standard_normal((12, 3))
    K = kron_explicit(As)
    np.testing.assert_allclose(implicit_response(As, X, 0.0, 1, 2), K @ X, rtol=1e-13, atol=1e-13)
    b = implicit_response(As, X, 0.25, 1, 2)
    np.testing.assert_allclose((b - K @ X) / 0.25, noise(np.arange(60), 3, 1, 2), rtol=1e-10, atol=1e-10)
    v = implicit_response(As, X[:, 0], 0.25, 1, 2)
    np.testing.assert_allclose(v, b[:, 0], rtol=0, atol=0)
