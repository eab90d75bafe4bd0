"""The oracle's moment maps against the matrices the paper prints
(fixtures under tests/golden/, transcribed from arXiv 2208.03562:
Appendix A eq. 62 for P, eq. 72 for P^-1, eq. S-matrix for S)."""
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def load(name):
    return np.loadtxt(os.path.join(GOLDEN, name), comments="#")


P = load("appendix_a_raw_moments.txt")
PINV = load("appendix_a_populations.txt")
SEXP = load("scaling_exponents.txt")


def test_printed_matrices_are_inverse():
    """The two printed maps are each other's inverse (a check of the
    transcription as much as of the paper)."""
    np.testing.assert_array_equal(P @ PINV, np.eye(9))
    np.testing.assert_array_equal(PINV @ P, np.eye(9))


def test_raw_moments_are_the_printed_map(O):
    for a in range(9):
        e = np.zeros(9)
        e[a] = 1.0
        np.testing.assert_array_equal(O.raw_moments_square(e), P[:, a])


def test_populations_are_the_printed_map(O):
    for m in range(9):
        e = np.zeros(9)
        e[m] = 1.0
        np.testing.assert_array_equal(O.populations_from_square_raw(e), PINV[:, m])


@pytest.mark.parametrize("r", [0.2, 0.5, 1.6, 4.0])
def test_scaling_is_the_printed_diagonal(O, r):
    m = np.arange(1.0, 10.0)
    np.testing.assert_allclose(O.scale_rect(r, m), m * r ** SEXP, rtol=1e-15)
    np.testing.assert_allclose(O.unscale_rect(r, m), m * r ** -SEXP, rtol=1e-15)
