"""Pins for the oracle's moment transforms (Appendix A sub-steps 1-3, 5-7).

The oracle chains closed-form maps: square raw moments (eq. 62), scaling S,
binomial shift F(u), and back through F(-u), S^-1 and eq. 72.  Here they are
checked against the *definition* of the central moments (eq. 9B, direct sums
over the rectangular velocity set) and against a generic linear solve of that
definition, on random populations, velocities and aspect ratios.
"""
import numpy as np
import pytest

EX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1], dtype=float)
EYB = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1], dtype=float)
ORDERS = [(0, 0), (1, 0), (0, 1), (2, 0), (0, 2), (1, 1), (2, 1), (1, 2), (2, 2)]
RS = [0.2, 0.5, 1.0, 1.6, 2.0, 4.0]


def definition_matrix(r, ux, uy):
    """M[mn, alpha] = (e_ax - ux)^m (e_ay - uy)^n with e_ay = r * (0, +-1)."""
    ey = r * EYB
    return np.array([(EX - ux) ** m * (ey - uy) ** n for m, n in ORDERS])


@pytest.mark.parametrize("r", RS)
def test_central_moments_match_definition(O, r):
    rng = np.random.default_rng(int(r * 100))
    for _ in range(20):
        f = rng.uniform(0.01, 0.5, 9)
        ux, uy = rng.uniform(-0.2, 0.2, 2)
        m = O.scale_rect(r, O.raw_moments_square(f))
        k = O.central_from_raw(m, ux, uy)
        ref = definition_matrix(r, ux, uy) @ f
        np.testing.assert_allclose(k, ref, rtol=1e-13, atol=1e-14)


@pytest.mark.parametrize("r", RS)
def test_raw_moments_match_definition(O, r):
    rng = np.random.default_rng(7)
    f = rng.uniform(0.01, 0.5, 9)
    m = O.scale_rect(r, O.raw_moments_square(f))
    np.testing.assert_allclose(m, definition_matrix(r, 0.0, 0.0) @ f, rtol=1e-14,
                               atol=1e-15)


@pytest.mark.parametrize("r", RS)
def test_inverse_chain_matches_linear_solve(O, r):
    rng = np.random.default_rng(11 + int(10 * r))
    for _ in range(20):
        k = rng.normal(size=9)
        ux, uy = rng.uniform(-0.2, 0.2, 2)
        m = O.raw_from_central(k, ux, uy)
        f = O.populations_from_square_raw(O.unscale_rect(r, m))
        ref = np.linalg.solve(definition_matrix(r, ux, uy), k)
        np.testing.assert_allclose(f, ref, rtol=1e-11, atol=1e-12)


def test_square_inverse_is_inverse(O):
    """P P^-1 = I: eq. 62 followed by eq. 72 on unit vectors."""
    for a in range(9):
        e = np.zeros(9)
        e[a] = 1.0
        np.testing.assert_allclose(
            O.populations_from_square_raw(O.raw_moments_square(e)), e, atol=1e-15)


def test_shift_inverse_is_negated_velocity(O):
    """F(u)^-1 = F(-u) (Sec. 4.2)."""
    rng = np.random.default_rng(3)
    k = rng.normal(size=9)
    ux, uy = 0.13, -0.07
    back = O.central_from_raw(O.raw_from_central(k, ux, uy), ux, uy)
    np.testing.assert_allclose(back, k, rtol=1e-14, atol=1e-15)


@pytest.mark.parametrize("r", RS)
def test_rest_state_moments(O, r):
    """The rest state has central moments (rho, 0, 0, c2, c2, 0, 0, 0, c2^2)
    with c2 = q^2/3, q = min(1, r) (eq. 2)."""
    q = min(1.0, r)
    c2 = q * q / 3.0
    p = O.params(4, 4, r, 1.0, 1.0, rho0=1.3)
    w = O.rest_populations(p)
    assert np.all(w > 0)
    k = definition_matrix(r, 0.0, 0.0) @ w
    np.testing.assert_allclose(
        k, 1.3 * np.array([1, 0, 0, c2, c2, 0, 0, 0, c2 * c2]), atol=1e-15)
