"""Pins for the oracle's per-node collision (Appendix A, collision sub-step).

* reduction to the textbook product-form equilibrium at gamma = 1 with all
  rates one and no corrections (the D2Q9 central-moment scheme on a square
  lattice, extended to r by the one-dimensional weights);
* exact conservation of mass and momentum, and a momentum gain of F/gamma
  under a body force (eq. 6, eq. hydrodynamicfields);
* lattice symmetries: mirror images in x and y for every r, the 90-degree
  rotation at r = 1 -- these catch sign and index slips in any term that is
  odd in a velocity or gradient component;
* which correction terms vanish where (eq. 38-40 with eq. 2).
"""
import numpy as np
import pytest

EX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1])
EYB = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1])
RS = [0.2, 0.5, 1.0, 1.6, 2.0, 4.0]

# index permutations of the velocity set: population of the image node
MIRROR_X = np.array([0, 3, 2, 1, 4, 6, 5, 8, 7])      # e_x -> -e_x
MIRROR_Y = np.array([0, 1, 4, 3, 2, 8, 7, 6, 5])      # e_y -> -e_y
ROT90 = np.array([0, 4, 1, 2, 3, 8, 5, 6, 7])         # new[a] = old[ROT90[a]]


def c2_of(r):
    q = min(1.0, r)
    return q * q / 3.0


def product_equilibrium(rho, ux, uy, r):
    """rho * phi_x(e_x) * phi_y(e_y): one-dimensional three-velocity
    distributions with mean u and variance c2 along x (lattice speed 1) and
    mean u, variance c2 along y (lattice speed r)."""
    c2 = c2_of(r)
    px = {0: 1 - c2 - ux * ux, 1: 0.5 * (c2 + ux * ux + ux), -1: 0.5 * (c2 + ux * ux - ux)}
    sy = (c2 + uy * uy) / (r * r)
    py = {0: 1 - sy, 1: 0.5 * (sy + uy / r), -1: 0.5 * (sy - uy / r)}
    return np.array([rho * px[EX[a]] * py[EYB[a]] for a in range(9)])


def random_state(rng, r, amp=0.3):
    """positive populations near a moving equilibrium"""
    rho = rng.uniform(0.9, 1.1)
    ux, uy = rng.uniform(-0.08, 0.08, 2) * min(1.0, r)
    feq = product_equilibrium(rho, ux, uy, r)
    return feq * (1.0 + amp * rng.uniform(-1, 1, 9))


@pytest.mark.parametrize("r", RS)
@pytest.mark.parametrize("frame", [0, 1])
def test_gamma1_unit_rates_gives_product_equilibrium(O, r, frame):
    """Central (PRC) and raw (PRNR) frames alike: with every rate one the
    collision lands on the equilibrium, the product form at gamma = 1."""
    rng = np.random.default_rng(int(r * 10))
    p = O.params(4, 4, r, 1.0, 1.0, corrections=0, frame=frame)
    for _ in range(10):
        f = random_state(rng, r)
        ft, d = O.collide_node(p, f)
        rho = f.sum()
        ux = (f * EX).sum() / rho
        uy = (f * EYB * r).sum() / rho
        np.testing.assert_allclose(ft, product_equilibrium(rho, ux, uy, r),
                                   rtol=1e-12, atol=1e-15)


@pytest.mark.parametrize("r", RS)
@pytest.mark.parametrize("gamma", [1.0, 0.5, 0.1])
@pytest.mark.parametrize("frame", [0, 1])
def test_collision_conserves_mass_and_momentum(O, r, gamma, frame):
    rng = np.random.default_rng(5)
    p = O.params(4, 4, r, gamma, 1.3, omega_xi=1.1, omega_1=0.9, omega_3=1.2,
                 omega_4=0.8, frame=frame)
    for _ in range(10):
        f = random_state(rng, r)
        gx, gy = rng.normal(scale=1e-3, size=2)
        ft, _ = O.collide_node(p, f, gx, gy)
        ey = EYB * r
        assert abs(ft.sum() - f.sum()) < 1e-14
        assert abs((ft * EX).sum() - (f * EX).sum()) < 1e-14
        assert abs((ft * ey).sum() - (f * ey).sum()) < 1e-14


@pytest.mark.parametrize("frame", [0, 1])
@pytest.mark.parametrize("omega_1", [1.0, 0.7])
def test_body_force_adds_force_over_gamma(O, frame, omega_1):
    rng = np.random.default_rng(9)
    r, gamma, fx, fy = 2.0, 0.3, 2e-5, -3e-5
    p = O.params(4, 4, r, gamma, 1.2, fx=fx, fy=fy, omega_1=omega_1, frame=frame)
    f = random_state(rng, r)
    ft, _ = O.collide_node(p, f, 0.0, 0.0)
    ey = EYB * r
    assert abs(ft.sum() - f.sum()) < 1e-14
    assert abs((ft * EX).sum() - (f * EX).sum() - fx / gamma) < 1e-14
    assert abs((ft * ey).sum() - (f * ey).sum() - fy / gamma) < 1e-14


def _mirror_check(O, p, perm, gsign, rng, r):
    f = random_state(rng, r)
    gx, gy = rng.normal(scale=2e-3, size=2)
    ft, _ = O.collide_node(p, f, gx, gy)
    ft_img, _ = O.collide_node(p, f[perm], gsign[0] * gx, gsign[1] * gy)
    np.testing.assert_allclose(ft_img, ft[perm], rtol=1e-12, atol=1e-15)


@pytest.mark.parametrize("r", RS)
@pytest.mark.parametrize("gamma", [1.0, 0.4])
@pytest.mark.parametrize("frame", [0, 1])
def test_mirror_symmetry(O, r, gamma, frame):
    rng = np.random.default_rng(21)
    p = O.params(4, 4, r, gamma, 1.4, omega_xi=1.2, frame=frame)
    for _ in range(5):
        _mirror_check(O, p, MIRROR_X, (-1, 1), rng, r)
        _mirror_check(O, p, MIRROR_Y, (1, -1), rng, r)


@pytest.mark.parametrize("gamma", [1.0, 0.3])
def test_rotation_symmetry_square_lattice(O, gamma):
    """At r = 1 the scheme is invariant under a quarter turn: populations
    rotate and the density gradient (gx, gy) becomes (-gy, gx)."""
    rng = np.random.default_rng(33)
    p = O.params(4, 4, 1.0, gamma, 1.5, omega_xi=1.3)
    for _ in range(10):
        f = random_state(rng, 1.0)
        gx, gy = rng.normal(scale=2e-3, size=2)
        ft, _ = O.collide_node(p, f, gx, gy)
        ft_rot, _ = O.collide_node(p, f[ROT90], -gy, gx)
        np.testing.assert_allclose(ft_rot, ft[ROT90], rtol=1e-12, atol=1e-15)


@pytest.mark.parametrize("r", RS)
def test_k11_corrections_vanish_without_preconditioning(O, r):
    """eq. 40: every k11 coefficient carries (1/gamma^2 - 1/gamma) or
    (1/gamma - 1), so at gamma = 1 switching them off changes nothing."""
    rng = np.random.default_rng(2)
    p_all = O.params(4, 4, r, 1.0, 1.3)
    p_no11 = O.params(4, 4, r, 1.0, 1.3, corrections=3)
    for _ in range(5):
        f = random_state(rng, r)
        gx, gy = rng.normal(scale=2e-3, size=2)
        np.testing.assert_allclose(O.collide_node(p_all, f, gx, gy)[0],
                                   O.collide_node(p_no11, f, gx, gy)[0], rtol=1e-13)


@pytest.mark.parametrize("r,axis", [(1.0, "x"), (1.0, "y"), (1.6, "x"), (2.0, "x"),
                                    (4.0, "x"), (0.5, "y"), (0.2, "y")])
def test_density_gradient_drops_out_where_factor_vanishes(O, r, axis):
    """At gamma = 1, U_gamma c2 - 1 = 3 c2 - 1 = 0 for r >= 1 and
    U_gamma c2 - r^2 = 0 for r <= 1 (eq. 2, eq. 38-39), so the collision does
    not depend on d_x rho (r >= 1), resp. d_y rho (r <= 1)."""
    rng = np.random.default_rng(4)
    p = O.params(4, 4, r, 1.0, 1.3)
    f = random_state(rng, r)
    base, _ = O.collide_node(p, f, 0.0, 0.0)
    g = (3e-3, 0.0) if axis == "x" else (0.0, 3e-3)
    moved, _ = O.collide_node(p, f, *g)
    np.testing.assert_allclose(moved, base, rtol=1e-13, atol=1e-16)
    # and the other component does matter when r != 1 or gamma != 1
    if r != 1.0:
        g2 = (0.0, 3e-3) if axis == "x" else (3e-3, 0.0)
        other, _ = O.collide_node(p, f, *g2)
        assert np.max(np.abs(other - base)) > 1e-9


def test_corrections_matter_off_the_square_lattice(O):
    rng = np.random.default_rng(8)
    f = random_state(rng, 2.0)
    on, _ = O.collide_node(O.params(4, 4, 2.0, 0.2, 1.3), f, 1e-3, -1e-3)
    off, _ = O.collide_node(O.params(4, 4, 2.0, 0.2, 1.3, corrections=0), f, 1e-3, -1e-3)
    assert np.max(np.abs(on - off)) > 1e-6


@pytest.mark.parametrize("r", RS)
@pytest.mark.parametrize("gamma", [1.0, 0.2])
def test_equilibrium_is_fixed_point_without_corrections(O, r, gamma):
    """Populations at the preconditioned equilibrium (eq. 14) are unchanged by
    a collision when the corrections are off."""
    p = O.params(4, 4, r, gamma, 0.7, omega_xi=1.3, corrections=0)
    feq = O.equilibrium_node(p, 1.02, 0.03 * min(1, r), -0.02 * min(1, r))
    ft, _ = O.collide_node(p, feq)
    np.testing.assert_allclose(ft, feq, rtol=1e-13, atol=1e-16)


@pytest.mark.parametrize("r", [0.5, 2.0])
def test_where_raw_and_central_frames_differ(O, r):
    """Relaxing raw (PRNR) or central (PRC) moments gives the same result at
    gamma = 1 when every moment is fully relaxed (all rates one, no
    corrections); it differs once the shear rate or the corrections leave the
    second-order moments off their base equilibria (the higher raw moments
    then inherit them only in the central frame), and under preconditioning
    even with full relaxation: the central k22
    equilibrium c2^2 rho (below eq. 14) maps to a raw k22 with
    (4/gamma^2 - 6/gamma + 3) rho ux^2 uy^2, the raw one (eq. 12) keeps 1."""
    rng = np.random.default_rng(5)
    f = random_state(rng, r)

    def both(gamma, omega_nu, corrections=0):
        return [O.collide_node(O.params(4, 4, r, gamma, omega_nu, frame=fr,
                                        corrections=corrections), f, 1e-3, -2e-3)[0]
                for fr in (0, 1)]

    a, b = both(1.0, 1.0)
    np.testing.assert_allclose(a, b, rtol=1e-12, atol=1e-15)
    a, b = both(1.0, 1.6)
    assert np.abs(a - b).max() > 1e-6
    # the corrections enter the higher raw moments only in the central frame
    a, b = both(1.0, 1.0, corrections=7)
    assert np.abs(a - b).max() > 1e-7
    a, b = both(0.5, 1.0)
    # the full-relaxation difference is exactly the fourth-order one
    rho = f.sum()
    ux = (f * EX).sum() / rho
    uy = (f * EYB * r).sum() / rho
    g = 0.5
    dm22 = (4 / g ** 2 - 6 / g + 3 - 1) * rho * ux ** 2 * uy ** 2
    # a change dm22 of the raw moment m22 alone changes f by P^-1 S^-1 of it
    e = np.zeros(9)
    e[8] = 1.0
    basis = O.populations_from_square_raw(O.unscale_rect(r, e))
    np.testing.assert_allclose(a - b, dm22 * basis, rtol=1e-9, atol=1e-16)
