"""Pins for the density-gradient path of the oracle: the isotropic finite
difference for grad rho (Sec. 3.6 below eq. 43; Appendix A, collision
sub-step) and everything built from it -- the lambda coefficients of eq. 38-39,
the lambda~ coefficients of eq. 40 and the e_b, e_s terms of eq. 43/45 that
enter the strain-rate solve of eq. 46-48.

What fixes the expected values (none of them is the oracle's own formula):

* the gradient stencil is exact on a linear density and second-order
  accurate, with an isotropic leading error at r = 1 ("isotropic second-order
  finite difference"); the wall clamp (our reading where the paper is silent)
  halves the one-sided difference of a linear field, which follows from the
  clamp itself;
* acoustic waves: the corrections exist so that the scheme reproduces the
  preconditioned Navier-Stokes equations (eq. 17a-17c for the inviscid
  fluxes; eq. 18a-18c with the physical parts of eq.
  2ndordernoneqmmomentswitherrorterms for the viscous stresses, transport
  coefficients of eq. transport-coefficients).  Linearised about a uniform
  flow, those equations give a 3 x 3 eigenproblem per wavevector: the
  frequencies and damping rates of the two sound modes and the shear mode,
  and how a sound wave drags the velocity component across it.  The oracle's
  modes, extracted from a small-amplitude run by a least-squares fit of the
  Fourier amplitudes (dynamic mode decomposition), must match them.  On a
  moving background the u . grad rho errors of eq. truncationerrors-nonGI
  change the damping by 10-30 % unless the lambda terms cancel them, and the
  transverse drag of a sound wave is set by the lambda~ terms;
* the local strain rate of eq. 48 in a sound wave on a moving background
  against the spectral derivative of the oracle's own velocity field (the e_b,
  e_s terms carry the u . grad rho part of the non-equilibrium moments).

The Chapman-Enskog analysis behind the corrections keeps terms up to third
order in the velocity; the backgrounds here keep the preconditioned Mach
number U / (gamma c_s) at 0.3 or below, where the neglected orders stay
under the tolerances (at 0.6 they reach 18 % in the damping).
"""
from __future__ import annotations

import numpy as np
import pytest


def c2_of(r):
    q = min(1.0, r)
    return q * q / 3.0


# ------------------------------------------------------------ gradient ----

def _positions(nx, ny, r):
    X, Y = np.meshgrid(np.arange(nx) + 0.5, (np.arange(ny) + 0.5) * r)
    return X, Y


def linear_gradient_errors(O, r, a=0.013, b=-0.021, nx=9, ny=8):
    """Largest deviation of the stencil from the exact gradient (a, b) of
    rho = 1 + a x + b y: interior nodes, and the wall nodes against the
    clamped reading (half the gradient normal to the wall, the tangential one
    exact)."""
    p = O.params(nx, ny, r, 1.0, 1.0, bc=O.BC_CAVITY)
    X, Y = _positions(nx, ny, r)
    gx, gy = O.grad_rho(p, 1.0 + a * X + b * Y)
    ex = np.full((ny, nx), a)
    ey = np.full((ny, nx), b)
    # clamped neighbours: at a wall column the outer neighbour is the node
    # itself, so the central difference spans one spacing instead of two
    ex[:, 0] = ex[:, -1] = a / 2
    ey[0, :] = ey[-1, :] = b / 2
    inner = (slice(1, -1), slice(1, -1))
    return {
        "interior": max(np.abs(gx - ex)[inner].max() / abs(a), np.abs(gy - ey)[inner].max() / abs(b)),
        "walls": max(np.abs(gx - ex).max() / abs(a), np.abs(gy - ey).max() / abs(b)),
    }


@pytest.mark.parametrize("r", [0.5, 1.0, 2.0])
def test_grad_rho_exact_on_linear_density(O, r):
    e = linear_gradient_errors(O, r)
    assert e["interior"] < 1e-11, e
    assert e["walls"] < 1e-11, e


def test_grad_rho_channel_wraps_along_x(O):
    """Channel: periodic along x, walls along y.  A density linear in y and
    periodic in x keeps the exact gradient in every column, halved next to
    the walls."""
    nx, ny, r, b = 6, 7, 2.0, 0.02
    p = O.params(nx, ny, r, 1.0, 1.0, bc=O.BC_CHANNEL)
    X, Y = _positions(nx, ny, r)
    gx, gy = O.grad_rho(p, 1.0 + b * Y + 1e-3 * np.sin(2 * np.pi * X / nx))
    ey = np.full((ny, nx), b)
    ey[0, :] = ey[-1, :] = b / 2
    assert np.abs(gy - ey).max() < 1e-12
    # the x part is the periodic sine's derivative, wrapped at the ends
    k = 2 * np.pi / nx
    assert np.abs(gx - 1e-3 * k * np.cos(k * X)).max() < 0.25 * 1e-3 * k


def sine_gradient_error(O, r, kind, n):
    """Largest relative error of the stencil on a periodic plane wave of one
    wavelength across an n-node (or n-node-per-side) grid."""
    if kind == "x":
        nx, ny = n, 4
    elif kind == "y":
        nx, ny = 4, n
    else:
        nx, ny = n, int(round(n / r))
    p = O.params(nx, ny, r, 1.0, 1.0, bc=O.BC_PERIODIC)
    X, Y = _positions(nx, ny, r)
    kx = 2 * np.pi / nx if kind in "xd" else 0.0
    ky = 2 * np.pi / (ny * r) if kind in "yd" else 0.0
    eps = 1e-3
    ph = kx * X + ky * Y
    gx, gy = O.grad_rho(p, 1.0 + eps * np.sin(ph))
    scale = eps * np.hypot(kx, ky)
    return max(np.abs(gx - eps * kx * np.cos(ph)).max(),
               np.abs(gy - eps * ky * np.cos(ph)).max()) / scale


@pytest.mark.parametrize("r", [0.5, 1.0, 2.0])
@pytest.mark.parametrize("kind", ["x", "y", "d"])
def test_grad_rho_second_order(O, r, kind):
    e1 = sine_gradient_error(O, r, kind, 16)
    e2 = sine_gradient_error(O, r, kind, 32)
    # leading error (k h)^2 / 6 with h the coarser spacing along the wave
    # (16 nodes per wavelength at worst on the diagonal grids): about 0.026
    assert e2 < 0.03, (e1, e2)
    assert 3.6 < e1 / e2 < 4.4, (e1, e2)


def test_grad_rho_leading_error_isotropic_on_square_grid(O):
    """At r = 1 the stencil's leading error is (|k|^2 / 6) times the gradient
    whatever the direction of the wave: the computed gradient of a plane wave
    stays parallel to k and its relative shortfall does not depend on the
    angle (a five-point central difference would be off by a factor of two
    between the axis and the diagonal)."""
    n, eps = 64, 1e-3
    p = O.params(n, n, 1.0, 1.0, 1.0, bc=O.BC_PERIODIC)
    X, Y = _positions(n, n, 1.0)
    short = []
    for mx, my in ((4, 0), (0, 4), (3, 3), (4, 2), (2, 4)):
        kx, ky = 2 * np.pi * mx / n, 2 * np.pi * my / n
        kk = np.hypot(kx, ky)
        ph = kx * X + ky * Y
        gx, gy = O.grad_rho(p, 1.0 + eps * np.sin(ph))
        c = np.cos(ph)
        w = c * c
        # least-squares amplitude of each component along cos(phase)
        ax = (gx * c).sum() / w.sum() / (eps * kx) if kx else None
        ay = (gy * c).sum() / w.sum() / (eps * ky) if ky else None
        amps = [a for a in (ax, ay) if a is not None]
        # parallel to k: the components' shortfalls agree to 2 % of their size
        # (the five-point difference would leave them 75 % apart at (4, 2))
        assert max(amps) - min(amps) < 0.02 * (1 - min(amps)), (mx, my, amps)
        short.append((1 - amps[0]) / (kk * kk / 6))
    # leading term k^2/6 in every direction (higher orders: a few per cent)
    assert max(short) < 1.0 + 1e-9 and min(short) > 0.9, short


# ------------------------------------------------------------ acoustics ---

def linear_modes(k, r, gamma, omega_nu, omega_xi, U):
    """Eigenvalues s and eigenvectors (d rho, d u_x, d u_y) of the preconditioned
    Navier-Stokes equations linearised about rho = 1, u = U, for perturbations
    exp(i k . x + s t) (k in units of 1/dx):

        d_t rho + div(rho u) = 0                                   (eq. 17a)
        d_t(rho u) + div(rho u u / gamma) + c2 grad rho = div tau   (eq. 17b-c)
        tau_xx = c2 rho [h_xi div u + h_nu (d_x u_x - d_y u_y)]
        tau_yy = c2 rho [h_xi div u - h_nu (d_x u_x - d_y u_y)]
        tau_xy = c2 rho h_nu (d_x u_y + d_y u_x)        (eq. 18b-c with the
        physical parts of the second-order non-equilibrium moments)

    with h = 1/omega - 1/2 and c2 = q^2/3 (eq. 2)."""
    c2 = c2_of(r)
    hn, hx = 1.0 / omega_nu - 0.5, 1.0 / omega_xi - 0.5
    ikx, iky = 1j * k[0], 1j * k[1]
    U0, V0 = U
    g = gamma
    L = np.zeros((3, 3), complex)
    # mass
    L[0] = [-(ikx * U0 + iky * V0), -ikx, -iky]
    # x momentum: convective flux rho u_x u / gamma, pressure c2 rho, stresses
    L[1] = [-(ikx * U0 * U0 + iky * U0 * V0) / g - c2 * ikx,
            -(2 * ikx * U0 + iky * V0) / g, -iky * U0 / g]
    L[1] += ikx * c2 * np.array([0, (hx + hn) * ikx, (hx - hn) * iky])
    L[1] += iky * c2 * hn * np.array([0, iky, ikx])
    # y momentum
    L[2] = [-(iky * V0 * V0 + ikx * U0 * V0) / g - c2 * iky,
            -ikx * V0 / g, -(2 * iky * V0 + ikx * U0) / g]
    L[2] += iky * c2 * np.array([0, (hx - hn) * ikx, (hx + hn) * iky])
    L[2] += ikx * c2 * hn * np.array([0, iky, ikx])
    # the time derivative acts on (rho, rho u_x, rho u_y)
    M = np.array([[1, 0, 0], [U0, 1, 0], [V0, 0, 1]], float)
    return np.linalg.eig(np.linalg.solve(M, L))


def _wave_grid(kind, n, r):
    if kind == "x":
        return n, 3
    if kind == "y":
        return 3, n
    return n, int(round(n / r))


def oracle_modes(O, r, gamma, omega_nu, kind, n, U, corrections=7, t0=60, nsnap=120, dt=2):
    """Complex rates s and eigenvectors of the oracle's three hydrodynamic
    modes at the grid's longest wave along x, y or the diagonal: a
    small-amplitude perturbation exciting all three on a uniform flow U, the
    Fourier amplitudes of (rho, u_x, u_y) sampled every dt steps once the
    non-hydrodynamic moments have relaxed, and the 3 x 3 map between
    consecutive samples fitted by least squares."""
    nx, ny = _wave_grid(kind, n, r)
    p = O.params(nx, ny, r, gamma, omega_nu, bc=O.BC_PERIODIC, corrections=corrections)
    X, Y = _positions(nx, ny, r)
    kx = 2 * np.pi / nx if kind in "xd" else 0.0
    ky = 2 * np.pi / (ny * r) if kind in "yd" else 0.0
    ph = kx * X + ky * Y
    rng = np.random.default_rng(3)
    c = rng.normal(size=3) + 1j * rng.normal(size=3)
    amp = 1e-6
    pert = [np.real(ci * np.exp(1j * ph)) for ci in c]
    ft = O.equilibrium_field(p, 1.0 + amp * pert[0], U[0] + amp * pert[1], U[1] + amp * pert[2])
    E = np.exp(-1j * ph)
    O.step(p, ft, t0)
    snaps = []
    for _ in range(nsnap):
        rho, ux, uy = O.velocity(p, ft)
        snaps.append([(rho * E).mean(), (ux * E).mean(), (uy * E).mean()])
        O.step(p, ft, dt)
    S = np.array(snaps).T
    A = S[:, 1:] @ np.linalg.pinv(S[:, :-1])
    lam, vec = np.linalg.eig(A)
    return np.log(lam) / dt, vec, (kx, ky)


def acoustic_errors(O, r, gamma, omega_nu, kind, n, U, corrections=7):
    """Per mode of the oracle, matched to the nearest mode of the linearised
    equations: relative error of the damping rate, error of the frequency in
    units of the sound frequency c_s |k|, and relative error of the velocity
    component across the wave (per unit of the component along it)."""
    s, v, k = oracle_modes(O, r, gamma, omega_nu, kind, n, U, corrections)
    st, vt = linear_modes(k, r, gamma, omega_nu, 1.0, U)
    kk = np.hypot(*k)
    along, across = (1, 2) if kind == "x" else (2, 1)
    out = []
    for i in range(3):
        j = int(np.argmin(abs(st - s[i])))
        e = {"damping": abs(s[i].real - st[j].real) / abs(st[j].real),
             "frequency": abs(s[i].imag - st[j].imag) / (np.sqrt(c2_of(r)) * kk)}
        sound = abs(vt[0, j]) > 0.1 * np.linalg.norm(vt[:, j])   # carries density
        if kind != "d" and sound:
            a = v[across, i] / v[along, i]
            b = vt[across, j] / vt[along, j]
            if abs(b) > 1e-3:
                e["transverse"] = abs(a - b) / abs(b)
        out.append(e)
    return out


# (r, gamma, omega_nu, wave, nodes per wavelength, background); the
# preconditioned Mach number U / (gamma c_s) stays at or below 0.3
ACOUSTIC = [
    (0.5, 0.3, 1.2, "x", 32, (0.025, 0.0)),
    (0.5, 0.3, 1.2, "y", 32, (0.0, 0.0125)),
    (2.0, 0.3, 1.2, "y", 32, (0.0, 0.05)),
    (2.0, 0.3, 1.2, "x", 32, (0.05, 0.0)),
    (1.0, 0.3, 1.2, "x", 32, (0.05, 0.0)),
    (1.0, 0.3, 1.2, "d", 24, (0.04, 0.03)),
    (0.5, 0.5, 1.5, "d", 24, (0.015, -0.01)),
    (2.0, 0.5, 1.5, "d", 24, (-0.04, 0.03)),
]
# a sound wave across a background flow: the transverse drag is set by the
# lambda~ terms of eq. 40 (gamma < 1)
TRANSVERSE = [
    (0.5, 0.3, 0.8, "x", 32, (0.0, 0.025)),
    (2.0, 0.3, 0.8, "y", 32, (0.05, 0.0)),
]
TOL_DAMPING, TOL_FREQUENCY, TOL_TRANSVERSE = 0.03, 0.02, 0.02


def acoustic_pins_hold(O, cases=ACOUSTIC + TRANSVERSE):
    """True if every mode of every case is within the tolerances."""
    for case in cases:
        for e in acoustic_errors(O, *case):
            if e["damping"] > TOL_DAMPING or e["frequency"] > TOL_FREQUENCY:
                return False
            if e.get("transverse", 0.0) > TOL_TRANSVERSE:
                return False
    return True


@pytest.mark.parametrize("case", ACOUSTIC + TRANSVERSE, ids=lambda c: f"r{c[0]}_{c[3]}_{c[5]}")
def test_sound_and_shear_modes_match_preconditioned_navier_stokes(O, case):
    errs = acoustic_errors(O, *case)
    for e in errs:
        assert e["damping"] < TOL_DAMPING, errs
        assert e["frequency"] < TOL_FREQUENCY, errs
        assert e.get("transverse", 0.0) < TOL_TRANSVERSE, errs
    if case in TRANSVERSE:
        assert sum("transverse" in e for e in errs) == 2, errs


@pytest.mark.parametrize("case", [ACOUSTIC[0], ACOUSTIC[2], ACOUSTIC[4]],
                         ids=lambda c: f"r{c[0]}_{c[3]}")
def test_sound_damping_on_moving_background_needs_lambda(O, case):
    """Without the lambda terms the u . grad rho errors of eq.
    truncationerrors-nonGI stay in the viscous stress, and a sound wave on a
    moving background is damped at the wrong rate."""
    errs = acoustic_errors(O, *case, corrections=O.CORR_ALL & ~O.CORR_LAMBDA)
    assert max(e["damping"] for e in errs) > 0.1, errs


def test_sound_damping_at_rest_does_not_depend_on_lambda(O):
    """At rest every lambda term is zero (they are proportional to u)."""
    case = (0.5, 0.3, 1.2, "x", 32, (0.0, 0.0))
    a = acoustic_errors(O, *case)
    b = acoustic_errors(O, *case, corrections=O.CORR_ALL & ~O.CORR_LAMBDA)
    for ea, eb in zip(sorted(a, key=lambda e: e["damping"]), sorted(b, key=lambda e: e["damping"])):
        assert abs(ea["damping"] - eb["damping"]) < 1e-9


def strain_rate_errors(O, r, gamma, omega_nu, kind, n, U, steps=200):
    """Largest error of the local strain rates of eq. 48 against the spectral
    derivative of the velocity field, relative to the largest true value, in
    a sound wave (one wavelength, started at rest relative to U) after
    `steps` steps."""
    nx, ny = _wave_grid(kind, n, r)
    p = O.params(nx, ny, r, gamma, omega_nu, bc=O.BC_PERIODIC)
    X, Y = _positions(nx, ny, r)
    kx = 2 * np.pi / nx if kind in "xd" else 0.0
    ky = 2 * np.pi / (ny * r) if kind in "yd" else 0.0
    ph = kx * X + ky * Y
    ft = O.equilibrium_field(p, 1.0 + 1e-4 * np.cos(ph), U[0], U[1])
    O.step(p, ft, steps)
    f = O.stream(p, ft)
    rho, ux, uy = O.macros(p, f)
    gx, gy = O.grad_rho(p, rho)
    dx = np.zeros((ny, nx))
    dy = np.zeros((ny, nx))
    for j in range(ny):
        for i in range(nx):
            _, d = O.collide_node(p, f[:, j, i], gx[j, i], gy[j, i])
            dx[j, i], dy[j, i] = d["dxux"], d["dyuy"]
    E = np.exp(-1j * ph)
    ex = np.real(2j * kx * (ux * E).mean() * np.exp(1j * ph))
    ey = np.real(2j * ky * (uy * E).mean() * np.exp(1j * ph))
    out = {}
    if kx:
        out["dxux"] = np.abs(dx - ex).max() / np.abs(ex).max()
    if ky:
        out["dyuy"] = np.abs(dy - ey).max() / np.abs(ey).max()
    return out


STRAIN = [
    (0.5, 0.3, 1.2, "x", 32, (0.025, 0.0)),
    (1.0, 0.3, 1.2, "x", 32, (0.05, 0.0)),
    (2.0, 0.3, 1.2, "x", 32, (0.05, 0.0)),
    (2.0, 0.3, 1.2, "y", 32, (0.0, 0.05)),
]
TOL_STRAIN = 0.08


def strain_pins_hold(O):
    return all(max(strain_rate_errors(O, *c).values()) < TOL_STRAIN for c in STRAIN)


@pytest.mark.parametrize("case", STRAIN, ids=lambda c: f"r{c[0]}_{c[3]}")
def test_strain_rate_in_sound_wave_on_moving_background(O, case):
    e = strain_rate_errors(O, *case)
    assert max(e.values()) < TOL_STRAIN, e
