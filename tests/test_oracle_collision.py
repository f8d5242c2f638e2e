"""Pins for the oracle's single-cell collision (Sec. 2.2 and 2.3).

Each check is a fact that follows from the equations, not a re-typing of
them: moment identities of the flow source Xi, the exact momentum and pressure
updates, the cumulants of the post-collision set recomputed by brute force, the
closed-form product distribution reached at omega = 1, axis-permutation
equivariance, and the zeroth/first moments of the phase-field collision."""
import numpy as np
import pytest

import oracle
from tests.test_oracle_cumulants import brute_cumulant

CS2 = 1.0 / 3.0
D = oracle.D


def cell_state(dim, seed, noise=0.02, sigma=2e-3, g=(1e-4, -2e-4, 3e-4), nu=0.05, rho_l=0.1,
               collision=0):
    rng = np.random.default_rng(seed)
    p = oracle.make_params(dim, (1, 1, 1), rho_h=1.0, rho_l=rho_l, nu_h=nu, nu_l=2 * nu, W=4.0,
                           M=0.07, sigma=sigma, g=g, collision=collision)
    phi = rng.uniform(0.2, 0.8)
    u = np.zeros(3)
    u[:dim] = rng.uniform(-0.05, 0.05, dim)
    ph = rng.uniform(-1e-3, 1e-3)
    f, gg = oracle.init(p, np.full((1, 1, 1), phi), u.reshape(3, 1, 1, 1), np.full((1, 1, 1), ph))
    f = f.ravel() * (1 + noise * rng.uniform(-1, 1, f.size))
    gg = gg.ravel() * (1 + noise * rng.uniform(-1, 1, gg.size))
    gg *= phi / gg.sum()  # phi is the zeroth moment of g
    grad = np.zeros(3)
    grad[:dim] = rng.uniform(-0.1, 0.1, dim)
    lap = rng.uniform(-0.02, 0.02)
    return p, f, gg, phi, grad, lap


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("seed", [0, 1])
def test_source_moments(dim, seed):
    p, f, g, phi, grad, lap = cell_state(dim, seed)
    c, w, _ = oracle.lattice(dim)
    fo, go, dg = oracle.collide_cell(p, f, g, phi, grad, lap)
    Xi = dg[D["Xi"]:D["Xi"] + len(w)]
    u = dg[D["u"]:D["u"] + 3]
    F = dg[D["F"]:D["F"] + 3]
    grad_rho = (p.rho_h - p.rho_l) * grad
    assert abs(Xi.sum() - CS2 * u @ grad_rho) < 1e-16
    assert np.abs(c.T @ Xi - CS2 * F).max() < 1e-16


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("collision", [0, 1])
def test_pressure_and_momentum_update(dim, collision):
    p, f, g, phi, grad, lap = cell_state(dim, 5, collision=collision)
    c, w, _ = oracle.lattice(dim)
    fo, go, dg = oracle.collide_cell(p, f, g, phi, grad, lap)
    Xi = dg[D["Xi"]:D["Xi"] + len(w)]
    F = dg[D["F"]:D["F"] + 3]
    # zeroth moment gains the source; first moment gains cs^2 F per step
    assert abs(fo.sum() - (f.sum() + Xi.sum())) < 1e-16
    assert np.abs(c.T @ fo - (c.T @ f + CS2 * F)).max() < 1e-16
    # and the velocity is the first moment of the preconditioned set
    rho = dg[D["rho"]]
    u = dg[D["u"]:D["u"] + 3]
    assert np.abs(u - ((c.T @ f) / (rho * CS2) + F / (2 * rho))).max() < 1e-15


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("seed", [2, 3])
def test_post_collision_cumulants(dim, seed):
    p, f, g, phi, grad, lap = cell_state(dim, seed, noise=0.05)
    c, w, _ = oracle.lattice(dim)
    fo, go, dg = oracle.collide_cell(p, f, g, phi, grad, lap)
    q = len(w)
    u = dg[D["u"]:D["u"] + 3]
    om = dg[D["omega"]]
    h = dg[D["h"]:D["h"] + q]
    hs = dg[D["hstar"]:D["hstar"] + q]
    # unit mass and velocity u conserved through the collision
    assert abs(h.sum() - 1) < 1e-14 and abs(hs.sum() - 1) < 1e-14
    assert np.abs(c.T @ hs - u).max() < 1e-15
    K = lambda hh, axes: brute_cumulant(c, hh, u, axes)
    ax = list(range(dim))
    for i in ax:
        for j in ax:
            if i < j:
                assert abs(K(hs, [i, j]) - (1 - om) * K(h, [i, j])) < 1e-15
    # deviatoric parts relax with omega, the trace goes to dim * cs^2
    for j in ax[1:]:
        assert abs((K(hs, [0, 0]) - K(hs, [j, j])) - (1 - om) * (K(h, [0, 0]) - K(h, [j, j]))) < 1e-15
    assert abs(sum(K(hs, [i, i]) for i in ax) - dim * CS2) < 1e-15
    # every cumulant of order 3..2*dim vanishes
    for a in range(3):
        for b in range(3):
            for cc in range(3 if dim == 3 else 1):
                if a + b + cc >= 3:
                    axes = [0] * a + [1] * b + [2] * cc
                    assert abs(K(hs, axes)) < 1e-14, (a, b, cc, K(hs, axes))


@pytest.mark.parametrize("dim", [2, 3])
def test_omega_one_gives_product_of_1d_distributions(dim):
    # nu = 1/6 -> tau = 1/2, omega = 1: every cumulant is at equilibrium, so
    # h* is the product of D1Q3 sets with mean u_i and variance cs^2
    p, f, g, phi, grad, lap = cell_state(dim, 4, nu=1.0 / 6.0)
    p.nu_l = p.nu_h
    c, w, _ = oracle.lattice(dim)
    fo, go, dg = oracle.collide_cell(p, f, g, phi, grad, lap)
    assert abs(dg[D["omega"]] - 1.0) < 1e-15
    u = dg[D["u"]:D["u"] + 3]
    hs = dg[D["hstar"]:D["hstar"] + len(w)]

    def d1q3(ci, ui):
        return 1 - ui * ui - CS2 if ci == 0 else (ui * ui + ci * ui + CS2) / 2

    want = np.array([np.prod([d1q3(c[a, i], u[i]) for i in range(dim)]) for a in range(len(w))])
    assert np.abs(hs - want).max() < 1e-15
    # raw second moments of f^p* are those of the BGK equilibrium: P cs^2 delta + u u
    P = dg[D["P"]]
    fps = hs + w * (P - 1)
    m2 = np.einsum("a,ai,aj->ij", fps, c, c)
    want2 = P * CS2 * np.diag([1.0] * dim + [0.0] * (3 - dim)) + np.outer(u, u)
    assert np.abs(m2 - want2).max() < 1e-14


def test_rate_one_second_moments_match_bgk_equilibrium_at_any_omega():
    # with omega != 1 the off-equilibrium part is scaled, but the trace and the
    # higher orders are at equilibrium: check the trace of the raw moments
    p, f, g, phi, grad, lap = cell_state(3, 8, noise=0.05)
    c, w, _ = oracle.lattice(3)
    fo, go, dg = oracle.collide_cell(p, f, g, phi, grad, lap)
    u = dg[D["u"]:D["u"] + 3]
    P = dg[D["P"]]
    fps = dg[D["hstar"]:D["hstar"] + 27] + w * (P - 1)
    m2 = np.einsum("a,ai,aj->ij", fps, c, c)
    assert abs(np.trace(m2) - (3 * P * CS2 + u @ u)) < 1e-14


def test_axis_permutation_equivariance_3d():
    p, f, g, phi, grad, lap = cell_state(3, 9, noise=0.05, g=(0.0, 0.0, 0.0))
    c, w, _ = oracle.lattice(3)
    fo, go, _ = oracle.collide_cell(p, f, g, phi, grad, lap)
    index = {tuple(v): a for a, v in enumerate(c)}
    for perm in [(1, 2, 0), (2, 0, 1), (1, 0, 2)]:
        # relabel axes: new axis k is old axis perm[k]
        mp = np.array([index[tuple(c[a][list(perm)])] for a in range(27)])
        f2 = np.empty(27)
        g2 = np.empty(27)
        f2[mp] = f
        g2[mp] = g
        fo2, go2, _ = oracle.collide_cell(p, f2, g2, phi, grad[list(perm)], lap)
        assert np.abs(fo2[mp] - fo).max() < 1e-16
        assert np.abs(go2[mp] - go).max() < 1e-16


@pytest.mark.parametrize("dim", [2, 3])
def test_phase_field_collision_moments(dim):
    p, f, g, phi, grad, lap = cell_state(dim, 6)
    c, w, _ = oracle.lattice(dim)
    fo, go, dg = oracle.collide_cell(p, f, g, phi, grad, lap)
    tb = dg[D["taubar_phi"]]
    assert abs(tb - (p.M / CS2 + 0.5)) < 1e-15
    u = dg[D["u"]:D["u"] + 3]
    n = dg[D["n"]:D["n"] + 3]
    assert abs(go.sum() - phi) < 1e-15
    flux = (1 - 1 / tb) * (c.T @ g) + phi * u / tb + (1 - 1 / (2 * tb)) * CS2 * n * 4 * phi * (1 - phi) / p.W
    assert np.abs(c.T @ go - flux).max() < 1e-16
