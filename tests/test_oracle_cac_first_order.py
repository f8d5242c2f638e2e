"""Pins for the first-order phase-field equilibrium with the correction term
(Sec. 2.2, the alternative to the second-order equilibrium): its moments, the
correction's moments, agreement with the second-order scheme where the two
must coincide, and the same interface transport."""
import numpy as np
import pytest

import oracle
from tests.test_oracle_collision import cell_state
from tests.test_oracle_physics import flat_interface

CS2 = 1.0 / 3.0
D = oracle.D


def first_order(p):
    q = oracle.make_params(p.dim, tuple(p.n), rho_h=p.rho_h, rho_l=p.rho_l, nu_h=p.nu_h,
                           nu_l=p.nu_l, W=p.W, M=p.M, sigma=p.sigma, g=tuple(p.g),
                           cac_edf=1)
    return q


@pytest.mark.parametrize("dim", [2, 3])
def test_first_order_equilibrium_moments(dim):
    p, f, g, phi, grad, lap = cell_state(dim, 4)
    c, w, _ = oracle.lattice(dim)
    _, _, dg = oracle.collide_cell(first_order(p), f, g, phi, grad, lap)
    geq = dg[D["geq"]:D["geq"] + len(w)]
    u = dg[D["u"]:D["u"] + 3]
    # zeroth and first moments as the second-order equilibrium; the second
    # moment lacks the phi u u term: cs^2 phi I
    assert abs(geq.sum() - phi) < 1e-15
    assert np.abs(c.T @ geq - phi * u).max() < 1e-16
    M2 = np.einsum("a,ai,aj->ij", geq, c, c)
    assert np.abs(M2 - CS2 * phi * np.diag((np.arange(3) < dim).astype(float))).max() < 1e-15


@pytest.mark.parametrize("dim", [2, 3])
def test_correction_term_moments(dim):
    p, f, g, phi, grad, lap = cell_state(dim, 5)
    q = first_order(p)
    c, w, _ = oracle.lattice(dim)
    _, _, dg = oracle.collide_cell(q, f, g, phi, grad, lap)
    u = dg[D["u"]:D["u"] + 3]
    tb = dg[D["taubar_phi"]]
    d = np.zeros(3)
    d[:dim] = [3e-4, -1e-4, 2e-4][:dim]
    # no time change of (phi u): no correction; a change d: C = (1 - 1/(2 tb)) w c.d / cs^2
    _, g0, _ = oracle.collide_cell(q, f, g, phi, grad, lap, phiu_prev=phi * u)
    _, g1, _ = oracle.collide_cell(q, f, g, phi, grad, lap, phiu_prev=phi * u - d)
    _, gn, _ = oracle.collide_cell(q, f, g, phi, grad, lap)
    assert np.array_equal(g0, gn)
    C = g1 - g0  # a difference of two O(1e-2) sets: rounding ~1e-17
    assert abs(C.sum()) < 1e-16
    assert np.abs(c.T @ C - (1 - 1 / (2 * tb)) * d).max() < 1e-16


def test_both_equilibria_coincide_for_a_fluid_at_rest():
    # no force, no flow: u = 0 up to the round-off of the initial equilibria
    # (~1e-16), so both equilibria and the correction reduce to w phi and the
    # runs agree to round-off
    params, phi, uu = flat_interface(n=32, W=4.0, u=0.0)
    params = dict(params, sigma=0.0, g=(0.0, 0.0, 0.0))
    p2 = oracle.params_from_dict(params)
    p1 = oracle.params_from_dict(dict(params, cac_edf=1))
    f, g = oracle.init(p2, phi, uu, np.zeros_like(phi))
    a = oracle.step(p2, f, g, 20)
    b = oracle.step(p1, f, g, 20)
    assert np.array_equal(a[0], b[0])
    assert np.abs(a[1] - b[1]).max() < 1e-15


def test_first_order_scheme_transports_a_flat_interface_like_the_second_order_one():
    U, T, n = 0.02, 800, 64
    params, phi, uu = flat_interface(n=n, W=4.0, u=U)
    out = []
    for edf in (0, 1):
        p = oracle.params_from_dict(dict(params, cac_edf=edf))
        f, g = oracle.init(p, phi, uu, np.zeros_like(phi))
        f, g = oracle.step(p, f, g, T)
        out.append(oracle.fields(p, f, g)["phi"][0, 0])
    # same macroscopic equation: the profiles agree to the discretisation
    # error of the two schemes (3e-3, as the second-order scheme's own
    # distance from the exactly shifted profile), while the interface moved
    # U T = 16 cells
    assert np.abs(out[0] - out[1]).max() < 3e-3
    shifted = np.roll(phi[0, 0], int(round(U * T)))
    assert np.abs(out[1] - shifted).max() < 1e-2
