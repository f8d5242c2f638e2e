"""Degenerate cases of the method on the GPU, through the C ABI, against the
FP64 oracle or against what the equations fix exactly:

* a single phase (phi = 1 everywhere, or phi = 0): the interface terms of
  Sec. 2.2-2.3 vanish (grad phi = 0, so the normal of the sharpening source
  is zero and the surface force is zero); one step from a non-equilibrium
  state matches the oracle to the one-step bars (FP64 1e-12, FP32 2e-6);
* a single phase at rest (phi 0 or 1, u = 0, p = 0, no gravity, periodic):
  the equilibria of both sets are a fixed point of the step up to rounding:
  after 20 steps f' is zero to 1e-12 (exactly for phi = 0) in every storage
  format and g is w phi to a few ulps per step, alone and in a batch (bit for
  bit the solo run); an empty light phase with walls stays exactly zero;
* lattices one and two cells wide along an axis, and a single cell: every
  neighbour is the cell itself or its mirror; one step against the oracle;
* equal densities (density ratio 1): the single-fluid limit, one step
  against the oracle.
"""
import numpy as np
import pytest

import oracle
from paper_2101_06769_amd import inputs
from tests.helpers import from_abi, gpu_available, rel_err, to_abi
from tests.test_gpu_parity import TOL1, gpu_solver, noisy_state

pytestmark = pytest.mark.gpu

if gpu_available():
    from paper_2101_06769_amd import mplb


def params_for(dim, n, bc, rho_l=0.2, sigma=2e-3, grav=2e-5):
    g = [0.0, 0.0, 0.0]
    g[dim - 1] = -grav
    return dict(dim=dim, n=tuple(n), bc=tuple(bc), rho_h=1.0, rho_l=rho_l, nu_h=0.03, nu_l=0.08,
                W=4.0, M=0.08, sigma=sigma, g=tuple(g))


def one_step_vs_oracle(params, phi, u, p, storage, seed):
    dim = params["dim"]
    po, f, g = noisy_state(params, phi, u, p, seed=seed)
    s = gpu_solver(params, storage, state=(f, g))
    s.step(1)
    f1, g1 = oracle.step(po, f, g, 1)
    ef = rel_err(from_abi(dim, s.get_populations(0)), f1)
    eg = rel_err(from_abi(dim, s.get_populations(1)), g1)
    return ef, eg


@pytest.mark.parametrize("storage", ["fp64", "fp32"])
@pytest.mark.parametrize("phase", [0.0, 1.0])
@pytest.mark.parametrize("dim,n,bc", [(2, (17, 13, 1), (0, 1, 0)), (3, (11, 9, 8), (0, 2, 1))])
def test_single_phase_one_step(storage, phase, dim, n, bc):
    params = params_for(dim, n, bc)
    _, u, p = inputs.random_state(params, seed=21)
    phi = np.full(u.shape[1:], phase)
    ef, eg = one_step_vs_oracle(params, phi, u, p, storage, seed=4)
    print("single phase %.0f %s %s: f' %.2e g %.2e" % (phase, storage, n, ef, eg))
    assert ef < TOL1[storage] and eg < TOL1[storage]


ULP = {"fp64": 2.0 ** -52, "fp32": 2.0 ** -23, "fp16s": 2.0 ** -23, "fp16s_all": 2.0 ** -23}


@pytest.mark.parametrize("storage", ["fp64", "fp32", "fp16s", "fp16s_all"])
@pytest.mark.parametrize("phase", [0.0, 1.0])
@pytest.mark.parametrize("dim,n", [(2, (24, 16, 1)), (3, (128, 8, 6))])
def test_fluid_at_rest_is_a_fixed_point(storage, phase, dim, n):
    # a single phase at rest, periodic on every axis.  The order parameter is
    # summed in orders that differ between the rows of a tile (the partial
    # sums of the update), so after a step it is uniform only to a rounding;
    # where it is then not exactly uniform the interface normal of the
    # sharpening source is of order one (grad phi against the 1e-24 floor of
    # its normalisation), and the source itself carries phi (1 - phi), a
    # rounding in a single phase.  So f' stays zero to the square of a
    # rounding and g stays w phi to a few ulps per step.  (A uniform phi of
    # 1/2, all interface, has an O(1) source there: no fixed point then.)
    params = params_for(dim, n, (0, 0, 0), grav=0.0)
    nx, ny, nz = n
    phi = np.full((nz, ny, nx), phase)
    s = mplb.Solver(params, storage=storage)
    s.init(phi, np.zeros((3, nz, ny, nx)), np.zeros((nz, ny, nx)))
    g0 = s.get_populations(1)
    s.step(20)  # past the step graph's 16-step runs
    f1, g1 = s.get_populations(0), s.get_populations(1)
    if phase == 0.0:
        assert np.all(f1 == 0.0) and np.all(g1 == 0.0)
    assert np.abs(f1).max() <= 1e-12
    assert np.abs(g1 - g0).max() <= 20 * 8 * ULP[storage] * max(phase, 1e-300)
    red, rc = s.reduce()
    assert rc == mplb.OK and red[4] <= 1e-12  # max |u|


@pytest.mark.parametrize("storage", ["fp64", "fp32", "fp16s", "fp16s_all"])
@pytest.mark.parametrize("dim,n,bc", [(2, (24, 16, 1), (1, 1, 0)), (3, (128, 8, 6), (0, 1, 1))])
def test_empty_light_phase_at_rest_with_walls_stays_exactly_zero(storage, dim, n, bc):
    params = params_for(dim, n, bc, grav=0.0)
    nx, ny, nz = n
    z = np.zeros((nz, ny, nx))
    s = mplb.Solver(params, storage=storage)
    s.init(z, np.zeros((3, nz, ny, nx)), z)
    s.step(20)
    assert np.all(s.get_populations(0) == 0.0) and np.all(s.get_populations(1) == 0.0)


@pytest.mark.parametrize("storage", ["fp64", "fp32"])
@pytest.mark.parametrize("dim,n,bc", [
    (3, (1, 1, 1), (0, 0, 0)),     # one cell, its own neighbour in every direction
    (3, (2, 2, 2), (1, 1, 1)),     # every cell a corner of walls
    (3, (1, 5, 3), (0, 2, 1)),     # one cell wide in x
    (2, (1, 1, 1), (0, 0, 0)),
    (2, (2, 7, 1), (2, 1, 0)),     # two cells between symmetry planes
])
def test_one_and_two_cell_lattices_one_step(storage, dim, n, bc):
    params = params_for(dim, n, bc)
    phi, u, p = inputs.random_state(params, seed=sum(n) + 3)
    ef, eg = one_step_vs_oracle(params, phi, u, p, storage, seed=9)
    print("tiny %s %s %s: f' %.2e g %.2e" % (storage, n, bc, ef, eg))
    assert ef < TOL1[storage] and eg < TOL1[storage]


@pytest.mark.parametrize("storage", ["fp64", "fp32"])
@pytest.mark.parametrize("dim,n,bc", [(2, (19, 11, 1), (0, 1, 0)), (3, (10, 9, 8), (0, 0, 1))])
def test_equal_densities_one_step(storage, dim, n, bc):
    params = params_for(dim, n, bc, rho_l=1.0)
    phi, u, p = inputs.random_state(params, seed=31)
    ef, eg = one_step_vs_oracle(params, phi, u, p, storage, seed=13)
    assert ef < TOL1[storage] and eg < TOL1[storage]


def test_fluid_at_rest_stays_at_rest_in_a_batch():
    # the same fixed point when the domain steps in a batch's shared launches,
    # bit for bit the solo run
    params = params_for(3, (128, 8, 6), (0, 0, 0), grav=0.0)
    phi = np.full((6, 8, 128), 1.0)
    z = np.zeros((3, 6, 8, 128))
    b = mplb.Batch(3, "fp32", capacity=2, max_tiles=1 << 12)
    s = mplb.Solver(params, storage="fp32", stream=b.stream)
    s.init(phi, z, np.zeros((6, 8, 128)))
    f0, g0 = s.get_populations(0), s.get_populations(1)
    slot = b.attach(s, 20)
    b.step(20)
    b.detach(slot)
    solo = mplb.Solver(params, storage="fp32")
    solo.init(phi, z, np.zeros((6, 8, 128)))
    solo.step(20)
    f1, g1 = s.get_populations(0), s.get_populations(1)
    assert np.array_equal(f1, solo.get_populations(0)) and np.abs(f1).max() <= 1e-12
    assert np.array_equal(g1, solo.get_populations(1))
    assert np.abs(g1 - g0).max() <= 20 * 8 * ULP["fp32"]
