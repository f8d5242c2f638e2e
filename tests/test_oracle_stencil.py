"""Pins for the isotropic finite differences of the order parameter (Sec. 2.2):
the gradient is exact on quadratics, the Laplacian exact on cubics, both are
second-order accurate on smooth periodic fields, and walls mirror the first
fluid layer into the ghost layer."""
import numpy as np
import pytest

import oracle


def _grid(n):
    nx, ny, nz = n
    zz, yy, xx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return xx.astype(float), yy.astype(float), zz.astype(float)


def _interior(n, dim):
    nx, ny, nz = n
    sl = [slice(1, nz - 1) if dim == 3 else slice(None), slice(1, ny - 1), slice(1, nx - 1)]
    return tuple(sl)


@pytest.mark.parametrize("dim", [2, 3])
def test_gradient_exact_on_quadratics_laplacian_exact_on_cubics(dim):
    n = (9, 8, 7) if dim == 3 else (9, 8, 1)
    x, y, z = _grid(n)
    if dim == 2:
        z = np.zeros_like(z)
    rng = np.random.default_rng(1)
    a = rng.normal(size=20)
    phi = (a[0] + a[1] * x + a[2] * y + a[3] * z + a[4] * x * x + a[5] * y * y + a[6] * z * z +
           a[7] * x * y + a[8] * x * z + a[9] * y * z)
    cub = (a[10] * x ** 3 + a[11] * y ** 3 + a[12] * z ** 3 + a[13] * x * x * y + a[14] * x * y * z +
           a[15] * y * y * z + a[16] * x * z * z)
    p = oracle.make_params(dim, n, bc=(1, 1, 1 if dim == 3 else 0))
    grad, lap = oracle.gradients(p, phi)
    gx = a[1] + 2 * a[4] * x + a[7] * y + a[8] * z
    gy = a[2] + 2 * a[5] * y + a[7] * x + a[9] * z
    gz = a[3] + 2 * a[6] * z + a[8] * x + a[9] * y
    want = [gx, gy, gz][:dim]
    sl = _interior(n, dim)
    for i in range(dim):
        assert np.abs(grad[i][sl] - want[i][sl]).max() < 1e-11
    lap_want = 2 * (a[4] + a[5] + (a[6] if dim == 3 else 0.0))
    assert np.abs(lap[sl] - lap_want).max() < 1e-11
    # Laplacian of the cubic part: 6a10 x + 6a11 y + 6a12 z + 2a13 y + 2a15 z + 2a16 x
    _, lapc = oracle.gradients(p, phi + cub)
    lapc_want = lap_want + 6 * a[10] * x + 6 * a[11] * y + 2 * a[13] * y
    if dim == 3:
        lapc_want = lapc_want + 6 * a[12] * z + 2 * a[15] * z + 2 * a[16] * x
    assert np.abs(lapc[sl] - lapc_want[sl]).max() < 1e-10


@pytest.mark.parametrize("dim", [2, 3])
def test_second_order_convergence_on_periodic_sine(dim):
    errs = []
    for N in (8, 16, 32):
        n = (N, N, N if dim == 3 else 1)
        x, y, z = _grid(n)
        k = 2 * np.pi / N
        phi = np.sin(k * x) * np.cos(k * y) * (np.cos(k * z) if dim == 3 else 1.0)
        p = oracle.make_params(dim, n)
        grad, lap = oracle.gradients(p, phi)
        gx = k * np.cos(k * x) * np.cos(k * y) * (np.cos(k * z) if dim == 3 else 1.0)
        lap_want = -dim * k * k * phi
        # errors relative to the exact derivative scale (k and k^2)
        errs.append((np.abs(grad[0] - gx).max() / k, np.abs(lap - lap_want).max() / (k * k)))
    for j in range(2):
        r1 = errs[0][j] / errs[1][j]
        r2 = errs[1][j] / errs[2][j]
        assert 3.4 < r1 < 4.6 and 3.8 < r2 < 4.2, (errs, j)


def test_wall_ghost_mirrors_first_fluid_layer():
    n = (4, 6, 1)
    x, y, z = _grid(n)
    phi = y.copy()  # linear in the wall-normal direction
    p = oracle.make_params(2, n, bc=(0, 1, 0))
    grad, lap = oracle.gradients(p, phi)
    # ghost value at y=-1 equals phi(y=0)=0: one-sided stencil gives 1/2
    assert np.allclose(grad[1][0, 0, :], 0.5, atol=1e-14)
    assert np.allclose(grad[1][0, -1, :], 0.5, atol=1e-14)
    assert np.allclose(grad[1][0, 2, :], 1.0, atol=1e-14)
    # Laplacian at the first layer: 6 * sum_{c_y=-1} w * (phi(0) - phi(0)) + 6 * sum_{c_y=+1} w * 1
    assert np.allclose(lap[0, 0, :], 6 * (1 / 9 + 2 / 36), atol=1e-14)
