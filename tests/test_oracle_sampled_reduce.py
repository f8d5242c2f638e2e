"""Pins for the two oracle entry points the full-size GPU checks rest on.

* ``step_sampled`` (one step evaluated only at chosen cells, for lattices too
  large for a full oracle step) must equal ``step`` at every cell: the pulled
  value of direction a at x is the post-collision value that left the source
  cell x - c_a (Sec. 2.2, 2.3; pull streaming), with bounce-back at walls,
  mirroring at symmetry planes and periodic wrap.  A wrong source decoding, a
  wrong direction at a boundary, or the order parameter taken from the wrong
  time level would break the equality.
* ``reduce`` (sum phi, sum rho u, max |u|) must equal fixed-order serial sums
  of the per-cell fields: a density-weighted momentum (not a plain sum of u)
  is checked on a lattice whose density varies by a factor of five.
"""
import numpy as np
import pytest

import oracle
from paper_2101_06769_amd import inputs


def _state(dim, n, bc, seed, rho_l=0.2):
    g = [0.0, 0.0, 0.0]
    g[dim - 1] = -2e-5
    params = dict(dim=dim, n=n, bc=bc, rho_h=1.0, rho_l=rho_l, nu_h=0.03, nu_l=0.08, W=4.0,
                  M=0.08, sigma=2e-3, g=tuple(g))
    phi, u, p = inputs.random_state(params, seed=seed)
    po = oracle.params_from_dict(params)
    f, gg = oracle.init(po, phi, u, p)
    q = f.shape[0]
    f = f * (1 + inputs.population_noise(q, n, seed + 1, 0.05))
    gg = gg * (1 + inputs.population_noise(q, n, seed + 2, 0.05))
    return po, f, gg


MIXES = [
    (2, (9, 7, 1), (0, 1, 0)),     # periodic x, walls y
    (2, (8, 6, 1), (1, 2, 0)),     # walls x, symmetry y (corners of both kinds)
    (3, (9, 7, 6), (0, 0, 1)),     # walls z
    (3, (6, 5, 7), (1, 2, 0)),     # wall / symmetry / periodic
    (3, (5, 6, 4), (2, 1, 1)),     # symmetry x, walls y and z
]


@pytest.mark.parametrize("dim,n,bc", MIXES)
def test_step_sampled_equals_full_step_at_every_cell(dim, n, bc):
    po, f, g = _state(dim, n, bc, seed=sum(n))
    f1, g1 = oracle.step(po, f, g, 1)
    N = n[0] * n[1] * n[2]
    cells = np.arange(N)
    fo, go = oracle.step_sampled(po, f, g, cells)
    q = f.shape[0]
    assert np.array_equal(fo, f1.reshape(q, N).T)
    assert np.array_equal(go, g1.reshape(q, N).T)
    # any order, repeats allowed
    perm = np.random.default_rng(0).permutation(np.concatenate([cells, cells[:5]]))
    fp, gp = oracle.step_sampled(po, f, g, perm)
    assert np.array_equal(fp, f1.reshape(q, N).T[perm])
    assert np.array_equal(gp, g1.reshape(q, N).T[perm])


@pytest.mark.parametrize("dim,n,bc", [MIXES[0], MIXES[2], MIXES[3]])
def test_reduce_equals_serial_sums_of_fields(dim, n, bc):
    po, f, g = _state(dim, n, bc, seed=3, rho_l=0.2)
    fl = oracle.fields(po, f, g)
    phi, rho, u = fl["phi"].ravel(), fl["rho"].ravel(), fl["u"].reshape(3, -1)
    assert rho.max() / rho.min() > 1.5  # density weighting matters here
    s = [0.0, 0.0, 0.0, 0.0]
    umax = 0.0
    for i in range(phi.size):  # cell order, one addition at a time
        s[0] += float(phi[i])
        for k in range(3):
            s[1 + k] += float(rho[i]) * float(u[k, i])
        umax = max(umax, float(np.sqrt(u[0, i] ** 2 + u[1, i] ** 2 + u[2, i] ** 2)))
    got = oracle.reduce(po, f, g)
    want = np.array(s + [umax])
    assert np.allclose(got, want, rtol=1e-14, atol=1e-17), (got, want)
    # not the undensity-weighted momentum
    plain = u.sum(axis=1)
    assert np.abs(got[1:4] - plain).max() > 1e-3 * np.abs(plain).max()
