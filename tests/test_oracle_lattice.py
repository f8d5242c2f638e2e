"""Pins for the oracle's lattice tables (Sec. 2.3, D3Q27; D2Q9 in 2-D).

The weights are typed out by hand in the oracle; these tests check them
against the Gauss-Hermite quadrature conditions they must satisfy and against
the tensor-product construction from the 1-D weights (2/3, 1/6, 1/6)."""
import itertools

import numpy as np
import pytest

import oracle

CS2 = 1.0 / 3.0


@pytest.mark.parametrize("dim", [2, 3])
def test_velocity_set_complete_and_opposites(dim):
    c, w, opp = oracle.lattice(dim)
    q = 9 if dim == 2 else 27
    assert c.shape == (q, 3)
    want = set(itertools.product((-1, 0, 1), repeat=dim))
    assert {tuple(v[:dim]) for v in c} == want
    if dim == 2:
        assert np.all(c[:, 2] == 0)
    for a in range(q):
        assert np.all(c[opp[a]] == -c[a])


@pytest.mark.parametrize("dim", [2, 3])
def test_weights_are_tensor_products_of_1d_weights(dim):
    c, w, _ = oracle.lattice(dim)
    w1 = {-1: 1.0 / 6.0, 0: 2.0 / 3.0, 1: 1.0 / 6.0}
    for a in range(len(w)):
        want = np.prod([w1[int(c[a, i])] for i in range(dim)])
        assert abs(w[a] - want) < 1e-16


@pytest.mark.parametrize("dim", [2, 3])
def test_isotropy_up_to_fourth_order(dim):
    c, w, _ = oracle.lattice(dim)
    c = c[:, :dim].astype(np.float64)
    d = np.eye(dim)
    assert abs(w.sum() - 1.0) < 1e-15
    assert np.abs(np.einsum("a,ai->i", w, c)).max() < 1e-16
    assert np.abs(np.einsum("a,ai,aj->ij", w, c, c) - CS2 * d).max() < 1e-15
    assert np.abs(np.einsum("a,ai,aj,ak->ijk", w, c, c, c)).max() < 1e-16
    m4 = np.einsum("a,ai,aj,ak,al->ijkl", w, c, c, c, c)
    iso = CS2 ** 2 * (np.einsum("ij,kl->ijkl", d, d) + np.einsum("ik,jl->ijkl", d, d) +
                      np.einsum("il,jk->ijkl", d, d))
    assert np.abs(m4 - iso).max() < 1e-15
