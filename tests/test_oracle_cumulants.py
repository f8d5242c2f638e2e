"""Pins for the oracle's moment / cumulant transforms (Sec. 2.3).

* forward transform vs joint cumulants by brute-force enumeration of set
  partitions (the general moment-cumulant formula), on random populations;
* backward transform is the inverse of the forward one;
* with all cumulants above second order at zero, the backward transform gives
  Isserlis (Wick) moments, checked against a brute-force sum over perfect
  matchings;
* the populations rebuilt from central moments reproduce those moments.
"""
import itertools
import math

import numpy as np
import pytest

import oracle


def set_partitions(items):
    if not items:
        yield []
        return
    first, rest = items[0], items[1:]
    for part in set_partitions(rest):
        yield [[first]] + part
        for i in range(len(part)):
            yield part[:i] + [[first] + part[i]] + part[i + 1:]


def perfect_matchings(items):
    if not items:
        yield []
        return
    a = items[0]
    for i in range(1, len(items)):
        rest = items[1:i] + items[i + 1:]
        for m in perfect_matchings(rest):
            yield [(a, items[i])] + m


def random_populations(dim, seed):
    c, w, _ = oracle.lattice(dim)
    rng = np.random.default_rng(seed)
    h = w * (1.0 + 0.6 * rng.uniform(-1, 1, size=len(w)))
    h /= h.sum()
    u = (c * h[:, None]).sum(axis=0)
    return c, h, u


def raw_central(c, h, u, axes):
    """E[prod_i (c_axis_i - u_axis_i)] over the unit-mass set h."""
    v = np.ones(len(h))
    for ax in axes:
        v = v * (c[:, ax] - u[ax])
    return float((v * h).sum())


def brute_cumulant(c, h, u, axes):
    total = 0.0
    for part in set_partitions(list(range(len(axes)))):
        k = len(part)
        term = (-1) ** (k - 1) * math.factorial(k - 1)
        for block in part:
            term *= raw_central(c, h, u, [axes[i] for i in block])
        total += term
    return total


def exps(dim):
    return [(a, b, cc) for a in range(3) for b in range(3) for cc in range(3 if dim == 3 else 1)]


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_forward_matches_set_partition_cumulants(dim, seed):
    c, h, u = random_populations(dim, seed)
    Pi = oracle.central_moments(dim, h, u)
    K = oracle.cumulants_from_central(dim, Pi)
    for (a, b, cc) in exps(dim):
        if a + b + cc < 2:
            continue
        axes = [0] * a + [1] * b + [2] * cc
        want = brute_cumulant(c, h, u, axes)
        got = K[a * 9 + b * 3 + cc]
        assert abs(got - want) < 1e-13, ((a, b, cc), got, want)
    # first central moments vanish, zeroth is one
    assert abs(Pi[0] - 1.0) < 1e-14
    assert max(abs(Pi[9]), abs(Pi[3]), abs(Pi[1])) < 1e-15


@pytest.mark.parametrize("dim", [2, 3])
def test_backward_inverts_forward(dim):
    c, h, u = random_populations(dim, 7)
    Pi = oracle.central_moments(dim, h, u)
    Pi2 = oracle.central_from_cumulants(dim, oracle.cumulants_from_central(dim, Pi))
    assert np.abs(Pi2 - Pi).max() < 1e-14


@pytest.mark.parametrize("dim", [2, 3])
def test_backward_with_gaussian_cumulants_gives_isserlis_moments(dim):
    rng = np.random.default_rng(3)
    K = np.zeros(27)
    K[0] = 1.0
    cov = np.zeros((3, 3))
    for i in range(dim):
        cov[i, i] = rng.uniform(0.2, 0.5)
    for i in range(dim):
        for j in range(i + 1, dim):
            cov[i, j] = cov[j, i] = rng.uniform(-0.05, 0.05)
    for i in range(dim):
        for j in range(i, dim):
            e = [0, 0, 0]
            e[i] += 1
            e[j] += 1
            K[e[0] * 9 + e[1] * 3 + e[2]] = cov[i, j]
    Pi = oracle.central_from_cumulants(dim, K)
    for (a, b, cc) in exps(dim):
        axes = [0] * a + [1] * b + [2] * cc
        if len(axes) % 2:
            want = 0.0
        else:
            want = sum(np.prod([cov[axes[i], axes[j]] for i, j in m]) if m else 1.0
                       for m in perfect_matchings(list(range(len(axes)))))
        assert abs(Pi[a * 9 + b * 3 + cc] - want) < 1e-15, ((a, b, cc), Pi[a * 9 + b * 3 + cc], want)


@pytest.mark.parametrize("dim", [2, 3])
def test_populations_from_central_reproduce_moments(dim):
    c, h, u = random_populations(dim, 11)
    Pi = oracle.central_moments(dim, h, u)
    h2 = oracle.populations_from_central(dim, Pi, u)
    assert np.abs(h2 - h).max() < 1e-14
