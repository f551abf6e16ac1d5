"""Pins of the null-space oracle against null spaces known in closed form."""
import numpy as np

import gen
from oracle import nullspace as N


def test_periodic_difference_operator_has_the_constant_null_vector():
    # T(-1) = D^T D with D the periodic first difference: N = span(1) (Example 4.2)
    n = 60
    Z = N.null_basis(gen.tridiag_T(n, -1.0))
    assert Z.shape == (n, 1)
    assert N.subspace_distance(Z, np.ones((n, 1))) < 1e-12


def test_zero_variant_null_space_is_the_zero_columns_of_q2():
    f = gen.dense_factors(80, 1012, n_zero_m=8)
    M = (f.q2 * f.m) @ f.q2.T
    Z = N.null_basis(M)
    assert Z.shape[1] == 8
    assert N.subspace_distance(Z, f.null_basis_M()) < 1e-11


def test_diagonal_zeros_give_coordinate_vectors_and_definite_gives_none():
    d = np.linspace(1.0, 2.0, 30)
    d[[4, 19]] = 0.0
    Z = N.null_basis(np.diag(d))
    E = np.zeros((30, 2))
    E[4, 0] = E[19, 1] = 1.0
    assert N.subspace_distance(Z, E) < 1e-14
    assert N.null_basis(np.diag(np.linspace(1.0, 2.0, 30))).shape[1] == 0


def test_subspace_distance():
    rng = np.random.default_rng(0)
    Q, _ = np.linalg.qr(rng.standard_normal((20, 3)))
    assert N.subspace_distance(Q, Q @ rng.standard_normal((3, 3))) < 1e-13   # same span
    e = np.zeros((20, 1))
    e[0] = 1.0
    f = np.zeros((20, 1))
    f[0], f[1] = np.cos(0.3), np.sin(0.3)
    assert abs(N.subspace_distance(e, f) - np.sin(0.3)) < 1e-14
    assert N.subspace_distance(Q, Q[:, :2]) == 1.0
