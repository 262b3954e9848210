"""Pins of the oracle's reference element (GLL tables, SBP, mortars) against
closed forms and identities that the mathematics fixes."""

import math

import numpy as np
import pytest

from oracle.refelem import gll, mortar_matrices, mass_matrix, lagrange_eval


def test_gll_closed_form_N3():
    xi, w, _ = gll(3)
    s = 1.0 / math.sqrt(5.0)
    np.testing.assert_allclose(xi, [-1.0, -s, s, 1.0], rtol=0, atol=1e-15)
    np.testing.assert_allclose(w, [1 / 6, 5 / 6, 5 / 6, 1 / 6], rtol=0, atol=1e-15)


def test_gll_closed_form_N4():
    xi, w, _ = gll(4)
    s = math.sqrt(3.0 / 7.0)
    np.testing.assert_allclose(xi, [-1.0, -s, 0.0, s, 1.0], rtol=0, atol=1e-15)
    np.testing.assert_allclose(w, [1 / 10, 49 / 90, 32 / 45, 49 / 90, 1 / 10], rtol=0, atol=1e-15)


@pytest.mark.parametrize("N", range(1, 8))
def test_sbp_and_exactness(N):
    xi, w, D = gll(N)
    W = np.diag(w)
    B = np.zeros((N + 1, N + 1))
    B[0, 0], B[N, N] = -1.0, 1.0
    # summation by parts: W D + D^T W = B
    assert np.abs(W @ D + D.T @ W - B).max() < 1e-14 * max(1, N)
    # D annihilates constants and differentiates x^k exactly for k <= N
    assert np.abs(D @ np.ones(N + 1)).max() < 1e-13
    for k in range(1, N + 1):
        assert np.abs(D @ xi ** k - k * xi ** (k - 1)).max() < 1e-12
    # the weights integrate polynomials of degree 2N-1 exactly
    for k in range(0, 2 * N):
        exact = (1 - (-1) ** (k + 1)) / (k + 1)
        assert abs(np.dot(w, xi ** k) - exact) < 1e-14


def test_norm_of_D():
    # ||D||_inf (end rows) in closed form: N=3: 7/2 + 5 sqrt(5)/2, N=4: 49/3
    for N, ref in ((3, 3.5 + 2.5 * math.sqrt(5.0)), (4, 49.0 / 3.0)):
        _, _, D = gll(N)
        assert abs(np.abs(D).sum(axis=1).max() - ref) < 1e-13


@pytest.mark.parametrize("N", [1, 2, 3, 4, 5])
def test_mortar_projection_identity(N):
    Pf, Pr = mortar_matrices(N)
    # projecting back the interpolated polynomial recovers it
    assert np.abs(Pr[0] @ Pf[0] + Pr[1] @ Pf[1] - np.eye(N + 1)).max() < 1e-14 * (N + 1)
    # constants are preserved both ways
    one = np.ones(N + 1)
    for k in range(2):
        assert np.abs(Pf[k] @ one - one).max() < 1e-14
    assert np.abs(Pr[0] @ one + Pr[1] @ one - one).max() < 1e-14
    # forward operator interpolates polynomials of degree N exactly
    xi, _, _ = gll(N)
    for k, s in ((0, (xi - 1) / 2), (1, (xi + 1) / 2)):
        for p in range(N + 1):
            assert np.abs(Pf[k] @ xi ** p - s ** p).max() < 1e-13


def test_mass_matrix_exact():
    # M = int l_i l_j; sum of all entries = length 2; against a fine quadrature
    N = 3
    xi, _, _ = gll(N)
    M = mass_matrix(N)
    assert abs(M.sum() - 2.0) < 1e-15
    xq = np.linspace(-1, 1, 20001)
    L = lagrange_eval(xi, xq)
    Mt = np.trapezoid(L[:, :, None] * L[:, None, :], xq, axis=0)
    assert np.abs(M - Mt).max() < 1e-7
