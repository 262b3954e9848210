"""Reference element: Gauss-Lobatto-Legendre (GLL) nodes, weights, the nodal
derivative matrix, Lagrange evaluation and the 2:1 mortar projections.

Follows the paper's description of the DGSEM reference element (GPU
Implementation section: tensor-product GLL collocation with the 1-D derivative
matrix D and quadrature weights w, summation-by-parts structure) and its mortar
paragraph (Surface Fluxes: forward interpolation to the mortars, reverse L2
projection carrying the area ratio).

Pinned by: closed-form GLL tables for N=3,4 and the SBP identity
W D + D^T W = diag(-1,0,..,0,1), D.1 = 0, exactness of D on x^k for k<=N, and
sum_k P^{k->c} P^{c->k} = I (tests/test_oracle_refelem.py).
"""

import numpy as np


def legendre(N, x):
    """P_N(x) and P_{N-1}(x) by the three-term (Bonnet) recurrence."""
    x = np.asarray(x, dtype=np.float64)
    p_prev = np.ones_like(x)
    if N == 0:
        return p_prev, np.zeros_like(x)
    p = x.copy()
    for k in range(1, N):
        p_prev, p = p, ((2 * k + 1) * x * p - k * p_prev) / (k + 1)
    return p, p_prev


def gll(N):
    """GLL nodes xi_0..xi_N (ascending), weights w and derivative matrix D.

    Nodes: the end points +-1 and the N-1 roots of P_N'.  Weights:
    w_i = 2 / (N (N+1) P_N(xi_i)^2).  Derivative matrix of the Lagrange basis at
    the nodes: D_ij = P_N(xi_i) / (P_N(xi_j) (xi_i - xi_j)) off the diagonal,
    D_00 = -N(N+1)/4, D_NN = +N(N+1)/4, other diagonal entries 0.
    """
    if N < 1:
        raise ValueError("GLL needs N >= 1")
    # interior nodes: roots of P_N', polished by Newton with P_N'' from the
    # Legendre equation (1-x^2) P'' = 2 x P' - N(N+1) P
    if N >= 2:
        c = np.zeros(N + 1)
        c[N] = 1.0
        guess = np.sort(np.real(np.polynomial.legendre.Legendre(c).deriv().roots()))
        x = guess.astype(np.float64)
        for _ in range(50):
            p, pm = legendre(N, x)
            dp = N * (x * p - pm) / (x * x - 1.0)
            d2p = (2.0 * x * dp - N * (N + 1) * p) / (1.0 - x * x)
            dx = dp / d2p
            x = x - dx
            if np.max(np.abs(dx)) < 1e-17:
                break
        interior = np.sort(x)
    else:
        interior = np.zeros(0)
    xi = np.concatenate([[-1.0], interior, [1.0]])
    # symmetrise (the node set is symmetric about 0)
    xi = 0.5 * (xi - xi[::-1])
    if N % 2 == 0:
        xi[N // 2] = 0.0
    pN, _ = legendre(N, xi)
    w = 2.0 / (N * (N + 1) * pN ** 2)
    n = N + 1
    D = np.zeros((n, n))
    for i in range(n):
        for j in range(n):
            if i != j:
                D[i, j] = pN[i] / (pN[j] * (xi[i] - xi[j]))
    D[0, 0] = -N * (N + 1) / 4.0
    D[N, N] = N * (N + 1) / 4.0
    return xi, w, D


def lagrange_eval(xi, x):
    """Matrix L[q, j] = l_j(x_q) of the Lagrange basis on nodes xi."""
    xi = np.asarray(xi, dtype=np.float64)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    n = len(xi)
    L = np.ones((len(x), n))
    for j in range(n):
        for k in range(n):
            if k != j:
                L[:, j] *= (x - xi[k]) / (xi[j] - xi[k])
    return L


def mass_matrix(N):
    """Exact mass matrix M_ij = int_{-1}^{1} l_i l_j of the GLL Lagrange basis,
    integrated with N+2 Gauss-Legendre points (exact for degree 2N+3 >= 2N)."""
    xi, _, _ = gll(N)
    xq, wq = np.polynomial.legendre.leggauss(N + 2)
    L = lagrange_eval(xi, xq)
    return L.T @ (wq[:, None] * L)


def mortar_matrices(N):
    """2:1 mortar operators (reading of the Surface Fluxes paragraph).

    Forward (coarse face -> mortar k, k = 0 lower half, 1 upper half):
        Pf[k][i, j] = l_j(s_k(xi_i)),  s_0(r) = (r-1)/2, s_1(r) = (r+1)/2.
    Reverse (mortar k -> coarse face), the L2 projection over half the face:
        Pr[k] = 1/2 M^{-1} Pf[k]^T M, with M the exact mass matrix.
    The factor 1/2 is the half-face Jacobian of the sub-face parametrisation.
    """
    xi, _, _ = gll(N)
    M = mass_matrix(N)
    Minv = np.linalg.inv(M)
    Pf, Pr = [], []
    for k in range(2):
        s = (xi - 1.0) / 2.0 if k == 0 else (xi + 1.0) / 2.0
        P = lagrange_eval(xi, s)
        Pf.append(P)
        Pr.append(0.5 * Minv @ P.T @ M)
    return Pf, Pr
