"""A second, scalar-loop evaluation of the Euler DGSEM right-hand side on
uniform periodic Cartesian meshes, written separately from the oracle: its own
GLL construction (numpy's Legendre roots, barycentric derivative matrix), its
own element/node indexing, one node at a time.  It follows the same equations
(eq. vol_weak, the Rusanov flux with the unnormalised normal, eq. surf_int) so
that agreement with the vectorised oracle pins the oracle's indexing, signs
and scalings against an independent transcription.
"""

import math

import numpy as np


def gll_barycentric(N):
    c = np.zeros(N + 1)
    c[N] = 1.0
    inner = np.polynomial.legendre.Legendre(c).deriv().roots() if N >= 2 else np.zeros(0)
    x = np.concatenate([[-1.0], np.sort(np.real(inner)), [1.0]])
    PN = np.polynomial.legendre.legval(x, c)
    w = 2.0 / (N * (N + 1) * PN ** 2)
    n = N + 1
    lam = np.array([1.0 / np.prod([x[j] - x[k] for k in range(n) if k != j]) for j in range(n)])
    D = np.zeros((n, n))
    for i in range(n):
        for j in range(n):
            if i != j:
                D[i, j] = (lam[j] / lam[i]) / (x[i] - x[j])
        D[i, i] = -sum(D[i, j] for j in range(n) if j != i)
    return x, w, D


def _flux(u, l, dim, gamma):
    rho = u[0]
    vel = [u[1 + d] / rho for d in range(dim)]
    p = (gamma - 1.0) * (u[dim + 1] - 0.5 * rho * sum(v * v for v in vel))
    f = [u[1 + l]]
    for d in range(dim):
        f.append(u[1 + d] * vel[l] + (p if d == l else 0.0))
    f.append((u[dim + 1] + p) * vel[l])
    c = abs(vel[l]) + math.sqrt(gamma * p / rho)
    return np.array(f), c


def _rusanov(uL, uR, l, dim, gamma, nmag):
    fL, cL = _flux(uL, l, dim, gamma)
    fR, cR = _flux(uR, l, dim, gamma)
    lam = max(cL, cR)
    return 0.5 * nmag * (fL + fR) - 0.5 * nmag * lam * (uR - uL)


def rhs(U, dim, N, nel, lo, hi, gamma=1.4):
    """U: (nv, E, n^dim) in element order x-fastest, node order i-fastest."""
    x, w, D = gll_barycentric(N)
    n = N + 1
    nv = dim + 2
    h = [(hi[d] - lo[d]) / nel[d] for d in range(dim)]
    J = np.prod([hd / 2.0 for hd in h])
    Ja = [2.0 * J / h[d] for d in range(dim)]
    E = int(np.prod(nel))
    out = np.zeros_like(U)

    def eidx(c):
        e = 0
        for d in reversed(range(dim)):
            e = e * nel[d] + (c[d] % nel[d])
        return e

    def ecoord(e):
        c = []
        for d in range(dim):
            c.append(e % nel[d])
            e //= nel[d]
        return c

    def nidx(a):
        k = 0
        for d in reversed(range(dim)):
            k = k * n + a[d]
        return k

    def ncoord(k):
        a = []
        for d in range(dim):
            a.append(k % n)
            k //= n
        return a

    for e in range(E):
        ce = ecoord(e)
        for q in range(n ** dim):
            a = ncoord(q)
            acc = np.zeros(nv)
            for l in range(dim):
                for m in range(n):
                    b = list(a)
                    b[l] = m
                    f, _ = _flux(U[:, e, nidx(b)], l, dim, gamma)
                    acc -= D[a[l], m] * Ja[l] * f / J
                fown, _ = _flux(U[:, e, q], l, dim, gamma)
                if a[l] == N:
                    cn = list(ce)
                    cn[l] += 1
                    b = list(a)
                    b[l] = 0
                    fs = _rusanov(U[:, e, q], U[:, eidx(cn), nidx(b)], l, dim, gamma, Ja[l])
                    acc -= (fs - Ja[l] * fown) / (J * w[N])
                if a[l] == 0:
                    cn = list(ce)
                    cn[l] -= 1
                    b = list(a)
                    b[l] = N
                    fs = _rusanov(U[:, eidx(cn), nidx(b)], U[:, e, q], l, dim, gamma, Ja[l])
                    acc += (fs - Ja[l] * fown) / (J * w[0])
            out[:, e, q] = acc
    return out
