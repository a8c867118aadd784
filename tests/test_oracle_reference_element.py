"""Pins for the oracle's reference element (GLL nodes, weights, D matrix).

Independent anchors: tabulated GLL values (tests/golden/gll_tables.txt),
polynomial exactness of the quadrature, and a derivative matrix rebuilt from
the Lagrange polynomials with numpy's polynomial module.
"""
import os

import numpy as np
import pytest

import oracle

HERE = os.path.dirname(__file__)


def _table():
    rows = {}
    for line in open(os.path.join(HERE, "golden", "gll_tables.txt")):
        if line.startswith("#") or not line.strip():
            continue
        N, x, w = line.split()
        rows.setdefault(int(N), []).append((float(x), float(w)))
    return rows


@pytest.mark.parametrize("N", [5, 7])
def test_gll_matches_table(N):
    xi, w = oracle.gll(N)
    tab = sorted(_table()[N])
    pos = sorted([(x, ww) for x, ww in zip(xi, w) if x >= 0])
    for (x0, w0), (x1, w1) in zip(tab, pos):
        assert abs(x0 - x1) < 1e-11
        assert abs(w0 - w1) < 1e-11
    assert np.allclose(xi, -xi[::-1], atol=0, rtol=0)


@pytest.mark.parametrize("N", range(1, 16))
def test_gll_quadrature_exactness(N):
    xi, w = oracle.gll(N)
    assert np.all(np.diff(xi) > 0) and xi[0] == -1.0 and xi[-1] == 1.0
    for k in range(0, 2 * N):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(np.dot(w, xi ** k) - exact) < 1e-13 * max(1, 2 ** k / 1e3)
    # degree 2N is NOT integrated exactly (Lobatto, not Gauss)
    k = 2 * N
    assert abs(np.dot(w, xi ** k) - 2.0 / (k + 1)) > 1e-10


@pytest.mark.parametrize("N", [2, 3, 5, 7, 9])
def test_deriv_against_lagrange_polynomials(N):
    xi, _ = oracle.gll(N)
    D = oracle.deriv(N)
    P = np.polynomial.polynomial
    # Lagrange basis l_j from the Vandermonde inverse, then differentiated
    V = np.vander(xi, N + 1, increasing=True)
    C = np.linalg.inv(V)   # column j = coefficients of l_j
    Dref = np.zeros((N + 1, N + 1))
    for j in range(N + 1):
        dc = P.polyder(C[:, j])
        Dref[:, j] = P.polyval(xi, dc)
    assert np.max(np.abs(D - Dref)) < 1e-9 * N ** 2


@pytest.mark.parametrize("N", [5, 7])
def test_deriv_identities(N):
    xi, w = oracle.gll(N)
    D = oracle.deriv(N)
    assert np.max(np.abs(D @ np.ones(N + 1))) < 1e-12
    for k in range(1, N + 1):
        assert np.max(np.abs(D @ xi ** k - k * xi ** (k - 1))) < 1e-11
    # summation by parts: W D + D^T W = diag(-1, 0, ..., 0, 1)
    W = np.diag(w)
    Q = W @ D + D.T @ W
    E = np.zeros_like(Q)
    E[0, 0], E[-1, -1] = -1.0, 1.0
    assert np.max(np.abs(Q - E)) < 1e-13
    assert D[0, 0] == -N * (N + 1) / 4 and D[N, N] == N * (N + 1) / 4


def test_table1_unique_count_formula():
    for line in open(os.path.join(HERE, "golden", "table1_unique_points.txt")):
        if line.startswith("#") or not line.strip():
            continue
        _, N, E, n = line.split()
        assert int(E) * int(N) ** 3 == int(n)
