"""Pins for the oracle's local operator, dssum, mask, Jacobi diagonal, dot."""
import itertools

import numpy as np
import pytest

import oracle
from paper_2405_05640_amd import workloads as wl
from tests import brute


def _mesh(spec):
    return oracle.Mesh(spec.nelx, spec.nely, spec.nelz, spec.order, spec.vertices,
                       spec.periodic, spec.dirichlet)


def _int_mono(p, lo, hi):
    return (hi ** (p + 1) - lo ** (p + 1)) / (p + 1)


def _mono(m, pw):
    x, y, z = m.xyz
    return x ** pw[0] * y ** pw[1] * z ** pw[2]


def _grad_integral(pu, pv, ext):
    """int over box of grad(x^pu) . grad(x^pv), pu/pv exponent triples."""
    total = 0.0
    for d in range(3):
        if pu[d] == 0 or pv[d] == 0:
            continue
        term = pu[d] * pv[d]
        for c in range(3):
            e = pu[c] + pv[c] - (2 if c == d else 0)
            term *= _int_mono(e, 0.0, ext[c])
        total += term
    return total


@pytest.mark.parametrize("N", [2, 3, 5])
def test_stiffness_quadrature_exactness_on_affine_mesh(N):
    ext = (0.6, 1.0, 1.4)
    m = _mesh(wl.box(2, 3, 2, N, extent=ext))
    rng = np.random.default_rng(N)
    checked = 0
    for _ in range(40):
        pu = rng.integers(0, N + 1, size=3)
        pv = rng.integers(0, N + 1, size=3)
        if np.any(pu + pv > 2 * N - 1):
            continue  # require deg_d(u) + deg_d(v) <= 2N-1 in every direction
        u, v = _mono(m, pu), _mono(m, pv)
        got = float(np.sum(u * m.ax(v, 1.0, 0.0)))
        ref = _grad_integral(pu, pv, ext)
        assert abs(got - ref) <= 1e-12 * max(1.0, abs(ref)), (pu, pv)
        checked += 1
    assert checked > 10


@pytest.mark.parametrize("N", [3, 5])
def test_mass_quadrature_exactness_and_failure(N):
    ext = (0.6, 1.0, 1.4)
    m = _mesh(wl.box(2, 3, 2, N, extent=ext))
    for pw in [(2 * N - 1, 0, 0), (1, 2 * N - 1, 3), (N, N - 1, 2 * N - 1)]:
        ref = np.prod([_int_mono(p, 0, e) for p, e in zip(pw, ext)])
        assert abs(np.sum(m.B * _mono(m, pw)) - ref) < 1e-13 * max(1, abs(ref))
    pw = (2 * N, 0, 0)
    ref = np.prod([_int_mono(p, 0, e) for p, e in zip(pw, ext)])
    assert abs(np.sum(m.B * _mono(m, pw)) - ref) > 1e-10 * abs(ref)


@pytest.mark.parametrize("N", [2, 4])
def test_element_matrix_kronecker_closed_form(N):
    hx, hy, hz = 0.5, 0.25, 0.75
    m = _mesh(wl.box(1, 1, 1, N, extent=(hx, hy, hz)))
    n = N + 1
    A = np.zeros((n ** 3, n ** 3))
    for c in range(n ** 3):
        e = np.zeros(n ** 3)
        e[c] = 1.0
        A[:, c] = m.ax(e, 1.0, 0.0).ravel()
    W = np.diag(m.w)
    K1 = m.D.T @ W @ m.D
    ref = (hy * hz / (2 * hx)) * np.kron(W, np.kron(W, K1)) \
        + (hx * hz / (2 * hy)) * np.kron(W, np.kron(K1, W)) \
        + (hx * hy / (2 * hz)) * np.kron(K1, np.kron(W, W))
    assert np.max(np.abs(A - ref)) < 1e-12 * np.max(np.abs(ref))
    # Helmholtz part: h2 B on the diagonal
    A2 = np.zeros_like(A)
    for c in range(n ** 3):
        e = np.zeros(n ** 3)
        e[c] = 1.0
        A2[:, c] = m.ax(e, 0.0, 1.0).ravel()
    assert np.allclose(A2, np.diag(m.B.ravel()), rtol=1e-15, atol=0)


@pytest.mark.parametrize("seed", [0, 3])
def test_constants_in_null_space_on_deformed_mesh(seed):
    m = _mesh(wl.random_deformed_box(3, 3, 2, 5, seed=seed, amp=0.25))
    w = m.ax(np.ones(m.shape), 1.0, 0.0)
    scale = np.max(np.abs(m.G))
    assert np.max(np.abs(w)) < 1e-12 * scale * (m.N + 1) ** 2


def test_coordinate_fields_give_volume_on_deformed_mesh():
    # for isoparametric trilinear elements, x_c is in the discrete space and
    # grad x_c . grad x_d = delta_cd, so x_c^T A_L x_d = delta_cd * sum(B)
    m = _mesh(wl.deformed_cube(3, 5, amp=0.2))
    vol = m.B.sum()
    for c in range(3):
        for d in range(3):
            got = float(np.sum(m.xyz[c] * m.ax(m.xyz[d], 1.0, 0.0)))
            assert abs(got - (vol if c == d else 0.0)) < 1e-12 * vol


@pytest.mark.parametrize("h2", [0.0, 0.1])
def test_assembled_operator_symmetric(h2):
    m = _mesh(wl.random_deformed_box(3, 2, 3, 4, seed=7, amp=0.2))
    rng = np.random.default_rng(1)
    u, v = brute.continuous_random(m, rng), brute.continuous_random(m, rng)
    a = m.dot(u, m.apply_S(v, 1.0, h2))
    b = m.dot(v, m.apply_S(u, 1.0, h2))
    assert abs(a - b) < 1e-13 * abs(a)
    # positive definite on masked continuous vectors
    assert m.dot(u, m.apply_S(u, 1.0, h2)) > 0


def test_dssum_properties():
    m = _mesh(wl.random_deformed_box(3, 2, 2, 3, seed=2, periodic=(1, 0, 0)))
    assert np.array_equal(m.dssum(np.ones(m.shape)), m.mult.astype(np.float64))
    rng = np.random.default_rng(0)
    u = brute.continuous_random(m, rng, masked=False)
    assert np.allclose(m.dssum(u), m.mult * u, rtol=1e-15, atol=0)
    # sum of copies equals the gathered sum
    v = rng.standard_normal(m.shape)
    s = np.zeros(m.n_global)
    np.add.at(s, m.glo.ravel(), v.ravel())
    assert np.allclose(m.dssum(v).ravel(), s[m.glo.ravel()], rtol=1e-14, atol=1e-15)


def test_dot_equals_global_euclidean():
    m = _mesh(wl.random_deformed_box(2, 3, 2, 4, seed=4))
    rng = np.random.default_rng(5)
    u, v = brute.continuous_random(m, rng), brute.continuous_random(m, rng)
    assert abs(m.dot(u, v) - m.gather_global(u) @ m.gather_global(v)) < 1e-13 * abs(m.dot(u, u))


@pytest.mark.parametrize("h2", [0.0, 0.3])
def test_jacobi_diagonal_matches_dense(h2):
    m = _mesh(wl.random_deformed_box(2, 2, 2, 3, seed=8, amp=0.2))
    S, free = brute.dense_S(m, 1.0, h2)
    dinv = m.jacobi_inv(1.0, h2)
    d = m.gather_global(1.0 / dinv)[free]
    assert np.allclose(d, np.diag(S), rtol=1e-13, atol=0)
    assert np.allclose(S, S.T, rtol=0, atol=1e-13 * np.abs(S).max())
    assert np.min(np.linalg.eigvalsh(S)) > 0
    # masked nodes carry d = 1
    assert np.all(dinv[m.mask == 1] == 1.0)


def test_neumann_null_space_is_constants():
    m = _mesh(wl.random_deformed_box(2, 2, 2, 2, seed=9, amp=0.2, dirichlet=0))
    S, free = brute.dense_S(m, 1.0, 0.0)
    ev = np.linalg.eigvalsh(S)
    assert abs(ev[0]) < 1e-12 * ev[-1] and ev[1] > 1e-6 * ev[-1]
