"""Pins for the oracle's geometry and gather-scatter numbering."""
import itertools

import numpy as np
import pytest

import oracle
from paper_2405_05640_amd import workloads as wl
from tests import brute


def _mesh(spec):
    return oracle.Mesh(spec.nelx, spec.nely, spec.nelz, spec.order, spec.vertices,
                       spec.periodic, spec.dirichlet)


def test_undeformed_box_closed_forms():
    spec = wl.box(3, 2, 4, 5, extent=(0.6, 1.0, 2.0))
    m = _mesh(spec)
    hx, hy, hz = 0.2, 0.5, 0.5
    W = np.einsum("k,j,i->kji", m.w, m.w, m.w)
    assert np.allclose(m.G[0], W * hy * hz / (2 * hx), rtol=1e-13, atol=0)
    assert np.allclose(m.G[3], W * hx * hz / (2 * hy), rtol=1e-13, atol=0)
    assert np.allclose(m.G[5], W * hx * hy / (2 * hz), rtol=1e-13, atol=0)
    for q in (1, 2, 4):
        assert np.max(np.abs(m.G[q])) < 1e-15
    assert np.allclose(m.B, W * hx * hy * hz / 8, rtol=1e-13, atol=0)
    assert abs(m.B.sum() - 0.6 * 1.0 * 2.0) < 1e-13


@pytest.mark.parametrize("seed", [0, 1])
def test_deformed_geometry_matches_trilinear_map(seed):
    spec = wl.random_deformed_box(3, 2, 2, 4, seed=seed, amp=0.2)
    m = _mesh(spec)
    n = m.N + 1
    for e in range(m.E):
        X = brute.element_corners(spec.vertices, spec.nelx, spec.nely, e)
        for k, j, i in itertools.product(range(n), repeat=3):
            x, J = brute.trilinear(X, m.xi[i], m.xi[j], m.xi[k])
            assert np.allclose(m.xyz[:, e, k, j, i], x, atol=1e-14)
            det = np.linalg.det(J)
            assert abs(m.jac[e, k, j, i] - det) < 1e-13 * abs(det)
            Ji = np.linalg.inv(J)
            Gref = m.w[i] * m.w[j] * m.w[k] * det * (Ji @ Ji.T)
            got = np.array([[m.G[0, e, k, j, i], m.G[1, e, k, j, i], m.G[2, e, k, j, i]],
                            [m.G[1, e, k, j, i], m.G[3, e, k, j, i], m.G[4, e, k, j, i]],
                            [m.G[2, e, k, j, i], m.G[4, e, k, j, i], m.G[5, e, k, j, i]]])
            assert np.allclose(got, Gref, rtol=1e-12, atol=1e-13 * np.abs(Gref).max())


def test_inverted_element_rejected():
    spec = wl.box(2, 2, 2, 3)
    v = spec.vertices.copy()
    v[1, 1, 1, 0] = 1.3   # push the centre vertex past its neighbours
    with pytest.raises(ValueError):
        oracle.Mesh(2, 2, 2, 3, v, (0, 0, 0), 0x3F)


@pytest.mark.parametrize("per", [(0, 0, 0), (1, 0, 1), (1, 1, 1), (0, 1, 0)])
@pytest.mark.parametrize("N", [1, 3, 7])
def test_numbering_matches_closed_form(per, N):
    spec = wl.random_deformed_box(3, 2, 4, N, seed=5, amp=0.1, periodic=per)
    m = _mesh(spec)
    glo, ng = brute.closed_form_glo(3, 2, 4, N, per)
    assert m.n_global == ng
    assert np.array_equal(m.glo, glo)
    counts = np.bincount(m.glo.ravel(), minlength=ng)
    assert np.array_equal(m.mult, counts[m.glo])


@pytest.mark.parametrize("dims", [(2, 3, 4), (4, 4, 4), (5, 1, 3)])
@pytest.mark.parametrize("N", [3, 7])
def test_fully_periodic_count_is_E_N3(dims, N):
    # Table 1: n = E N^3 unique points
    m = _mesh(wl.box(*dims, N, periodic=(1, 1, 1), dirichlet=0))
    assert m.n_global == int(np.prod(dims)) * N ** 3
    assert np.all(m.mask == 0)


def test_mult_histogram_and_dirichlet_count():
    nel, N = 4, 5
    m = _mesh(wl.cube(nel, N))
    n = nel * N + 1
    assert m.n_global == n ** 3
    # global nodes by multiplicity: element vertices shared by 8 etc.
    g_mult = np.zeros(m.n_global, dtype=np.int64)
    g_mult[m.glo.ravel()] = m.mult.ravel()
    hist = np.bincount(g_mult, minlength=9)
    assert hist[8] == (nel - 1) ** 3
    # Dirichlet nodes on all six faces
    gm = np.zeros(m.n_global, dtype=bool)
    gm[m.glo.ravel()[m.mask.ravel() == 1]] = True
    assert gm.sum() == n ** 3 - (n - 2) ** 3
    # shared local fraction 1 - ((N-1)/(N+1))^3 for an all-shared interior element
    interior = (m.mult > 1).reshape(m.E, -1)
    e_center = 1 + nel * (1 + nel * 1)
    assert interior[e_center].mean() == pytest.approx(1 - ((N - 1) / (N + 1)) ** 3)
