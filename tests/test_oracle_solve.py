"""Pins for the oracle's Jacobi-PCG: dense direct solve on tiny meshes,
manufactured-solution spectral convergence, termination and status codes."""
import numpy as np
import pytest

import oracle
from paper_2405_05640_amd import workloads as wl
from tests import brute


def _mesh(spec):
    return oracle.Mesh(spec.nelx, spec.nely, spec.nelz, spec.order, spec.vertices,
                       spec.periodic, spec.dirichlet)


@pytest.mark.parametrize("h2", [0.0, 0.1])
@pytest.mark.parametrize("per", [(0, 0, 0), (1, 0, 1)])
def test_pcg_matches_dense_direct_solve(h2, per):
    spec = wl.random_deformed_box(2, 2, 2, 3, seed=11, amp=0.2, periodic=per,
                                  dirichlet=wl.DIRICHLET_ALL if per == (0, 0, 0) else wl.DIRICHLET_Y_WALLS)
    m = _mesh(spec)
    rng = np.random.default_rng(3)
    f = rng.standard_normal(m.shape)
    b = m.rhs(f)
    S, free = brute.dense_S(m, 1.0, h2)
    xg = np.linalg.solve(S, m.gather_global(b)[free])
    x, info = m.pcg(b, 1.0, h2, tol=1e-13)
    assert info["status"] == 0
    assert info["true_rel_res"] <= 1e-13
    got = m.gather_global(x)[free]
    assert np.max(np.abs(got - xg)) < 1e-9 * np.max(np.abs(xg))
    # continuity and mask of the iterate
    assert np.allclose(x, x.ravel()[0] * 0 + m.gather_global(x)[m.glo], rtol=0, atol=0)
    assert np.all(x[m.mask == 1] == 0)
    # exact-arithmetic bound: at most n_unknowns iterations
    assert info["iterations"] <= len(free)


def test_manufactured_c0():
    spec = wl.config("c0")
    m = _mesh(spec)
    uex, f = wl.manufactured(*m.xyz)
    b = m.rhs(f)
    x, info = m.pcg(b, 1.0, 0.0, tol=1e-10)
    assert info["status"] == 0 and info["true_rel_res"] <= 1e-10
    err = np.max(np.abs(x - uex))
    assert err < 1e-7      # N=5, 4^3 elements (measured 7.8e-9)
    assert 20 < info["iterations"] < 200


def test_spectral_convergence_in_N():
    errs = []
    for N in range(2, 10):
        m = _mesh(wl.cube(2, N))
        uex, f = wl.manufactured(*m.xyz)
        x, info = m.pcg(m.rhs(f), 1.0, 0.0, tol=1e-13)
        errs.append(np.max(np.abs(x - uex)))
    errs = np.array(errs)
    # geometric decay: every two orders gain at least a factor 10
    assert np.all(errs[2:] < errs[:-2] / 10), errs
    assert errs[-1] < 1e-7


def test_residual_history_monotone_energy_and_statuses():
    m = _mesh(wl.deformed_cube(3, 4, amp=0.2))
    rng = np.random.default_rng(0)
    b = m.rhs(rng.standard_normal(m.shape))
    x, info = m.pcg(b, 1.0, 0.1, tol=1e-10, history=True)
    assert info["status"] == 0
    h = info["history"]
    assert h[0] == 1.0 and h[-1] <= 1e-10 and len(h) == info["iterations"] + 1
    # not converged within max_iter
    x2, info2 = m.pcg(b, 1.0, 0.1, tol=1e-10, max_iter=5)
    assert info2["status"] == 1 and info2["iterations"] == 5
    # zero right-hand side: zero solution, no iterations
    x3, info3 = m.pcg(np.zeros(m.shape), 1.0, 0.1)
    assert info3["status"] == 0 and info3["iterations"] == 0 and np.all(x3 == 0)
