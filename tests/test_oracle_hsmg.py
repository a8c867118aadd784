"""Pins for the oracle's hybrid Schwarz multigrid and flexible GMRES
(oracle/hsmg.py): interpolation exactness, prolongation of the coordinate
field, restriction as the exact transpose, the separable local solves equal
to the dense inverse of the assembled operator's principal submatrix on
rectilinear meshes, the coarse solve equal to the dense inverse of the
order-1 operator there, flexible GMRES against a dense solve and against the
minimal-residual definition, and the preconditioner's effect."""
import numpy as np
import pytest

import oracle
from oracle import cnn, hsmg
from paper_2405_05640_amd import workloads as wl
from tests import brute


def _mesh(spec):
    return oracle.Mesh(spec.nelx, spec.nely, spec.nelz, spec.order, spec.vertices, spec.periodic,
                       spec.dirichlet)


def _stretched(nelx, nely, nelz, order, periodic=(0, 0, 0), dirichlet=wl.DIRICHLET_ALL, seed=0):
    """Rectilinear tensor-product box with uneven plane spacing per axis."""
    rng = np.random.default_rng(seed)
    planes = []
    for n in (nelx, nely, nelz):
        h = rng.uniform(0.5, 1.5, n)
        planes.append(np.concatenate([[0.0], np.cumsum(h)]) / np.sum(h))
    v = wl.lattice(nelx, nely, nelz, *planes)
    return wl.MeshSpec(nelx, nely, nelz, order, v, tuple(periodic), dirichlet, "stretched")


@pytest.mark.parametrize("nc,nf", [(1, 3), (3, 7), (2, 5), (1, 7)])
def test_interpolation_is_exact_for_coarse_polynomials(nc, nf):
    J = hsmg.interp_matrix(nc, nf)
    xc, _ = oracle.gll(nc)
    xf, _ = oracle.gll(nf)
    for p in range(nc + 1):
        assert np.allclose(J @ xc ** p, xf ** p, rtol=0, atol=1e-13)
    assert not np.allclose(J @ xc ** (nc + 1), xf ** (nc + 1), atol=1e-6)
    # the GLL end points coincide on both grids
    assert np.array_equal(J[0], np.eye(nc + 1)[0]) and np.array_equal(J[-1], np.eye(nc + 1)[-1])


def test_prolongation_reproduces_the_coordinate_field():
    # the element map is trilinear (degree 1 in each reference coordinate),
    # so interpolating the coarse node coordinates gives the fine ones
    fine = _mesh(wl.random_deformed_box(3, 2, 2, 7, seed=3, amp=0.2))
    for nc in (3, 1):
        crs = hsmg.level_mesh(fine, nc)
        J = hsmg.interp_matrix(nc, 7)
        for d in range(3):
            xf = np.einsum("kc,jb,ia,ecba->ekji", J, J, J, crs.xyz[d])
            assert np.allclose(xf, fine.xyz[d], rtol=0, atol=1e-14)


@pytest.mark.parametrize("spec", [wl.random_deformed_box(3, 2, 2, 7, seed=5, amp=0.2),
                                  wl.channel(3, 5)], ids=["jitter", "channel"])
def test_restriction_is_the_transpose_of_prolongation(spec):
    # on assembled vectors (one value per global node): <R r, v> = <r, P v>
    fine = _mesh(spec)
    mid = hsmg.level_mesh(fine, 3)
    J = hsmg.interp_matrix(3, spec.order)
    rng = np.random.default_rng(1)
    for _ in range(3):
        r = brute.continuous_random(fine, rng)
        v = brute.continuous_random(mid, rng)
        lhs = np.dot(mid.gather_global(hsmg.restrict(J, fine, mid, r)), mid.gather_global(v))
        rhs = np.dot(fine.gather_global(r), fine.gather_global(hsmg.prolong(J, mid, fine, v)))
        assert abs(lhs - rhs) <= 1e-13 * (abs(lhs) + np.linalg.norm(r) * np.linalg.norm(v))
    # and the restricted residual is continuous and masked
    rr = hsmg.restrict(J, fine, mid, brute.continuous_random(fine, rng))
    assert np.array_equal(rr, mid.gather_global(rr)[mid.glo])
    assert np.all(rr[mid.mask == 1] == 0)


@pytest.mark.parametrize("periodic,dirichlet,h2", [
    ((0, 0, 0), wl.DIRICHLET_ALL, 0.0),
    ((1, 0, 0), wl.DIRICHLET_Y_WALLS, 0.0),
    ((0, 0, 1), 0x01 | 0x08, 0.3),          # x- and y+ Dirichlet, the rest Neumann, Helmholtz
    ((1, 0, 1), wl.DIRICHLET_Y_WALLS, 2.0),
], ids=["dirichlet", "periodic_x", "mixed_neumann_helm", "channel_like_helm"])
def test_fdm_is_the_inverse_of_the_principal_submatrix(periodic, dirichlet, h2):
    # rectilinear mesh with uneven spacing: the separable local matrix is the
    # restriction of the assembled operator to the element's nodes
    spec = _stretched(3, 2, 3, 3, periodic, dirichlet, seed=2)
    m = _mesh(spec)
    S, free = brute.dense_S(m, 1.0, h2)
    pos = {g: c for c, g in enumerate(free)}
    lev = hsmg.SchwarzLevel(m)
    rng = np.random.default_rng(4)
    for e in range(m.E):
        ids = m.glo[e].ravel()
        keep = np.array([g in pos for g in ids])
        sub = [pos[g] for g in ids[keep]]
        Ae = S[np.ix_(sub, sub)]
        re = rng.standard_normal(m.shape[1:])
        re.ravel()[~keep] = 0.0
        z = hsmg.fdm_solve(lev.factors[e], re, 1.0, h2)
        ref = np.zeros(re.size)
        ref[keep] = np.linalg.solve(Ae, re.ravel()[keep])
        assert np.allclose(z.ravel(), ref, rtol=0, atol=1e-11 * np.max(np.abs(ref)))


def test_fdm_on_deformed_elements_is_an_approximation():
    # off rectilinear meshes the separable solve only approximates the local
    # inverse; it must stay close on mildly deformed elements
    m = _mesh(wl.random_deformed_box(3, 3, 2, 3, seed=8, amp=0.05))
    S, free = brute.dense_S(m)
    pos = {g: c for c, g in enumerate(free)}
    lev = hsmg.SchwarzLevel(m)
    rng = np.random.default_rng(5)
    e = 4
    ids = m.glo[e].ravel()
    keep = np.array([g in pos for g in ids])
    sub = [pos[g] for g in ids[keep]]
    re = rng.standard_normal(m.shape[1:])
    re.ravel()[~keep] = 0.0
    z = hsmg.fdm_solve(lev.factors[e], re, 1.0, 0.0).ravel()[keep]
    ref = np.linalg.solve(S[np.ix_(sub, sub)], re.ravel()[keep])
    err = np.linalg.norm(z - ref) / np.linalg.norm(ref)
    assert 1e-6 < err < 0.3


@pytest.mark.parametrize("periodic,dirichlet,h2", [
    ((0, 0, 0), wl.DIRICHLET_ALL, 0.0),
    ((1, 0, 1), wl.DIRICHLET_Y_WALLS, 0.0),
    ((0, 1, 0), 0x01, 0.5),
], ids=["dirichlet", "channel_like", "neumann_helm"])
def test_coarse_solve_is_the_inverse_of_the_order1_operator(periodic, dirichlet, h2):
    spec = _stretched(4, 3, 3, 1, periodic, dirichlet, seed=6)
    m = _mesh(spec)
    S, free = brute.dense_S(m, 1.0, h2)
    cs = hsmg.CoarseSolver(m)
    rng = np.random.default_rng(7)
    r = brute.continuous_random(m, rng)
    z = cs.solve(r, 1.0, h2)
    ref = np.linalg.solve(S, m.gather_global(r)[free])
    assert np.allclose(m.gather_global(z)[free], ref, rtol=0, atol=1e-12 * np.max(np.abs(ref)))
    assert np.all(z[m.mask == 1] == 0)


def test_fgmres_identity_preconditioner_matches_dense_solve():
    m = _mesh(wl.random_deformed_box(2, 2, 2, 3, seed=9, amp=0.15))
    S, free = brute.dense_S(m, 1.0, 0.2)
    rng = np.random.default_rng(10)
    b = m.rhs(rng.standard_normal(m.shape))
    x, info = hsmg.fgmres(m, b, lambda r: r, 1.0, 0.2, tol=1e-12, restart=20)
    ref = np.linalg.solve(S, m.gather_global(b)[free])
    assert np.allclose(m.gather_global(x)[free], ref, rtol=0, atol=1e-9 * np.max(np.abs(ref)))
    assert info["true_rel_res"] <= 1e-12
    assert info["restarts"] >= 1
    h = np.array(info["history"])
    assert np.all(np.diff(h[:21]) <= 1e-15)          # non-increasing within a cycle


def test_fgmres_is_the_minimal_residual_over_its_search_space():
    # for a fixed linear preconditioner M, k steps of FGMRES from x = 0 give
    # the minimum of |b - S x| over x in span{M r0, M S M r0, ...} (k terms):
    # the explicit Krylov basis and a least-squares solve reproduce the
    # residual history
    m = _mesh(wl.channel(2, 4))
    pc = hsmg.HSMG(m, n_mid=2)
    rng = np.random.default_rng(11)
    b = m.rhs(rng.standard_normal(m.shape))
    _, info = hsmg.fgmres(m, b, lambda r: pc.apply(r), tol=1e-14, restart=12, max_iter=6)
    gb = lambda u: m.gather_global(u)
    free = np.nonzero(np.bincount(m.glo.ravel(), weights=(m.mask.ravel() == 0), minlength=m.n_global) > 0)[0]
    basis, v = [], b.copy()
    for k in range(1, 7):
        z = pc.apply(v)
        basis.append(z)
        v = m.apply_S(z)
        AZ = np.stack([gb(m.apply_S(q))[free] for q in basis], axis=1)
        y, *_ = np.linalg.lstsq(AZ, gb(b)[free], rcond=None)
        res = np.linalg.norm(gb(b)[free] - AZ @ y) / np.linalg.norm(gb(b)[free])
        assert abs(res - info["history"][k]) <= 1e-8 * info["history"][k] + 1e-14


def test_hsmg_composition_and_gain():
    # the preconditioner is the additive combination of its pinned parts, is
    # linear, keeps Dirichlet nodes at zero, and cuts the Krylov iterations
    # far below Jacobi-PCG's
    spec = wl.channel(4, 5)
    m = _mesh(spec)
    pc = hsmg.HSMG(m, n_mid=3)
    rng = np.random.default_rng(12)
    r = brute.continuous_random(m, rng)
    r2 = brute.continuous_random(m, rng)
    z = pc.apply(r)
    r1 = hsmg.restrict(pc.J_fm, m, pc.mid, r)
    zc = pc.coarse.solve(hsmg.restrict(pc.J_mc, pc.mid, pc.crs, r1), 1.0, 0.0)
    zm = pc.sw_m.smooth(r1, 1.0, 0.0) + hsmg.prolong(pc.J_mc, pc.crs, pc.mid, zc)
    ref = pc.sw_f.smooth(r, 1.0, 0.0) + hsmg.prolong(pc.J_fm, pc.mid, m, zm)
    assert np.allclose(z, ref, rtol=0, atol=1e-13 * np.max(np.abs(ref)))
    assert np.allclose(pc.apply(2.0 * r - 3.0 * r2), 2.0 * z - 3.0 * pc.apply(r2), rtol=0,
                       atol=1e-12 * np.max(np.abs(z)))
    assert np.all(z[m.mask == 1] == 0)
    b = m.rhs(rng.standard_normal(m.shape))
    _, pinfo = m.pcg(b, tol=1e-10)
    x, ginfo = hsmg.fgmres(m, b, lambda q: pc.apply(q), tol=1e-10, restart=30)
    res = b - m.apply_S(x)
    assert np.sqrt(m.dot(res, res) / m.dot(b, b)) <= 1.05e-10
    print("channel 4^3 N=5: Jacobi-PCG %d iterations, HSMG-FGMRES %d" % (pinfo["iterations"], ginfo["iterations"]))
    assert ginfo["iterations"] * 4 < pinfo["iterations"]


def test_block_jacobi_is_symmetric_positive_definite():
    # the velocity preconditioner (unweighted sum of local solves) as a dense
    # matrix on the free global nodes
    m = _mesh(wl.random_deformed_box(2, 2, 2, 3, seed=13, amp=0.1))
    lev = hsmg.SchwarzLevel(m)
    _, free = brute.dense_S(m)
    glo = m.glo.ravel()
    M = np.zeros((len(free), len(free)))
    for c, g in enumerate(free):
        u = (glo == g).astype(np.float64).reshape(m.shape)
        M[:, c] = m.gather_global(hsmg.block_jacobi(lev, u, 1.0, 0.5))[free]
    assert np.allclose(M, M.T, rtol=0, atol=1e-13 * np.max(np.abs(M)))
    assert np.min(np.linalg.eigvalsh(0.5 * (M + M.T))) > 0


def test_block_jacobi_pcg_solves_and_beats_point_jacobi():
    # CG with the block-Jacobi preconditioner reaches the tolerance on a
    # velocity-like Helmholtz problem, in fewer iterations than Jacobi-PCG
    m = _mesh(wl.random_deformed_box(3, 3, 2, 5, seed=14, amp=0.1))
    h1, h2 = 1.0, 50.0
    lev = hsmg.SchwarzLevel(m)
    rng = np.random.default_rng(15)
    b = m.rhs(rng.standard_normal(m.shape))
    x, info = hsmg.pcg(m, b, lambda r: hsmg.block_jacobi(lev, r, h1, h2), h1, h2, tol=1e-10)
    assert info["true_rel_res"] <= 1.05e-10
    _, pinfo = m.pcg(b, h1, h2, tol=1e-10)
    print("block-Jacobi PCG %d iterations, Jacobi-PCG %d" % (info["iterations"], pinfo["iterations"]))
    assert info["iterations"] < pinfo["iterations"]
    # with the identity preconditioner the routine is plain CG: it matches a
    # dense solve
    S, free = brute.dense_S(m, h1, h2)
    x0, _ = hsmg.pcg(m, b, lambda r: r, h1, h2, tol=1e-13)
    ref = np.linalg.solve(S, m.gather_global(b)[free])
    assert np.allclose(m.gather_global(x0)[free], ref, rtol=0, atol=1e-9 * np.max(np.abs(ref)))


def test_symmetric_hsmg_is_spd_and_serves_cg():
    # the symmetric weighting makes the three-level preconditioner symmetric
    # positive definite (dense matrix on the free global nodes); CG with it
    # reaches the tolerance in about as many iterations as flexible GMRES
    # with the averaged weighting
    m = _mesh(wl.random_deformed_box(2, 2, 2, 4, seed=16, amp=0.1))
    pc = hsmg.HSMG(m)
    _, free = brute.dense_S(m)
    glo = m.glo.ravel()
    M = np.zeros((len(free), len(free)))
    for c, g in enumerate(free):
        u = (glo == g).astype(np.float64).reshape(m.shape)
        M[:, c] = m.gather_global(pc.apply(u, sym=True))[free]
    assert np.allclose(M, M.T, rtol=0, atol=1e-13 * np.max(np.abs(M)))
    assert np.min(np.linalg.eigvalsh(0.5 * (M + M.T))) > 0
    m2 = _mesh(wl.channel(4, 5))
    pc2 = hsmg.HSMG(m2)
    rng = np.random.default_rng(17)
    b = m2.rhs(rng.standard_normal(m2.shape))
    _, ci = hsmg.pcg(m2, b, lambda r: pc2.apply(r, sym=True), tol=1e-10)
    _, gi = hsmg.fgmres(m2, b, lambda r: pc2.apply(r), tol=1e-10)
    print("channel 4^3 N=5: CG + symmetric HSMG %d iterations, FGMRES + averaged HSMG %d" %
          (ci["iterations"], gi["iterations"]))
    assert ci["true_rel_res"] <= 1.05e-10
    assert ci["iterations"] <= gi["iterations"] + 5


def test_learned_multigrid_composition():
    # the learned multigrid keeps the middle and coarse levels and puts the
    # learned smoother in place of the fine Schwarz level.  With a zero
    # network the fine level is Jacobi, and with the symmetric middle level
    # the whole preconditioner is then symmetric positive definite (a
    # transposed restriction or prolongation would break the symmetry)
    m = _mesh(wl.random_deformed_box(2, 2, 2, 4, seed=18, amp=0.1))
    pc = hsmg.HSMG(m)
    dinv = m.jacobi_inv()
    zero = cnn.Net.init(4, seed=0)
    _, free = brute.dense_S(m)
    glo = m.glo.ravel()
    M = np.zeros((len(free), len(free)))
    for c, g in enumerate(free):
        u = (glo == g).astype(np.float64).reshape(m.shape)
        M[:, c] = m.gather_global(pc.apply(u, sym=True, fine=lambda q: cnn.smoother(m, zero, q, dinv)))[free]
    assert np.allclose(M, M.T, rtol=0, atol=1e-13 * np.max(np.abs(M)))
    assert np.min(np.linalg.eigvalsh(0.5 * (M + M.T))) > 0
    # the coarser levels' part is what the full cycle adds to its fine level
    rng = np.random.default_rng(19)
    r = brute.continuous_random(m, rng)
    assert np.allclose(pc.apply(r) - pc.sw_f.smooth(r, 1.0, 0.0), pc.coarse_part(r), rtol=0, atol=1e-13)


def test_learned_multigrid_fgmres_converges():
    # flexible GMRES with the learned multigrid (a random network: a
    # nonlinear, non-symmetric preconditioner) reaches 1e-10, in far fewer
    # iterations than Jacobi-PCG
    m = _mesh(wl.random_deformed_box(3, 3, 2, 5, seed=20, amp=0.1, periodic=(1, 0, 0), dirichlet=0x3c))
    pc = hsmg.HSMG(m)
    dinv = m.jacobi_inv()
    net = cnn.Net.init(4, seed=3)
    net.W[2] = np.random.default_rng(21).standard_normal(net.W[2].shape) * 0.05
    rng = np.random.default_rng(22)
    b = m.rhs(rng.standard_normal(m.shape))
    x, info = hsmg.fgmres(m, b, lambda q: pc.apply(q, fine=lambda t: cnn.smoother(m, net, t, dinv)), tol=1e-10)
    _, pinfo = m.pcg(b, tol=1e-10)
    res = b - m.apply_S(x)
    print("learned multigrid FGMRES %d iterations, Jacobi-PCG %d" % (info["iterations"], pinfo["iterations"]))
    assert np.sqrt(m.dot(res, res) / m.dot(b, b)) <= 1.05e-10
    assert info["iterations"] < 0.6 * pinfo["iterations"]


def test_learned_multigrid_fcg_with_a_linear_spd_cycle_is_pcg():
    # flexible CG with the learned multigrid: with a zero network and the
    # symmetric middle level the preconditioner is linear and SPD, and the
    # Polak-Ribiere coefficient then equals the Fletcher-Reeves one, so the
    # iterates are those of PCG with the same preconditioner
    m = _mesh(wl.random_deformed_box(3, 2, 2, 4, seed=23, amp=0.1))
    pc = hsmg.HSMG(m)
    dinv = m.jacobi_inv()
    zero = cnn.Net.init(4, seed=0)
    rng = np.random.default_rng(24)
    b = m.rhs(rng.standard_normal(m.shape))
    x, info = cnn.fcg(m, zero, b, coarse=lambda q: pc.coarse_part(q, sym=True))
    xp, pinfo = hsmg.pcg(m, b, lambda q: dinv * q + pc.coarse_part(q, sym=True), tol=1e-10)
    print("FCG %d iterations, PCG %d" % (info["iterations"], pinfo["iterations"]))
    assert info["fallback_at"] == -1
    assert abs(info["iterations"] - pinfo["iterations"]) <= 1
    assert np.max(np.abs(x - xp)) <= 1e-8 * np.max(np.abs(xp))
