"""GPU parity of the paper's pressure solver (restarted flexible GMRES with
the hybrid Schwarz multigrid preconditioner) and the velocity solves'
block-Jacobi CG against the FP64 oracle (oracle/hsmg.py): the preconditioner
and its fine level, output by output, on meshes with Dirichlet walls,
periodic wraps, Neumann faces, deformed and stretched elements and orders
N = 3, 5, 7; solves to the oracle-evaluated FP64 true residual 1e-10 with
iteration counts next to the oracle's; argument checks."""
import numpy as np
import pytest

from oracle import hsmg
from paper_2405_05640_amd import sem
from paper_2405_05640_amd import workloads as wl
from tests import brute
from tests.gpu_util import dev, host, pair

pytestmark = pytest.mark.gpu

MESHES = {
    "channel3_N7": (wl.channel(3, 7), 1.0, 0.0),
    "jitter_3x2x3_N7_helm": (wl.random_deformed_box(3, 2, 3, 7, seed=3, amp=0.15), 1.0, 0.1),
    "deformed4_N5": (wl.deformed_cube(4, 5), 1.0, 0.0),
    "mixed_bc_N5": (wl.random_deformed_box(3, 3, 2, 5, seed=6, amp=0.1, periodic=(0, 0, 1),
                                           dirichlet=0x01 | 0x08), 1.0, 0.3),
    "box2x3x2_N3_periodic_y": (wl.random_deformed_box(2, 3, 2, 3, seed=8, amp=0.1, periodic=(0, 1, 0),
                                                      dirichlet=0x03 | 0x30), 2.0, 0.0),
}
IDS = list(MESHES)


@pytest.fixture(scope="module", params=IDS)
def case(request):
    spec, h1, h2 = MESHES[request.param]
    print("mesh", request.param, flush=True)
    om, gm = pair(spec, prepare=sem.SEM_PREP_HSMG)
    return request.param, om, gm, h1, h2, hsmg.HSMG(om)


def test_preconditioners_match_oracle(case):
    # the three-level preconditioner, its fine Schwarz level and the
    # unweighted block-Jacobi, every output against the oracle: the library
    # factors the local and coarse problems with its own eigen-solver, so
    # results agree to the conditioning of those factorisations
    import torch
    name, om, gm, h1, h2, pc = case
    rng = np.random.default_rng(11)
    r = brute.continuous_random(om, rng)
    z = torch.empty(gm.shape, dtype=torch.float64, device="cuda")
    refs = {sem.PRECOND_HSMG: pc.apply(r, h1, h2),
            sem.PRECOND_SCHWARZ: pc.sw_f.smooth(r, h1, h2),
            sem.PRECOND_BLOCK_JACOBI: hsmg.block_jacobi(pc.sw_f, r, h1, h2),
            sem.PRECOND_HSMG_SYM: pc.apply(r, h1, h2, sym=True)}
    for kind, ref in refs.items():
        gm.precond(dev(r), z, kind=kind, h1=h1, h2=h2)
        zh = host(z)
        err = np.max(np.abs(zh - ref)) / np.max(np.abs(ref))
        print("%s kind %d: max relative difference %.2e" % (name, kind, err))
        assert err <= 1e-10
        assert np.array_equal(zh, om.gather_global(zh)[om.glo])       # continuous
        assert np.all(zh[om.mask == 1] == 0)


def test_gmres_hsmg_solve_matches_oracle(case):
    import torch
    name, om, gm, h1, h2, pc = case
    rng = np.random.default_rng(12)
    b = om.rhs(rng.standard_normal(om.shape))
    xo, info = hsmg.fgmres(om, b, lambda q: pc.apply(q, h1, h2), h1, h2, tol=1e-10, restart=30)
    x = torch.zeros(gm.shape, dtype=torch.float64, device="cuda")
    rep = gm.pcg_solve(dev(b), x, h1=h1, h2=h2, rel_tol=1e-10, form=sem.FORM_GMRES_HSMG)
    xh = host(x)
    res = b - om.apply_S(xh, h1, h2)
    true_rel = np.sqrt(om.dot(res, res) / om.dot(b, b))
    d = xh - xo
    err_s = np.sqrt(om.dot(d, om.apply_S(d, h1, h2)) / om.dot(xo, om.apply_S(xo, h1, h2)))
    _, pinfo = om.pcg(b, h1, h2, tol=1e-10)
    print("%s: GMRES-HSMG %d iterations (oracle %d), Jacobi-PCG %d; true rel res %.2e, S-norm distance %.2e" %
          (name, rep.iterations, info["iterations"], pinfo["iterations"], true_rel, err_s))
    assert true_rel <= 1.05e-10
    assert abs(rep.true_rel_res - true_rel) <= 1e-3 * true_rel + 2e-13
    assert abs(rep.iterations - info["iterations"]) <= max(1, info["iterations"] // 20)
    assert err_s <= 1e-8
    assert rep.iterations < pinfo["iterations"]


def test_block_jacobi_cg_matches_oracle(case):
    import torch
    name, om, gm, h1, h2, pc = case
    rng = np.random.default_rng(13)
    b = om.rhs(rng.standard_normal(om.shape))
    xo, info = hsmg.pcg(om, b, lambda q: hsmg.block_jacobi(pc.sw_f, q, h1, h2), h1, h2, tol=1e-10)
    x = torch.zeros(gm.shape, dtype=torch.float64, device="cuda")
    rep = gm.pcg_solve(dev(b), x, h1=h1, h2=h2, rel_tol=1e-10, form=sem.FORM_PCG_BLOCK_JACOBI)
    xh = host(x)
    res = b - om.apply_S(xh, h1, h2)
    true_rel = np.sqrt(om.dot(res, res) / om.dot(b, b))
    print("%s: block-Jacobi CG %d iterations (oracle %d), true rel res %.2e" %
          (name, rep.iterations, info["iterations"], true_rel))
    assert true_rel <= 1.05e-10
    assert abs(rep.iterations - info["iterations"]) <= max(1, info["iterations"] // 50)


def test_pcg_hsmg_solve_matches_oracle(case):
    # CG with the symmetric multigrid preconditioner
    import torch
    name, om, gm, h1, h2, pc = case
    rng = np.random.default_rng(16)
    b = om.rhs(rng.standard_normal(om.shape))
    xo, info = hsmg.pcg(om, b, lambda q: pc.apply(q, h1, h2, sym=True), h1, h2, tol=1e-10)
    x = torch.zeros(gm.shape, dtype=torch.float64, device="cuda")
    rep = gm.pcg_solve(dev(b), x, h1=h1, h2=h2, rel_tol=1e-10, form=sem.FORM_PCG_HSMG)
    xh = host(x)
    res = b - om.apply_S(xh, h1, h2)
    true_rel = np.sqrt(om.dot(res, res) / om.dot(b, b))
    print("%s: CG + symmetric HSMG %d iterations (oracle %d), true rel res %.2e" %
          (name, rep.iterations, info["iterations"], true_rel))
    assert true_rel <= 1.05e-10
    assert abs(rep.iterations - info["iterations"]) <= max(1, info["iterations"] // 20)


def test_gmres_restart_and_history():
    # a short restart length forces several cycles; the residual history is
    # non-increasing within each cycle and ends below the tolerance
    import torch
    spec = wl.channel(3, 5)
    om, gm = pair(spec, prepare=sem.SEM_PREP_HSMG)
    rng = np.random.default_rng(14)
    b = om.rhs(rng.standard_normal(om.shape))
    x = torch.zeros(gm.shape, dtype=torch.float64, device="cuda")
    rep = gm.pcg_solve(dev(b), x, form=sem.FORM_GMRES_HSMG, restart=4, history=True)
    assert rep.restarts >= 1
    res = b - om.apply_S(host(x))
    assert np.sqrt(om.dot(res, res) / om.dot(b, b)) <= 1.05e-10
    h = rep.history
    assert h[0] == 1.0 and len(h) == rep.iterations + 1
    for c in range(0, rep.iterations, 4):
        seg = h[c + 1:c + 5] if c == 0 else h[c + 1:c + 5]
        assert np.all(np.diff(seg) <= 1e-14)


def test_gmres_hsmg_edge_cases_and_checks():
    import torch
    om, gm = pair(wl.channel(3, 5), prepare=sem.SEM_PREP_HSMG)
    b = torch.zeros(gm.shape, dtype=torch.float64, device="cuda")
    x = torch.ones_like(b)
    for form in (sem.FORM_GMRES_HSMG, sem.FORM_PCG_BLOCK_JACOBI, sem.FORM_PCG_HSMG):
        rep = gm.pcg_solve(b, x, form=form)
        assert rep.status == 0 and rep.iterations == 0 and torch.count_nonzero(x) == 0
    rng = np.random.default_rng(15)
    bb = dev(om.rhs(rng.standard_normal(om.shape)))
    rep = gm.pcg_solve(bb, x, form=sem.FORM_GMRES_HSMG, max_iter=3, raise_on_error=False)
    assert rep.status == sem.SEM_ERR_NOT_CONVERGED and rep.iterations == 3
    r = host(bb) - om.apply_S(host(x))
    assert abs(np.sqrt(om.dot(r, r) / om.dot(host(bb), host(bb))) - rep.true_rel_res) <= 1e-6 * rep.true_rel_res
    for bad in (dict(h1=0.0), dict(h2=-1.0), dict(restart=31)):
        with pytest.raises(sem.SemError):
            gm.pcg_solve(bb, x, form=sem.FORM_GMRES_HSMG, **bad)
    plain = sem.Mesh.from_spec(wl.channel(3, 5))
    with pytest.raises(sem.SemError):
        plain.pcg_solve(bb, x, form=sem.FORM_GMRES_HSMG)
    with pytest.raises(sem.SemError):
        plain.precond(bb, x)
    # a periodic direction with one element is refused at mesh creation
    with pytest.raises(sem.SemError):
        sem.Mesh.from_spec(wl.random_deformed_box(1, 2, 2, 5, seed=1, amp=0.0, periodic=(1, 0, 0)),
                           prepare=sem.SEM_PREP_HSMG)


@pytest.mark.parametrize("spec", [
    # 261 coarse planes along z (more than one workgroup's 256 threads) and a
    # 67 x 67 coarse plane (more than the 4,352 nodes a plane kernel holds in
    # LDS): both take the six single-axis coarse passes
    wl.box(2, 2, 260, 3, extent=(1.0, 1.0, 130.0), dirichlet=0x01 | 0x04 | 0x10 | 0x20),
    wl.box(66, 66, 1, 3, extent=(66.0, 66.0, 1.0), dirichlet=0x0F),
], ids=["column_2x2x260_N3", "plate_66x66x1_N3"])
def test_coarse_solve_without_plane_kernels(spec):
    import torch
    print("mesh", spec.name, flush=True)
    om, gm = pair(spec, prepare=sem.SEM_PREP_HSMG)
    pc = hsmg.HSMG(om)
    rng = np.random.default_rng(17)
    r = brute.continuous_random(om, rng)
    z = torch.empty(gm.shape, dtype=torch.float64, device="cuda")
    for kind, sym in ((sem.PRECOND_HSMG, False), (sem.PRECOND_HSMG_SYM, True)):
        ref = pc.apply(r, 1.0, 0.0, sym=sym)
        gm.precond(dev(r), z, kind=kind)
        err = np.max(np.abs(host(z) - ref)) / np.max(np.abs(ref))
        print("%s kind %d: max relative difference %.2e" % (spec.name, kind, err))
        assert err <= 1e-10
    b = om.rhs(rng.standard_normal(om.shape))
    xo, info = hsmg.pcg(om, b, lambda q: pc.apply(q, sym=True), tol=1e-10)
    x = torch.zeros(gm.shape, dtype=torch.float64, device="cuda")
    rep = gm.pcg_solve(dev(b), x, rel_tol=1e-10, form=sem.FORM_PCG_HSMG)
    res = b - om.apply_S(host(x))
    true_rel = np.sqrt(om.dot(res, res) / om.dot(b, b))
    print("%s: CG + symmetric HSMG %d iterations (oracle %d), true rel res %.2e" %
          (spec.name, rep.iterations, info["iterations"], true_rel))
    assert true_rel <= 1.05e-10
    assert abs(rep.iterations - info["iterations"]) <= max(1, info["iterations"] // 20)


@pytest.mark.parametrize("spec,h2", [(wl.deformed_cube(3, 7), 5.0), (wl.channel(3, 7), 0.0)],
                         ids=["deformed3_N7_helm", "channel3_N7"])
def test_batched_block_jacobi_matches_single_solves(spec, h2):
    # the velocity solves' form: three fields through one batched operator,
    # each with its own block-Jacobi CG, against separate solves and the oracle
    import torch
    om, gm = pair(spec, prepare=sem.SEM_PREP_HSMG)
    pc = hsmg.HSMG(om)
    rng = np.random.default_rng(27)
    bs = np.stack([om.rhs(rng.standard_normal(om.shape)) for _ in range(3)])
    X = torch.zeros(bs.shape, dtype=torch.float64, device="cuda")
    reps = sem.pcg_solve_batched(gm, dev(bs), X, h1=1.0, h2=h2, rel_tol=1e-10, form=sem.FORM_PCG_BLOCK_JACOBI)
    Xh = host(X)
    for c in range(3):
        xs = torch.zeros(gm.shape, dtype=torch.float64, device="cuda")
        rs = gm.pcg_solve(dev(bs[c]), xs, h1=1.0, h2=h2, rel_tol=1e-10, form=sem.FORM_PCG_BLOCK_JACOBI)
        _, info = hsmg.pcg(om, bs[c], lambda q: hsmg.block_jacobi(pc.sw_f, q, 1.0, h2), 1.0, h2, tol=1e-10)
        r = bs[c] - om.apply_S(Xh[c], 1.0, h2)
        true_rel = np.sqrt(om.dot(r, r) / om.dot(bs[c], bs[c]))
        print("%s field %d: batched block-Jacobi CG %d iterations, single %d, oracle %d, true rel res %.2e" %
              (spec.name, c, reps[c].iterations, rs.iterations, info["iterations"], true_rel))
        assert reps[c].status == 0 and true_rel <= 1.05e-10
        assert abs(reps[c].iterations - rs.iterations) <= 1
        assert abs(reps[c].iterations - info["iterations"]) <= max(1, info["iterations"] // 50)
        assert np.linalg.norm(Xh[c] - host(xs)) <= 1e-8 * np.linalg.norm(host(xs))
    # a plain (not multigrid-prepared) mesh cannot take the block-Jacobi form
    plain = sem.Mesh.from_spec(spec)
    with pytest.raises(sem.SemError):
        sem.pcg_solve_batched(plain, dev(bs), X, form=sem.FORM_PCG_BLOCK_JACOBI)
