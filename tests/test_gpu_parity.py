"""GPU parity: the HIP path through the C ABI against the FP64 CPU oracle on
the same seeded inputs.  Bars: integer/index data bit-exact; FP64 fields,
operator and gather-scatter within 1e-12 relative (max-norm); solves to a
true relative residual of 1e-10 as evaluated by the oracle."""
import numpy as np
import pytest

from paper_2405_05640_amd import sem
from paper_2405_05640_amd import workloads as wl
from tests.gpu_util import dev, host, pair, relmax

pytestmark = pytest.mark.gpu

TOL = 1e-12

SPECS = [
    wl.config("c0"),
    wl.random_deformed_box(3, 2, 4, 7, seed=1, amp=0.2),                      # ragged, N=7
    wl.random_deformed_box(5, 3, 2, 4, seed=2, amp=0.2, periodic=(1, 0, 1),
                           dirichlet=wl.DIRICHLET_Y_WALLS),
    wl.channel(4, 7),
    wl.box(1, 1, 1, 3),                                                       # single element
    wl.box(2, 1, 3, 1, periodic=(0, 1, 0)),                                   # N=1, periodic nel=1
    wl.deformed_cube(3, 9),
]
IDS = ["c0", "jitter_N7", "jitter_per_N4", "channel4_N7", "one_elem_N3", "N1_per", "deformed_N9"]


@pytest.fixture(scope="module", params=list(range(len(SPECS))), ids=IDS)
def meshes(request):
    spec = SPECS[request.param]
    print("mesh", spec.name, flush=True)
    return pair(spec)


def test_numbering_mult_mask_bit_exact(meshes):
    om, gm = meshes
    assert gm.n_global == om.n_global
    assert np.array_equal(gm.export(sem.FIELD_GLO_NUM), om.glo)
    assert np.array_equal(gm.export(sem.FIELD_MULT), om.mult)
    assert np.array_equal(gm.export(sem.FIELD_MASK), om.mask)


def test_reference_element_and_geometry(meshes):
    om, gm = meshes
    gll = gm.export(sem.FIELD_GLL)
    assert np.max(np.abs(gll[0] - om.xi)) < 1e-14
    assert np.max(np.abs(gll[1] - om.w)) < 1e-14
    assert relmax(gm.export(sem.FIELD_DERIV), om.D) < 1e-12
    assert relmax(gm.export(sem.FIELD_XYZ), om.xyz) < TOL
    assert relmax(gm.export(sem.FIELD_G), om.G) < TOL
    assert relmax(gm.export(sem.FIELD_B), om.B) < TOL


@pytest.mark.parametrize("h1,h2", [(1.0, 0.0), (1.0, 0.1), (0.7, 2.5)])
def test_ax_f64(meshes, h1, h2):
    import torch
    om, gm = meshes
    rng = np.random.default_rng(10)
    u = rng.standard_normal(om.shape)
    ref = om.ax(u, h1, h2)
    w = torch.empty(gm.shape, dtype=torch.float64, device="cuda")
    gm.ax(dev(u), w, h1, h2)
    assert relmax(host(w), ref) < TOL


def test_dssum_f64_bitwise_and_mask(meshes):
    import torch
    om, gm = meshes
    rng = np.random.default_rng(11)
    u = rng.standard_normal(om.shape)
    t = dev(u)
    gm.dssum(t, mask=False)
    assert np.array_equal(host(t), om.dssum(u))
    t = dev(u)
    gm.dssum(t, mask=True)
    assert np.array_equal(host(t), om.apply_mask(om.dssum(u)))


def test_rhs_jacobi_dot(meshes):
    import torch
    om, gm = meshes
    rng = np.random.default_rng(12)
    f = rng.standard_normal(om.shape)
    b = torch.empty(gm.shape, dtype=torch.float64, device="cuda")
    gm.rhs(dev(f), b)
    assert relmax(host(b), om.rhs(f)) < TOL
    for h2 in (0.0, 0.3):
        d = torch.empty_like(b)
        gm.jacobi(d, 1.0, h2)
        assert relmax(host(d), om.jacobi_inv(1.0, h2)) < TOL
    u, v = om.rhs(rng.standard_normal(om.shape)), om.rhs(rng.standard_normal(om.shape))
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    gm.dot(dev(u), dev(v), out)
    ref = om.dot(u, v)
    assert abs(host(out)[0] - ref) <= 1e-13 * np.sqrt(om.dot(u, u) * om.dot(v, v))


@pytest.mark.parametrize("h2", [0.0, 0.1])
def test_pcg_solve_parity(meshes, h2):
    import torch
    om, gm = meshes
    rng = np.random.default_rng(13)
    b = om.rhs(rng.standard_normal(om.shape))
    xo, info = om.pcg(b, 1.0, h2, tol=1e-10)
    x = torch.zeros(gm.shape, dtype=torch.float64, device="cuda")
    rep = gm.pcg_solve(dev(b), x, h1=1.0, h2=h2, rel_tol=1e-10, history=True)
    xg = host(x)
    # (i) true residual of the GPU solution, evaluated by the oracle
    r = b - om.apply_S(xg, 1.0, h2)
    true_rel = np.sqrt(om.dot(r, r) / om.dot(b, b))
    assert true_rel <= 1.05e-10
    # the reported true residual agrees with the oracle's (both at rounding
    # level when the solve is exact to machine precision)
    assert abs(rep.true_rel_res - true_rel) <= 1e-3 * true_rel + 1e-14
    # (ii) solutions agree within the residual-implied bound (S-norm)
    e = xg - xo
    en = np.sqrt(max(om.dot(e, om.apply_S(e, 1.0, h2)), 0.0))
    xn = np.sqrt(om.dot(xo, om.apply_S(xo, 1.0, h2)))
    bn = np.sqrt(om.dot(b, b))
    assert en <= 1e-6 * xn + 1e-300
    # (iii) iteration counts agree within 2 % (+1)
    assert abs(rep.iterations - info["iterations"]) <= max(1, 0.02 * info["iterations"])
    # continuity and mask of the GPU iterate
    assert np.array_equal(xg, om.gather_global(xg)[om.glo])
    assert np.all(xg[om.mask == 1] == 0.0)
    assert rep.history[0] == 1.0 and rep.history[-1] <= 1e-10


@pytest.mark.parametrize("h2", [0.0, 0.1])
def test_single_reduction_pcg_parity(meshes, h2):
    # the Chronopoulos-Gear form is the same Krylov method: same bars as the
    # standard form against the oracle (true residual, S-norm error, counts)
    import torch
    om, gm = meshes
    rng = np.random.default_rng(14)
    b = om.rhs(rng.standard_normal(om.shape))
    xo, info = om.pcg(b, 1.0, h2, tol=1e-10)
    x = torch.zeros(gm.shape, dtype=torch.float64, device="cuda")
    rep = gm.pcg_solve(dev(b), x, h1=1.0, h2=h2, rel_tol=1e-10, form=sem.FORM_PCG_1RED, history=True, check_every=8)
    xg = host(x)
    r = b - om.apply_S(xg, 1.0, h2)
    true_rel = np.sqrt(om.dot(r, r) / om.dot(b, b))
    assert true_rel <= 1.05e-10
    assert abs(rep.true_rel_res - true_rel) <= 1e-3 * true_rel + 1e-14
    e = xg - xo
    en = np.sqrt(max(om.dot(e, om.apply_S(e, 1.0, h2)), 0.0))
    assert en <= 1e-6 * np.sqrt(om.dot(xo, om.apply_S(xo, 1.0, h2))) + 1e-300
    assert abs(rep.iterations - info["iterations"]) <= max(2, 0.03 * info["iterations"])
    assert np.array_equal(xg, om.gather_global(xg)[om.glo])
    assert np.all(xg[om.mask == 1] == 0.0)
    assert rep.history[0] == 1.0 and rep.history[-1] <= 1e-10


def test_deterministic_repeat():
    import torch
    om, gm = pair(wl.deformed_cube(4, 7))
    rng = np.random.default_rng(0)
    u = dev(rng.standard_normal(om.shape))
    w1 = torch.empty_like(u)
    w2 = torch.empty_like(u)
    gm.ax(u, w1, 1.0, 0.1)
    gm.dssum(w1, mask=True)
    gm.ax(u, w2, 1.0, 0.1)
    gm.dssum(w2, mask=True)
    assert torch.equal(w1, w2)
    b = dev(om.rhs(rng.standard_normal(om.shape)))
    x1 = torch.zeros_like(b)
    x2 = torch.zeros_like(b)
    r1 = gm.pcg_solve(b, x1, h1=1.0, h2=0.1)
    r2 = gm.pcg_solve(b, x2, h1=1.0, h2=0.1)
    assert r1.iterations == r2.iterations and torch.equal(x1, x2)


def test_manufactured_c0_solution():
    import torch
    om, gm = pair(wl.config("c0"))
    uex, f = wl.manufactured(*om.xyz)
    b = torch.empty(gm.shape, dtype=torch.float64, device="cuda")
    gm.rhs(dev(f), b)
    x = torch.zeros_like(b)
    rep = gm.pcg_solve(b, x, rel_tol=1e-10)
    assert rep.status == 0 and rep.true_rel_res <= 1e-10
    assert np.max(np.abs(host(x) - uex)) < 1e-7


def test_status_codes_and_argument_checks():
    import torch
    om, gm = pair(wl.deformed_cube(2, 3))
    rng = np.random.default_rng(1)
    b = dev(om.rhs(rng.standard_normal(om.shape)))
    x = torch.zeros_like(b)
    rep = gm.pcg_solve(b, x, max_iter=3, raise_on_error=False)
    assert rep.status == sem.SEM_ERR_NOT_CONVERGED and rep.iterations == 3
    rep = gm.pcg_solve(torch.zeros_like(b), x)
    assert rep.status == 0 and rep.iterations == 0 and torch.count_nonzero(x) == 0
    with pytest.raises(ValueError):
        gm.ax(b[:-1], x)                       # wrong size caught on the host
    with pytest.raises(ValueError):
        gm.ax(b.float(), x)                    # wrong dtype
    with pytest.raises(sem.SemError):
        gm.ax(b.float(), x.float(), dtype=sem.SEM_F32)   # mesh not prepared for fp32
    v = wl.box(2, 2, 2, 3).vertices.copy()
    v[1, 1, 1, 0] = 1.3
    with pytest.raises(sem.SemError):
        sem.Mesh(2, 2, 2, 3, v)


def test_reliable_and_split_status_codes():
    # reliable-update forms: zero right-hand side, iteration cap, argument
    # checks; the split-BF16 operator needs a BF16-prepared N = 7 mesh
    import torch
    om, gm = pair(wl.deformed_cube(2, 7), prepare=sem.SEM_PREP_F32 | sem.SEM_PREP_BF16)
    rng = np.random.default_rng(2)
    b = dev(om.rhs(rng.standard_normal(om.shape)))
    x = torch.zeros_like(b)
    for form in (sem.FORM_RELIABLE_FP32, sem.FORM_RELIABLE_BF16):
        rep = gm.pcg_solve(torch.zeros_like(b), x, form=form, inner_tol=0.1)
        assert rep.status == 0 and rep.iterations == 0 and torch.count_nonzero(x) == 0
        rep = gm.pcg_solve(b, x, form=form, inner_tol=0.1, max_iter=5, check_every=1, raise_on_error=False)
        assert rep.status == sem.SEM_ERR_NOT_CONVERGED and rep.iterations >= 5
        r = host(b) - om.apply_S(host(x), 1.0, 0.0)   # x is the FP64 iterate the report describes
        assert abs(np.sqrt(om.dot(r, r) / om.dot(host(b), host(b))) - rep.true_rel_res) <= 1e-6 * rep.true_rel_res
        for bad in (0.0, 1.0):
            with pytest.raises(sem.SemError):
                gm.pcg_solve(b, x, form=form, inner_tol=bad)
    plain = sem.Mesh.from_spec(wl.deformed_cube(2, 7))
    with pytest.raises(sem.SemError):
        plain.pcg_solve(b, x, form=sem.FORM_RELIABLE_FP32, inner_tol=0.1)
    with pytest.raises(sem.SemError):
        plain.ax(b.float(), x.float(), dtype=sem.SEM_BF16_SPLIT)
    om5, gm5 = pair(wl.deformed_cube(2, 5), prepare=sem.SEM_PREP_BF16)
    u5 = torch.zeros(gm5.shape, dtype=torch.float32, device="cuda")
    with pytest.raises(sem.SemError):
        gm5.ax(u5, torch.empty_like(u5), dtype=sem.SEM_BF16_SPLIT)


def test_table1_unique_count_fully_periodic_64cube():
    # Table 1 (TGV row): E = 262,144 elements at N = 7 -> n = E N^3 = 89,915,392
    spec = wl.box(64, 64, 64, 7, periodic=(1, 1, 1), dirichlet=0)
    gm = sem.Mesh.from_spec(spec)
    assert gm.E == 262144 and gm.n_global == 89915392
    gm.close()


@pytest.mark.parametrize("h2", [0.0, 0.1])
def test_ax_f32_error_bound(h2):
    # |A32 u - A64 u| <= c eps32 (|D|^T |G| |D| |u|), c = 3 (N+1) + 6
    import torch
    spec = wl.deformed_cube(3, 7)
    om, gm = pair(spec, prepare=sem.SEM_PREP_F32)
    rng = np.random.default_rng(20)
    u = rng.standard_normal(om.shape).astype(np.float32).astype(np.float64)
    w = torch.empty(gm.shape, dtype=torch.float32, device="cuda")
    gm.ax(dev(u, torch.float32), w, 1.0, h2, dtype=sem.SEM_F32)
    err = np.abs(host(w).astype(np.float64) - om.ax(u, 1.0, h2))
    bound = (3 * (om.N + 1) + 6) * 2.0 ** -24 * om.ax_abs_bound(u, 1.0, h2)
    assert np.all(err <= bound + 1e-30)


@pytest.mark.parametrize("spec", [wl.config("c0"), wl.deformed_cube(4, 7), wl.channel(3, 7)],
                         ids=["c0", "deformed4_N7", "channel3_N7"])
def test_dc_fp32_solve_reaches_fp64_tolerance(spec):
    import torch
    om, gm = pair(spec, prepare=sem.SEM_PREP_F32)
    h2 = 0.1 if spec.name.startswith("deformed") else 0.0
    rng = np.random.default_rng(21)
    b = om.rhs(rng.standard_normal(om.shape))
    x = torch.zeros(gm.shape, dtype=torch.float64, device="cuda")
    rep = gm.pcg_solve(dev(b), x, h1=1.0, h2=h2, rel_tol=1e-10, form=sem.FORM_DC_FP32, inner_tol=1e-5)
    xg = host(x)
    r = b - om.apply_S(xg, 1.0, h2)
    true_rel = np.sqrt(om.dot(r, r) / om.dot(b, b))
    assert true_rel <= 1.05e-10
    assert rep.outer_iterations >= 2
    xo, info = om.pcg(b, 1.0, h2, tol=1e-10)
    e = xg - xo
    assert np.sqrt(om.dot(e, om.apply_S(e, 1.0, h2))) <= 1e-6 * np.sqrt(om.dot(xo, om.apply_S(xo, 1.0, h2)))
    print("DC-FP32 %s: inner its %d, outer %d; FP64 PCG its %d" % (spec.name, rep.iterations,
                                                                  rep.outer_iterations, info["iterations"]))


def test_ax_bf16_matrix_cores():
    # bound against FP64 as for FP32 with eps = 2^-8, and closer to the
    # oracle's BF16 emulation than that emulation is to FP64
    import torch
    from oracle import mixed
    spec = wl.deformed_cube(3, 7)
    om, gm = pair(spec, prepare=sem.SEM_PREP_BF16)
    rng = np.random.default_rng(22)
    u = mixed.bf16_round(rng.standard_normal(om.shape).astype(np.float32)).astype(np.float64)
    ub = dev(u.astype(np.float32)).to(torch.bfloat16).view(torch.int16)
    for h2 in (0.0, 0.1):
        w = torch.empty(gm.shape, dtype=torch.float32, device="cuda")
        gm.ax(ub, w, 1.0, h2, dtype=sem.SEM_BF16)
        wg = host(w).astype(np.float64)
        w64 = om.ax(u, 1.0, h2)
        bound = (3 * (om.N + 1) + 6) * 2.0 ** -8 * om.ax_abs_bound(u, 1.0, h2)
        assert np.all(np.abs(wg - w64) <= bound + 1e-30)
        we = mixed.ax_lowp(om, u, 1.0, h2, "bf16")
        assert np.linalg.norm(wg - we) <= np.linalg.norm(we - w64)


@pytest.mark.parametrize("spec", [wl.deformed_cube(3, 7), wl.channel(3, 7)], ids=["deformed3_N7", "channel3_N7"])
def test_ax_bf16_split_matrix_cores(spec):
    # the split-BF16 operator against the exact operator with its stored G and
    # B (half precision, per-element scale): within a 2^-15-level bound
    # (about 2^-8 tighter than the plain BF16 operator), and well closer to
    # it than that operator is to FP64 (storage 2^-11 against split 2^-16)
    import torch
    from oracle import mixed
    om, gm = pair(spec, prepare=sem.SEM_PREP_BF16)
    rng = np.random.default_rng(26)
    u32 = rng.standard_normal(om.shape).astype(np.float32)
    u = u32.astype(np.float64)
    for h2 in (0.0, 0.1):
        w = torch.empty(gm.shape, dtype=torch.float32, device="cuda")
        gm.ax(dev(u32, torch.float32), w, 1.0, h2, dtype=sem.SEM_BF16_SPLIT)
        wg = host(w).astype(np.float64)
        ref = mixed.ax_bf16_split_reference(om, u, 1.0, h2)
        bound = (3 * (om.N + 1) + 6) * 2.0 ** -15 * om.ax_abs_bound(u, 1.0, h2)
        assert np.all(np.abs(wg - ref) <= bound + 1e-30)
        w64 = om.ax(u, 1.0, h2)
        ratio = np.linalg.norm(wg - ref) / np.linalg.norm(ref - w64)
        print("split-BF16 %s h2=%g: |gpu - ref| / |ref - fp64| = %.4f" % (spec.name, h2, ratio))
        assert ratio <= 0.1


@pytest.mark.parametrize("spec", [wl.deformed_cube(4, 7), wl.channel(3, 7)], ids=["deformed4_N7", "channel3_N7"])
def test_dc_bf16_solve_reaches_fp64_tolerance(spec):
    import torch
    om, gm = pair(spec, prepare=sem.SEM_PREP_BF16)
    h2 = 0.1 if spec.name.startswith("deformed") else 0.0
    rng = np.random.default_rng(23)
    b = om.rhs(rng.standard_normal(om.shape))
    x = torch.zeros(gm.shape, dtype=torch.float64, device="cuda")
    rep = gm.pcg_solve(dev(b), x, h1=1.0, h2=h2, rel_tol=1e-10, form=sem.FORM_DC_BF16, inner_tol=1e-2,
                       max_outer=60)
    xg = host(x)
    r = b - om.apply_S(xg, 1.0, h2)
    assert np.sqrt(om.dot(r, r) / om.dot(b, b)) <= 1.05e-10
    print("DC-BF16 %s: inner its %d, outer %d" % (spec.name, rep.iterations, rep.outer_iterations))


@pytest.mark.parametrize("form,prep", [(sem.FORM_FCG_INNER_FP32, sem.SEM_PREP_F32),
                                       (sem.FORM_FCG_INNER_BF16, sem.SEM_PREP_BF16)], ids=["inner_fp32", "inner_bf16"])
@pytest.mark.parametrize("spec", [wl.deformed_cube(4, 7), wl.channel(3, 7)], ids=["deformed4_N7", "channel3_N7"])
def test_nested_fcg_reaches_fp64_tolerance(spec, form, prep):
    import torch
    om, gm = pair(spec, prepare=prep)
    h2 = 0.1 if spec.name.startswith("deformed") else 0.0
    rng = np.random.default_rng(24)
    b = om.rhs(rng.standard_normal(om.shape))
    x = torch.zeros(gm.shape, dtype=torch.float64, device="cuda")
    rep = gm.pcg_solve(dev(b), x, h1=1.0, h2=h2, rel_tol=1e-10, form=form, inner_iters=8, inner_tol=0.0)
    xg = host(x)
    r = b - om.apply_S(xg, 1.0, h2)
    assert np.sqrt(om.dot(r, r) / om.dot(b, b)) <= 1.05e-10
    assert rep.fallback_used == 0 and rep.outer_iterations > 0
    assert rep.iterations <= 8 * rep.outer_iterations + 8
    _, info = om.pcg(b, 1.0, h2)
    print("nested %s %s: %d outer, %d inner; FP64 PCG %d" % (spec.name, form, rep.outer_iterations, rep.iterations,
                                                            info["iterations"]))


@pytest.mark.parametrize("form,prep,delta", [(sem.FORM_RELIABLE_FP32, sem.SEM_PREP_F32, 1e-2),
                                             (sem.FORM_RELIABLE_BF16, sem.SEM_PREP_BF16, 0.1)],
                         ids=["reliable_fp32", "reliable_bf16split"])
@pytest.mark.parametrize("spec", [wl.deformed_cube(4, 7), wl.channel(3, 7)], ids=["deformed4_N7", "channel3_N7"])
def test_reliable_update_cg_reaches_fp64_tolerance(spec, form, prep, delta):
    # the FP64 true residual (evaluated by the oracle) meets 1e-10; with the
    # FP32 operator the kept search direction holds the iteration count near
    # the FP64 PCG count (a restarted defect correction would not)
    import torch
    om, gm = pair(spec, prepare=prep)
    h2 = 0.1 if spec.name.startswith("deformed") else 0.0
    rng = np.random.default_rng(25)
    b = om.rhs(rng.standard_normal(om.shape))
    x = torch.zeros(gm.shape, dtype=torch.float64, device="cuda")
    rep = gm.pcg_solve(dev(b), x, h1=1.0, h2=h2, rel_tol=1e-10, form=form, inner_tol=delta, check_every=4)
    xg = host(x)
    r = b - om.apply_S(xg, 1.0, h2)
    assert np.sqrt(om.dot(r, r) / om.dot(b, b)) <= 1.05e-10
    assert rep.outer_iterations >= 2
    _, info = om.pcg(b, 1.0, h2)
    if form == sem.FORM_RELIABLE_FP32:
        assert rep.iterations <= 1.25 * info["iterations"] + 8
    print("reliable %s %s: %d iterations, %d replacements; FP64 PCG %d" %
          (spec.name, form, rep.iterations, rep.outer_iterations, info["iterations"]))


@pytest.mark.parametrize("spec,h2", [(wl.deformed_cube(3, 7), 5.0), (wl.channel(3, 7), 0.0)],
                         ids=["deformed3_N7_helm", "channel3_N7"])
def test_batched_solve_matches_single_solves(spec, h2):
    import torch
    om, gm = pair(spec)
    rng = np.random.default_rng(25)
    bs = np.stack([om.rhs(rng.standard_normal(om.shape)) for _ in range(3)])
    X = torch.zeros(bs.shape, dtype=torch.float64, device="cuda")
    reps = sem.pcg_solve_batched(gm, dev(bs), X, h1=1.0, h2=h2, rel_tol=1e-10)
    Xh = host(X)
    for c in range(3):
        xs = torch.zeros(gm.shape, dtype=torch.float64, device="cuda")
        rs = gm.pcg_solve(dev(bs[c]), xs, h1=1.0, h2=h2, rel_tol=1e-10)
        assert abs(reps[c].iterations - rs.iterations) <= 1
        r = bs[c] - om.apply_S(Xh[c], 1.0, h2)
        assert np.sqrt(om.dot(r, r) / om.dot(bs[c], bs[c])) <= 1.05e-10
        assert np.linalg.norm(Xh[c] - host(xs)) <= 1e-8 * np.linalg.norm(host(xs))
