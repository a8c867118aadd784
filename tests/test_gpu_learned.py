"""GPU parity of the learned smoother against the FP64 oracle (oracle/cnn.py):
FP32 path within 1e-5 (forward, norm-wise, and an element-wise rounding
bound) / 1e-5 (gradient, norm-wise), BF16 inference path within 2e-2
(norm-wise, on the learned correction) and an element-wise bound; Adam
training steps element-wise against the oracle's Adam; the training
diagonal cache and checkpoint/resume; flexible CG reaches the FP64 true
residual 1e-10 in every mode, equals Jacobi-PCG for the zero network, and
falls back on a broken network; snapshot errors and training."""
import numpy as np
import pytest

import oracle
from oracle import cnn
from paper_2405_05640_amd import sem
from paper_2405_05640_amd import workloads as wl
from tests.gpu_util import dev, host, pair

pytestmark = pytest.mark.gpu


def _net_weights(seed, scale3=0.05):
    net = cnn.Net.init(16, seed=seed)
    rng = np.random.default_rng(seed + 100)
    net.W[2] = rng.standard_normal(net.W[2].shape) * scale3
    flat = np.concatenate([net.W[0].ravel(), net.W[1].ravel(), net.W[2].ravel()]).astype(np.float32)
    # the oracle evaluates the FP32-rounded weights too
    net.W = [flat[:864].reshape(16, 2, 3, 3, 3).astype(np.float64),
             flat[864:864 + 6912].reshape(16, 16, 3, 3, 3).astype(np.float64),
             flat[864 + 6912:].reshape(1, 16, 3, 3, 3).astype(np.float64)]
    return net, flat


def _abs_net_bound(om, net, r, dinv, rel):
    """rel * mask(dssum(t_e AbsNet(|X_e|) / mult)): AbsNet is the network
    with |W| and no ReLU on the absolute features."""
    X, s, t, live = cnn.features(r, dinv)
    absnet = cnn.Net(*[np.abs(w) for w in net.W])
    A = np.abs(X)
    for W in absnet.W:
        A = cnn.conv3d(A, W)
    c = t[:, None, None, None] * A[:, 0]
    c[~live] = 0.0
    return rel * om.apply_mask(om.dssum(c / om.mult))


@pytest.fixture(scope="module")
def mp():
    spec = wl.random_deformed_box(3, 2, 3, 7, seed=4, amp=0.15, periodic=(1, 0, 0),
                                  dirichlet=wl.DIRICHLET_Y_WALLS | 0x30)
    return pair(spec)


def test_smoother_forward_fp32_and_bf16(mp):
    import torch
    om, gm = mp
    net, flat = _net_weights(1)
    sm = sem.Smoother(gm)
    sm.set_weights(flat)
    assert np.array_equal(sm.get_weights(), flat)
    rng = np.random.default_rng(2)
    r = om.rhs(rng.standard_normal(om.shape))
    dinv = om.jacobi_inv()
    z_ref = cnn.smoother(om, net, r, dinv)
    corr_ref = z_ref - dinv * r
    z = torch.empty(gm.shape, dtype=torch.float64, device="cuda")
    sm.apply(dev(r), z, fp32=True)
    z32 = host(z)
    assert np.linalg.norm(z32 - z_ref) <= 1e-5 * np.linalg.norm(z_ref)
    assert np.linalg.norm((z32 - dinv * r) - corr_ref) <= 1e-5 * np.linalg.norm(corr_ref)
    # element-wise: every output point within a rounding bound built from the
    # network run on absolute values (|W|, |X|, no ReLU: ReLU is 1-Lipschitz)
    # times t_e.  FP32 path: the input rounding plus one rounding per term of
    # the three layers' sums (54 + 432 + 432 terms) gives fewer than 1024
    # units of 2^-24; averaging over node copies cannot raise the bound.
    bound32 = _abs_net_bound(om, net, r, dinv, 1024 * 2.0 ** -24) + 1e-14 * np.abs(z_ref)
    err32 = np.abs(z32 - z_ref)
    print("FP32 smoother: max error / element-wise bound = %.3g" % np.max(err32 / np.maximum(bound32, 1e-300)))
    assert np.all(err32 <= bound32)
    sm.apply(dev(r), z, fp32=False)
    zb = host(z)
    assert np.linalg.norm((zb - dinv * r) - corr_ref) <= 2e-2 * np.linalg.norm(corr_ref)
    # BF16 inference: the input of each layer (X, Y1, Y2) and its weights
    # (W1, W2, W3) are rounded to BF16 once (2^-9 relative each), six
    # roundings along any path through the network: below 2^-6 relative on
    # top of the FP32 bound
    boundb = _abs_net_bound(om, net, r, dinv, 2.0 ** -6 + 1024 * 2.0 ** -24) + 1e-14 * np.abs(z_ref)
    errb = np.abs(zb - z_ref)
    print("BF16 smoother: max error / element-wise bound = %.3g" % np.max(errb / np.maximum(boundb, 1e-300)))
    assert np.all(errb <= boundb)
    # continuity and Dirichlet nodes
    assert np.array_equal(zb, om.gather_global(zb)[om.glo])
    assert np.all(zb[om.mask == 1] == 0)
    # zero network is exactly Jacobi
    zero = flat.copy()
    zero[864 + 6912:] = 0
    sm.set_weights(zero)
    sm.apply(dev(r), z)
    # (the GPU's and the oracle's Jacobi diagonals agree to rounding)
    assert np.allclose(host(z), dinv * r, rtol=1e-12, atol=0)


@pytest.mark.parametrize("h2", [0.0, 0.1])
def test_loss_gradient_fp32_path(mp, h2):
    om, gm = mp
    net, flat = _net_weights(3, scale3=0.1)
    sm = sem.Smoother(gm)
    sm.set_weights(flat)
    rng = np.random.default_rng(4)
    from tests import brute
    e = brute.continuous_random(om, rng)
    r = om.apply_S(e, 1.0, h2)
    L_ref, g_ref = cnn.loss_and_grad(om, net, r, e, om.jacobi_inv(1.0, h2), 1.0, h2)
    L, g = sm.loss_grad(dev(e), 1.0, h2)
    assert abs(L - L_ref) <= 1e-5 * abs(L_ref)
    gr = np.concatenate([x.ravel() for x in g_ref])
    print("FP32 gradient: norm-wise relative error %.3g" % (np.linalg.norm(g - gr) / np.linalg.norm(gr)))
    assert np.linalg.norm(g - gr) <= 1e-5 * np.linalg.norm(gr)
    for lo, hi in ((0, 864), (864, 864 + 6912), (864 + 6912, 8208)):
        assert np.linalg.norm(g[lo:hi] - gr[lo:hi]) <= 1e-5 * np.linalg.norm(gr[lo:hi])


def _true_rel(om, b, x, h2=0.0):
    r = b - om.apply_S(x, 1.0, h2)
    return np.sqrt(om.dot(r, r) / om.dot(b, b))


def test_fcg_zero_net_matches_pcg_and_fallbacks(mp):
    import torch
    om, gm = mp
    rng = np.random.default_rng(5)
    b = om.rhs(rng.standard_normal(om.shape))
    _, info = om.pcg(b)
    sm = sem.Smoother(gm)   # fresh: last layer zero -> Jacobi
    x = torch.zeros(gm.shape, dtype=torch.float64, device="cuda")
    rep = gm.pcg_solve(dev(b), x, form=sem.FORM_FCG_LEARNED, smoother=sm)
    assert rep.fallback_used == 0
    assert abs(rep.iterations - info["iterations"]) <= 2
    assert _true_rel(om, b, host(x)) <= 1.05e-10
    # random network: converges, FP64 true residual decides
    net, flat = _net_weights(6)
    sm.set_weights(flat)
    x.zero_()
    rep = gm.pcg_solve(dev(b), x, form=sem.FORM_FCG_LEARNED, smoother=sm)
    assert _true_rel(om, b, host(x)) <= 1.05e-10
    # broken network (NaN last layer): rejected at once, Jacobi-PCG finishes
    bad = flat.copy()
    bad[864 + 6912:] = np.nan
    sm.set_weights(bad)
    x.zero_()
    rep = gm.pcg_solve(dev(b), x, form=sem.FORM_FCG_LEARNED, smoother=sm)
    assert rep.fallback_used == 1
    assert _true_rel(om, b, host(x)) <= 1.05e-10
    # stall test forced by an impossible rate: falls back, still converges
    sm2 = sem.Smoother(gm, stall_window=3, stall_rate=1e-6)
    sm2.set_weights(flat)
    x.zero_()
    rep = gm.pcg_solve(dev(b), x, form=sem.FORM_FCG_LEARNED, smoother=sm2)
    assert rep.fallback_used == 1
    assert _true_rel(om, b, host(x)) <= 1.05e-10


def test_pcg_snapshots_match_oracle(mp):
    import torch
    om, gm = mp
    rng = np.random.default_rng(7)
    b = om.rhs(rng.standard_normal(om.shape))
    xs, _ = om.pcg(b, tol=1e-10)
    iters = [0, 3, 10]
    e = torch.zeros(len(iters) * gm.n_global, dtype=torch.float64, device="cuda")
    rep = sem.pcg_snapshots(gm, dev(b), iters, e)
    assert rep.status == 0
    E = host(e).reshape(len(iters), -1)
    for q, k in enumerate(iters):
        if k == 0:
            xk = np.zeros(om.shape)
        else:
            xk, _ = om.pcg(b, tol=1e-30, max_iter=k)
        ref = om.gather_global(xs - xk)
        assert np.linalg.norm(E[q] - ref) <= 1e-7 * np.linalg.norm(om.gather_global(xs))


def test_training_gain_over_jacobi():
    # What the trained network gains over the method without it (the zero
    # network, which is exactly Jacobi): on held-out error fields, the A-norm
    # error left after one smoothing, |e - M(S e)|_S^2 / |e|_S^2, is lower.
    # The flexible-CG solve with the trained network still meets the FP64
    # true residual; its iteration count is reported, not asserted (no
    # iteration gain is measured for this per-element smoother).
    import torch
    spec = wl.channel(4, 7)
    om, gm = pair(spec)
    glo = torch.from_numpy(gm.export(sem.FIELD_GLO_NUM).ravel()).cuda()
    vm = wl.kolmogorov_velocity(2)
    iters = [1, 2, 4, 8]

    def errors(ts):
        out = []
        for t in ts:
            f = wl.fourier_on_elements(wl.divergence_source(vm, t), om.xyz, (4, 4, 4))
            b = torch.empty(gm.shape, dtype=torch.float64, device="cuda")
            gm.rhs(dev(f), b)
            e = torch.zeros(len(iters) * gm.n_global, dtype=torch.float64, device="cuda")
            sem.pcg_snapshots(gm, b, iters, e)
            out += [e[q * gm.n_global:(q + 1) * gm.n_global].contiguous() for q in range(len(iters))]
        return out

    train = errors(range(8))
    held = errors(range(40, 42))
    sm = sem.Smoother(gm, seed=0, lr=2e-3)

    def held_loss():
        return float(np.mean([sm.loss_grad(e[glo].reshape(gm.shape).contiguous())[0] for e in held]))

    jacobi = held_loss()   # fresh smoother: last layer zero -> Jacobi
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    first, last = [], []
    for epoch in range(8):
        for k, ep in enumerate(train):
            sm.train_step(ep.float().contiguous(), loss)
            if epoch == 0:
                first.append(float(loss.item()))
            if epoch == 7:
                last.append(float(loss.item()))
    trained = held_loss()
    print("training loss %.4f -> %.4f; held-out one-step A-norm error: Jacobi %.4f, trained %.4f" %
          (np.mean(first), np.mean(last), jacobi, trained))
    assert np.mean(last) < np.mean(first)
    assert trained < 0.97 * jacobi
    # held-out solve: FCG with the trained smoother vs Jacobi-PCG
    f = wl.fourier_on_elements(wl.divergence_source(vm, 50), om.xyz, (4, 4, 4))
    b = om.rhs(f)
    x = torch.zeros(gm.shape, dtype=torch.float64, device="cuda")
    rep = gm.pcg_solve(dev(b), x, form=sem.FORM_FCG_LEARNED, smoother=sm)
    assert _true_rel(om, b, host(x)) <= 1.05e-10
    x.zero_()
    rj = gm.pcg_solve(dev(b), x)
    print("held-out: FCG-learned %d iterations (fallback %d) vs Jacobi-PCG %d" %
          (rep.iterations, rep.fallback_used, rj.iterations))


def _fields_f32(om, gm, n, seed):
    """n continuous masked error fields with float32-representable values, as
    (global float32 torch vectors, local float64 numpy fields)."""
    import torch
    from tests import brute
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        e = brute.continuous_random(om, rng).astype(np.float32).astype(np.float64)
        eg = om.gather_global(e).astype(np.float32)
        out.append((torch.from_numpy(eg).cuda(), eg[om.glo].astype(np.float64)))
    return out


def test_train_step_adam_against_oracle(mp):
    # Three sem_smoother_train_step calls on fixed pairs.  (1) The Adam update
    # itself, element by element: the oracle's FP64 Adam fed the GPU's own
    # gradient at each step (sem_smoother_loss_grad gives the same bits as the
    # gradient inside train_step: same inputs, fixed reduction order) must
    # reproduce the GPU weights and moments to FP32 rounding.  (2) The whole
    # chain against the oracle's forward, backward and Adam in FP64, with a
    # large eps so the update is a smooth function of the gradient: every
    # weight within the FP32 gradient error propagated through three steps.
    om, gm = mp
    net, flat = _net_weights(8, scale3=0.05)
    pairs = _fields_f32(om, gm, 3, seed=21)
    lr = 1e-3
    # (1) default eps
    # the library holds the hyperparameters in FP32; the oracle takes the
    # same (FP32-rounded) values and runs in FP64
    f32 = lambda a: float(np.float32(a))
    hyper = dict(lr=f32(lr), beta1=f32(0.9), beta2=f32(0.999), eps=f32(1e-8))
    sm = sem.Smoother(gm, lr=lr)
    sm.set_weights(flat)
    opt = cnn.Adam([(8208,)], **hyper)
    opt_abs = cnn.Adam([(8208,)], **hyper)      # the same recursions on |g|
    W = [flat.astype(np.float64)]
    tol = np.zeros(8208)
    u32 = 2.0 ** -24
    for eg, el in pairs:
        L, g = sm.loss_grad(dev(el))
        sm.train_step(eg)
        g = g.astype(np.float64)
        W = opt.step(W, [g])
        opt_abs.step([np.zeros(8208)], [np.abs(g)])
        # FP32 rounding of one step: the moments carry a few units of 2^-24
        # of the recursion run on |g| (cancelling gradients make m small
        # next to its terms), the update a few more, and W one rounding
        t = opt.t
        m_abs = opt_abs.m[0] / (1 - opt.b1 ** t)
        v_hat = opt.v[0] / (1 - opt.b2 ** t)
        tol += 16 * u32 * lr * m_abs / (np.sqrt(v_hat) + opt.eps) + u32 * np.abs(W[0])
    w_gpu, m_gpu, v_gpu, step = sm.get_state()
    assert step == 3
    moved = np.abs(w_gpu - flat)
    assert np.count_nonzero(moved) > 8000
    err = np.abs(w_gpu - W[0])
    print("Adam (GPU gradient): max |W - W_oracle| = %.3g, max error / bound = %.3g (update scale %.3g)" %
          (err.max(), np.max(err / tol), moved.max()))
    assert np.all(err <= tol)
    assert np.all(np.abs(m_gpu - opt.m[0]) <= 16 * u32 * opt_abs.m[0])
    assert np.allclose(v_gpu, opt.v[0], rtol=1e-6, atol=1e-38)
    # (2) oracle forward + backward + Adam
    dinv = om.jacobi_inv()
    _, g0 = cnn.loss_and_grad(om, net, om.apply_S(pairs[0][1]), pairs[0][1], dinv)
    gmax = max(np.max(np.abs(x)) for x in g0)
    gnorm = np.sqrt(sum(np.sum(x * x) for x in g0))
    eps = 10.0 * gmax
    lib_eps = sem.Smoother(gm, lr=lr, eps=eps)
    lib_eps.set_weights(flat)
    onet = cnn.Net(*[w.copy() for w in net.W])
    oopt = cnn.Adam([w.shape for w in onet.W], lr=f32(lr), beta1=f32(0.9), beta2=f32(0.999), eps=f32(eps))
    for eg, el in pairs:
        lib_eps.train_step(eg)
        cnn.train_step(om, onet, oopt, el, dinv)
    wo = np.concatenate([w.ravel() for w in onet.W])
    wg = lib_eps.get_weights()
    # the update's derivative in g is at most 2 lr / eps per step; the FP32
    # gradient is within 1e-5 |g| (norm-wise) of the oracle's
    tol2 = 3 * 2 * lr * 1e-5 * gnorm / eps + 3 * 2.0 ** -22 * np.abs(wo)
    err2 = np.abs(wg - wo)
    print("train chain: max |W - W_oracle| = %.3g, bound %.3g, update %.3g" %
          (err2.max(), tol2.max(), np.abs(wo - flat).max()))
    assert np.all(err2 <= tol2)
    assert np.abs(wo - flat).max() > 100 * tol2.max()


def test_train_step_dinv_cache_follows_mesh_and_coefficients(mp):
    # the training Jacobi diagonal is rebuilt whenever the mesh or h1, h2
    # differ from what the buffer holds, including after sem_smoother_apply or
    # sem_smoother_loss_grad with other coefficients (which rebuild it too)
    import torch
    om, gm = mp
    net, flat = _net_weights(9, scale3=0.05)
    (eg, el), (eg2, el2) = _fields_f32(om, gm, 2, seed=31)
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    a = sem.Smoother(gm)
    a.set_weights(flat)
    a.train_step(eg, loss, h2=0.0)
    state = a.get_state()
    a.loss_grad(dev(el), 1.0, 0.1)            # rebuilds the buffer for h2 = 0.1
    a.train_step(eg2, loss, h2=0.0)
    la = float(loss.item())
    b = sem.Smoother(gm)
    b.set_state(*state)
    b.train_step(eg2, loss, h2=0.0)
    assert float(loss.item()) == la
    assert np.array_equal(a.get_state()[0], b.get_state()[0])
    # a second mesh of the same size (other vertices): a fresh smoother with
    # the same state on that mesh gives the same step
    spec2 = wl.random_deformed_box(3, 2, 3, 7, seed=5, amp=0.15, periodic=(1, 0, 0),
                                   dirichlet=wl.DIRICHLET_Y_WALLS | 0x30)
    gm2 = sem.Mesh.from_spec(spec2)
    b.set_state(*state)
    b.train_step(eg, loss, h2=0.0)             # buffer now holds gm's diagonal
    b.set_state(*state)
    b.train_step(eg2, loss, h2=0.0, mesh=gm2)
    lb = float(loss.item())
    c = sem.Smoother(gm2)
    c.set_state(*state)
    c.train_step(eg2, loss, h2=0.0)
    assert float(loss.item()) == lb
    assert np.array_equal(b.get_state()[0], c.get_state()[0])


def test_smoother_checkpoint_resume(mp):
    # weights, Adam moments and the step count round-trip: a resumed
    # smoother takes exactly the same next step as the original
    om, gm = mp
    net, flat = _net_weights(10, scale3=0.05)
    pairs = _fields_f32(om, gm, 3, seed=41)
    a = sem.Smoother(gm)
    a.set_weights(flat)
    for eg, _ in pairs[:2]:
        a.train_step(eg)
    st = a.get_state()
    assert st[3] == 2 and np.any(st[1] != 0) and np.any(st[2] != 0)
    b = sem.Smoother(gm)
    b.set_state(*st)
    for x, y in zip(b.get_state(), st):
        assert np.array_equal(np.asarray(x), np.asarray(y))
    a.train_step(pairs[2][0])
    b.train_step(pairs[2][0])
    for x, y in zip(a.get_state(), b.get_state()):
        assert np.array_equal(np.asarray(x), np.asarray(y))


# ---------------------------------------------------------------- learned multigrid


@pytest.fixture(scope="module")
def mpg():
    from oracle import hsmg
    spec = wl.random_deformed_box(3, 2, 3, 7, seed=4, amp=0.15, periodic=(1, 0, 0),
                                  dirichlet=wl.DIRICHLET_Y_WALLS | 0x30)
    om, gm = pair(spec, prepare=sem.SEM_PREP_HSMG)
    return om, gm, hsmg.HSMG(om)


def test_learned_multigrid_apply_matches_oracle(mpg):
    # the learned smoother on the fine level plus the hybrid Schwarz
    # multigrid's middle and coarse levels: the network part within the
    # element-wise rounding bounds of the plain smoother, the coarser levels
    # to the conditioning of their factorisations (1e-10 of their size)
    import torch
    om, gm, pc = mpg
    net, flat = _net_weights(1)
    sm = sem.Smoother(gm)
    sm.set_weights(flat)
    rng = np.random.default_rng(31)
    r = om.rhs(rng.standard_normal(om.shape))
    dinv = om.jacobi_inv()
    cp = pc.coarse_part(r)
    z_ref = cnn.smoother(om, net, r, dinv) + cp
    ref_fine = pc.apply(r, fine=lambda q: cnn.smoother(om, net, q, dinv))
    assert np.allclose(z_ref, ref_fine, rtol=0, atol=1e-14 * np.max(np.abs(z_ref)))
    z = torch.empty(gm.shape, dtype=torch.float64, device="cuda")
    floor = 1e-10 * np.max(np.abs(cp)) + 1e-14 * np.abs(z_ref)
    for fp32, rel in ((True, 1024 * 2.0 ** -24), (False, 2.0 ** -6 + 1024 * 2.0 ** -24)):
        sm.mg_apply(dev(r), z, fp32=fp32)
        zh = host(z)
        bound = _abs_net_bound(om, net, r, dinv, rel) + floor
        err = np.abs(zh - z_ref)
        print("learned multigrid (%s network): max error / bound = %.3g" %
              ("FP32" if fp32 else "BF16", np.max(err / np.maximum(bound, 1e-300))))
        assert np.all(err <= bound)
        assert np.array_equal(zh, om.gather_global(zh)[om.glo])
        assert np.all(zh[om.mask == 1] == 0)
    # zero network: Jacobi on the fine level
    zero = flat.copy()
    zero[864 + 6912:] = 0
    sm.set_weights(zero)
    sm.mg_apply(dev(r), z)
    assert np.allclose(host(z), dinv * r + cp, rtol=0, atol=1e-10 * np.max(np.abs(dinv * r + cp)))


@pytest.mark.parametrize("which", ["zero", "random"])
def test_gmres_learned_multigrid_matches_oracle(mpg, which):
    import torch
    from oracle import hsmg
    om, gm, pc = mpg
    net, flat = _net_weights(5, scale3=0.0 if which == "zero" else 0.05)
    sm = sem.Smoother(gm)
    sm.set_weights(flat)
    dinv = om.jacobi_inv()
    rng = np.random.default_rng(32)
    b = om.rhs(rng.standard_normal(om.shape))
    xo, info = hsmg.fgmres(om, b, lambda q: pc.apply(q, fine=lambda t: cnn.smoother(om, net, t, dinv)),
                           tol=1e-10, restart=30)
    x = torch.zeros(gm.shape, dtype=torch.float64, device="cuda")
    rep = gm.pcg_solve(dev(b), x, form=sem.FORM_GMRES_LEARNED_MG, smoother=sm, restart=30)
    true_rel = _true_rel(om, b, host(x))
    _, pinfo = om.pcg(b)
    print("%s network: learned-multigrid GMRES %d iterations (oracle %d), Jacobi-PCG %d, true rel res %.2e" %
          (which, rep.iterations, info["iterations"], pinfo["iterations"], true_rel))
    assert true_rel <= 1.05e-10
    assert abs(rep.true_rel_res - true_rel) <= 1e-3 * true_rel + 2e-13
    # zero network: the same linear preconditioner on both sides; a random
    # one runs its middle layer in BF16 on the GPU
    tol = 1 if which == "zero" else max(2, info["iterations"] // 10)
    assert abs(rep.iterations - info["iterations"]) <= tol
    assert rep.iterations < pinfo["iterations"]


@pytest.mark.parametrize("which", ["zero", "random"])
def test_fcg_learned_multigrid_matches_oracle(mpg, which):
    # flexible CG (Polak-Ribiere) with the learned multigrid
    import torch
    om, gm, pc = mpg
    net, flat = _net_weights(6, scale3=0.0 if which == "zero" else 0.05)
    sm = sem.Smoother(gm)
    sm.set_weights(flat)
    rng = np.random.default_rng(34)
    b = om.rhs(rng.standard_normal(om.shape))
    xo, info = cnn.fcg(om, net, b, coarse=lambda q: pc.coarse_part(q))
    x = torch.zeros(gm.shape, dtype=torch.float64, device="cuda")
    rep = gm.pcg_solve(dev(b), x, form=sem.FORM_FCG_LEARNED_MG, smoother=sm, check_every=4)
    true_rel = _true_rel(om, b, host(x))
    _, pinfo = om.pcg(b)
    print("%s network: learned-multigrid FCG %d iterations (oracle %d, fallback at %d), Jacobi-PCG %d, "
          "true rel res %.2e" % (which, rep.iterations, info["iterations"], info["fallback_at"], pinfo["iterations"],
                                 true_rel))
    assert true_rel <= 1.05e-10
    assert rep.fallback_used == (1 if info["fallback_at"] >= 0 else 0)
    if which == "zero":
        assert rep.iterations < pinfo["iterations"]
        assert abs(rep.iterations - info["iterations"]) <= 1
    elif info["fallback_at"] < 0:
        assert abs(rep.iterations - info["iterations"]) <= max(2, info["iterations"] // 10)
    # (an untrained network makes flexible CG with one stored direction
    # stagnate until (r, z) <= 0 hands over to Jacobi-PCG; the iterations
    # after that depend on the state at the switch, which the BF16 and FP64
    # networks reach differently)


@pytest.mark.parametrize("h2", [0.0, 0.1])
def test_mg_context_loss_gradient(mpg, h2):
    # training in the multigrid context: the loss of M(r) + C(r), C the
    # coarser levels' part, and its FP32 gradient against the oracle
    om, gm, pc = mpg
    from tests import brute
    net, flat = _net_weights(3, scale3=0.1)
    sm = sem.Smoother(gm, mg_context=True)
    sm.set_weights(flat)
    rng = np.random.default_rng(33)
    e = brute.continuous_random(om, rng)
    r = om.apply_S(e, 1.0, h2)
    L_ref, g_ref = cnn.loss_and_grad(om, net, r, e, om.jacobi_inv(1.0, h2), 1.0, h2, extra=pc.coarse_part(r, 1.0, h2))
    L, g = sm.loss_grad(dev(e), 1.0, h2)
    gr = np.concatenate([x.ravel() for x in g_ref])
    print("multigrid-context loss %.6f (oracle %.6f), gradient norm-wise relative error %.3g" %
          (L, L_ref, np.linalg.norm(g - gr) / np.linalg.norm(gr)))
    assert abs(L - L_ref) <= 1e-5 * abs(L_ref)
    assert np.linalg.norm(g - gr) <= 1e-5 * np.linalg.norm(gr)


def test_learned_multigrid_argument_checks(mp, mpg):
    import torch
    om, gm = mp
    _, gmh, _ = mpg
    with pytest.raises(sem.SemError):
        sem.Smoother(gm, mg_context=True)            # mesh without SEM_PREP_HSMG
    sm = sem.Smoother(gm)
    b = torch.ones(gm.shape, dtype=torch.float64, device="cuda")
    x = torch.zeros_like(b)
    with pytest.raises(sem.SemError):
        gm.pcg_solve(b, x, form=sem.FORM_GMRES_LEARNED_MG, smoother=sm)
    with pytest.raises(sem.SemError):
        gmh.pcg_solve(b, x, form=sem.FORM_GMRES_LEARNED_MG)    # no smoother
    smh = sem.Smoother(gmh)
    with pytest.raises(sem.SemError):
        smh.mg_apply(b, x, h1=0.0)
    with pytest.raises(sem.SemError):
        sm.mg_apply(b, x)                             # mesh without SEM_PREP_HSMG
