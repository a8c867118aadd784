"""GPU parity of the learned smoother against the FP64 oracle (oracle/cnn.py):
FP32 path within 1e-5 (forward) / 1e-4 (gradient, norm-wise), BF16 inference
path within 2e-2 (norm-wise, on the learned correction); flexible CG reaches
the FP64 true residual 1e-10 in every mode, equals Jacobi-PCG for the zero
network, and falls back on a broken network; snapshot errors and training."""
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
    sm.apply(dev(r), z, fp32=False)
    zb = host(z)
    assert np.linalg.norm((zb - dinv * r) - corr_ref) <= 2e-2 * np.linalg.norm(corr_ref)
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
    assert np.linalg.norm(g - gr) <= 1e-4 * np.linalg.norm(gr)
    for lo, hi in ((0, 864), (864, 864 + 6912), (864 + 6912, 8208)):
        assert np.linalg.norm(g[lo:hi] - gr[lo:hi]) <= 1e-4 * np.linalg.norm(gr[lo:hi])


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
