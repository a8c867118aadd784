"""Pins for the oracle's learned smoother: convolution against brute force
and a delta-kernel closed form, adjoint identities, finite-difference
gradients of the A-norm loss, positive homogeneity, the zero network being
Jacobi, and flexible CG (= Jacobi-PCG for the zero network, fallback paths)."""
import itertools

import numpy as np
import pytest

import oracle
from oracle import cnn
from paper_2405_05640_amd import workloads as wl
from tests import brute


def _mesh(spec):
    return oracle.Mesh(spec.nelx, spec.nely, spec.nelz, spec.order, spec.vertices,
                       spec.periodic, spec.dirichlet)


def test_conv3d_brute_force():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((2, 3, 4, 4, 4))
    W = rng.standard_normal((5, 3, 3, 3, 3))
    out = cnn.conv3d(x, W)
    ref = np.zeros_like(out)
    n = 4
    for e, o, k, j, i in itertools.product(range(2), range(5), range(n), range(n), range(n)):
        s = 0.0
        for c, a, b, d in itertools.product(range(3), range(3), range(3), range(3)):
            kk, jj, ii = k + a - 1, j + b - 1, i + d - 1
            if 0 <= kk < n and 0 <= jj < n and 0 <= ii < n:
                s += W[o, c, a, b, d] * x[e, c, kk, jj, ii]
        ref[e, o, k, j, i] = s
    assert np.max(np.abs(out - ref)) < 1e-12


def test_delta_kernel_is_channel_mixing():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((3, 2, 8, 8, 8))
    W = np.zeros((4, 2, 3, 3, 3))
    M = rng.standard_normal((4, 2))
    W[:, :, 1, 1, 1] = M
    assert np.allclose(cnn.conv3d(x, W), np.einsum("oc,ecxyz->eoxyz", M, x), rtol=0, atol=1e-14)


def test_conv_adjoints():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((2, 3, 5, 5, 5))
    W = rng.standard_normal((4, 3, 3, 3, 3))
    g = rng.standard_normal((2, 4, 5, 5, 5))
    lhs = np.sum(cnn.conv3d(x, W) * g)
    assert abs(lhs - np.sum(x * cnn.conv3d_grad_input(g, W))) < 1e-10 * abs(lhs)
    assert abs(lhs - np.sum(W * cnn.conv3d_grad_weight(x, g))) < 1e-10 * abs(lhs)


def _pair(m, rng, h2=0.0):
    e = brute.continuous_random(m, rng)
    r = m.apply_S(e, 1.0, h2)
    return r, e


def test_zero_net_is_jacobi_and_homogeneity():
    m = _mesh(wl.deformed_cube(2, 7, amp=0.2))
    rng = np.random.default_rng(3)
    r, _ = _pair(m, rng)
    dinv = m.jacobi_inv()
    z0 = cnn.smoother(m, cnn.Net.init(16, seed=0), r, dinv)
    assert np.array_equal(z0, dinv * r)
    net = cnn.Net.init(16, seed=1)
    net.W[2] = rng.standard_normal(net.W[2].shape) * 0.05
    z = cnn.smoother(m, net, r, dinv)
    assert np.array_equal(cnn.smoother(m, net, 2.0 * r, dinv), 2.0 * z)
    assert np.array_equal(cnn.smoother(m, net, 0.25 * r, dinv), 0.25 * z)
    # continuity and mask of the smoother output
    assert np.array_equal(z, m.gather_global(z)[m.glo])
    assert np.all(z[m.mask == 1] == 0)


@pytest.mark.parametrize("h2,with_extra", [(0.0, False), (0.1, False), (0.1, True)])
def test_loss_gradient_matches_finite_differences(h2, with_extra):
    # with_extra: the in-context loss of the learned multigrid, where a fixed
    # coarser-level field is added to the smoother output
    m = _mesh(wl.deformed_cube(2, 7, amp=0.2))
    rng = np.random.default_rng(4)
    net = cnn.Net.init(4, seed=2)
    net.W[2] = rng.standard_normal(net.W[2].shape) * 0.1
    r, e = _pair(m, rng, h2)
    dinv = m.jacobi_inv(1.0, h2)
    extra = None
    if with_extra:
        extra = brute.continuous_random(m, rng) * 0.3 * np.max(np.abs(e))
    L, grads = cnn.loss_and_grad(m, net, r, e, dinv, 1.0, h2, extra=extra)
    assert 0 < L
    if with_extra:
        L0, g0 = cnn.loss_and_grad(m, net, r, e, dinv, 1.0, h2)
        assert L != L0 and not np.allclose(grads[1], g0[1])
    h = 1e-6
    picks = [(0, (1, 0, 1, 1, 1)), (0, (3, 1, 0, 2, 1)), (1, (2, 3, 1, 1, 0)), (1, (0, 0, 2, 2, 2)),
             (2, (0, 1, 1, 1, 1)), (2, (0, 3, 0, 1, 2))]
    for layer, idx in picks:
        W0 = net.W[layer][idx]
        net.W[layer][idx] = W0 + h
        Lp, _ = cnn.loss_and_grad(m, net, r, e, dinv, 1.0, h2, extra=extra)
        net.W[layer][idx] = W0 - h
        Lm, _ = cnn.loss_and_grad(m, net, r, e, dinv, 1.0, h2, extra=extra)
        net.W[layer][idx] = W0
        fd = (Lp - Lm) / (2 * h)
        g = grads[layer][idx]
        assert abs(fd - g) <= 1e-6 * max(abs(g), 1e-3 * np.max(np.abs(grads[layer]))), (layer, idx, fd, g)


def test_fcg_zero_net_equals_pcg():
    m = _mesh(wl.deformed_cube(3, 5, amp=0.2))
    rng = np.random.default_rng(5)
    b = m.rhs(rng.standard_normal(m.shape))
    x, info = cnn.fcg(m, cnn.Net.init(16, seed=0), b, 1.0, 0.1)
    xo, io = m.pcg(b, 1.0, 0.1)
    assert abs(info["iterations"] - io["iterations"]) <= 2
    r = b - m.apply_S(x, 1.0, 0.1)
    assert np.sqrt(m.dot(r, r) / m.dot(b, b)) <= 1.05e-10


def test_fcg_fallback_paths_converge():
    m = _mesh(wl.deformed_cube(3, 5, amp=0.2))
    rng = np.random.default_rng(6)
    b = m.rhs(rng.standard_normal(m.shape))
    net = cnn.Net.init(8, seed=3)
    net.W[2] = rng.standard_normal(net.W[2].shape) * 0.05
    for kw in ({}, {"force_fallback_at": 7}):
        x, info = cnn.fcg(m, net, b, 1.0, 0.0, **kw)
        r = b - m.apply_S(x, 1.0, 0.0)
        assert np.sqrt(m.dot(r, r) / m.dot(b, b)) <= 1.05e-10
        if kw:
            assert info["fallback_at"] == 7
    bad = cnn.Net.init(8, seed=3)
    bad.W[2][:] = np.nan
    x, info = cnn.fcg(m, bad, b, 1.0, 0.0)
    assert info["fallback_at"] == 0
    r = b - m.apply_S(x, 1.0, 0.0)
    assert np.sqrt(m.dot(r, r) / m.dot(b, b)) <= 1.05e-10


def test_bf16_rounding_and_lowp_operator_bounds():
    from oracle import mixed
    # rounding: exact values stay, ties go to even, relative error <= 2^-9
    v = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 2 ** -7, 3.0, -2.5], dtype=np.float32)
    r = mixed.bf16_round(v)
    assert r[0] == 1.0 and r[1] == 1.0 and r[2] == 1.0 + 2 ** -7 and r[3] == 3.0 and r[4] == -2.5
    rng = np.random.default_rng(0)
    x = rng.standard_normal(10000).astype(np.float32)
    assert np.max(np.abs(mixed.bf16_round(x) - x) / np.abs(x)) <= 2 ** -8   # unit roundoff (8-bit significand)
    m = _mesh(wl.deformed_cube(2, 7, amp=0.2))
    u = rng.standard_normal(m.shape)
    w64 = m.ax(u, 1.0, 0.1)
    bound = m.ax_abs_bound(u, 1.0, 0.1)
    c = 3 * (m.N + 1) + 6
    for prec, eps in (("f32", 2.0 ** -24), ("bf16", 2.0 ** -8)):
        w = mixed.ax_lowp(m, u, 1.0, 0.1, prec)
        assert np.all(np.abs(w - w64) <= c * eps * bound + 1e-30), prec
    # bf16 is really coarser than f32
    e16 = np.linalg.norm(mixed.ax_lowp(m, u, 1.0, 0.1, "bf16") - w64)
    e32 = np.linalg.norm(mixed.ax_lowp(m, u, 1.0, 0.1, "f32") - w64)
    assert e16 > 100 * e32


def _half_grid_neighbours(y):
    """The two IEEE half grid points around each |y| (y below 65504), built
    from the format's definition: spacing 2^(e-10) in the binade [2^e, 2^(e+1)),
    2^-24 below 2^-14."""
    a = np.abs(y)
    _, x = np.frexp(a)
    spacing = np.ldexp(1.0, np.maximum(x - 11, -24))
    lo = np.floor(a / spacing) * spacing
    return lo, lo + spacing, spacing


def test_f16_scaled_storage_rounds_to_nearest_half():
    # the split operator's G and B storage: per element a power-of-two scale
    # that puts the largest magnitude in [2^14, 2^15), then round to nearest
    # half (ties to even) straight from float64.  Checked against the two
    # neighbouring grid points of every value (brute force over the format),
    # including double-rounding cases that a float32 detour would get wrong
    from oracle import mixed
    rng = np.random.default_rng(11)
    a = rng.standard_normal((5, 3, 40)) * np.logspace(-6, 2, 5)[:, None, None]
    a[1, 0, 0] = 0.0
    a[2, 1, :3] = [1e-12, -3e-13, 2e-9]           # below the element's half normal range
    a[4] = 0.0                                    # an element of zeros
    k = mixed.f16_scale_exponents(a, 0)
    for e in range(5):
        m = np.max(np.abs(a[e]))
        if m == 0:
            assert k[e] == 0
        else:
            assert 2.0 ** 14 <= m / 2.0 ** k[e] < 2.0 ** 15
    st = mixed.f16_scaled_storage(a, 0)
    y = a / 2.0 ** k[:, None, None]
    ys = st / 2.0 ** k[:, None, None]
    lo, hi, sp = _half_grid_neighbours(y)
    ay = np.abs(y)
    near = np.where(ay - lo < hi - ay, lo, np.where(ay - lo > hi - ay, hi,
                    np.where(np.mod(lo / sp, 2) == 0, lo, hi)))   # ties to the even significand
    assert np.array_equal(np.abs(ys), near)
    assert np.all(np.sign(ys) * np.sign(y) >= 0)
    # double rounding: 1 + 2^-11 + 2^-40 must go up; 1 + 2^-11 is a tie to 1
    b = np.array([[1 + 2.0 ** -11 + 2.0 ** -40, 1 + 2.0 ** -11, 2.0 ** 14]])
    sb = mixed.f16_scaled_storage(b, 0) / 2.0 ** mixed.f16_scale_exponents(b, 0)[0]
    assert np.array_equal(sb, [[1 + 2.0 ** -10, 1.0, 2.0 ** 14]])
    # relative error of a normal value: at most 2^-11
    normal = ay >= 2.0 ** -14
    assert np.all(np.abs(ys - y)[normal] <= 2.0 ** -11 * ay[normal])


def test_f16_storage_reference_operator():
    # the split-BF16 operator's reference: the exact operator with G and B in
    # the scaled half storage.  The operator stays symmetric and differs from
    # the FP64 one by at most the storage rounding (2^-11 relative, plus a
    # 2^-39-of-the-largest floor for values below the half normal range)
    from oracle import mixed
    m = _mesh(wl.deformed_cube(2, 7, amp=0.2))
    Gh = mixed.f16_scaled_storage(m.G, 1)
    Bh = mixed.f16_scaled_storage(m.B, 0)
    gmax = np.max(np.abs(m.G), axis=(0, 2, 3, 4))[None, :, None, None, None]
    assert np.all(np.abs(Gh - m.G) <= 2.0 ** -11 * np.abs(m.G) + 2.0 ** -39 * gmax)
    assert np.all(np.abs(Bh - m.B) <= 2.0 ** -11 * m.B)
    rng = np.random.default_rng(3)
    u, v = rng.standard_normal(m.shape), rng.standard_normal(m.shape)
    au = mixed.ax_bf16_split_reference(m, u, 1.0, 0.1)
    av = mixed.ax_bf16_split_reference(m, v, 1.0, 0.1)
    assert abs(np.sum(v * au) - np.sum(u * av)) <= 1e-12 * np.sum(np.abs(v * au))
    w64 = m.ax(u, 1.0, 0.1)
    assert np.all(np.abs(au - w64) <= 2.0 ** -11 * m.ax_abs_bound(u, 1.0, 0.1) + 1e-30)
    assert np.linalg.norm(au - w64) > 0.0


def test_bf16_storage_reference_operator():
    # the exact operator with G and B rounded to BF16 (the plain BF16
    # operator's storage).  Rounding is idempotent, the operator stays
    # symmetric (G12, G13, G23 are shared by both of their uses), and it
    # differs from the FP64 operator by at most the storage rounding
    from oracle import mixed
    m = _mesh(wl.deformed_cube(2, 7, amp=0.2))
    Gb = mixed.bf16_storage(m.G)
    Bb = mixed.bf16_storage(m.B)
    assert np.array_equal(mixed.bf16_storage(Gb), Gb)
    assert np.all(np.abs(Gb - m.G) <= 2.0 ** -8 * np.abs(m.G) + 1e-37)   # float32 underflow of ~0 entries
    rng = np.random.default_rng(3)
    u, v = rng.standard_normal(m.shape), rng.standard_normal(m.shape)
    au = m.ax(u, 1.0, 0.1, G=Gb, B=Bb)
    av = m.ax(v, 1.0, 0.1, G=Gb, B=Bb)
    assert abs(np.sum(v * au) - np.sum(u * av)) <= 1e-12 * np.sum(np.abs(v * au))
    w64 = m.ax(u, 1.0, 0.1)
    assert np.all(np.abs(au - w64) <= 2.0 ** -8 * m.ax_abs_bound(u, 1.0, 0.1) + 1e-30)
    assert np.linalg.norm(au - w64) > 0.0


# ---------------------------------------------------------------- Adam

def _adam_run(grads, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8, W0=None):
    shape = np.shape(grads[0])
    opt = cnn.Adam([shape], lr, b1, b2, eps)
    W = [np.zeros(shape) if W0 is None else np.array(W0, dtype=np.float64)]
    out = []
    for g in grads:
        W = opt.step(W, [g])
        out.append(W[0].copy())
    return out, opt


def test_adam_first_step_closed_form():
    # bias correction makes the first estimates m_hat = g, v_hat = g^2, so the
    # first step is -lr g / (|g| + eps) in every component (a sign step for
    # |g| >> eps), whatever beta1 and beta2 are
    rng = np.random.default_rng(0)
    g = rng.standard_normal(50) * np.logspace(-10, 2, 50)
    g[3] = 0.0
    W0 = rng.standard_normal(50)
    for b1, b2 in ((0.9, 0.999), (0.5, 0.7)):
        (W1,), _ = _adam_run([g], lr=2e-3, b1=b1, b2=b2, eps=1e-8, W0=W0)
        assert np.allclose(W1, W0 - 2e-3 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    assert W1[3] == W0[3]


def test_adam_constant_gradient_closed_form():
    # a constant gradient g gives m_t = (1 - b1^t) g and v_t = (1 - b2^t) g^2
    # (geometric sums), so every bias-corrected step is the first one again:
    # W_k = W_0 - k lr g / (|g| + eps).  Missing or wrong bias corrections
    # break this from step 2 on.
    rng = np.random.default_rng(1)
    g = rng.standard_normal(20)
    Ws, _ = _adam_run([g] * 7, lr=1e-2, eps=1e-8)
    for k, W in enumerate(Ws, start=1):
        assert np.allclose(W, -k * 1e-2 * g / (np.abs(g) + 1e-8), rtol=1e-13, atol=0)


def test_adam_impulse_closed_form():
    # gradient g at step 1, then zeros: m_k = b1^(k-1) (1 - b1) g and
    # v_k = b2^(k-1) (1 - b2) g^2, so step k moves by
    # lr a_k g / (sqrt(c_k) |g| + eps) with a_k = b1^(k-1)(1-b1)/(1-b1^k) and
    # c_k = b2^(k-1)(1-b2)/(1-b2^k).  Tells beta1 from beta2 (a swap fails).
    g = np.array([0.3, -2.0, 1e-3])
    b1, b2, lr, eps = 0.9, 0.99, 1e-3, 1e-8
    Ws, opt = _adam_run([g] + [np.zeros(3)] * 5, lr=lr, b1=b1, b2=b2, eps=eps)
    W = np.zeros(3)
    for k in range(1, 7):
        a = b1 ** (k - 1) * (1 - b1) / (1 - b1 ** k)
        c = b2 ** (k - 1) * (1 - b2) / (1 - b2 ** k)
        W = W - lr * a * g / (np.sqrt(c) * np.abs(g) + eps)
        assert np.allclose(Ws[k - 1], W, rtol=1e-12, atol=0)
    assert opt.t == 6
    assert np.allclose(opt.m[0], b1 ** 5 * (1 - b1) * g, rtol=1e-14)
    assert np.allclose(opt.v[0], b2 ** 5 * (1 - b2) * g * g, rtol=1e-14)
    swapped, _ = _adam_run([g] + [np.zeros(3)] * 5, lr=lr, b1=b2, b2=b1, eps=eps)
    assert not np.allclose(swapped[-1], Ws[-1], rtol=1e-6)


def test_adam_scale_invariance_without_eps():
    # with eps = 0 the update depends on the gradient sequence only through
    # its direction: scaling every gradient by c > 0 leaves the path unchanged
    rng = np.random.default_rng(2)
    gs = [rng.standard_normal(30) for _ in range(5)]
    a, _ = _adam_run(gs, eps=0.0)
    b, _ = _adam_run([1e4 * g for g in gs], eps=0.0)
    for x, y in zip(a, b):
        assert np.allclose(x, y, rtol=1e-12, atol=1e-18)


def test_train_step_is_loss_grad_then_adam():
    # cnn.train_step = loss and gradient at the current weights (the pinned
    # loss_and_grad), then the pinned Adam update; the loss it returns is the
    # one before the update, and a small step lowers the loss of the same pair
    m = _mesh(wl.random_deformed_box(2, 2, 2, 7, seed=1, amp=0.1))
    rng = np.random.default_rng(3)
    e = brute.continuous_random(m, rng)
    dinv = m.jacobi_inv()
    net = cnn.Net.init(16, seed=0)
    net.W[2] = np.random.default_rng(9).standard_normal(net.W[2].shape) * 0.05
    W0 = [w.copy() for w in net.W]
    L0, g0 = cnn.loss_and_grad(m, net, m.apply_S(e), e, dinv)
    opt = cnn.Adam([w.shape for w in net.W], lr=1e-4)
    L = cnn.train_step(m, net, opt, e, dinv)
    assert L == L0
    ref = cnn.Adam([w.shape for w in W0], lr=1e-4).step(W0, g0)
    for a, b in zip(net.W, ref):
        assert np.array_equal(a, b)
    L1, _ = cnn.loss_and_grad(m, net, m.apply_S(e), e, dinv)
    assert L1 < L0


# ---------------------------------------------------------------- BF16 rounding order

def _rn(x, bits):
    """Round a Fraction to the nearest binary number with `bits` significant
    bits, ties to even (no exponent limits: the values here are moderate)."""
    from fractions import Fraction
    if x == 0:
        return Fraction(0)
    s = -1 if x < 0 else 1
    a = abs(x)
    e = 0
    while a >= 2:
        a /= 2
        e += 1
    while a < 1:
        a *= 2
        e -= 1
    scaled = a * 2 ** (bits - 1)          # in [2^(bits-1), 2^bits)
    q, r = divmod(scaled.numerator, scaled.denominator)
    frac = Fraction(r, scaled.denominator)
    if frac > Fraction(1, 2) or (frac == Fraction(1, 2) and q % 2 == 1):
        q += 1
    return s * Fraction(q) * Fraction(2) ** (e - (bits - 1))


def test_bf16_operator_rounding_sequence_one_element():
    # The plain BF16 emulation rounds at five places: u, D, G and B to BF16 on
    # entry, and the three G-combination results to BF16 before the
    # transposed contractions; every other operation is one FP32 rounding.
    # On one N = 1 element (two-term contractions, so the FP32 sum order
    # cannot matter) the expected result is evaluated here in exact rational
    # arithmetic with those roundings written out (BF16: 8 significant bits,
    # FP32: 24, nearest-even).  The emulation must match it bit for bit, and
    # leaving out any one of the five roundings must change the result.
    from fractions import Fraction
    from types import SimpleNamespace

    from oracle import mixed
    rng = np.random.default_rng(5)
    f32 = np.float32
    D = rng.uniform(-1, 1, (2, 2)).astype(f32)
    G = rng.uniform(-1, 1, (6, 1, 2, 2, 2)).astype(f32)
    G[[0, 3, 5]] = np.abs(G[[0, 3, 5]]) + 1
    B = rng.uniform(0.5, 1.5, (1, 2, 2, 2)).astype(f32)
    u = rng.standard_normal((1, 2, 2, 2)).astype(f32)
    h1, h2 = 1.0, 0.5
    fake = SimpleNamespace(D=D.astype(np.float64), G=G.astype(np.float64), B=B.astype(np.float64))
    got = mixed.ax_lowp(fake, u.astype(np.float64), h1, h2, "bf16")

    def expected(skip=()):
        b16 = lambda x: _rn(x, 8)
        r32 = lambda x: _rn(x, 24)
        F = lambda a: Fraction(float(a))
        rd = lambda name, x: x if name in skip else b16(x)
        Dq = [[rd("D", F(D[a, b])) for b in range(2)] for a in range(2)]
        Gq = [[[[rd("G", F(G[c, 0, k, j, i])) for i in range(2)] for j in range(2)] for k in range(2)] for c in range(6)]
        Bq = [[[rd("B", F(B[0, k, j, i])) for i in range(2)] for j in range(2)] for k in range(2)]
        uq = [[[rd("u", F(u[0, k, j, i])) for i in range(2)] for j in range(2)] for k in range(2)]
        idx = [(k, j, i) for k in range(2) for j in range(2) for i in range(2)]
        ur, us, ut = {}, {}, {}
        for (k, j, i) in idx:   # two exact BF16 x BF16 products, one FP32 rounding of the sum
            ur[k, j, i] = r32(sum(Dq[i][m] * uq[k][j][m] for m in range(2)))
            us[k, j, i] = r32(sum(Dq[j][m] * uq[k][m][i] for m in range(2)))
            ut[k, j, i] = r32(sum(Dq[k][m] * uq[m][j][i] for m in range(2)))
        flux = {}
        for name, (a, b, c) in (("r", (0, 1, 2)), ("s", (1, 3, 4)), ("t", (2, 4, 5))):
            for (k, j, i) in idx:   # numpy: ((Ga ur + Gb us) + Gc ut), each op rounded to FP32
                p = r32(r32(r32(Gq[a][k][j][i] * ur[k, j, i]) + r32(Gq[b][k][j][i] * us[k, j, i]))
                        + r32(Gq[c][k][j][i] * ut[k, j, i]))
                flux[name, k, j, i] = p if "comb" in skip else b16(p)
        out = np.zeros((1, 2, 2, 2))
        for (k, j, i) in idx:
            wr = r32(sum(Dq[m][i] * flux["r", k, j, m] for m in range(2)))
            ws = r32(sum(Dq[m][j] * flux["s", k, m, i] for m in range(2)))
            wt = r32(sum(Dq[m][k] * flux["t", m, j, i] for m in range(2)))
            w = r32(r32(wr + ws) + wt)
            helm = r32(r32(Fraction(h2) * Bq[k][j][i]) * uq[k][j][i])
            out[0, k, j, i] = float(r32(r32(Fraction(h1) * w) + helm))
        return out

    ref = expected()
    assert np.array_equal(got, ref)
    for step in ("u", "D", "G", "B", "comb"):
        assert not np.array_equal(expected(skip=(step,)), ref), step
