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


@pytest.mark.parametrize("h2", [0.0, 0.1])
def test_loss_gradient_matches_finite_differences(h2):
    m = _mesh(wl.deformed_cube(2, 7, amp=0.2))
    rng = np.random.default_rng(4)
    net = cnn.Net.init(4, seed=2)
    net.W[2] = rng.standard_normal(net.W[2].shape) * 0.1
    r, e = _pair(m, rng, h2)
    dinv = m.jacobi_inv(1.0, h2)
    L, grads = cnn.loss_and_grad(m, net, r, e, dinv, 1.0, h2)
    assert 0 < L
    h = 1e-6
    picks = [(0, (1, 0, 1, 1, 1)), (0, (3, 1, 0, 2, 1)), (1, (2, 3, 1, 1, 0)), (1, (0, 0, 2, 2, 2)),
             (2, (0, 1, 1, 1, 1)), (2, (0, 3, 0, 1, 2))]
    for layer, idx in picks:
        W0 = net.W[layer][idx]
        net.W[layer][idx] = W0 + h
        Lp, _ = cnn.loss_and_grad(m, net, r, e, dinv, 1.0, h2)
        net.W[layer][idx] = W0 - h
        Lm, _ = cnn.loss_and_grad(m, net, r, e, dinv, 1.0, h2)
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
