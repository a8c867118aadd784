"""FP64 oracle of the learned smoother and of flexible CG (test infrastructure).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The paper itself solves the pressure equation with preconditioned Krylov
methods (section 3.1); a learned per-element smoother inside a flexible CG is
not in the paper.  Every definition below is this project's reading, written
out plainly:

* Per element e the assembled residual r and the Jacobi-scaled residual
  q = dinv o r are taken on the element's (N+1)^3 tile; s_e = max|r_e|,
  t_e = max|q_e|.  The network input is X_e = [r_e / s_e, q_e / t_e]
  (2 channels); an element with s_e = 0 or t_e = 0 gets c_e = 0.
* Net: three 3x3x3 convolutions (cross-correlation, stride 1, zero padding 1,
  no bias), 2 -> C -> C -> 1 channels, ReLU after the first two.
* c_e = t_e Net(X_e); the smoother is
      M(r) = dinv o r + mask(Q^T (c / mult))
  i.e. the element outputs are averaged over the copies of every node.  A
  zero network gives exactly Jacobi, and M(a r) = a M(r) for a > 0.
* Loss of one pair (r, e) with e the error that r belongs to (S e = r):
      L = ||e - M(r)||_S^2 / ||e||_S^2,
  or, trained in the context of the learned multigrid, with M(r) + C(r) in
  place of M(r), C the fixed coarser-level part,
  dL/dz = -2 S (e - M(r)) / ||e||_S^2 (z = M(r)), and
  dL/dc_l = dL/dz_{glo(l)} / mult_l on free nodes.
* Training updates the weights with Adam (Kingma & Ba 2015): with gradient
  g at step t (t = 1, 2, ...), m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
  W -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps); moments start at 0.
* Flexible CG (Notay 2000; Golub & Ye 1999): CG with z_k = M(r_k) and the
  Polak-Ribiere coefficient beta = (z_k, r_k - r_{k-1}) / (z_{k-1}, r_{k-1}).
  Fallback: on a non-finite value, (r, z) <= 0, or a residual reduction over
  `window` iterations worse than rho^window, the solve continues as plain
  Jacobi-PCG from the current iterate.

Vectors here are local-form continuous fields (all copies equal), as in the
rest of the oracle; conv tensors are [E][C][k][j][i].
"""
from __future__ import annotations

import numpy as np

OFFSETS = [(dk, dj, di) for dk in (-1, 0, 1) for dj in (-1, 0, 1) for di in (-1, 0, 1)]


def _pad(a):
    return np.pad(a, ((0, 0), (0, 0), (1, 1), (1, 1), (1, 1)))


def conv3d(x, W):
    """out[e,o,k,j,i] = sum_c sum_off W[o,c,off] x[e,c,k+dk,j+dj,i+di] (zero outside)."""
    E, C, n = x.shape[0], x.shape[1], x.shape[2]
    O = W.shape[0]
    xp = _pad(x)
    out = np.zeros((E, O, n, n, n))
    for (dk, dj, di) in OFFSETS:
        sl = xp[:, :, 1 + dk:1 + dk + n, 1 + dj:1 + dj + n, 1 + di:1 + di + n]
        out += np.einsum("oc,ecxyz->eoxyz", W[:, :, dk + 1, dj + 1, di + 1], sl)
    return out


def conv3d_grad_input(g, W):
    """Adjoint of conv3d in its input: dx[e,c,p] = sum_o sum_off W[o,c,off] g[e,o,p-off]."""
    E, O, n = g.shape[0], g.shape[1], g.shape[2]
    C = W.shape[1]
    gp = _pad(g)
    dx = np.zeros((E, C, n, n, n))
    for (dk, dj, di) in OFFSETS:
        sl = gp[:, :, 1 - dk:1 - dk + n, 1 - dj:1 - dj + n, 1 - di:1 - di + n]
        dx += np.einsum("oc,eoxyz->ecxyz", W[:, :, dk + 1, dj + 1, di + 1], sl)
    return dx


def conv3d_grad_weight(x, g):
    """dW[o,c,off] = sum_e sum_p g[e,o,p] x[e,c,p+off]."""
    n = x.shape[2]
    xp = _pad(x)
    dW = np.zeros((g.shape[1], x.shape[1], 3, 3, 3))
    for (dk, dj, di) in OFFSETS:
        sl = xp[:, :, 1 + dk:1 + dk + n, 1 + dj:1 + dj + n, 1 + di:1 + di + n]
        dW[:, :, dk + 1, dj + 1, di + 1] = np.einsum("eoxyz,ecxyz->oc", g, sl)
    return dW


class Net:
    """Weights W1 (C,2,3,3,3), W2 (C,C,3,3,3), W3 (1,C,3,3,3)."""

    def __init__(self, W1, W2, W3):
        self.W = [np.asarray(W1, dtype=np.float64), np.asarray(W2, dtype=np.float64),
                  np.asarray(W3, dtype=np.float64)]

    @classmethod
    def init(cls, channels=16, seed=0):
        """He-normal layers 1 and 2 (fan-in 27 C_in), zero last layer."""
        rng = np.random.default_rng(seed)
        W1 = rng.standard_normal((channels, 2, 3, 3, 3)) * np.sqrt(2.0 / (27 * 2))
        W2 = rng.standard_normal((channels, channels, 3, 3, 3)) * np.sqrt(2.0 / (27 * channels))
        W3 = np.zeros((1, channels, 3, 3, 3))
        return cls(W1, W2, W3)

    def forward(self, X, keep=False):
        A1 = conv3d(X, self.W[0])
        Y1 = np.maximum(A1, 0.0)
        A2 = conv3d(Y1, self.W[1])
        Y2 = np.maximum(A2, 0.0)
        Y3 = conv3d(Y2, self.W[2])
        if keep:
            return Y3, (X, Y1, Y2)
        return Y3

    def backward(self, cache, g3):
        """Gradients of sum(g3 * Y3) w.r.t. the three weight tensors."""
        X, Y1, Y2 = cache
        dW3 = conv3d_grad_weight(Y2, g3)
        g2 = conv3d_grad_input(g3, self.W[2]) * (Y2 > 0)
        dW2 = conv3d_grad_weight(Y1, g2)
        g1 = conv3d_grad_input(g2, self.W[1]) * (Y1 > 0)
        dW1 = conv3d_grad_weight(X, g1)
        return [dW1, dW2, dW3]


def features(r, dinv):
    """Per-element input X, and the scales s, t (local-form r, dinv)."""
    E = r.shape[0]
    q = dinv * r
    s = np.max(np.abs(r.reshape(E, -1)), axis=1)
    t = np.max(np.abs(q.reshape(E, -1)), axis=1)
    live = (s > 0) & (t > 0)
    X = np.zeros((E, 2) + r.shape[1:])
    X[live, 0] = r[live] / s[live, None, None, None]
    X[live, 1] = q[live] / t[live, None, None, None]
    return X, s, t, live


def smoother(mesh, net, r, dinv, keep=False):
    """z = M(r) (local form).  dinv: the oracle's Jacobi inverse (1 on masked
    nodes); r is masked, so dinv o r is 0 there."""
    X, s, t, live = features(r, dinv)
    Y3, cache = net.forward(X, keep=True)
    c = t[:, None, None, None] * Y3[:, 0]
    c[~live] = 0.0
    corr = mesh.apply_mask(mesh.dssum(c / mesh.mult))
    z = dinv * r + corr
    if keep:
        return z, (cache, t, live)
    return z


def loss_and_grad(mesh, net, r, e, dinv, h1=1.0, h2=0.0, extra=None):
    """A-norm loss of one (r, e) pair and its weight gradients.  extra: a
    fixed field added to the smoother output before the loss (training in
    context: the coarser levels' part of the learned multigrid, so that the
    network learns what those levels leave over)."""
    z, (cache, t, live) = smoother(mesh, net, r, dinv, keep=True)
    if extra is not None:
        z = z + extra
    Se = mesh.apply_S(e, h1, h2)
    en = mesh.dot(e, Se)
    d = e - z
    Sd = mesh.apply_S(d, h1, h2)
    L = mesh.dot(d, Sd) / en
    # dL/dz_g = -2 (S d)_g / en; dL/dc_l = dL/dz_glo(l) / mult_l (0 on masked)
    gz = -2.0 * Sd / en
    gc = np.where(mesh.mask == 1, 0.0, gz / mesh.mult)
    g3 = (t[:, None, None, None] * gc)[:, None]
    g3[~live] = 0.0
    grads = net.backward(cache, g3)
    return L, grads


class Adam:
    """Adam optimiser state over a list of arrays (Kingma & Ba 2015,
    Algorithm 1), in FP64: first and second moment estimates, bias-corrected
    by 1 - beta^t at step t."""

    def __init__(self, shapes, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps = float(lr), float(beta1), float(beta2), float(eps)
        self.m = [np.zeros(sh) for sh in shapes]
        self.v = [np.zeros(sh) for sh in shapes]
        self.t = 0

    def step(self, params, grads):
        """Returns the updated parameters (new arrays)."""
        self.t += 1
        out = []
        for q, (W, g) in enumerate(zip(params, grads)):
            g = np.asarray(g, dtype=np.float64)
            self.m[q] = self.b1 * self.m[q] + (1.0 - self.b1) * g
            self.v[q] = self.b2 * self.v[q] + (1.0 - self.b2) * g * g
            m_hat = self.m[q] / (1.0 - self.b1 ** self.t)
            v_hat = self.v[q] / (1.0 - self.b2 ** self.t)
            out.append(np.asarray(W, dtype=np.float64) - self.lr * m_hat / (np.sqrt(v_hat) + self.eps))
        return out


def train_step(mesh, net, opt, e, dinv, h1=1.0, h2=0.0):
    """One training step on the pair (S e, e): loss and gradient at the
    current weights, then an Adam update of net.W in place.  Returns the loss
    before the update."""
    r = mesh.apply_S(e, h1, h2)
    L, grads = loss_and_grad(mesh, net, r, e, dinv, h1, h2)
    net.W = opt.step(net.W, grads)
    return L


def fcg(mesh, net, b, h1=1.0, h2=0.0, tol=1e-10, max_iter=20000, window=25, rho=None,
        force_fallback_at=None, coarse=None):
    """Flexible CG with the learned smoother; Jacobi-PCG fallback.
    Returns (x, info).  `rho`: per-iteration residual reduction rate of plain
    Jacobi-PCG used by the stall test (None disables it).  coarse: a callable
    r -> C(r) added to the smoother output (the learned multigrid's middle
    and coarse levels); the fallback is plain Jacobi-PCG either way."""
    dinv = mesh.jacobi_inv(h1, h2)

    def learned(q):
        z = smoother(mesh, net, q, dinv)
        return z if coarse is None else z + coarse(q)

    x = np.zeros(mesh.shape)
    bn = np.sqrt(mesh.dot(b, b))
    info = {"iterations": 0, "fallback_at": -1, "status": 0}
    if bn == 0.0:
        return x, info
    r = b.copy()
    use_net = True
    z = learned(r)
    rz = mesh.dot(r, z)
    if not (rz > 0) or not np.isfinite(rz):
        use_net = False
        info["fallback_at"] = 0
        z = dinv * r
        rz = mesh.dot(r, z)
    p = z.copy()
    hist = [1.0]
    it = 0
    while it < max_iter:
        w = mesh.apply_S(p, h1, h2)
        pw = mesh.dot(p, w)
        if not (pw > 0) or not np.isfinite(pw):
            info["status"] = 2
            break
        alpha = rz / pw
        x = x + alpha * p
        r_old = r
        r = r - alpha * w
        it += 1
        rel = np.sqrt(mesh.dot(r, r)) / bn
        hist.append(rel)
        if rel <= tol:
            break
        stall = False
        if use_net and rho is not None and it >= window and hist[-1] > hist[-1 - window] * rho ** window:
            stall = True
        if use_net and force_fallback_at is not None and it == force_fallback_at:
            stall = True
        if use_net and not stall:
            zn = learned(r)
            rzn = mesh.dot(r, zn)
            if not (rzn > 0) or not np.isfinite(rzn):
                stall = True
        if stall:
            use_net = False
            info["fallback_at"] = it
            zn = dinv * r
            rzn = mesh.dot(r, zn)
            beta = 0.0   # restart the search direction
        elif use_net:
            beta = mesh.dot(zn, r - r_old) / rz
        else:
            zn = dinv * r
            rzn = mesh.dot(r, zn)
            beta = rzn / rz
        rz = rzn
        p = zn + beta * p
    info["iterations"] = it
    info["history"] = np.array(hist)
    return x, info
