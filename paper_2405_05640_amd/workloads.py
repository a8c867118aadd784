"""Seeded synthetic inputs: mesh vertices, boundary flags and right-hand sides.

This module is the only thing the HIP path and the CPU oracle share.  It holds
none of the method's arithmetic (no GLL points, no geometry, no operator): it
produces element-vertex lattices and evaluates closed-form source fields at
point coordinates handed to it by the caller.

The paper's workloads (Table 1: turbulent pipe, Taylor-Green vortex,
Rayleigh-Benard convection, all at N = 7) use mesh files that are not
available; these synthetic stand-ins keep their structure:

* ``cube``      -- uniform hexahedra on [0,1]^3, Dirichlet on all faces
                   (manufactured solution sin(pi x) sin(pi y) sin(pi z));
* ``deformed``  -- the same cube with every vertex displaced by
                   0.05 h sin(2 pi .) sin(2 pi .) (cyclic in x, y, z);
* ``channel``   -- aspect-ratio-1 box, periodic in x and z, walls at y = 0, 1
                   with tanh stretching toward the walls (the RBC case's
                   periodic-sided, walled cube of section 3.2);
* right-hand sides: random Fourier series with Gaussian amplitudes (k <= 8),
  and velocity-like k^-5/3 fields whose divergence is the pressure source,
  advected by a uniform shift per time index.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

DIRICHLET_ALL = 0x3F          # bits 0..5 = x-, x+, y-, y+, z-, z+
DIRICHLET_Y_WALLS = 0x0C      # y- and y+


@dataclass(frozen=True)
class MeshSpec:
    nelx: int
    nely: int
    nelz: int
    order: int
    vertices: np.ndarray          # [(nelz+1)][(nely+1)][(nelx+1)][3], float64
    periodic: tuple
    dirichlet: int
    name: str = ""

    @property
    def nelem(self) -> int:
        return self.nelx * self.nely * self.nelz

    @property
    def n_local(self) -> int:
        return self.nelem * (self.order + 1) ** 3


def lattice(nelx, nely, nelz, xs=None, ys=None, zs=None):
    """Tensor-product vertex lattice; ``xs`` etc. are the 1-D vertex planes."""
    xs = np.linspace(0.0, 1.0, nelx + 1) if xs is None else np.asarray(xs, dtype=np.float64)
    ys = np.linspace(0.0, 1.0, nely + 1) if ys is None else np.asarray(ys, dtype=np.float64)
    zs = np.linspace(0.0, 1.0, nelz + 1) if zs is None else np.asarray(zs, dtype=np.float64)
    v = np.zeros((nelz + 1, nely + 1, nelx + 1, 3))
    v[..., 0] = xs[None, None, :]
    v[..., 1] = ys[None, :, None]
    v[..., 2] = zs[:, None, None]
    return v


def cube(nel: int, order: int, dirichlet: int = DIRICHLET_ALL) -> MeshSpec:
    return MeshSpec(nel, nel, nel, order, lattice(nel, nel, nel), (0, 0, 0), dirichlet,
                    "cube%d_N%d" % (nel, order))


def box(nelx, nely, nelz, order, extent=(1.0, 1.0, 1.0), periodic=(0, 0, 0),
        dirichlet=DIRICHLET_ALL) -> MeshSpec:
    v = lattice(nelx, nely, nelz, np.linspace(0, extent[0], nelx + 1),
                np.linspace(0, extent[1], nely + 1), np.linspace(0, extent[2], nelz + 1))
    return MeshSpec(nelx, nely, nelz, order, v, tuple(periodic), dirichlet,
                    "box%dx%dx%d_N%d" % (nelx, nely, nelz, order))


def deformed_cube(nel: int, order: int, amp: float = 0.05,
                  dirichlet: int = DIRICHLET_ALL) -> MeshSpec:
    """Cube with vertices moved simultaneously (from undeformed positions):
    x += amp h sin(2 pi y) sin(2 pi z), y += amp h sin(2 pi z) sin(2 pi x),
    z += amp h sin(2 pi x) sin(2 pi y), h = 1/nel."""
    v = lattice(nel, nel, nel)
    h = 1.0 / nel
    x, y, z = v[..., 0].copy(), v[..., 1].copy(), v[..., 2].copy()
    s = lambda a: np.sin(2.0 * math.pi * a)
    v[..., 0] = x + amp * h * s(y) * s(z)
    v[..., 1] = y + amp * h * s(z) * s(x)
    v[..., 2] = z + amp * h * s(x) * s(y)
    return MeshSpec(nel, nel, nel, order, v, (0, 0, 0), dirichlet,
                    "deformed%d_N%d" % (nel, order))


def random_deformed_box(nelx, nely, nelz, order, seed, amp=0.15, periodic=(0, 0, 0),
                        dirichlet=DIRICHLET_ALL) -> MeshSpec:
    """Unit box with interior vertices jittered uniformly by up to amp*h
    (boundary vertices move only tangentially; periodic planes stay matched)."""
    rng = np.random.default_rng(seed)
    v = lattice(nelx, nely, nelz)
    nel = (nelx, nely, nelz)
    d = rng.uniform(-1.0, 1.0, size=v.shape)
    for c in range(3):
        axis = 2 - c  # vertex array is [z][y][x]
        h = 1.0 / nel[c]
        d[..., c] *= amp * h
        if periodic[c]:
            # keep the far plane the exact periodic image of the near one
            idx_first = [slice(None)] * 3
            idx_last = [slice(None)] * 3
            idx_first[axis] = 0
            idx_last[axis] = nel[c]
            d[tuple(idx_last) + (c,)] = d[tuple(idx_first) + (c,)]
        else:
            for end in (0, nel[c]):
                idx = [slice(None)] * 3
                idx[axis] = end
                d[tuple(idx) + (c,)] = 0.0
    v = v + d
    return MeshSpec(nelx, nely, nelz, order, v, tuple(periodic), dirichlet,
                    "jitter%dx%dx%d_N%d_s%d" % (nelx, nely, nelz, order, seed))


def channel(nel: int, order: int, beta: float = 2.0) -> MeshSpec:
    """Unit cube, periodic in x and z, walls (Dirichlet) at y = 0 and 1,
    y_j = (1 + tanh(beta (2j/nel - 1)) / tanh(beta)) / 2."""
    j = np.arange(nel + 1)
    ys = 0.5 * (1.0 + np.tanh(beta * (2.0 * j / nel - 1.0)) / math.tanh(beta))
    ys[0], ys[-1] = 0.0, 1.0
    v = lattice(nel, nel, nel, ys=ys)
    return MeshSpec(nel, nel, nel, order, v, (1, 0, 1), DIRICHLET_Y_WALLS,
                    "channel%d_N%d" % (nel, order))


# --------------------------------------------------------------------------
# Right-hand sides (evaluated at caller-provided point coordinates)


def manufactured(x, y, z):
    """Exact u = sin(pi x) sin(pi y) sin(pi z) and f = -lap u = 3 pi^2 u."""
    xp = _xp(x)
    u = xp.sin(math.pi * x) * xp.sin(math.pi * y) * xp.sin(math.pi * z)
    return u, 3.0 * math.pi ** 2 * u


def half_space_modes(kmax: int = 8):
    """Integer wave vectors with 1 <= |k| <= kmax whose first nonzero
    component is positive, in lexicographic (kx, ky, kz) order."""
    ks = []
    for kx in range(-kmax, kmax + 1):
        for ky in range(-kmax, kmax + 1):
            for kz in range(-kmax, kmax + 1):
                n2 = kx * kx + ky * ky + kz * kz
                if n2 < 1 or n2 > kmax * kmax:
                    continue
                first = kx if kx != 0 else (ky if ky != 0 else kz)
                if first > 0:
                    ks.append((kx, ky, kz))
    return np.array(ks, dtype=np.int64)


@dataclass(frozen=True)
class FourierField:
    """f(x) = sum_k a_k cos(2 pi k.x) + b_k sin(2 pi k.x)."""
    k: np.ndarray   # (M, 3) int
    a: np.ndarray   # (M,)
    b: np.ndarray   # (M,)


def gaussian_fourier(seed: int, kmax: int = 8) -> FourierField:
    """Unit-variance Gaussian amplitudes; per mode, a then b, modes in
    lexicographic order."""
    k = half_space_modes(kmax)
    rng = np.random.default_rng(seed)
    ab = rng.standard_normal((len(k), 2))
    return FourierField(k, ab[:, 0].copy(), ab[:, 1].copy())


@dataclass(frozen=True)
class VelocityModes:
    """Velocity-like field v = sum_k A_k cos(2 pi k.x) + B_k sin(2 pi k.x),
    A_k, B_k in R^3 with amplitude |k|^(-11/6) (shell energy ~ k^(-5/3))."""
    k: np.ndarray   # (M, 3)
    A: np.ndarray   # (M, 3)
    B: np.ndarray   # (M, 3)


def kolmogorov_velocity(seed: int, kmax: int = 8) -> VelocityModes:
    k = half_space_modes(kmax)
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((len(k), 6))
    sig = np.linalg.norm(k, axis=1) ** (-11.0 / 6.0)
    return VelocityModes(k, g[:, :3] * sig[:, None], g[:, 3:] * sig[:, None])


ADVECTION_SHIFT = (1.0 / 97.0, 0.0, 1.0 / 89.0)


def divergence_source(vm: VelocityModes, t: int, shift=ADVECTION_SHIFT) -> FourierField:
    """Pressure source f_t(x) = (div v)(x - c t): a scalar Fourier series.
    d/dx_j [A cos(th) + B sin(th)]_j = 2 pi k_j (-A_j sin(th) + B_j cos(th)),
    with th = 2 pi k.(x - c t) = 2 pi k.x - phi."""
    k = vm.k.astype(np.float64)
    ca = 2.0 * math.pi * np.sum(k * vm.B, axis=1)    # coefficient of cos(th)
    sa = -2.0 * math.pi * np.sum(k * vm.A, axis=1)   # coefficient of sin(th)
    phi = 2.0 * math.pi * t * (k @ np.asarray(shift, dtype=np.float64))
    # cos(th) = cos(kx) cos(phi) + sin(kx) sin(phi); sin(th) = sin(kx) cos(phi) - cos(kx) sin(phi)
    a = ca * np.cos(phi) - sa * np.sin(phi)
    b = ca * np.sin(phi) + sa * np.cos(phi)
    return FourierField(vm.k, a, b)


def _xp(x):
    mod = type(x).__module__
    if mod.startswith("torch"):
        import torch
        return torch
    return np


def fourier_eval(ff: FourierField, x, y, z, chunk: int = 64):
    """Evaluate at arbitrary points (numpy or torch arrays of equal shape).
    Uses exp(2 pi i k.x) = e_x^kx e_y^ky e_z^kz with per-axis power tables."""
    xp = _xp(x)
    kmax = int(np.abs(ff.k).max())
    if xp is np:
        shape = np.shape(x)
        xs, ys, zs = (np.ravel(np.asarray(c, dtype=np.float64)) for c in (x, y, z))
        out = np.zeros(xs.shape)
        ex = [np.exp(2j * math.pi * kk * xs) for kk in range(-kmax, kmax + 1)]
        ey = [np.exp(2j * math.pi * kk * ys) for kk in range(-kmax, kmax + 1)]
        ez = [np.exp(2j * math.pi * kk * zs) for kk in range(-kmax, kmax + 1)]
        for (kx, ky, kz), a, b in zip(ff.k, ff.a, ff.b):
            ph = ex[kx + kmax] * ey[ky + kmax] * ez[kz + kmax]
            out += a * ph.real + b * ph.imag
        return out.reshape(shape)
    import torch
    shape = x.shape
    xs, ys, zs = (c.reshape(-1).to(torch.float64) for c in (x, y, z))
    out = torch.zeros_like(xs)
    kr = torch.arange(-kmax, kmax + 1, device=xs.device, dtype=torch.float64)
    for lo in range(0, xs.numel(), 1 << 22):
        sl = slice(lo, min(lo + (1 << 22), xs.numel()))
        ex = torch.polar(torch.ones(1, device=xs.device, dtype=torch.float64), 2 * math.pi * kr[:, None] * xs[None, sl])
        ey = torch.polar(torch.ones(1, device=xs.device, dtype=torch.float64), 2 * math.pi * kr[:, None] * ys[None, sl])
        ez = torch.polar(torch.ones(1, device=xs.device, dtype=torch.float64), 2 * math.pi * kr[:, None] * zs[None, sl])
        acc = torch.zeros(sl.stop - sl.start, device=xs.device, dtype=torch.float64)
        ks = torch.as_tensor(ff.k + kmax, device=xs.device)
        ca = torch.as_tensor(ff.a, device=xs.device, dtype=torch.float64)
        cb = torch.as_tensor(ff.b, device=xs.device, dtype=torch.float64)
        for m0 in range(0, len(ff.k), chunk):
            m1 = min(m0 + chunk, len(ff.k))
            ph = ex[ks[m0:m1, 0]] * ey[ks[m0:m1, 1]] * ez[ks[m0:m1, 2]]
            acc += (ca[m0:m1, None] * ph.real + cb[m0:m1, None] * ph.imag).sum(0)
        out[sl] = acc
    return out.reshape(shape)


def fourier_eval_separable(ff: FourierField, x1, y1, z1):
    """Evaluate on a tensor grid: returns F[iz, iy, ix] = f(x1[ix], y1[iy], z1[iz])
    (numpy).  exp(i k.x) factorises, so this is three small contractions."""
    kmax = int(np.abs(ff.k).max())
    K = 2 * kmax + 1
    C = np.zeros((K, K, K), dtype=np.complex128)     # [kz, ky, kx]
    # a cos + b sin = Re((a - i b) e^{i th})
    np.add.at(C, (ff.k[:, 2] + kmax, ff.k[:, 1] + kmax, ff.k[:, 0] + kmax), ff.a - 1j * ff.b)
    kr = np.arange(-kmax, kmax + 1)
    Ex = np.exp(2j * math.pi * np.outer(kr, np.asarray(x1, dtype=np.float64)))  # [kx, ix]
    Ey = np.exp(2j * math.pi * np.outer(kr, np.asarray(y1, dtype=np.float64)))
    Ez = np.exp(2j * math.pi * np.outer(kr, np.asarray(z1, dtype=np.float64)))
    T = np.einsum("zyx,xi->zyi", C, Ex)
    T = np.einsum("zyi,yj->zji", T, Ey)
    T = np.einsum("zji,zk->kji", T, Ez)
    return T.real.copy()


def fourier_on_elements(ff: FourierField, xyz, nel):
    """Evaluate on local-form coordinates ``xyz`` of shape (3, E, n, n, n)
    (numpy or torch) for an element grid ``nel = (nelx, nely, nelz)``.
    When x depends only on (ex, i), y only on (ey, j) and z only on (ez, k)
    to within 1e-13 (undeformed tensor meshes) the separable path is used on
    the first slice's coordinates; otherwise the general point evaluation."""
    nelx, nely, nelz = nel
    is_torch = type(xyz).__module__.startswith("torch")
    X = xyz.detach().cpu().numpy() if is_torch else np.asarray(xyz)
    n = X.shape[-1]
    Xr = X.reshape(3, nelz, nely, nelx, n, n, n)
    x1 = Xr[0, 0, 0, :, 0, 0, :]          # (nelx, n) over (ex, i)
    y1 = Xr[1, 0, :, 0, 0, :, 0]          # (nely, n) over (ey, j)
    z1 = Xr[2, :, 0, 0, :, 0, 0]          # (nelz, n) over (ez, k)
    tol = 1e-13 * max(1.0, float(np.max(np.abs(X))))
    sep = (np.max(np.abs(Xr[0] - x1[None, None, :, None, None, :])) <= tol
           and np.max(np.abs(Xr[1] - y1[None, :, None, None, :, None])) <= tol
           and np.max(np.abs(Xr[2] - z1[:, None, None, :, None, None])) <= tol)
    if not sep:
        if is_torch:
            return fourier_eval(ff, xyz[0], xyz[1], xyz[2])
        return fourier_eval(ff, X[0], X[1], X[2])
    F = fourier_eval_separable(ff, x1.ravel(), y1.ravel(), z1.ravel())   # [(ez,k), (ey,j), (ex,i)]
    F = F.reshape(nelz, n, nely, n, nelx, n).transpose(0, 2, 4, 1, 3, 5)
    out = np.ascontiguousarray(F).reshape(-1, n, n, n)
    if is_torch:
        import torch
        return torch.from_numpy(out).to(xyz.device)
    return out


# --------------------------------------------------------------------------
# The five workload configurations


def config(name: str) -> MeshSpec:
    """c0: 4^3 cube, N=5, Dirichlet, Poisson (manufactured solution);
    c1/c2: 32^3 deformed cube, N=7, Dirichlet, Helmholtz h1=1, h2=0.1;
    c3: 16^3 channel, N=7; c4: 64^3 channel, N=7 (Poisson)."""
    if name == "c0":
        return cube(4, 5)
    if name in ("c1", "c2"):
        return deformed_cube(32, 7)
    if name == "c3":
        return channel(16, 7)
    if name == "c4":
        return channel(64, 7)
    raise KeyError(name)


HELMHOLTZ = {"c0": (1.0, 0.0), "c1": (1.0, 0.1), "c2": (1.0, 0.1), "c3": (1.0, 0.0), "c4": (1.0, 0.0)}
RHS_SEED = {"c1": 1, "c2": 1, "c3": 2, "c4": 4}
