"""FP64 CPU oracle for the spectral-element pressure-solve hot path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package.  It shares no
code with the HIP library in ``paper_2405_05640_amd`` and imports nothing from
it; the two meet only through the seeded input generators.

The arithmetic lives in ``sem_oracle.c`` (plain loops, FP64) and ``cnn.py`` /
``mixed.py`` (numpy); this module only marshals numpy arrays.  The method is
the one the paper builds on (section 3.1, "Neko": E hexahedral elements,
order-N GLL collocation, element-by-element operators, gather-scatter
coupling, preconditioned Krylov solve of Ax=b), with the textbook definitions
of Deville, Fischer & Mund (2002) for the spectral-element pieces.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sem_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libsem_oracle.so")
_lib = None

_d = ctypes.POINTER(ctypes.c_double)
_i64 = ctypes.POINTER(ctypes.c_int64)
_i32 = ctypes.POINTER(ctypes.c_int32)
_u8 = ctypes.POINTER(ctypes.c_uint8)


def build(force: bool = True) -> str:
    """Compile ``sem_oracle.c`` into ``libsem_oracle.so`` with gcc."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O3", "-march=x86-64-v3", "-fopenmp", "-fPIC", "-shared",
               "-std=c11", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
            build(force=True)
        L = ctypes.CDLL(_LIB_PATH)
        L.ora_gll.argtypes = [ctypes.c_int, _d, _d]
        L.ora_gll.restype = ctypes.c_int
        L.ora_deriv.argtypes = [ctypes.c_int, _d, _d]
        L.ora_deriv.restype = None
        L.ora_geometry.argtypes = [ctypes.c_int] * 4 + [_d, _d, _d, _d, _d]
        L.ora_geometry.restype = ctypes.c_int64
        L.ora_numbering.argtypes = [ctypes.c_int] * 4 + [_u8, ctypes.c_uint8, _i64, _i32, _u8]
        L.ora_numbering.restype = ctypes.c_int64
        L.ora_ax.argtypes = [ctypes.c_int64, ctypes.c_int, _d, _d, _d, ctypes.c_double,
                             ctypes.c_double, _d, _d]
        L.ora_ax.restype = None
        L.ora_dssum.argtypes = [ctypes.c_int64, _i64, ctypes.c_int64, _d]
        L.ora_dssum.restype = None
        L.ora_mask.argtypes = [ctypes.c_int64, _u8, _d]
        L.ora_mask.restype = None
        L.ora_apply_S.argtypes = [ctypes.c_int64, ctypes.c_int, _d, _d, _d, ctypes.c_double,
                                  ctypes.c_double, _i64, ctypes.c_int64, _u8, _d, _d]
        L.ora_apply_S.restype = None
        L.ora_diag_local.argtypes = [ctypes.c_int64, ctypes.c_int, _d, _d, _d, ctypes.c_double,
                                     ctypes.c_double, _d]
        L.ora_diag_local.restype = None
        L.ora_jacobi_inv.argtypes = [ctypes.c_int64, ctypes.c_int, _d, _d, _d, ctypes.c_double,
                                     ctypes.c_double, _i64, ctypes.c_int64, _u8, _d]
        L.ora_jacobi_inv.restype = None
        L.ora_dot.argtypes = [ctypes.c_int64, _d, _d, _i32]
        L.ora_dot.restype = ctypes.c_double
        L.ora_pcg.argtypes = [ctypes.c_int64, ctypes.c_int, _d, _d, _d, ctypes.c_double,
                              ctypes.c_double, _i64, ctypes.c_int64, _u8, _i32, _d, _d, _d,
                              ctypes.c_double, ctypes.c_int, _d, _d]
        L.ora_pcg.restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a, t=_d):
    return a.ctypes.data_as(t)


def _c(a, dtype):
    a = np.ascontiguousarray(a, dtype=dtype)
    return a


# --------------------------------------------------------------------------
# Reference element


def gll(N: int):
    """GLL nodes and weights on [-1, 1] (N+1 points)."""
    xi = np.zeros(N + 1)
    w = np.zeros(N + 1)
    if lib().ora_gll(N, _p(xi), _p(w)) != 0:
        raise ValueError("order must be >= 1")
    return xi, w


def deriv(N: int):
    """Derivative matrix D[i, j] = l_j'(xi_i) on the GLL nodes."""
    xi, _ = gll(N)
    D = np.zeros((N + 1, N + 1))
    lib().ora_deriv(N, _p(xi), _p(D))
    return D


# --------------------------------------------------------------------------
# Mesh


@dataclass
class Mesh:
    """Oracle mesh: geometry, numbering, mult and mask, all on the host."""

    nelx: int
    nely: int
    nelz: int
    N: int
    vertices: np.ndarray
    periodic: tuple = (0, 0, 0)
    dirichlet: int = 0x3F
    xi: np.ndarray = field(init=False)
    w: np.ndarray = field(init=False)
    D: np.ndarray = field(init=False)
    xyz: np.ndarray = field(init=False)
    G: np.ndarray = field(init=False)
    B: np.ndarray = field(init=False)
    jac: np.ndarray = field(init=False)
    glo: np.ndarray = field(init=False)
    mult: np.ndarray = field(init=False)
    mask: np.ndarray = field(init=False)
    n_global: int = field(init=False)

    def __post_init__(self):
        n = self.N + 1
        self.E = self.nelx * self.nely * self.nelz
        self.np_ = n ** 3
        self.nl = self.E * self.np_
        self.vertices = _c(self.vertices, np.float64)
        assert self.vertices.shape == (self.nelz + 1, self.nely + 1, self.nelx + 1, 3)
        self.xi, self.w = gll(self.N)
        self.D = deriv(self.N)
        self.xyz = np.zeros((3, self.E, n, n, n))
        self.G = np.zeros((6, self.E, n, n, n))
        self.B = np.zeros((self.E, n, n, n))
        self.jac = np.zeros((self.E, n, n, n))
        bad = lib().ora_geometry(self.nelx, self.nely, self.nelz, self.N, _p(self.vertices),
                                 _p(self.xyz), _p(self.G), _p(self.B), _p(self.jac))
        if bad != 0:
            raise ValueError("element %d has a non-positive Jacobian" % (bad - 1))
        self.glo = np.zeros((self.E, n, n, n), dtype=np.int64)
        self.mult = np.zeros((self.E, n, n, n), dtype=np.int32)
        self.mask = np.zeros((self.E, n, n, n), dtype=np.uint8)
        per = np.array([1 if q else 0 for q in self.periodic], dtype=np.uint8)
        ng = lib().ora_numbering(self.nelx, self.nely, self.nelz, self.N, _p(per, _u8),
                                 int(self.dirichlet), _p(self.glo, _i64), _p(self.mult, _i32),
                                 _p(self.mask, _u8))
        if ng < 0:
            raise ValueError("bad mesh description")
        self.n_global = int(ng)

    @property
    def shape(self):
        n = self.N + 1
        return (self.E, n, n, n)

    # ---------------------------------------------------------------- ops
    def ax(self, u, h1=1.0, h2=0.0, G=None, B=None):
        """Unassembled local operator w = h1 sum_ab D_a^T G_ab D_b u + h2 B u
        (optionally with other geometric factors G [6, E, ...] and B)."""
        u = _c(u, np.float64).reshape(self.shape)
        G = self.G if G is None else _c(G, np.float64)
        B = self.B if B is None else _c(B, np.float64)
        w = np.zeros(self.shape)
        lib().ora_ax(self.E, self.N, _p(self.D), _p(G), _p(B), h1, h2, _p(u), _p(w))
        return w

    def ax_abs_bound(self, u, h1=1.0, h2=0.0):
        """The local operator with |D|, |G|, |B| and |u|: the magnitude that
        bounds rounding errors of any evaluation order of A_L u."""
        u = np.abs(_c(u, np.float64).reshape(self.shape))
        Da, Ga, Ba = np.abs(self.D), np.abs(self.G), np.abs(self.B)
        w = np.zeros(self.shape)
        lib().ora_ax(self.E, self.N, _p(Da), _p(Ga), _p(Ba), abs(h1), abs(h2), _p(u), _p(w))
        return w

    def dssum(self, u):
        """Direct-stiffness summation (returns a new array)."""
        v = _c(u, np.float64).reshape(self.shape).copy()
        lib().ora_dssum(self.nl, _p(self.glo, _i64), self.n_global, _p(v))
        return v

    def apply_mask(self, u):
        v = _c(u, np.float64).reshape(self.shape).copy()
        lib().ora_mask(self.nl, _p(self.mask, _u8), _p(v))
        return v

    def apply_S(self, u, h1=1.0, h2=0.0):
        """Assembled, masked operator S u = mask(dssum(A_L u))."""
        u = _c(u, np.float64).reshape(self.shape)
        w = np.zeros(self.shape)
        lib().ora_apply_S(self.E, self.N, _p(self.D), _p(self.G), _p(self.B), h1, h2,
                          _p(self.glo, _i64), self.n_global, _p(self.mask, _u8), _p(u), _p(w))
        return w

    def diag_local(self, h1=1.0, h2=0.0):
        d = np.zeros(self.shape)
        lib().ora_diag_local(self.E, self.N, _p(self.D), _p(self.G), _p(self.B), h1, h2, _p(d))
        return d

    def jacobi_inv(self, h1=1.0, h2=0.0):
        d = np.zeros(self.shape)
        lib().ora_jacobi_inv(self.E, self.N, _p(self.D), _p(self.G), _p(self.B), h1, h2,
                             _p(self.glo, _i64), self.n_global, _p(self.mask, _u8), _p(d))
        return d

    def dot(self, u, v):
        """Inner product of continuous local-form vectors (each node once)."""
        u = _c(u, np.float64).reshape(self.shape)
        v = _c(v, np.float64).reshape(self.shape)
        return float(lib().ora_dot(self.nl, _p(u), _p(v), _p(self.mult, _i32)))

    def rhs(self, f):
        """b = mask(dssum(B f)) for f sampled at the local GLL nodes."""
        return self.apply_mask(self.dssum(self.B * np.asarray(f, dtype=np.float64).reshape(self.shape)))

    def pcg(self, b, h1=1.0, h2=0.0, tol=1e-10, max_iter=20000, history=False):
        """Jacobi-PCG from x = 0.  Returns (x, info dict)."""
        b = _c(b, np.float64).reshape(self.shape)
        dinv = self.jacobi_inv(h1, h2)
        x = np.zeros(self.shape)
        out = np.zeros(4)
        hist = np.zeros(max_iter + 1) if history else None
        st = lib().ora_pcg(self.E, self.N, _p(self.D), _p(self.G), _p(self.B), h1, h2,
                           _p(self.glo, _i64), self.n_global, _p(self.mask, _u8),
                           _p(self.mult, _i32), _p(dinv), _p(b), _p(x), tol, max_iter, _p(out),
                           _p(hist) if hist is not None else None)
        info = {"status": int(st), "iterations": int(out[0]), "rel_res": float(out[1]),
                "true_rel_res": float(out[2]), "restarts": int(out[3])}
        if hist is not None:
            info["history"] = hist[: int(out[0]) + 1].copy()
        return x, info

    def gather_global(self, u):
        """Global vector from a continuous local-form one (value of any copy)."""
        g = np.zeros(self.n_global)
        g[self.glo.ravel()] = np.asarray(u).ravel()
        return g
