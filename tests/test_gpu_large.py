"""GPU parity at the largest single-GPU size: the 64^3-element N = 7
tanh-stretched channel (periodic x and z, Dirichlet walls in y; 134,217,728
local points), in the launch configuration of the large benchmark (FP64
Poisson, h1 = 1, h2 = 0).  The oracle cannot take the whole mesh in a
test's time, so:
* the numbering and the Dirichlet mask are checked at every point against
  their closed form on the structured lattice;
* the operator is compared on sampled blocks of elements against oracle
  meshes built from the same vertices (the local operator of an element
  depends only on its corners and its values), in two parts.  The kernel's
  arithmetic: against the oracle's operator fed the library's own G and B,
  elementwise within 1e-14 (|D|^T |G| |D| |u|), FP64 rounding of the
  contractions.  The geometric factors: against the oracle's, which takes
  the Jacobian by differentiating absolute GLL coordinates with D and so
  carries an absolute error of about eps |D|_inf max|x| in J; relative to a
  thin wall element far from the origin (h about 0.005, |x| about 1) that
  is about 1e-12 in G, so the bar per element is
  64 eps |D|_inf max|x_e| / h_min,e times max |G_e|;
* the gather-scatter is compared at every point, bit for bit, with sums
  over the closed-form numbering taken in ascending local index
  (numpy's bincount adds its weights in input order)."""
import numpy as np
import pytest

import oracle
from paper_2405_05640_amd import sem
from paper_2405_05640_amd import workloads as wl
from tests.gpu_util import dev, host, relmax

pytestmark = pytest.mark.gpu

N = 7
NP = N + 1


@pytest.fixture(scope="module")
def c4():
    print("building the 64^3 N=7 channel (library)", flush=True)
    spec = wl.config("c4")
    return spec, sem.Mesh.from_spec(spec)


def closed_form_numbering(spec):
    """glo = gi + nx (gj + ny gk) with gi = ex N + i (wrapped when periodic),
    and the wall mask, for the [E][k][j][i] local layout."""
    per = spec.periodic
    nx = spec.nelx * N + (0 if per[0] else 1)
    ny = spec.nely * N + (0 if per[1] else 1)
    nz = spec.nelz * N + (0 if per[2] else 1)
    l = np.arange(NP)
    gi = (np.arange(spec.nelx)[:, None] * N + l[None, :]) % nx       # [ex][i]
    gj = (np.arange(spec.nely)[:, None] * N + l[None, :]) % ny       # [ey][j]
    gk = (np.arange(spec.nelz)[:, None] * N + l[None, :]) % nz       # [ez][k]
    # [ez][ey][ex][k][j][i]
    glo = (gi[None, None, :, None, None, :]
           + nx * (gj[None, :, None, None, :, None] + ny * gk[:, None, None, :, None, None]))
    glo = glo.reshape(-1, NP, NP, NP)
    walls = np.zeros((spec.nely, NP), dtype=bool)
    if not per[1]:
        walls = (gj == 0) | (gj == ny - 1)
    mask = np.broadcast_to(walls[None, :, None, None, :, None],
                           (spec.nelz, spec.nely, spec.nelx, NP, NP, NP)).reshape(-1, NP, NP, NP)
    return glo, mask, nx * ny * nz


def test_large_numbering_and_mask(c4):
    spec, gm = c4
    glo, mask, ng = closed_form_numbering(spec)
    assert gm.n_local == 134217728 and gm.n_global == ng
    assert np.array_equal(gm.export(sem.FIELD_GLO_NUM), glo)
    assert np.array_equal(gm.export(sem.FIELD_MASK) != 0, mask)


def test_large_operator_on_sampled_blocks(c4):
    import torch
    spec, gm = c4
    rng = np.random.default_rng(60)
    u = rng.standard_normal(gm.shape)
    w = torch.empty(gm.shape, dtype=torch.float64, device="cuda")
    gm.ax(dev(u), w, 1.0, 0.0)
    wh = host(w)
    del w
    Glib = gm.export(sem.FIELD_G)
    Blib = gm.export(sem.FIELD_B)
    V = np.asarray(spec.vertices).reshape(spec.nelz + 1, spec.nely + 1, spec.nelx + 1, 3)
    eps = 2.0 ** -53
    b = 3
    # blocks at the first wall and the periodic seams, in the interior, and at
    # the last wall and the far seams
    for x0, y0, z0 in ((0, 0, 0), (30, 31, 29), (spec.nelx - b, spec.nely - b, spec.nelz - b)):
        sub = np.ascontiguousarray(V[z0:z0 + b + 1, y0:y0 + b + 1, x0:x0 + b + 1])
        om = oracle.Mesh(b, b, b, N, sub, (0, 0, 0), 0)
        ez, ey, ex = np.meshgrid(np.arange(z0, z0 + b), np.arange(y0, y0 + b), np.arange(x0, x0 + b),
                                 indexing="ij")
        e = (ex + spec.nelx * (ey + spec.nely * ez)).ravel()      # sub-mesh element order (x fastest)
        # the kernel's arithmetic, on the library's own factors
        ref = om.ax(u[e], 1.0, 0.0, G=Glib[:, e], B=Blib[e])
        scale = om.ax_abs_bound(u[e], 1.0, 0.0)
        err_k = np.max(np.abs(wh[e] - ref) / scale)
        # the factors against the oracle's, within the oracle's own rounding of J
        dn = np.max(np.sum(np.abs(om.D), axis=1))
        edges = np.concatenate([np.diff(sub, axis=a).reshape(-1, 3) for a in range(3)])
        hmin = np.min(np.linalg.norm(edges, axis=1))
        xmax = np.max(np.abs(sub))
        tol_g = 64 * eps * dn * xmax / hmin
        gmax = np.max(np.abs(om.G), axis=(0, 2, 3, 4))[None, :, None, None, None]
        err_g = np.max(np.abs(Glib[:, e] - om.G) / gmax)
        print("block at", (x0, y0, z0), "kernel |err| / abs-operator %.2e; G rel. diff %.2e (bar %.2e)"
              % (err_k, err_g, tol_g), flush=True)
        assert np.all(np.abs(wh[e] - ref) <= 1e-14 * scale)
        assert err_g <= tol_g
        assert relmax(Blib[e], om.B) <= tol_g


def test_large_dssum_every_point(c4):
    spec, gm = c4
    glo, mask, ng = closed_form_numbering(spec)
    rng = np.random.default_rng(61)
    u = rng.standard_normal(gm.shape)
    s = np.bincount(glo.ravel(), weights=u.ravel(), minlength=ng)
    ref = s[glo]
    mult = np.bincount(glo.ravel(), minlength=ng)[glo]
    ref[mult == 1] = u[mult == 1]          # a node with one copy keeps its value
    ref[mask] = 0.0
    t = dev(u)
    gm.dssum(t, mask=True)
    assert np.array_equal(host(t), ref)
