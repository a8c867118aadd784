"""Brute-force helpers that pin the oracle: closed forms written out in numpy,
independent of the oracle's C code (tests only)."""
import numpy as np


def closed_form_glo(nelx, nely, nelz, N, periodic):
    """Lexicographic structured numbering: gi = ex N + i (mod nx if periodic),
    glo = gi + nx (gj + ny gk)."""
    n = N + 1
    nd = [nel * N + (0 if per else 1) for nel, per in zip((nelx, nely, nelz), periodic)]
    ez, ey, ex, k, j, i = np.meshgrid(np.arange(nelz), np.arange(nely), np.arange(nelx),
                                      np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    gi = (ex * N + i) % nd[0]
    gj = (ey * N + j) % nd[1]
    gk = (ez * N + k) % nd[2]
    glo = gi + nd[0] * (gj + nd[1] * gk)
    # reorder to [e][k][j][i] with e = ex + nelx (ey + nely ez)
    glo = glo.reshape(nelz, nely, nelx, n, n, n).reshape(-1, n, n, n)
    return glo, int(np.prod(nd))


def trilinear(X, r, s, t):
    """Trilinear map of one hexahedron with corners X[c3][c2][c1][xyz] at
    reference point (r, s, t); returns x (3,) and J[c][a] = dx_c/dr_a."""
    phi = lambda q: np.array([(1 - q) / 2, (1 + q) / 2])
    dphi = np.array([-0.5, 0.5])
    pr, ps, pt = phi(r), phi(s), phi(t)
    x = np.einsum("zyxc,x,y,z->c", X, pr, ps, pt)
    J = np.stack([np.einsum("zyxc,x,y,z->c", X, dphi, ps, pt),
                  np.einsum("zyxc,x,y,z->c", X, pr, dphi, pt),
                  np.einsum("zyxc,x,y,z->c", X, pr, ps, dphi)], axis=1)
    return x, J


def element_corners(vert, nelx, nely, e):
    ex = e % nelx
    ey = (e // nelx) % nely
    ez = e // (nelx * nely)
    return vert[ez:ez + 2, ey:ey + 2, ex:ex + 2, :]


def dense_S(mesh, h1=1.0, h2=0.0):
    """Dense assembled operator on the global unmasked unknowns, by applying
    the oracle's S to every continuous unit vector.  Returns (S, free_ids)."""
    glo = mesh.glo.ravel()
    maskg = np.zeros(mesh.n_global, dtype=bool)
    maskg[glo[mesh.mask.ravel() == 1]] = True
    free = np.nonzero(~maskg)[0]
    S = np.zeros((len(free), len(free)))
    for c, g in enumerate(free):
        u = (glo == g).astype(np.float64).reshape(mesh.shape)
        w = mesh.apply_S(u, h1, h2)
        S[:, c] = mesh.gather_global(w)[free]
    return S, free


def continuous_random(mesh, rng, masked=True):
    g = rng.standard_normal(mesh.n_global)
    u = g[mesh.glo]
    if masked:
        u = np.where(mesh.mask == 1, 0.0, u)
    return u
