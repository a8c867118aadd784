"""FP64 oracle of the pressure preconditioner and Krylov method the paper
names (section 3.1, "Neko": restarted GMRES with a hybrid-Schwarz
multigrid preconditioner; CG with block-Jacobi for the velocity solves).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The paper names the methods and cites the spectral-element literature for
them; it gives no formulas.  The definitions below are this project's
readings of the textbook constructions (Deville, Fischer & Mund 2002, ch. 4
and 8; Lottes & Fischer 2005 for the Schwarz/multigrid combination; Saad 2003,
Algorithm 9.6, for flexible GMRES), written out plainly over the oracle
meshes of ``oracle.Mesh``.  Vectors are local-form continuous fields, as in
the rest of the oracle.

Levels.  The same vertices at polynomial orders N (fine), N_mid and 1
(coarse); each level is an ``oracle.Mesh`` with its own GLL points,
numbering, multiplicity and Dirichlet mask.

Prolongation P (coarse -> fine): on every element, tensor-product Lagrange
interpolation J (x) J (x) J from the coarse GLL points to the fine ones,
J[f, c] = l_c(xi_f).  The interpolant of a continuous field is continuous.
Restriction R = P^T on assembled (one value per global node) vectors; for a
continuous local-form residual r it is R r = dssum_c(J^T (r / mult_f)) on
every element, then the coarse Dirichlet mask (a face value of P depends
only on the coarse nodes of that face, so every element holding a fine node
also holds every coarse node it interpolates from).

Schwarz smoother (one level).  The subdomains are the elements' own node
sets, which overlap on shared faces, edges and vertices (minimal overlap:
each subdomain reaches one GLL point into its neighbours, where it is
closed by homogeneous Dirichlet conditions).  The local matrix is the
principal submatrix of the assembled operator on those nodes, approximated
by a separable one built from one length per element and direction:

  A_d = (2/L) Ahat + [left neighbour] (2/L_l) Ahat[N,N] e_0 e_0^T
                   + [right neighbour] (2/L_r) Ahat[0,0] e_N e_N^T,
  B_d = (L/2) W   + [left] (L_l/2) w_N e_0 e_0^T + [right] (L_r/2) w_0 e_N e_N^T

with Ahat = D^T W D the 1-D GLL stiffness and W = diag(w); a node on a
Dirichlet face is removed, a domain boundary without Dirichlet condition
gets no neighbour term.  The local solve is the fast diagonalisation
(Lynch, Rice & Thomas 1964): A_d S_d = B_d S_d Lambda_d with
S_d^T B_d S_d = I, and

  z_e = (S_z (x) S_y (x) S_x) [h1 (lx_i + ly_j + lz_k) + h2]^-1 (S_z (x) S_y (x) S_x)^T r_e.

On a rectilinear tensor-product mesh (boxes whose widths depend only on
their index along each axis) this is exactly the inverse of the principal
submatrix.  The element length L along an axis is the mean length of the
element's four edges in that direction.  The smoother adds the local
corrections of all elements (dssum) and averages them over the copies of
each node (weight 1/mult), then applies the mask.

Coarse solve (order 1).  The coarse operator is approximated by the
separable operator of a rectilinear grid whose vertex planes are the
averages of the mesh's vertex planes (global 1-D linear-element stiffness
and lumped mass per axis, periodic wraps and Dirichlet ends as the mesh),
inverted by global fast diagonalisation.  On rectilinear meshes this is the
exact inverse of the order-1 spectral-element operator.

Hybrid Schwarz multigrid (additive over levels, as the paper's Neko solver
combines them): for a fine residual r,

  z = Sw_0(r) + P_01 [ Sw_1(R_10 r) + P_12 C^-1 R_21 R_10 r ]

with Sw_l the level-l Schwarz smoother and C^-1 the coarse solve.  The
learned multigrid (not in the paper) keeps the two coarser levels and puts
the learned smoother of oracle/cnn.py in place of Sw_0.  In the
symmetric variant each Sw_l = W^1/2 K_l W^1/2 (W = 1/mult) instead of W K_l,
which makes the whole preconditioner symmetric positive definite, so that CG
can use it.

Flexible GMRES(m) with right preconditioning (Saad 2003, Algorithm 9.6),
modified Gram-Schmidt, Givens rotations, restarts from the true residual;
inner products are the mult-weighted ones of the assembled vectors.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

import oracle


def lagrange_interp(x_from, x_to):
    """J[f, c] = l_c(x_to[f]) for the Lagrange basis on the points x_from."""
    x_from = np.asarray(x_from, dtype=np.float64)
    x_to = np.asarray(x_to, dtype=np.float64)
    J = np.ones((len(x_to), len(x_from)))
    for c in range(len(x_from)):
        for m in range(len(x_from)):
            if m != c:
                J[:, c] *= (x_to - x_from[m]) / (x_from[c] - x_from[m])
    return J


def interp_matrix(Nc, Nf):
    """Interpolation from the order-Nc GLL points to the order-Nf ones."""
    xc, _ = oracle.gll(Nc)
    xf, _ = oracle.gll(Nf)
    return lagrange_interp(xc, xf)


def _apply3(J, u):
    """Tensor product J (x) J (x) J on every element of u[E, k, j, i]."""
    return np.einsum("kc,jb,ia,ecba->ekji", J, J, J, u)


def _apply3T(J, u):
    return np.einsum("kc,jb,ia,ekji->ecba", J, J, J, u)


def level_mesh(spec_like, order):
    """Oracle mesh of the same vertices at another order."""
    m = spec_like
    return oracle.Mesh(m.nelx, m.nely, m.nelz, order, m.vertices, m.periodic, m.dirichlet)


def prolong(J, coarse, fine, zc):
    """P zc: continuous coarse field -> continuous fine field (masked)."""
    return fine.apply_mask(_apply3(J, np.asarray(zc).reshape(coarse.shape)))


def restrict(J, fine, coarse, rf):
    """R rf = P^T rf for a continuous fine residual (masked coarse result)."""
    t = _apply3T(J, np.asarray(rf).reshape(fine.shape) / fine.mult)
    return coarse.apply_mask(coarse.dssum(t))


# --------------------------------------------------------------------------
# Fast-diagonalisation local solves


def element_lengths(mesh):
    """L[e, d]: mean length of element e's four edges along axis d."""
    V = mesh.vertices
    L = np.zeros((mesh.E, 3))
    for e in range(mesh.E):
        ex = e % mesh.nelx
        ey = (e // mesh.nelx) % mesh.nely
        ez = e // (mesh.nelx * mesh.nely)
        C = V[ez:ez + 2, ey:ey + 2, ex:ex + 2, :]        # [c][b][a][xyz]
        L[e, 0] = np.mean([np.linalg.norm(C[c, b, 1] - C[c, b, 0]) for b in (0, 1) for c in (0, 1)])
        L[e, 1] = np.mean([np.linalg.norm(C[c, 1, a] - C[c, 0, a]) for a in (0, 1) for c in (0, 1)])
        L[e, 2] = np.mean([np.linalg.norm(C[1, b, a] - C[0, b, a]) for a in (0, 1) for b in (0, 1)])
    return L


def _elem_index(mesh, e):
    return e % mesh.nelx, (e // mesh.nelx) % mesh.nely, e // (mesh.nelx * mesh.nely)


def _neighbour(mesh, idx, d, side):
    """Element index along axis d of the left (side=0) / right (1) neighbour,
    or None at a domain boundary."""
    nel = (mesh.nelx, mesh.nely, mesh.nelz)[d]
    q = idx[d] + (1 if side else -1)
    if 0 <= q < nel:
        return q
    return (q % nel) if mesh.periodic[d] else None


def local_1d(mesh, L, e, d):
    """(A_d, B_d, keep) of element e along axis d (see module docstring)."""
    N = mesh.N
    _, w = oracle.gll(N)
    D = oracle.deriv(N)
    Ahat = D.T @ np.diag(w) @ D
    idx = _elem_index(mesh, e)
    Le = L[e, d]
    A = (2.0 / Le) * Ahat
    B = np.diag((Le / 2.0) * w)
    keep = np.ones(N + 1, dtype=bool)
    stride = [1, mesh.nelx, mesh.nelx * mesh.nely][d]
    for side, node, other in ((0, 0, N), (1, N, 0)):
        q = _neighbour(mesh, idx, d, side)
        if q is None:
            if (mesh.dirichlet >> (2 * d + side)) & 1:
                keep[node] = False
            continue
        en = e + (q - idx[d]) * stride
        Ln = L[en, d]
        A[node, node] += (2.0 / Ln) * Ahat[other, other]
        B[node, node] += (Ln / 2.0) * w[other]
    return A, B, keep


def fdm_factors(A, B, keep):
    """S (columns B-orthonormal eigenvectors) and eigenvalues of the kept block."""
    k = np.nonzero(keep)[0]
    lam, S = scipy.linalg.eigh(A[np.ix_(k, k)], B[np.ix_(k, k)])
    return S, lam, k


def fdm_solve(factors, re, h1, h2):
    """Separable local solve on one element's tile re[k, j, i]."""
    (Sx, lx, kx), (Sy, ly, ky), (Sz, lz, kz) = factors
    sub = re[np.ix_(kz, ky, kx)]
    t = np.einsum("ai,kja->kji", Sx, sub)
    t = np.einsum("bj,kbi->kji", Sy, t)
    t = np.einsum("ck,cji->kji", Sz, t)
    d = h1 * (lz[:, None, None] + ly[None, :, None] + lx[None, None, :]) + h2
    with np.errstate(divide="ignore"):
        t = np.where(d != 0.0, t / np.where(d != 0.0, d, 1.0), 0.0)
    t = np.einsum("ai,kji->kja", Sx, t)
    t = np.einsum("bj,kji->kbi", Sy, t)
    t = np.einsum("ck,kji->cji", Sz, t)
    out = np.zeros_like(re)
    out[np.ix_(kz, ky, kx)] = t
    return out


class SchwarzLevel:
    """Per-element separable local solvers of one level."""

    def __init__(self, mesh):
        self.mesh = mesh
        self.L = element_lengths(mesh)
        self.factors = [[fdm_factors(*local_1d(mesh, self.L, e, d)) for d in range(3)]
                        for e in range(mesh.E)]

    def local_solves(self, r, h1, h2):
        """Unassembled local corrections: element e's FDM solve of r_e."""
        r = np.asarray(r).reshape(self.mesh.shape)
        return np.stack([fdm_solve(self.factors[e], r[e], h1, h2) for e in range(self.mesh.E)])

    def smooth(self, r, h1, h2, weighted=True, sym=False):
        """Additive Schwarz: sum of the local corrections, averaged over the
        copies of every node (weighted) or plainly summed, masked.  sym: the
        symmetric weighting W^1/2 K W^1/2 with W = 1/mult (the residual and
        the summed corrections each divided by sqrt(mult))."""
        if sym:
            ms = np.sqrt(self.mesh.mult)
            z = self.mesh.dssum(self.local_solves(np.asarray(r).reshape(self.mesh.shape) / ms, h1, h2)) / ms
            return self.mesh.apply_mask(z)
        z = self.mesh.dssum(self.local_solves(r, h1, h2))
        if weighted:
            z = z / self.mesh.mult
        return self.mesh.apply_mask(z)


# --------------------------------------------------------------------------
# Coarse solve


def axis_planes(mesh, d):
    """Vertex-plane coordinates along axis d, averaged over the other two
    vertex indices."""
    V = mesh.vertices[..., d]
    axes = {0: (0, 1), 1: (0, 2), 2: (1, 2)}[d]
    return V.mean(axis=axes)


def coarse_1d(mesh, d):
    """Global 1-D linear-element stiffness and lumped mass along axis d on
    the averaged planes, restricted to the kept (non-Dirichlet) nodes, and
    the kept node indices of the order-1 lattice."""
    X = axis_planes(mesh, d)
    nel = len(X) - 1
    per = bool(mesh.periodic[d])
    n = nel if per else nel + 1
    A = np.zeros((n, n))
    B = np.zeros((n, n))
    for q in range(nel):
        h = X[q + 1] - X[q]
        a, b = q, (q + 1) % n
        A[a, a] += 1.0 / h
        A[b, b] += 1.0 / h
        A[a, b] -= 1.0 / h
        A[b, a] -= 1.0 / h
        B[a, a] += h / 2.0
        B[b, b] += h / 2.0
    keep = np.ones(n, dtype=bool)
    if not per:
        if mesh.dirichlet >> (2 * d) & 1:
            keep[0] = False
        if mesh.dirichlet >> (2 * d + 1) & 1:
            keep[n - 1] = False
    k = np.nonzero(keep)[0]
    return A[np.ix_(k, k)], B[np.ix_(k, k)], k, n


class CoarseSolver:
    """Global fast diagonalisation of the separable order-1 operator."""

    def __init__(self, coarse_mesh):
        self.mesh = coarse_mesh
        assert coarse_mesh.N == 1
        self.axes = []
        for d in range(3):
            A, B, k, n = coarse_1d(coarse_mesh, d)
            lam, S = scipy.linalg.eigh(A, B)
            self.axes.append((S, lam, k, n))

    def solve(self, rc, h1, h2):
        m = self.mesh
        (Sx, lx, kx, nx), (Sy, ly, ky, ny), (Sz, lz, kz, nz) = self.axes
        g = m.gather_global(np.asarray(rc).reshape(m.shape)).reshape(nz, ny, nx)
        t = g[np.ix_(kz, ky, kx)]
        t = np.einsum("ai,kja->kji", Sx, t)
        t = np.einsum("bj,kbi->kji", Sy, t)
        t = np.einsum("ck,cji->kji", Sz, t)
        d = h1 * (lz[:, None, None] + ly[None, :, None] + lx[None, None, :]) + h2
        small = np.abs(d) <= 1e-12 * np.max(np.abs(d))
        t = np.where(small, 0.0, t / np.where(small, 1.0, d))
        t = np.einsum("ai,kji->kja", Sx, t)
        t = np.einsum("bj,kji->kbi", Sy, t)
        t = np.einsum("ck,kji->cji", Sz, t)
        out = np.zeros((nz, ny, nx))
        out[np.ix_(kz, ky, kx)] = t
        return m.apply_mask(out.ravel()[m.glo])


# --------------------------------------------------------------------------
# Hybrid Schwarz multigrid


class HSMG:
    """Three-level hybrid Schwarz multigrid (orders N, n_mid, 1); the middle
    order defaults to min(3, N - 1)."""

    def __init__(self, fine, n_mid=None):
        if n_mid is None:
            n_mid = min(3, fine.N - 1)
        self.fine = fine
        self.mid = level_mesh(fine, n_mid)
        self.crs = level_mesh(fine, 1)
        self.J_fm = interp_matrix(n_mid, fine.N)
        self.J_mc = interp_matrix(1, n_mid)
        self.sw_f = SchwarzLevel(fine)
        self.sw_m = SchwarzLevel(self.mid)
        self.coarse = CoarseSolver(self.crs)

    def apply(self, r, h1=1.0, h2=0.0, sym=False, fine=None):
        """z = M r; sym: the symmetric weighting on the fine and mid levels
        (a symmetric positive definite M, for CG).  fine: a callable r -> z
        that replaces the fine Schwarz level (the learned multigrid puts the
        learned smoother there); the coarser levels are unchanged."""
        r = np.asarray(r).reshape(self.fine.shape)
        z = self.sw_f.smooth(r, h1, h2, sym=sym) if fine is None else fine(r)
        return z + self.coarse_part(r, h1, h2, sym)

    def coarse_part(self, r, h1=1.0, h2=0.0, sym=False):
        """P_01 [Sw_1(R_10 r) + P_12 C^-1 R_21 R_10 r]: what the middle and
        coarse levels add to the fine level's output."""
        r = np.asarray(r).reshape(self.fine.shape)
        r1 = restrict(self.J_fm, self.fine, self.mid, r)
        z1 = self.sw_m.smooth(r1, h1, h2, sym=sym)
        r2 = restrict(self.J_mc, self.mid, self.crs, r1)
        z2 = self.coarse.solve(r2, h1, h2)
        z1 = z1 + prolong(self.J_mc, self.crs, self.mid, z2)
        return prolong(self.J_fm, self.mid, self.fine, z1)


def block_jacobi(level, r, h1, h2):
    """The velocity preconditioner: unweighted sum of the element-local
    separable solves (symmetric positive definite, for CG)."""
    return level.smooth(r, h1, h2, weighted=False)


# --------------------------------------------------------------------------
# Flexible GMRES


def fgmres(mesh, b, precond, h1=1.0, h2=0.0, tol=1e-10, restart=30, max_iter=2000):
    """Right-preconditioned flexible GMRES(m) on S x = b (x from zero).
    precond(r) -> z.  Returns (x, info) with the iteration count, the
    residual-norm estimate per iteration and the final true residual."""
    dot = mesh.dot
    x = np.zeros(mesh.shape)
    bn = np.sqrt(dot(b, b))
    info = {"iterations": 0, "history": [1.0], "restarts": 0}
    if bn == 0.0:
        info["true_rel_res"] = 0.0
        return x, info
    r = np.asarray(b, dtype=np.float64).reshape(mesh.shape).copy()
    beta = bn
    it = 0
    while it < max_iter:
        V = [r / beta]
        Z = []
        H = np.zeros((restart + 1, restart))
        cs = np.zeros(restart)
        sn = np.zeros(restart)
        g = np.zeros(restart + 1)
        g[0] = beta
        j = -1
        for j in range(restart):
            Z.append(precond(V[j]))
            w = mesh.apply_S(Z[j], h1, h2)
            for i in range(j + 1):
                H[i, j] = dot(w, V[i])
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.sqrt(dot(w, w))
            V.append(w / H[j + 1, j] if H[j + 1, j] > 0 else w)
            for i in range(j):
                a, c = H[i, j], H[i + 1, j]
                H[i, j] = cs[i] * a + sn[i] * c
                H[i + 1, j] = -sn[i] * a + cs[i] * c
            den = np.hypot(H[j, j], H[j + 1, j])
            cs[j], sn[j] = H[j, j] / den, H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            it += 1
            info["history"].append(abs(g[j + 1]) / bn)
            if abs(g[j + 1]) <= tol * bn or it >= max_iter:
                break
        k = j + 1
        y = scipy.linalg.solve_triangular(H[:k, :k], g[:k])
        for i in range(k):
            x = x + y[i] * Z[i]
        r = np.asarray(b).reshape(mesh.shape) - mesh.apply_S(x, h1, h2)
        beta = np.sqrt(dot(r, r))
        if beta <= tol * bn:
            break
        info["restarts"] += 1
    info["iterations"] = it
    info["true_rel_res"] = beta / bn
    return x, info


def pcg(mesh, b, precond, h1=1.0, h2=0.0, tol=1e-10, max_iter=20000):
    """Preconditioned CG (Hestenes & Stiefel) with a symmetric positive
    definite precond(r) -> z; recursive-residual stop ||r|| <= tol ||b||.
    Returns (x, info)."""
    dot = mesh.dot
    x = np.zeros(mesh.shape)
    r = np.asarray(b, dtype=np.float64).reshape(mesh.shape).copy()
    bn = np.sqrt(dot(r, r))
    info = {"iterations": 0}
    if bn == 0.0:
        info["true_rel_res"] = 0.0
        return x, info
    z = precond(r)
    p = z.copy()
    rz = dot(r, z)
    it = 0
    while it < max_iter:
        w = mesh.apply_S(p, h1, h2)
        alpha = rz / dot(p, w)
        x = x + alpha * p
        r = r - alpha * w
        it += 1
        if np.sqrt(dot(r, r)) <= tol * bn:
            break
        z = precond(r)
        rz_new = dot(r, z)
        p = z + (rz_new / rz) * p
        rz = rz_new
    res = np.asarray(b).reshape(mesh.shape) - mesh.apply_S(x, h1, h2)
    info["iterations"] = it
    info["true_rel_res"] = np.sqrt(dot(res, res)) / bn
    return x, info
