/*
 * sem_oracle.c -- plain, slow, obviously correct FP64 CPU oracle for the
 * spectral-element pressure-solve hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes
 * or calls this file; only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark load it.  It shares no code, header, table or constant
 * generator with the HIP library.
 *
 * What it follows:
 *  - The paper (Karp et al., "Experience and Analysis of Scalable High-Fidelity
 *    CFD on Modular Supercomputing Architectures"), section 3.1 "Neko": the
 *    domain is split into E non-overlapping hexahedra, the solution is an
 *    order-N polynomial collocated on the Gauss-Lobatto-Legendre (GLL) points,
 *    operators are evaluated element by element (matrix-free), the only
 *    coupling between elements is a unit-depth gather-scatter, and a
 *    preconditioned Krylov method solves Ax=b.  The paper defers the method
 *    itself to Deville, Fischer & Mund (2002), "High-Order Methods for
 *    Incompressible Fluid Flow"; the definitions below are the textbook ones.
 *  - Conjugate gradients: Hestenes & Stiefel (1952), point-Jacobi
 *    preconditioned.
 *
 * Layout: local ("E-vector") arrays are [E][k][j][i] with i (r direction)
 * fastest; element e = ex + nelx*(ey + nely*ez).  Geometric factors are six
 * arrays of n_local values in the order G11 G12 G13 G22 G23 G33.
 *
 * Every loop is written in the order of the definition it implements.  OpenMP
 * is used only over independent elements (no reduction changes order).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define NP(N) ((N) + 1)

/* ------------------------------------------------------------------------ */
/* Reference element: GLL nodes, weights, derivative matrix (Deville et al.
 * 2002, sec. 2.4; the paper's sec. 3.1 places the unknowns on these points). */

/* Legendre P_n(x) and P_{n-1}(x) by the three-term recurrence
 * (k+1) P_{k+1} = (2k+1) x P_k - k P_{k-1}. */
static void legendre_pair(int n, double x, double *pn, double *pnm1)
{
    double p0 = 1.0, p1 = x;
    if (n == 0) { *pn = 1.0; *pnm1 = 0.0; return; }
    for (int k = 1; k < n; ++k) {
        double p2 = ((2.0 * k + 1.0) * x * p1 - k * p0) / (k + 1.0);
        p0 = p1;
        p1 = p2;
    }
    *pn = p1;
    *pnm1 = p0;
}

/* GLL nodes: xi_0 = -1, xi_N = +1, interior = roots of P_N'.  Newton on
 * f(x) = (1-x^2) P_N'(x) = N (P_{N-1} - x P_N), whose derivative by the
 * Legendre equation is -N(N+1) P_N, so the step is
 * x += (P_{N-1} - x P_N) / ((N+1) P_N).  Weights w_j = 2/(N(N+1) P_N(xi_j)^2).
 * Returns 0, or -1 for N < 1. */
int ora_gll(int N, double *xi, double *w)
{
    if (N < 1) return -1;
    const double pi = 3.14159265358979323846;
    for (int j = 0; j <= N; ++j) {
        double x;
        if (j == 0) x = -1.0;
        else if (j == N) x = 1.0;
        else {
            x = -cos(pi * j / N);
            for (int it = 0; it < 100; ++it) {
                double pn, pnm1;
                legendre_pair(N, x, &pn, &pnm1);
                double dx = (pnm1 - x * pn) / ((N + 1.0) * pn);
                x += dx;
                if (fabs(dx) < 1e-17) break;
            }
        }
        xi[j] = x;
    }
    /* symmetric pairs: enforce exact antisymmetry of the node set */
    for (int j = 0; j <= N / 2; ++j) {
        double a = 0.5 * (xi[N - j] - xi[j]);
        xi[j] = -a;
        xi[N - j] = a;
    }
    if (N % 2 == 0) xi[N / 2] = 0.0;
    for (int j = 0; j <= N; ++j) {
        double pn, pnm1;
        legendre_pair(N, xi[j], &pn, &pnm1);
        w[j] = 2.0 / (N * (N + 1.0) * pn * pn);
    }
    return 0;
}

/* D[i*(N+1)+j] = l_j'(xi_i) for the Lagrange basis on the GLL nodes:
 * P_N(xi_i) / (P_N(xi_j) (xi_i - xi_j)) off the diagonal,
 * -N(N+1)/4 at (0,0), +N(N+1)/4 at (N,N), 0 elsewhere on the diagonal. */
void ora_deriv(int N, const double *xi, double *D)
{
    const int n = NP(N);
    double *pn = (double *)malloc(sizeof(double) * n);
    for (int j = 0; j < n; ++j) {
        double q;
        legendre_pair(N, xi[j], &pn[j], &q);
    }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            double d;
            if (i != j) d = pn[i] / (pn[j] * (xi[i] - xi[j]));
            else if (i == 0) d = -0.25 * N * (N + 1.0);
            else if (i == N) d = 0.25 * N * (N + 1.0);
            else d = 0.0;
            D[i * n + j] = d;
        }
    free(pn);
}

/* ------------------------------------------------------------------------ */
/* Mesh geometry (Deville et al. 2002, sec. 4.1-4.3): trilinear map of each
 * hexahedron evaluated at the GLL points, isoparametric Jacobian from the
 * derivative matrix, and the metric terms of the weak Laplacian. */

static inline int64_t vtx(int nelx, int nely, int ix, int iy, int iz)
{
    return ((int64_t)iz * (nely + 1) + iy) * (nelx + 1) + ix;
}

/* xyz: 3 arrays of n_local; G: 6 arrays of n_local (G11 G12 G13 G22 G23 G33);
 * B: n_local; jac: optional n_local detJ.  Returns 0, or the 1-based index of
 * the first element with detJ <= 0 at some node. */
int64_t ora_geometry(int nelx, int nely, int nelz, int N, const double *vert,
                     double *xyz, double *G, double *B, double *jac)
{
    const int n = NP(N);
    const int64_t p = (int64_t)n * n * n;
    const int64_t E = (int64_t)nelx * nely * nelz;
    const int64_t nl = E * p;
    double xi[32], wq[32], D[32 * 32];
    ora_gll(N, xi, wq);
    ora_deriv(N, xi, D);
    int64_t bad = 0;

#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < E; ++e) {
        const int ex = (int)(e % nelx);
        const int ey = (int)((e / nelx) % nely);
        const int ez = (int)(e / ((int64_t)nelx * nely));
        double X[3][2][2][2]; /* corner coordinates X[c][ct][cs][cr] */
        for (int c3 = 0; c3 < 2; ++c3)
            for (int c2 = 0; c2 < 2; ++c2)
                for (int c1 = 0; c1 < 2; ++c1) {
                    const double *v = vert + 3 * vtx(nelx, nely, ex + c1, ey + c2, ez + c3);
                    for (int c = 0; c < 3; ++c) X[c][c3][c2][c1] = v[c];
                }
        double *x = (double *)malloc(sizeof(double) * 3 * p);
        for (int k = 0; k < n; ++k)
            for (int j = 0; j < n; ++j)
                for (int i = 0; i < n; ++i) {
                    const double pr[2] = {0.5 * (1.0 - xi[i]), 0.5 * (1.0 + xi[i])};
                    const double ps[2] = {0.5 * (1.0 - xi[j]), 0.5 * (1.0 + xi[j])};
                    const double pt[2] = {0.5 * (1.0 - xi[k]), 0.5 * (1.0 + xi[k])};
                    const int64_t l = i + n * (j + n * k);
                    for (int c = 0; c < 3; ++c) {
                        double s = 0.0;
                        for (int c3 = 0; c3 < 2; ++c3)
                            for (int c2 = 0; c2 < 2; ++c2)
                                for (int c1 = 0; c1 < 2; ++c1)
                                    s += X[c][c3][c2][c1] * pr[c1] * ps[c2] * pt[c3];
                        x[c * p + l] = s;
                        xyz[c * nl + e * p + l] = s;
                    }
                }
        for (int k = 0; k < n; ++k)
            for (int j = 0; j < n; ++j)
                for (int i = 0; i < n; ++i) {
                    const int64_t l = i + n * (j + n * k);
                    double J[3][3]; /* J[c][a] = d x_c / d r_a */
                    for (int c = 0; c < 3; ++c) {
                        double dr = 0.0, ds = 0.0, dt = 0.0;
                        for (int m = 0; m < n; ++m) {
                            dr += D[i * n + m] * x[c * p + (m + n * (j + n * k))];
                            ds += D[j * n + m] * x[c * p + (i + n * (m + n * k))];
                            dt += D[k * n + m] * x[c * p + (i + n * (j + n * m))];
                        }
                        J[c][0] = dr;
                        J[c][1] = ds;
                        J[c][2] = dt;
                    }
                    const double det =
                        J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                        J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                        J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
                    if (!(det > 0.0)) {
#pragma omp critical
                        {
                            if (bad == 0 || e + 1 < bad) bad = e + 1;
                        }
                    }
                    /* rows of J^{-1}: gradients of r, s, t in physical space */
                    double gr[3][3];
                    gr[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / det;
                    gr[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
                    gr[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
                    gr[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / det;
                    gr[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
                    gr[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
                    gr[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / det;
                    gr[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
                    gr[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
                    const double wdet = wq[i] * wq[j] * wq[k] * det;
                    const int ab[6][2] = {{0, 0}, {0, 1}, {0, 2}, {1, 1}, {1, 2}, {2, 2}};
                    for (int q = 0; q < 6; ++q) {
                        const int a = ab[q][0], b = ab[q][1];
                        G[q * nl + e * p + l] =
                            wdet * (gr[a][0] * gr[b][0] + gr[a][1] * gr[b][1] + gr[a][2] * gr[b][2]);
                    }
                    B[e * p + l] = wdet;
                    if (jac) jac[e * p + l] = det;
                }
        free(x);
    }
    return bad;
}

/* ------------------------------------------------------------------------ */
/* Global numbering for the gather-scatter (paper sec. 3.1: the only coupling
 * between elements).  Derived from coordinates, not index arithmetic: every
 * local node gets its position on the undeformed element lattice in element
 * units, X = ex + (1 + xi_i)/2 (exact at element faces), wrapped to 0 at the
 * far plane of a periodic direction.  All local nodes are sorted
 * lexicographically by (Z, Y, X); equal positions are one global node, and
 * global ids are assigned in that sorted order. */

typedef struct {
    double key[3]; /* Z, Y, X */
    int64_t l;
} node_key;

static int cmp_key(const void *a, const void *b)
{
    const node_key *p = (const node_key *)a, *q = (const node_key *)b;
    for (int c = 0; c < 3; ++c) {
        if (p->key[c] < q->key[c]) return -1;
        if (p->key[c] > q->key[c]) return 1;
    }
    return (p->l < q->l) ? -1 : (p->l > q->l);
}

/* glo (n_local int64), mult (n_local int32), mask (n_local uint8: 1 = the
 * node lies on a non-periodic face whose Dirichlet bit is set; bits 0..5 =
 * x-, x+, y-, y+, z-, z+).  Returns n_global, or -1 on bad input. */
int64_t ora_numbering(int nelx, int nely, int nelz, int N, const uint8_t *periodic,
                      uint8_t dirichlet, int64_t *glo, int32_t *mult, uint8_t *mask)
{
    if (nelx < 1 || nely < 1 || nelz < 1 || N < 1) return -1;
    const int n = NP(N);
    const int64_t p = (int64_t)n * n * n;
    const int64_t E = (int64_t)nelx * nely * nelz;
    const int64_t nl = E * p;
    const int nel[3] = {nelx, nely, nelz};
    double xi[32], wq[32];
    ora_gll(N, xi, wq);
    node_key *keys = (node_key *)malloc(sizeof(node_key) * nl);
    if (!keys) return -1;
    for (int64_t e = 0; e < E; ++e) {
        const int ec[3] = {(int)(e % nelx), (int)((e / nelx) % nely), (int)(e / ((int64_t)nelx * nely))};
        for (int64_t l = 0; l < p; ++l) {
            const int ic[3] = {(int)(l % n), (int)((l / n) % n), (int)(l / (n * n))};
            node_key *kk = &keys[e * p + l];
            for (int d = 0; d < 3; ++d) {
                double X = ec[d] + 0.5 * (1.0 + xi[ic[d]]);
                if (periodic[d] && X == (double)nel[d]) X = 0.0;
                kk->key[2 - d] = X;
            }
            kk->l = e * p + l;
            uint8_t m = 0;
            for (int d = 0; d < 3; ++d) {
                if (periodic[d]) continue;
                const double X = kk->key[2 - d];
                if (X == 0.0 && (dirichlet >> (2 * d) & 1)) m = 1;
                if (X == (double)nel[d] && (dirichlet >> (2 * d + 1) & 1)) m = 1;
            }
            mask[e * p + l] = m;
        }
    }
    qsort(keys, (size_t)nl, sizeof(node_key), cmp_key);
    int64_t g = -1;
    for (int64_t q = 0; q < nl; ++q) {
        if (q == 0 || keys[q].key[0] != keys[q - 1].key[0] || keys[q].key[1] != keys[q - 1].key[1] ||
            keys[q].key[2] != keys[q - 1].key[2])
            ++g;
        glo[keys[q].l] = g;
    }
    free(keys);
    const int64_t ng = g + 1;
    int32_t *cnt = (int32_t *)calloc((size_t)ng, sizeof(int32_t));
    for (int64_t l = 0; l < nl; ++l) cnt[glo[l]]++;
    for (int64_t l = 0; l < nl; ++l) mult[l] = cnt[glo[l]];
    free(cnt);
    return ng;
}

/* ------------------------------------------------------------------------ */
/* Local operator (Deville et al. 2002, sec. 4.4): for each element
 *   w = h1 * sum_a D_a^T ( sum_b G_ab (D_b u) ) + h2 * B u
 * with D_r = I(x)I(x)D, D_s = I(x)D(x)I, D_t = D(x)I(x)I.  Unassembled. */
void ora_ax(int64_t E, int N, const double *D, const double *G, const double *B,
            double h1, double h2, const double *u, double *w)
{
    const int n = NP(N);
    const int64_t p = (int64_t)n * n * n;
    const int64_t nl = E * p;
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < E; ++e) {
        const double *ue = u + e * p;
        double *ur = (double *)malloc(sizeof(double) * 6 * p);
        double *us = ur + p, *ut = ur + 2 * p, *fr = ur + 3 * p, *fs = ur + 4 * p, *ft = ur + 5 * p;
        for (int k = 0; k < n; ++k)
            for (int j = 0; j < n; ++j)
                for (int i = 0; i < n; ++i) {
                    const int l = i + n * (j + n * k);
                    double a = 0.0, b = 0.0, c = 0.0;
                    for (int m = 0; m < n; ++m) {
                        a += D[i * n + m] * ue[m + n * (j + n * k)];
                        b += D[j * n + m] * ue[i + n * (m + n * k)];
                        c += D[k * n + m] * ue[i + n * (j + n * m)];
                    }
                    ur[l] = a;
                    us[l] = b;
                    ut[l] = c;
                }
        for (int64_t l = 0; l < p; ++l) {
            const int64_t q = e * p + l;
            const double g11 = G[0 * nl + q], g12 = G[1 * nl + q], g13 = G[2 * nl + q];
            const double g22 = G[3 * nl + q], g23 = G[4 * nl + q], g33 = G[5 * nl + q];
            fr[l] = g11 * ur[l] + g12 * us[l] + g13 * ut[l];
            fs[l] = g12 * ur[l] + g22 * us[l] + g23 * ut[l];
            ft[l] = g13 * ur[l] + g23 * us[l] + g33 * ut[l];
        }
        for (int k = 0; k < n; ++k)
            for (int j = 0; j < n; ++j)
                for (int i = 0; i < n; ++i) {
                    const int l = i + n * (j + n * k);
                    double s = 0.0;
                    for (int m = 0; m < n; ++m) {
                        s += D[m * n + i] * fr[m + n * (j + n * k)];
                        s += D[m * n + j] * fs[i + n * (m + n * k)];
                        s += D[m * n + k] * ft[i + n * (j + n * m)];
                    }
                    w[e * p + l] = h1 * s + h2 * B[e * p + l] * ue[l];
                }
        free(ur);
    }
}

/* ------------------------------------------------------------------------ */
/* Direct-stiffness summation w <- Q Q^T w: every global node receives the sum
 * of its local copies, accumulated in ascending local index, and the sum is
 * written back to every copy. */
void ora_dssum(int64_t nl, const int64_t *glo, int64_t ng, double *u)
{
    double *s = (double *)calloc((size_t)ng, sizeof(double));
    for (int64_t l = 0; l < nl; ++l) s[glo[l]] += u[l];
    for (int64_t l = 0; l < nl; ++l) u[l] = s[glo[l]];
    free(s);
}

void ora_mask(int64_t nl, const uint8_t *mask, double *u)
{
    for (int64_t l = 0; l < nl; ++l)
        if (mask[l]) u[l] = 0.0;
}

/* Assembled operator S u = mask(dssum(A_L u)). */
static void apply_S(int64_t E, int N, const double *D, const double *G, const double *B,
                    double h1, double h2, const int64_t *glo, int64_t ng, const uint8_t *mask,
                    const double *u, double *w)
{
    const int64_t nl = E * NP(N) * NP(N) * NP(N);
    ora_ax(E, N, D, G, B, h1, h2, u, w);
    ora_dssum(nl, glo, ng, w);
    ora_mask(nl, mask, w);
}

void ora_apply_S(int64_t E, int N, const double *D, const double *G, const double *B,
                 double h1, double h2, const int64_t *glo, int64_t ng, const uint8_t *mask,
                 const double *u, double *w)
{
    apply_S(E, N, D, G, B, h1, h2, glo, ng, mask, u, w);
}

/* Diagonal of the unassembled element matrices, written out from the
 * operator definition (the cross terms survive only where D_ii != 0, i.e. on
 * element faces). */
void ora_diag_local(int64_t E, int N, const double *D, const double *G, const double *B,
                    double h1, double h2, double *d)
{
    const int n = NP(N);
    const int64_t p = (int64_t)n * n * n;
    const int64_t nl = E * p;
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < E; ++e)
        for (int k = 0; k < n; ++k)
            for (int j = 0; j < n; ++j)
                for (int i = 0; i < n; ++i) {
                    const int64_t q = e * p + i + n * (j + n * k);
                    double s = 0.0;
                    for (int m = 0; m < n; ++m) {
                        s += G[0 * nl + e * p + m + n * (j + n * k)] * D[m * n + i] * D[m * n + i];
                        s += G[3 * nl + e * p + i + n * (m + n * k)] * D[m * n + j] * D[m * n + j];
                        s += G[5 * nl + e * p + i + n * (j + n * m)] * D[m * n + k] * D[m * n + k];
                    }
                    s += 2.0 * G[1 * nl + q] * D[i * n + i] * D[j * n + j];
                    s += 2.0 * G[2 * nl + q] * D[i * n + i] * D[k * n + k];
                    s += 2.0 * G[4 * nl + q] * D[j * n + j] * D[k * n + k];
                    d[q] = h1 * s + h2 * B[q];
                }
}

/* Assembled Jacobi diagonal: d = mask(dssum(diag A_L)), with d = 1 on the
 * masked nodes; returns its reciprocal. */
void ora_jacobi_inv(int64_t E, int N, const double *D, const double *G, const double *B,
                    double h1, double h2, const int64_t *glo, int64_t ng, const uint8_t *mask,
                    double *dinv)
{
    const int64_t nl = E * NP(N) * NP(N) * NP(N);
    ora_diag_local(E, N, D, G, B, h1, h2, dinv);
    ora_dssum(nl, glo, ng, dinv);
    for (int64_t l = 0; l < nl; ++l) dinv[l] = mask[l] ? 1.0 : 1.0 / dinv[l];
}

/* Inner product of two continuous local-form vectors: every global node
 * counted once, (u,v) = sum_l u_l v_l / mult_l, summed in ascending l. */
double ora_dot(int64_t nl, const double *u, const double *v, const int32_t *mult)
{
    double s = 0.0;
    for (int64_t l = 0; l < nl; ++l) s += u[l] * v[l] / (double)mult[l];
    return s;
}

/* ------------------------------------------------------------------------ */
/* Point-Jacobi preconditioned conjugate gradients (Hestenes & Stiefel 1952)
 * on S x = b in local form.  x starts at zero; stops when the recursive
 * residual satisfies ||r|| <= tol ||b||; the true residual ||b - S x|| is then
 * evaluated and, while it exceeds tol ||b||, CG restarts from the current x
 * (at most 3 restarts).
 * out[0] = iterations (operator applications inside the loop),
 * out[1] = final recursive relative residual, out[2] = true relative residual,
 * out[3] = number of restarts.  hist (optional, length max_iter+1) receives
 * the recursive relative residual after every iteration (hist[0] = 1).
 * Returns 0 (converged), 1 (max_iter reached), 2 (breakdown). */
int ora_pcg(int64_t E, int N, const double *D, const double *G, const double *B,
            double h1, double h2, const int64_t *glo, int64_t ng, const uint8_t *mask,
            const int32_t *mult, const double *dinv, const double *b, double *x,
            double tol, int max_iter, double *out, double *hist)
{
    const int64_t nl = E * NP(N) * NP(N) * NP(N);
    double *r = (double *)malloc(sizeof(double) * nl);
    double *z = (double *)malloc(sizeof(double) * nl);
    double *pv = (double *)malloc(sizeof(double) * nl);
    double *w = (double *)malloc(sizeof(double) * nl);
    const double bnorm = sqrt(ora_dot(nl, b, b, mult));
    int it = 0, status = 1, restarts = 0;
    double rel = 0.0, true_rel = 0.0;
    for (int64_t l = 0; l < nl; ++l) x[l] = 0.0;
    if (hist) hist[0] = 1.0;
    if (bnorm == 0.0) {
        out[0] = 0; out[1] = 0; out[2] = 0; out[3] = 0;
        free(r); free(z); free(pv); free(w);
        return 0;
    }
    for (int64_t l = 0; l < nl; ++l) r[l] = b[l];
    for (;;) {
        for (int64_t l = 0; l < nl; ++l) z[l] = dinv[l] * r[l];
        for (int64_t l = 0; l < nl; ++l) pv[l] = z[l];
        double rz = ora_dot(nl, r, z, mult);
        rel = sqrt(ora_dot(nl, r, r, mult)) / bnorm;
        int converged = rel <= tol;
        while (!converged && it < max_iter) {
            apply_S(E, N, D, G, B, h1, h2, glo, ng, mask, pv, w);
            const double pw = ora_dot(nl, pv, w, mult);
            if (!(pw > 0.0) || !isfinite(pw)) { status = 2; goto done; }
            const double alpha = rz / pw;
            for (int64_t l = 0; l < nl; ++l) x[l] += alpha * pv[l];
            for (int64_t l = 0; l < nl; ++l) r[l] -= alpha * w[l];
            ++it;
            rel = sqrt(ora_dot(nl, r, r, mult)) / bnorm;
            if (hist) hist[it] = rel;
            if (rel <= tol) { converged = 1; break; }
            for (int64_t l = 0; l < nl; ++l) z[l] = dinv[l] * r[l];
            const double rz_new = ora_dot(nl, r, z, mult);
            const double beta = rz_new / rz;
            rz = rz_new;
            for (int64_t l = 0; l < nl; ++l) pv[l] = z[l] + beta * pv[l];
        }
        if (!converged) { status = 1; break; }
        /* true residual */
        apply_S(E, N, D, G, B, h1, h2, glo, ng, mask, x, w);
        for (int64_t l = 0; l < nl; ++l) r[l] = b[l] - w[l];
        true_rel = sqrt(ora_dot(nl, r, r, mult)) / bnorm;
        if (true_rel <= tol) { status = 0; break; }
        if (restarts == 3 || it >= max_iter) { status = 1; break; }
        ++restarts;
    }
done:
    if (status != 0) {
        apply_S(E, N, D, G, B, h1, h2, glo, ng, mask, x, w);
        for (int64_t l = 0; l < nl; ++l) r[l] = b[l] - w[l];
        true_rel = sqrt(ora_dot(nl, r, r, mult)) / bnorm;
    }
    out[0] = it;
    out[1] = rel;
    out[2] = true_rel;
    out[3] = restarts;
    free(r); free(z); free(pv); free(w);
    return status;
}
