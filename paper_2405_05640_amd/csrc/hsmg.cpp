// hsmg.cpp -- host setup of the hybrid Schwarz multigrid preconditioner
// (the paper's pressure preconditioner, section 3.1; the construction is the
// textbook one of Deville, Fischer & Mund 2002, ch. 8, and Lottes & Fischer
// 2005): per-element separable local solvers at orders N and 3, the
// GLL-to-GLL interpolation matrices between the levels, and the separable
// order-1 coarse solver, all factored by fast diagonalisation.
#include <algorithm>
#include <cmath>
#include <limits>
#include <new>

#include "hsmg.hpp"

namespace sem {
namespace {

// C = Q diag(d) Q^T for a symmetric n x n C (row-major) by cyclic Jacobi
// rotations (Golub & Van Loan, Matrix Computations, sec. 8.5); the columns
// of Q are the eigenvectors.
void sym_eig(int n, std::vector<double> C, std::vector<double> &Q, std::vector<double> &d)
{
    Q.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) Q[(size_t)i * n + i] = 1.0;
    auto at = [&](int r, int c) -> double & { return C[(size_t)r * n + c]; };
    for (int sweep = 0; sweep < 64; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int r = 0; r < n; ++r)
            for (int c = 0; c < n; ++c) {
                const double v = at(r, c) * at(r, c);
                tot += v;
                if (r != c) off += v;
            }
        if (off <= 1e-32 * tot || off == 0.0) break;
        for (int p = 0; p < n - 1; ++p)
            for (int q = p + 1; q < n; ++q) {
                const double apq = at(p, q);
                if (apq == 0.0) continue;
                const double theta = (at(q, q) - at(p, p)) / (2.0 * apq);
                const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
                for (int r = 0; r < n; ++r) {   // columns p, q
                    const double arp = at(r, p), arq = at(r, q);
                    at(r, p) = c * arp - s * arq;
                    at(r, q) = s * arp + c * arq;
                }
                for (int r = 0; r < n; ++r) {   // rows p, q
                    const double apr = at(p, r), aqr = at(q, r);
                    at(p, r) = c * apr - s * aqr;
                    at(q, r) = s * apr + c * aqr;
                }
                at(p, q) = at(q, p) = 0.0;
                for (int r = 0; r < n; ++r) {
                    const double vrp = Q[(size_t)r * n + p], vrq = Q[(size_t)r * n + q];
                    Q[(size_t)r * n + p] = c * vrp - s * vrq;
                    Q[(size_t)r * n + q] = s * vrp + c * vrq;
                }
            }
    }
    d.resize(n);
    for (int i = 0; i < n; ++i) d[i] = at(i, i);
}

// Generalised problem A s = lam B s with B diagonal positive, on the kept
// indices of an n-point axis: S (n x n, row = node, column = mode slot) with
// S^T B S = I on the kept block, eigenvalues lam (+inf for unused slots,
// whose columns are zero; tiny eigenvalues of a singular A are set to 0).
void gen_eig(int n, const std::vector<double> &A, const std::vector<double> &Bd, const std::vector<char> &keep,
             double *S, double *lam)
{
    std::vector<int> k;
    for (int a = 0; a < n; ++a)
        if (keep[a]) k.push_back(a);
    const int nk = (int)k.size();
    for (int q = 0; q < n * n; ++q) S[q] = 0.0;
    for (int q = 0; q < n; ++q) lam[q] = std::numeric_limits<double>::infinity();
    if (nk == 0) return;
    std::vector<double> C((size_t)nk * nk), Q, d;
    for (int r = 0; r < nk; ++r)
        for (int c = 0; c < nk; ++c)
            C[(size_t)r * nk + c] = A[(size_t)k[r] * n + k[c]] / std::sqrt(Bd[k[r]] * Bd[k[c]]);
    sym_eig(nk, C, Q, d);
    double dmax = 0.0;
    for (double v : d) dmax = std::max(dmax, std::fabs(v));
    for (int q = 0; q < nk; ++q) {
        lam[q] = std::fabs(d[q]) <= 1e-12 * dmax ? 0.0 : d[q];
        for (int r = 0; r < nk; ++r) S[(size_t)k[r] * n + q] = Q[(size_t)r * nk + q] / std::sqrt(Bd[k[r]]);
    }
}

// mean length of element (ex, ey, ez)'s four edges along axis d
double edge_length(const sem_mesh_desc &ds, int ex, int ey, int ez, int d)
{
    auto vtx = [&](int x, int y, int z) { return ds.vertices + 3 * (((int64_t)z * (ds.nely + 1) + y) * (ds.nelx + 1) + x); };
    double s = 0.0;
    for (int u = 0; u < 2; ++u)
        for (int v = 0; v < 2; ++v) {
            int a[3] = {ex, ey, ez}, b[3] = {ex, ey, ez};
            const int o1 = (d + 1) % 3, o2 = (d + 2) % 3;
            a[o1] += u; a[o2] += v;
            b[o1] += u; b[o2] += v;
            b[d] += 1;
            const double *p = vtx(a[0], a[1], a[2]), *q = vtx(b[0], b[1], b[2]);
            s += std::sqrt((q[0] - p[0]) * (q[0] - p[0]) + (q[1] - p[1]) * (q[1] - p[1]) + (q[2] - p[2]) * (q[2] - p[2]));
        }
    return 0.25 * s;
}

// Per-element separable local solvers of an order-N level:
// out[e] = [S_x | S_y | S_z | l_x | l_y | l_z].
void element_factors(const sem_mesh_desc &ds, const Mesh &m, int N, const std::vector<double> &L, double *out)
{
    const int NP = N + 1;
    std::vector<double> x, w;
    gll_rule(N, x, w);
    const std::vector<double> D = deriv_matrix(x);
    std::vector<double> Ahat((size_t)NP * NP, 0.0);   // D^T W D
    for (int a = 0; a < NP; ++a)
        for (int b = 0; b < NP; ++b) {
            double s = 0.0;
            for (int q = 0; q < NP; ++q) s += D[(size_t)q * NP + a] * w[q] * D[(size_t)q * NP + b];
            Ahat[(size_t)a * NP + b] = s;
        }
    const int nel[3] = {m.nelx, m.nely, m.nelz};
    const int64_t stride[3] = {1, m.nelx, (int64_t)m.nelx * m.nely};
    const int64_t per_elem = 3 * NP * NP + 3 * NP;
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < m.E; ++e) {
        const int idx[3] = {(int)(e % m.nelx), (int)((e / m.nelx) % m.nely), (int)(e / ((int64_t)m.nelx * m.nely))};
        double *blk = out + e * per_elem;
        for (int d = 0; d < 3; ++d) {
            const double Le = L[(size_t)e * 3 + d];
            std::vector<double> A((size_t)NP * NP), Bd(NP);
            for (int q = 0; q < NP * NP; ++q) A[q] = (2.0 / Le) * Ahat[q];
            for (int q = 0; q < NP; ++q) Bd[q] = 0.5 * Le * w[q];
            std::vector<char> keep(NP, 1);
            for (int side = 0; side < 2; ++side) {
                const int node = side ? N : 0, other = side ? 0 : N;
                int q = idx[d] + (side ? 1 : -1);
                if (q < 0 || q >= nel[d]) {
                    if (!m.periodic[d]) {
                        if ((m.dirichlet >> (2 * d + side)) & 1) keep[node] = 0;
                        continue;
                    }
                    q = (q + nel[d]) % nel[d];
                }
                const double Ln = L[(size_t)(e + (int64_t)(q - idx[d]) * stride[d]) * 3 + d];
                A[(size_t)node * NP + node] += (2.0 / Ln) * Ahat[(size_t)other * NP + other];
                Bd[node] += 0.5 * Ln * w[other];
            }
            gen_eig(NP, A, Bd, keep, blk + d * NP * NP, blk + 3 * NP * NP + d * NP);
        }
    }
}

// J[f][c] = l_c(xf[f]) on the points xc, barycentric form.
std::vector<double> interp(const std::vector<double> &xc, const std::vector<double> &xf)
{
    const int nc = (int)xc.size(), nf = (int)xf.size();
    std::vector<double> lam(nc, 1.0), J((size_t)nf * nc, 0.0);
    for (int c = 0; c < nc; ++c)
        for (int k = 0; k < nc; ++k)
            if (k != c) lam[c] /= (xc[c] - xc[k]);
    for (int f = 0; f < nf; ++f) {
        int hit = -1;
        for (int c = 0; c < nc; ++c)
            if (xf[f] == xc[c]) hit = c;
        if (hit >= 0) {
            J[(size_t)f * nc + hit] = 1.0;
            continue;
        }
        double den = 0.0;
        for (int c = 0; c < nc; ++c) den += lam[c] / (xf[f] - xc[c]);
        for (int c = 0; c < nc; ++c) J[(size_t)f * nc + c] = (lam[c] / (xf[f] - xc[c])) / den;
    }
    return J;
}

template <typename T>
sem_status put(T **dst, const std::vector<T> &src, size_t &acc)
{
    hipError_t e = hipMalloc((void **)dst, src.size() * sizeof(T));
    if (e != hipSuccess) return fail(SEM_ERR_OUT_OF_MEMORY, std::string("hipMalloc (multigrid): ") + hipGetErrorString(e));
    acc += src.size() * sizeof(T);
    SEM_HIP_TRY(hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice));
    return SEM_OK;
}

#define SEM_TRY(x)                   \
    do {                             \
        sem_status _s = (x);         \
        if (_s != SEM_OK) return _s; \
    } while (0)

Lattice level_lattice(const Mesh &m, int N)
{
    const int64_t nx = (int64_t)m.nelx * N + (m.periodic[0] ? 0 : 1);
    const int64_t ny = (int64_t)m.nely * N + (m.periodic[1] ? 0 : 1);
    const int64_t nz = (int64_t)m.nelz * N + (m.periodic[2] ? 0 : 1);
    return Lattice{m.nelx, m.nely, m.nelz, N, N + 1, nx, ny, nz, (int64_t)(N + 1) * (N + 1) * (N + 1),
                   {m.periodic[0], m.periodic[1], m.periodic[2]}, m.dirichlet, {nullptr, nullptr, nullptr}, 0};
}

}  // namespace

sem_status hsmg_setup(const sem_mesh_desc &ds, Mesh &m)
{
    const int nel[3] = {m.nelx, m.nely, m.nelz};
    for (int d = 0; d < 3; ++d) {
        if (m.periodic[d] && nel[d] < 2)
            return fail(SEM_ERR_UNSUPPORTED, "the multigrid preconditioner needs two or more elements along a periodic "
                                             "direction");
        if (nel[d] > 1024) return fail(SEM_ERR_UNSUPPORTED, "the multigrid coarse solve supports up to 1024 elements "
                                                            "per direction");
    }
    if (m.N < 2) return fail(SEM_ERR_UNSUPPORTED, "the multigrid preconditioner needs order N >= 2");
    Hsmg *h = new (std::nothrow) Hsmg();
    if (!h) return fail(SEM_ERR_OUT_OF_MEMORY, "host allocation");
    m.hsmg = h;
    h->Nm = std::min(kHsmgMidOrder, m.N - 1);
    h->lat_m = level_lattice(m, h->Nm);
    h->lat_c = level_lattice(m, 1);
    h->ng_m = h->lat_m.nx * h->lat_m.ny * h->lat_m.nz;
    h->ng_c = h->lat_c.nx * h->lat_c.ny * h->lat_c.nz;
    size_t acc = 0;

    // element lengths
    std::vector<double> L((size_t)m.E * 3);
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < m.E; ++e) {
        const int ex = (int)(e % m.nelx), ey = (int)((e / m.nelx) % m.nely), ez = (int)(e / ((int64_t)m.nelx * m.nely));
        for (int d = 0; d < 3; ++d) L[(size_t)e * 3 + d] = edge_length(ds, ex, ey, ez, d);
    }
    // fine and mid local solvers
    for (int lev = 0; lev < 2; ++lev) {
        const int N = lev == 0 ? m.N : h->Nm, NP = N + 1;
        std::vector<double> f((size_t)m.E * (3 * NP * NP + 3 * NP));
        element_factors(ds, m, N, L, f.data());
        SEM_TRY(put(lev == 0 ? &h->d_fdm_f : &h->d_fdm_m, f, acc));
    }
    // interpolation matrices
    {
        std::vector<double> xf, wf, xm, wm, xc, wc;
        gll_rule(m.N, xf, wf);
        gll_rule(h->Nm, xm, wm);
        gll_rule(1, xc, wc);
        SEM_TRY(put(&h->d_Jfm, interp(xm, xf), acc));
        SEM_TRY(put(&h->d_Jmc, interp(xc, xm), acc));
    }
    // coarse solver: linear elements on the averaged vertex planes
    for (int d = 0; d < 3; ++d) {
        const int ne = nel[d];
        const bool per = m.periodic[d] != 0;
        const int n = per ? ne : ne + 1;
        std::vector<double> X(ne + 1, 0.0);
        const int nv[3] = {m.nelx + 1, m.nely + 1, m.nelz + 1};
        for (int q = 0; q <= ne; ++q) {
            double s = 0.0;
            int64_t cnt = 0;
            const int o1 = (d + 1) % 3, o2 = (d + 2) % 3;
            for (int u = 0; u < nv[o1]; ++u)
                for (int v = 0; v < nv[o2]; ++v) {
                    int c[3];
                    c[d] = q; c[o1] = u; c[o2] = v;
                    s += ds.vertices[3 * (((int64_t)c[2] * (m.nely + 1) + c[1]) * (m.nelx + 1) + c[0]) + d];
                    ++cnt;
                }
            X[q] = s / (double)cnt;
        }
        std::vector<double> A((size_t)n * n, 0.0), Bd(n, 0.0);
        for (int q = 0; q < ne; ++q) {
            const double hq = X[q + 1] - X[q];
            if (!(hq > 0.0)) return fail(SEM_ERR_INVALID_ARG, "vertex planes are not increasing along an axis");
            const int a = q, b = (q + 1) % n;
            A[(size_t)a * n + a] += 1.0 / hq;
            A[(size_t)b * n + b] += 1.0 / hq;
            A[(size_t)a * n + b] -= 1.0 / hq;
            A[(size_t)b * n + a] -= 1.0 / hq;
            Bd[a] += 0.5 * hq;
            Bd[b] += 0.5 * hq;
        }
        std::vector<char> keep(n, 1);
        if (!per) {
            if ((m.dirichlet >> (2 * d)) & 1) keep[0] = 0;
            if ((m.dirichlet >> (2 * d + 1)) & 1) keep[n - 1] = 0;
        }
        std::vector<double> S((size_t)n * n), lam(n);
        gen_eig(n, A, Bd, keep, S.data(), lam.data());
        h->cn[d] = n;
        SEM_TRY(put(&h->d_cS[d], S, acc));
        SEM_TRY(put(&h->d_clam[d], lam, acc));
    }
    h->bytes = acc;
    if (hipHostMalloc((void **)&h->h_flag, 2 * sizeof(int), hipHostMallocDefault) != hipSuccess) {
        h->h_flag = nullptr;
        return fail(SEM_ERR_OUT_OF_MEMORY, "pinned host flag of the GMRES solve");
    }
    for (hipEvent_t *e : {&h->ev[0], &h->ev[1], &h->fork, &h->join})
        if (hipEventCreateWithFlags(e, hipEventDisableTiming) != hipSuccess) {
            *e = nullptr;
            return fail(SEM_ERR_HIP, "event creation for the multigrid solves");
        }
    if (hipStreamCreateWithFlags(&h->side, hipStreamNonBlocking) != hipSuccess) {
        h->side = nullptr;
        return fail(SEM_ERR_HIP, "side stream creation for the learned multigrid");
    }
    return SEM_OK;
}

void hsmg_release(Mesh &m)
{
    Hsmg *h = m.hsmg;
    if (!h) return;
    void *ptrs[] = {h->d_fdm_f, h->d_fdm_m, h->d_Jfm, h->d_Jmc, h->d_cS[0], h->d_cS[1], h->d_cS[2],
                    h->d_clam[0], h->d_clam[1], h->d_clam[2]};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    if (h->h_flag) (void)hipHostFree(h->h_flag);
    for (hipEvent_t e : {h->ev[0], h->ev[1], h->fork, h->join})
        if (e) (void)hipEventDestroy(e);
    if (h->side) (void)hipStreamDestroy(h->side);
    delete h;
    m.hsmg = nullptr;
}

}  // namespace sem
