// mesh.cpp -- host-side mesh setup of libsem and the mesh entry points.
//
// Reference element, trilinear geometry, geometric factors, structured
// global numbering and the per-axis copy tables of the gather-scatter
// (paper section 3.1: hexahedral
// elements, GLL collocation, gather-scatter coupling; the spectral-element
// definitions follow Deville, Fischer & Mund 2002, chapters 2 and 4).
#include <atomic>
#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <new>

#include "hsmg.hpp"
#include "sem_internal.hpp"

namespace sem {

static thread_local std::string g_err;

void set_error(const std::string &msg) { g_err = msg; }

sem_status fail(sem_status st, const std::string &msg)
{
    g_err = msg;
    return st;
}

// ---------------------------------------------------------------------------
// Reference element.

// Legendre P_N and its first two derivatives by the recurrences
// P_{k+1} = ((2k+1) x P_k - k P_{k-1}) / (k+1),
// P'_{k+1} = P'_{k-1} + (2k+1) P_k,  P''_{k+1} = P''_{k-1} + (2k+1) P'_k.
static void legendre3(int N, double x, double &p, double &dp, double &ddp)
{
    double p0 = 1.0, p1 = x, d0 = 0.0, d1 = 1.0, dd0 = 0.0, dd1 = 0.0;
    if (N == 0) { p = 1.0; dp = 0.0; ddp = 0.0; return; }
    for (int k = 1; k < N; ++k) {
        const double p2 = ((2 * k + 1) * x * p1 - k * p0) / (k + 1);
        const double d2 = d0 + (2 * k + 1) * p1;
        const double dd2 = dd0 + (2 * k + 1) * d1;
        p0 = p1; p1 = p2; d0 = d1; d1 = d2; dd0 = dd1; dd1 = dd2;
    }
    p = p1; dp = d1; ddp = dd1;
}

// GLL nodes (endpoints and the zeros of P_N', by Newton on P_N') and weights
// 2 / (N (N+1) P_N^2).
void gll_rule(int N, std::vector<double> &x, std::vector<double> &w)
{
    x.assign(N + 1, 0.0);
    w.assign(N + 1, 0.0);
    x[0] = -1.0;
    x[N] = 1.0;
    for (int j = 1; j < N; ++j) {
        double t = -std::cos(M_PI * j / N);
        for (int it = 0; it < 60; ++it) {
            double p, dp, ddp;
            legendre3(N, t, p, dp, ddp);
            const double step = dp / ddp;
            t -= step;
            if (std::fabs(step) <= 1e-16) break;
        }
        x[j] = t;
    }
    for (int j = 0; j < (N + 1) / 2; ++j) {   // exact mirror symmetry
        const double a = 0.5 * (x[N - j] - x[j]);
        x[j] = -a;
        x[N - j] = a;
    }
    if (N % 2 == 0) x[N / 2] = 0.0;
    for (int j = 0; j <= N; ++j) {
        double p, dp, ddp;
        legendre3(N, x[j], p, dp, ddp);
        w[j] = 2.0 / (N * (N + 1.0) * p * p);
    }
}

// Derivative of the Lagrange basis at the nodes in barycentric form:
// D_ij = (lam_j / lam_i) / (x_i - x_j) for i != j, D_ii = -sum_{j!=i} D_ij,
// lam_j = 1 / prod_{k != j} (x_j - x_k).
std::vector<double> deriv_matrix(const std::vector<double> &x)
{
    const int n = (int)x.size();
    std::vector<double> lam(n, 1.0), D(n * n, 0.0);
    for (int j = 0; j < n; ++j)
        for (int k = 0; k < n; ++k)
            if (k != j) lam[j] /= (x[j] - x[k]);
    for (int i = 0; i < n; ++i) {
        double diag = 0.0;
        for (int j = 0; j < n; ++j) {
            if (j == i) continue;
            D[i * n + j] = (lam[j] / lam[i]) / (x[i] - x[j]);
            diag -= D[i * n + j];
        }
        D[i * n + i] = diag;
    }
    return D;
}

static uint16_t to_bf16(float f)
{
    uint32_t u;
    std::memcpy(&u, &f, 4);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
    const uint32_t lsb = (u >> 16) & 1u;
    u += 0x7fffu + lsb;   // round to nearest, ties to even
    return (uint16_t)(u >> 16);
}

// IEEE half bits of a double, rounded to nearest (ties to even) straight from
// the double.  |v| must be below 65520 (no overflow handling: the callers
// scale their values into [0, 2^15)).
static uint16_t to_f16(double v)
{
    const uint16_t sign = std::signbit(v) ? 0x8000u : 0u;
    const double a = std::fabs(v);
    if (a == 0.0) return sign;
    int x;
    std::frexp(a, &x);                               // a in [2^(x-1), 2^x)
    const int qexp = std::max(x - 11, -24);          // grid spacing 2^qexp (normal: 11 bits; subnormal: 2^-24)
    const double r = std::nearbyint(std::ldexp(a, -qexp));   // exact scaling, then ties to even
    const double val = std::ldexp(r, qexp);
    if (val < 0x1p-14) return (uint16_t)(sign | (uint16_t)r);   // subnormal (r < 1024)
    int y;
    std::frexp(val, &y);                             // val in [2^(y-1), 2^y)
    const uint32_t mant = (uint32_t)std::ldexp(val, 11 - y) - 1024u;
    return (uint16_t)(sign | (uint16_t)((y - 1 + 15) << 10) | (uint16_t)mant);
}

// Per-element power-of-two scale of the half storage: exponent k with
// max |a| / 2^k in [2^14, 2^15) (0 for an element of zeros).
static int f16_exponent(const double *a, int64_t n)
{
    double mx = 0.0;
    for (int64_t q = 0; q < n; ++q) mx = std::max(mx, std::fabs(a[q]));
    if (mx == 0.0) return 0;
    int x;
    std::frexp(mx, &x);
    return x - 15;
}

// ---------------------------------------------------------------------------
// Structured numbering: gi = ex N + i (mod nx if periodic), glo = gi + nx (gj + ny gk).

static inline int64_t ndir(int nel, int N, bool per) { return (int64_t)nel * N + (per ? 0 : 1); }

int64_t Mesh::glo(int64_t e, int i, int j, int k) const
{
    const int64_t ex = e % nelx, ey = (e / nelx) % nely, ez = e / ((int64_t)nelx * nely);
    const int64_t nx = ndir(nelx, N, periodic[0]), ny = ndir(nely, N, periodic[1]),
                  nz = ndir(nelz, N, periodic[2]);
    const int64_t gi = (ex * N + i) % nx, gj = (ey * N + j) % ny, gk = (ez * N + k) % nz;
    return gi + nx * (gj + ny * gk);
}

// copies of a structured node along one direction
static inline int copies1(int64_t g, int nel, int N, bool per)
{
    if (g % N != 0) return 1;
    if (per) return 2;
    return (g == 0 || g == (int64_t)nel * N) ? 1 : 2;
}

static inline bool masked1(int64_t g, int nel, int N, bool per, uint8_t bits, int d)
{
    if (per) return false;
    if (g == 0 && ((bits >> (2 * d)) & 1)) return true;
    if (g == (int64_t)nel * N && ((bits >> (2 * d + 1)) & 1)) return true;
    return false;
}

template <typename T>
static sem_status upload(T **dst, const T *src, size_t count, size_t &acc)
{
    if (count == 0) { *dst = nullptr; return SEM_OK; }
    hipError_t e = hipMalloc((void **)dst, count * sizeof(T));
    if (e != hipSuccess) return fail(SEM_ERR_OUT_OF_MEMORY, std::string("hipMalloc: ") + hipGetErrorString(e));
    acc += count * sizeof(T);
    SEM_HIP_TRY(hipMemcpy(*dst, src, count * sizeof(T), hipMemcpyHostToDevice));
    return SEM_OK;
}

static void release(Mesh &m)
{
    void *ptrs[] = {m.d_D, m.d_D32, m.d_Dbf, m.d_G, m.d_B, m.d_xyz, m.d_wcode, m.d_mult,
                    m.d_G32, m.d_B32, m.d_Gbf, m.d_Bbf, m.d_Gh, m.d_Bh, m.d_hscale, m.d_scratch, m.d_tab};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    hsmg_release(m);
}

#define SEM_TRY(x)                      \
    do {                                \
        sem_status _s = (x);            \
        if (_s != SEM_OK) return _s;    \
    } while (0)

static sem_status build(const sem_mesh_desc &d, Mesh &m)
{
    m.nelx = d.nelx; m.nely = d.nely; m.nelz = d.nelz;
    m.N = d.order; m.NP = d.order + 1;
    for (int c = 0; c < 3; ++c) m.periodic[c] = d.periodic[c] ? 1 : 0;
    m.dirichlet = d.dirichlet_faces & 0x3f;
    m.E = (int64_t)m.nelx * m.nely * m.nelz;
    m.P = (int64_t)m.NP * m.NP * m.NP;
    m.nl = m.E * m.P;
    const int N = m.N, NP = m.NP;
    const int64_t P = m.P, E = m.E, nl = m.nl;
    SEM_HIP_TRY(hipGetDevice(&m.device));

    gll_rule(N, m.xi, m.wq);
    m.D = deriv_matrix(m.xi);

    // ---- geometry: trilinear map and its analytic Jacobian at the GLL nodes
    std::unique_ptr<double[]> G(new (std::nothrow) double[(size_t)6 * nl]);
    std::unique_ptr<double[]> B(new (std::nothrow) double[(size_t)nl]);
    std::unique_ptr<double[]> X(new (std::nothrow) double[(size_t)3 * nl]);
    if (!G || !B || !X) return fail(SEM_ERR_OUT_OF_MEMORY, "host allocation for geometry");
    const double *V = d.vertices;
    int64_t first_bad = -1;
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < E; ++e) {
        const int64_t ex = e % m.nelx, ey = (e / m.nelx) % m.nely, ez = e / ((int64_t)m.nelx * m.nely);
        double C[8][3];   // corner c = a + 2 b + 4 c'
        for (int c = 0; c < 8; ++c) {
            const int64_t vx = ex + (c & 1), vy = ey + ((c >> 1) & 1), vz = ez + ((c >> 2) & 1);
            const double *v = V + 3 * ((vz * (m.nely + 1) + vy) * (m.nelx + 1) + vx);
            C[c][0] = v[0]; C[c][1] = v[1]; C[c][2] = v[2];
        }
        bool bad = false;
        for (int k = 0; k < NP; ++k)
            for (int j = 0; j < NP; ++j)
                for (int i = 0; i < NP; ++i) {
                    const double r = m.xi[i], s = m.xi[j], t = m.xi[k];
                    const double fr[2] = {0.5 * (1 - r), 0.5 * (1 + r)};
                    const double fs[2] = {0.5 * (1 - s), 0.5 * (1 + s)};
                    const double ft[2] = {0.5 * (1 - t), 0.5 * (1 + t)};
                    const double dfl[2] = {-0.5, 0.5};
                    double x[3] = {0, 0, 0}, J[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
                    for (int c = 0; c < 8; ++c) {
                        const int a = c & 1, b = (c >> 1) & 1, cc = (c >> 2) & 1;
                        const double phi = fr[a] * fs[b] * ft[cc];
                        const double dr = dfl[a] * fs[b] * ft[cc];
                        const double ds = fr[a] * dfl[b] * ft[cc];
                        const double dt = fr[a] * fs[b] * dfl[cc];
                        for (int q = 0; q < 3; ++q) {
                            x[q] += C[c][q] * phi;
                            J[q][0] += C[c][q] * dr;
                            J[q][1] += C[c][q] * ds;
                            J[q][2] += C[c][q] * dt;
                        }
                    }
                    // cofactors: inverse = adj(J) / det
                    const double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
                    const double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
                    const double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
                    const double det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
                    if (!(det > 0.0)) bad = true;
                    const double inv = 1.0 / det;
                    // rows of J^{-1} = gradients of r, s, t
                    const double g[3][3] = {
                        {c00 * inv, (J[0][2] * J[2][1] - J[0][1] * J[2][2]) * inv,
                         (J[0][1] * J[1][2] - J[0][2] * J[1][1]) * inv},
                        {c01 * inv, (J[0][0] * J[2][2] - J[0][2] * J[2][0]) * inv,
                         (J[0][2] * J[1][0] - J[0][0] * J[1][2]) * inv},
                        {c02 * inv, (J[0][1] * J[2][0] - J[0][0] * J[2][1]) * inv,
                         (J[0][0] * J[1][1] - J[0][1] * J[1][0]) * inv}};
                    const double wj = m.wq[i] * m.wq[j] * m.wq[k] * det;
                    const int64_t l = i + NP * (j + (int64_t)NP * k);
                    const int pairs[6][2] = {{0, 0}, {0, 1}, {0, 2}, {1, 1}, {1, 2}, {2, 2}};
                    for (int q = 0; q < 6; ++q) {
                        const double *ga = g[pairs[q][0]], *gb = g[pairs[q][1]];
                        G[(size_t)(e * 6 + q) * P + l] = wj * (ga[0] * gb[0] + ga[1] * gb[1] + ga[2] * gb[2]);
                    }
                    B[e * P + l] = wj;
                    for (int q = 0; q < 3; ++q) X[(size_t)q * nl + e * P + l] = x[q];
                }
        if (bad) {
#pragma omp critical(sem_bad)
            if (first_bad < 0 || e < first_bad) first_bad = e;
        }
    }
    if (first_bad >= 0)
        return fail(SEM_ERR_INVALID_ARG, "element " + std::to_string(first_bad) +
                                             " has a non-positive Jacobian (inverted or degenerate)");

    // ---- numbering, multiplicity, mask (closed form; the kernels recompute
    //      copies from the lattice description, no index lists are stored)
    const bool px = m.periodic[0], py = m.periodic[1], pz = m.periodic[2];
    const int64_t nx = ndir(m.nelx, N, px), ny = ndir(m.nely, N, py), nz = ndir(m.nelz, N, pz);
    m.ng = nx * ny * nz;
    m.lat = Lattice{m.nelx, m.nely, m.nelz, N, NP, nx, ny, nz, P, {m.periodic[0], m.periodic[1], m.periodic[2]},
                    m.dirichlet, {nullptr, nullptr, nullptr}, 0};
    std::vector<int2> tab(nx + ny + nz);
    {
        const int nel[3] = {m.nelx, m.nely, m.nelz};
        const int64_t nd[3] = {nx, ny, nz};
        int64_t base = 0;
        for (int d = 0; d < 3; ++d) {
            for (int64_t g = 0; g < nd[d]; ++g) {
                int ec[2] = {0, 0}, lc[2] = {0, 0};
                const int cnt = lattice_copies(g, nel[d], N, m.periodic[d] != 0, ec, lc);
                const bool msk = masked1(g, nel[d], N, m.periodic[d] != 0, m.dirichlet, d);
                tab[base + g].x = ec[0] | (ec[1] << 16);
                tab[base + g].y = lc[0] | (lc[1] << 8) | (cnt << 16) | ((msk ? 1 : 0) << 24);
            }
            base += nd[d];
            if (m.periodic[d] && nel[d] == 1) m.lat.unsorted = 1;
        }
    }
    std::vector<uint8_t> wcode(nl), mult(nl);
    int64_t ns = 0, nmask = 0, nsl = 0;
#pragma omp parallel for schedule(static) reduction(+ : ns, nmask)
    for (int64_t gk = 0; gk < nz; ++gk)
        for (int64_t gj = 0; gj < ny; ++gj)
            for (int64_t gi = 0; gi < nx; ++gi) {
                const int c = copies1(gi, m.nelx, N, px) * copies1(gj, m.nely, N, py) *
                              copies1(gk, m.nelz, N, pz);
                if (c > 1) ++ns;
                if (masked1(gi, m.nelx, N, px, m.dirichlet, 0) || masked1(gj, m.nely, N, py, m.dirichlet, 1) ||
                    masked1(gk, m.nelz, N, pz, m.dirichlet, 2))
                    ++nmask;
            }
#pragma omp parallel for schedule(static) reduction(+ : nsl)
    for (int64_t e = 0; e < E; ++e) {
        const int64_t ex = e % m.nelx, ey = (e / m.nelx) % m.nely, ez = e / ((int64_t)m.nelx * m.nely);
        for (int k = 0; k < NP; ++k)
            for (int j = 0; j < NP; ++j)
                for (int i = 0; i < NP; ++i) {
                    const int64_t gi = (ex * N + i) % nx, gj = (ey * N + j) % ny, gk = (ez * N + k) % nz;
                    const int c = copies1(gi, m.nelx, N, px) * copies1(gj, m.nely, N, py) *
                                  copies1(gk, m.nelz, N, pz);
                    const bool msk = masked1(gi, m.nelx, N, px, m.dirichlet, 0) ||
                                     masked1(gj, m.nely, N, py, m.dirichlet, 1) ||
                                     masked1(gk, m.nelz, N, pz, m.dirichlet, 2);
                    const int64_t l = e * P + i + NP * (j + (int64_t)NP * k);
                    mult[l] = (uint8_t)c;
                    wcode[l] = msk ? 0 : (uint8_t)(1 + (c == 1 ? 0 : c == 2 ? 1 : c == 4 ? 2 : 3));
                    if (c > 1) ++nsl;
                }
    }
    m.n_shared_global = ns;
    m.n_masked_global = nmask;
    m.n_shared_local = nsl;

    // ---- upload
    size_t acc = 0;
    SEM_TRY(upload(&m.d_tab, tab.data(), tab.size(), acc));
    m.lat.tab[0] = m.d_tab;
    m.lat.tab[1] = m.d_tab + nx;
    m.lat.tab[2] = m.d_tab + nx + ny;
    SEM_TRY(upload(&m.d_D, m.D.data(), m.D.size(), acc));
    // element-blocked geometric factors are already [E][6][P]
    SEM_TRY(upload(&m.d_G, G.get(), (size_t)6 * nl, acc));
    SEM_TRY(upload(&m.d_B, B.get(), (size_t)nl, acc));
    SEM_TRY(upload(&m.d_xyz, X.get(), (size_t)3 * nl, acc));
    SEM_TRY(upload(&m.d_wcode, wcode.data(), (size_t)nl, acc));
    SEM_TRY(upload(&m.d_mult, mult.data(), (size_t)nl, acc));
    {
        std::vector<float> D32(m.D.begin(), m.D.end());
        // BF16 D as hi | lo pairs: hi = bf16(D), lo = bf16(D - hi)
        std::vector<uint16_t> Dbf(2 * m.D.size());
        for (size_t q = 0; q < m.D.size(); ++q) {
            Dbf[q] = to_bf16((float)m.D[q]);
            uint32_t hb = (uint32_t)Dbf[q] << 16;
            float hf;
            std::memcpy(&hf, &hb, 4);
            Dbf[m.D.size() + q] = to_bf16((float)(m.D[q] - (double)hf));
        }
        SEM_TRY(upload(&m.d_D32, D32.data(), D32.size(), acc));
        SEM_TRY(upload(&m.d_Dbf, Dbf.data(), Dbf.size(), acc));
    }
    if (d.prepare & SEM_PREP_F32) {
        std::vector<float> g32((size_t)6 * nl), b32(nl);
#pragma omp parallel for schedule(static)
        for (int64_t q = 0; q < 6 * nl; ++q) g32[q] = (float)G[q];
#pragma omp parallel for schedule(static)
        for (int64_t q = 0; q < nl; ++q) b32[q] = (float)B[q];
        SEM_TRY(upload(&m.d_G32, g32.data(), g32.size(), acc));
        SEM_TRY(upload(&m.d_B32, b32.data(), b32.size(), acc));
    }
    if (d.prepare & SEM_PREP_BF16) {
        std::vector<uint16_t> gb((size_t)6 * nl), bb(nl);
#pragma omp parallel for schedule(static)
        for (int64_t q = 0; q < 6 * nl; ++q) gb[q] = to_bf16((float)G[q]);
#pragma omp parallel for schedule(static)
        for (int64_t q = 0; q < nl; ++q) bb[q] = to_bf16((float)B[q]);
        SEM_TRY(upload(&m.d_Gbf, gb.data(), gb.size(), acc));
        SEM_TRY(upload(&m.d_Bbf, bb.data(), bb.size(), acc));
        // half storage with one power-of-two scale per element and array
        // (the split-BF16 operator's G and B)
        std::vector<uint16_t> gh((size_t)6 * nl), bh(nl);
        std::vector<float> sc((size_t)2 * m.E);
#pragma omp parallel for schedule(static)
        for (int64_t e = 0; e < m.E; ++e) {
            const double *Ge = G.get() + e * 6 * P, *Be = B.get() + e * P;
            const int kg = f16_exponent(Ge, 6 * P), kb = f16_exponent(Be, P);
            for (int64_t q = 0; q < 6 * P; ++q) gh[e * 6 * P + q] = to_f16(std::ldexp(Ge[q], -kg));
            for (int64_t q = 0; q < P; ++q) bh[e * P + q] = to_f16(std::ldexp(Be[q], -kb));
            sc[2 * e] = std::ldexp(1.0f, kg);
            sc[2 * e + 1] = std::ldexp(1.0f, kb);
        }
        SEM_TRY(upload(&m.d_Gh, gh.data(), gh.size(), acc));
        SEM_TRY(upload(&m.d_Bh, bh.data(), bh.size(), acc));
        SEM_TRY(upload(&m.d_hscale, sc.data(), sc.size(), acc));
    }
    if (d.prepare & SEM_PREP_HSMG) {
        SEM_TRY(hsmg_setup(d, m));
        acc += m.hsmg->bytes;
    }
    m.scratch_len = dot_blocks(m) + 1;
    {
        hipError_t e = hipMalloc((void **)&m.d_scratch, sizeof(double) * m.scratch_len);
        if (e != hipSuccess) return fail(SEM_ERR_OUT_OF_MEMORY, "hipMalloc scratch");
        acc += sizeof(double) * m.scratch_len;
    }
    m.device_bytes = acc;
    return SEM_OK;
}

}  // namespace sem

using namespace sem;

extern "C" {

const char *sem_last_error(void) { return sem::g_err.c_str(); }

const char *sem_version(void) { return "sem 0.1 gfx950"; }

sem_status sem_mesh_create(const sem_mesh_desc *desc, sem_mesh **out)
{
    set_error("");
    if (!desc || !out) return fail(SEM_ERR_INVALID_ARG, "null desc or out");
    *out = nullptr;
    if (!desc->vertices) return fail(SEM_ERR_INVALID_ARG, "null vertices");
    if (desc->nelx < 1 || desc->nely < 1 || desc->nelz < 1)
        return fail(SEM_ERR_INVALID_ARG, "element counts must be >= 1");
    if (desc->order < 1 || desc->order > kMaxOrder)
        return fail(SEM_ERR_INVALID_ARG, "order must be in 1..15");
    const int64_t np = desc->order + 1;
    const int64_t nl = (int64_t)desc->nelx * desc->nely * desc->nelz * np * np * np;
    if (nl >= ((int64_t)1 << 31))
        return fail(SEM_ERR_UNSUPPORTED, "more than 2^31 local nodes");
    if (desc->nelx > 32767 || desc->nely > 32767 || desc->nelz > 32767)
        return fail(SEM_ERR_UNSUPPORTED, "more than 32767 elements along one direction");
    sem_mesh *h = new (std::nothrow) sem_mesh();
    if (!h) return fail(SEM_ERR_OUT_OF_MEMORY, "host allocation");
    sem_status st = build(*desc, h->m);
    if (st != SEM_OK) {
        release(h->m);
        delete h;
        return st;
    }
    static std::atomic<uint64_t> next_serial{1};
    h->m.serial = next_serial.fetch_add(1);
    *out = h;
    return SEM_OK;
}

sem_status sem_mesh_destroy(sem_mesh *mesh)
{
    if (!mesh) return SEM_OK;
    release(mesh->m);
    delete mesh;
    return SEM_OK;
}

sem_status sem_mesh_query(const sem_mesh *mesh, sem_mesh_info *out)
{
    if (!mesh || !out) return fail(SEM_ERR_INVALID_ARG, "null mesh or out");
    const Mesh &m = mesh->m;
    out->nelem = m.E;
    out->n_local = m.nl;
    out->n_global = m.ng;
    out->n_shared_global = m.n_shared_global;
    out->n_shared_local = m.n_shared_local;
    out->n_masked_global = m.n_masked_global;
    out->order = m.N;
    out->npts_elem = (int32_t)m.P;
    out->device_bytes = m.device_bytes;
    return SEM_OK;
}

sem_status sem_mesh_export(const sem_mesh *mesh, int field, void *host_dst, size_t bytes)
{
    if (!mesh || !host_dst) return fail(SEM_ERR_INVALID_ARG, "null mesh or destination");
    const Mesh &m = mesh->m;
    const size_t nl = (size_t)m.nl;
    auto need = [&](size_t b) -> sem_status {
        if (b != bytes)
            return fail(SEM_ERR_INVALID_ARG, "export size mismatch: need " + std::to_string(b) +
                                                 " bytes, got " + std::to_string(bytes));
        return SEM_OK;
    };
    switch (field) {
    case SEM_FIELD_GLO_NUM: {
        SEM_TRY(need(nl * 8));
        int64_t *o = (int64_t *)host_dst;
#pragma omp parallel for schedule(static)
        for (int64_t e = 0; e < m.E; ++e)
            for (int64_t q = 0; q < m.P; ++q)
                o[e * m.P + q] = m.glo(e, (int)(q % m.NP), (int)((q / m.NP) % m.NP), (int)(q / (m.NP * m.NP)));
        return SEM_OK;
    }
    case SEM_FIELD_MULT: {
        SEM_TRY(need(nl * 4));
        std::vector<uint8_t> t(nl);
        SEM_HIP_TRY(hipMemcpy(t.data(), m.d_mult, nl, hipMemcpyDeviceToHost));
        int32_t *o = (int32_t *)host_dst;
        for (size_t q = 0; q < nl; ++q) o[q] = t[q];
        return SEM_OK;
    }
    case SEM_FIELD_MASK: {
        SEM_TRY(need(nl));
        std::vector<uint8_t> t(nl);
        SEM_HIP_TRY(hipMemcpy(t.data(), m.d_wcode, nl, hipMemcpyDeviceToHost));
        uint8_t *o = (uint8_t *)host_dst;
        for (size_t q = 0; q < nl; ++q) o[q] = t[q] == 0 ? 1 : 0;
        return SEM_OK;
    }
    case SEM_FIELD_G: {
        SEM_TRY(need(nl * 6 * 8));
        double *o = (double *)host_dst;
        // device [E][6][P] -> host [6][E][P]
        for (int q = 0; q < 6; ++q)
            SEM_HIP_TRY(hipMemcpy2D(o + (size_t)q * nl, m.P * sizeof(double), m.d_G + (size_t)q * m.P,
                                    6 * m.P * sizeof(double), m.P * sizeof(double), m.E,
                                    hipMemcpyDeviceToHost));
        return SEM_OK;
    }
    case SEM_FIELD_B:
        SEM_TRY(need(nl * 8));
        SEM_HIP_TRY(hipMemcpy(host_dst, m.d_B, nl * 8, hipMemcpyDeviceToHost));
        return SEM_OK;
    case SEM_FIELD_XYZ:
        SEM_TRY(need(nl * 3 * 8));
        SEM_HIP_TRY(hipMemcpy(host_dst, m.d_xyz, nl * 3 * 8, hipMemcpyDeviceToHost));
        return SEM_OK;
    case SEM_FIELD_GLL: {
        SEM_TRY(need((size_t)2 * m.NP * 8));
        double *o = (double *)host_dst;
        for (int q = 0; q < m.NP; ++q) { o[q] = m.xi[q]; o[m.NP + q] = m.wq[q]; }
        return SEM_OK;
    }
    case SEM_FIELD_DERIV:
        SEM_TRY(need((size_t)m.NP * m.NP * 8));
        std::memcpy(host_dst, m.D.data(), (size_t)m.NP * m.NP * 8);
        return SEM_OK;
    default:
        return fail(SEM_ERR_INVALID_ARG, "unknown field " + std::to_string(field));
    }
}

}  // extern "C"
