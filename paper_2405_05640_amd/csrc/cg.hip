// cg.hip -- assembled-vector kernels of the Krylov solvers.
//
// Inside the solvers every Krylov vector is stored once per unique (global)
// node instead of once per element copy: at N = 7 that is 68 % of the local
// points, so every vector update moves a third fewer bytes.  The operator
// reads its input through the closed-form numbering (ax kernel, gather mode)
// and writes the unassembled element result w; the assembly Q^T w (the
// gather half of the gather-scatter, paper section 3.1) is fused into the
// kernel that consumes w.  One thread per global node, lexicographic order:
// neighbouring lanes read neighbouring element rows, so the pass is
// coalesced.  Copies are summed in ascending local index, the same order as
// sem_dssum.
//
// Dirichlet nodes carry dinv = 0: r, p, x are forced to zero there and they
// drop out of every inner product.  Partial sums are per block in FP64
// (cross-lane shuffles within a wavefront) and are reduced in a fixed order
// by one-workgroup finalize kernels, so every run is bitwise reproducible.
#include "cg.hpp"
#include "reduce.hpp"

namespace sem {
namespace cg {

__device__ __forceinline__ void g_to_ijk(const Lattice &L, int64_t g, int64_t &gi, int64_t &gj, int64_t &gk)
{
    gi = g % L.nx;
    const int64_t t = g / L.nx;
    gj = t % L.ny;
    gk = t / L.ny;
}

// sum of the copies of node (gi, gj, gk) of a local [E][k][j][i] field
template <typename T>
__device__ __forceinline__ double assemble_at(const Lattice &L, const T *__restrict__ w, int gi, int gj, int gk,
                                              bool &masked)
{
    int loc[8];
    const int n = node_locals(L, gi, gj, gk, loc, masked);
    T s = T(0);
    for (int c = 0; c < n; ++c) s += w[loc[c]];
    return (double)s;
}

// Block sums of NV values per thread: a butterfly of cross-lane shuffles in
// each wavefront, then the wavefronts' sums in order; thread 0 stores
// out[q * stride + block].
template <int NV>
__device__ __forceinline__ void block_store(double (&v)[NV], double *out, int stride)
{
    __shared__ double red[NV][kBS / 64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        double x = v[q];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
        if (lane == 0) red[q][wv] = x;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < NV; ++q) {
            double x = red[q][0];
#pragma unroll
            for (int w = 1; w < kBS / 64; ++w) x += red[q][w];
            out[q * stride + blockIdx.x] = x;
        }
    }
}

__device__ double block_sum(const double *__restrict__ a, int64_t n)
{
    __shared__ double red[kBS];
    double s = 0.0;
    for (int64_t q = threadIdx.x; q < n; q += kBS) s += a[q];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = kBS / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

#define GRID_STRIDE(g, n) for (int64_t g = (int64_t)blockIdx.x * kBS + threadIdx.x; g < (n); g += (int64_t)gridDim.x * kBS)

// ---------------------------------------------------------------- layout moves

// ug[g] = u at the first copy of g (u continuous)
template <typename Tin, typename Tout>
__global__ void __launch_bounds__(kBS) gather_kernel(const Tin *__restrict__ u, Tout *__restrict__ ug, Lattice L)
{
    SEM_FOR_EACH_NODE(L, gi, gj, gk, g)
    {
        int loc[8];
        bool msk;
        node_locals(L, gi, gj, gk, loc, msk);
        ug[g] = (Tout)u[loc[0]];
    }
}

// u[l] = ug[glo(l)]
template <typename Tin, typename Tout>
__global__ void __launch_bounds__(kBS) scatter_kernel(const Tin *__restrict__ ug, Tout *__restrict__ u, Lattice L, int64_t nl)
{
    GRID_STRIDE(l, nl)
    {
        const int64_t e = l / L.P;
        const int q = (int)(l - e * L.P);
        const int i = q % L.NP, j = (q / L.NP) % L.NP, k = q / (L.NP * L.NP);
        u[l] = (Tout)ug[lattice_glo(L, e, i, j, k)];
    }
}

// dinv[g] = 1 / sum of local diagonal copies, 0 on Dirichlet nodes
template <typename T>
__global__ void __launch_bounds__(kBS) dinv_kernel(const double *__restrict__ dl, T *__restrict__ dinv, Lattice L)
{
    SEM_FOR_EACH_NODE(L, gi, gj, gk, g)
    {
        bool msk;
        const double d = assemble_at(L, dl, gi, gj, gk, msk);
        dinv[g] = msk ? T(0) : (T)(1.0 / d);
    }
}

// ---------------------------------------------------------------- CG steps

// x = 0, r = b (0 on Dirichlet nodes), p = dinv r; partials (r,r), (r,z)
template <typename T>
__global__ void __launch_bounds__(kBS)
init_kernel(const T *__restrict__ b, T *__restrict__ x, T *__restrict__ r, T *__restrict__ p,
            const T *__restrict__ dinv, int64_t ng, double *__restrict__ part)
{
    double acc[2] = {0.0, 0.0};
    GRID_STRIDE(g, ng)
    {
        const T d = dinv[g];
        const T rg = d == T(0) ? T(0) : b[g];
        x[g] = T(0);
        r[g] = rg;
        const T z = d * rg;
        p[g] = z;
        acc[0] += (double)rg * (double)rg;
        acc[1] += (double)rg * (double)z;
    }
    block_store<2>(acc, part, gridDim.x);
}

__global__ void __launch_bounds__(kBS) init_finalize(CgState *st, const double *__restrict__ part, int nb, double tol, double *hist)
{
    const double rr = block_sum(part, nb);
    const double rz = block_sum(part + nb, nb);
    if (threadIdx.x == 0) {
        st->bb = rr;
        st->rr = rr;
        st->rz = rz;
        st->tol2 = tol * tol * rr;
        st->it = 0;
        st->status = 0;
        st->done = (rr == 0.0) ? 1 : 0;
        if (hist && st->hist_len > 0) hist[0] = 1.0;
    }
}

// first stage of a two-stage reduction: kStage blocks, fixed chunks
__global__ void __launch_bounds__(kBS) reduce_stage_kernel(const double *__restrict__ part, int64_t n, int nv,
                                                            double *__restrict__ stage)
{
    const int64_t chunk = (n + kStage - 1) / kStage;
    const int64_t lo = blockIdx.x * chunk, hi = std::min<int64_t>(n, lo + chunk);
    for (int q = 0; q < nv; ++q) {
        const double v = lo < hi ? block_sum(part + q * n + lo, hi - lo) : 0.0;
        if (threadIdx.x == 0) stage[q * kStage + blockIdx.x] = v;
    }
}

__device__ __forceinline__ void alpha_finalize(CgState *st, double pw)
{
    st->pw = pw;
    if (!(pw > 0.0) || !isfinite(pw) || !isfinite(st->rz)) {
        st->done = 2;
        st->status = SEM_ERR_BREAKDOWN;
    } else {
        st->alpha = st->rz / pw;
    }
}

// alpha = rz / (p, S p) from n partials (per element, or the stage sums)
__global__ void __launch_bounds__(kWide) alpha_direct_kernel(CgState *st, const double *__restrict__ part, int64_t n)
{
    const double pw = wide_sum(part, n);
    if (threadIdx.x == 0 && !st->done) alpha_finalize(st, pw);
}

// iteration count, residual history, convergence test and beta
__device__ __forceinline__ void beta_finalize(CgState *st, double rr, double rz, double *hist)
{
    const int it = st->it + 1;
    st->it = it;
    st->rr = rr;
    if (hist && it < st->hist_len) hist[it] = sqrt(rr / st->bb);
    if (!isfinite(rr) || !isfinite(rz)) {
        st->done = 2;
        st->status = SEM_ERR_BREAKDOWN;
    } else if (rr <= st->tol2) {
        st->done = 1;
    } else if (it >= st->max_it) {
        st->done = 3;
    } else {
        st->beta = rz / st->rz;
        st->rz = rz;
    }
}

// wg = Q^T w (w in the row layout); x += alpha p; r -= alpha wg; partials
// (r,r), (r, dinv r).  RPB rows per workgroup, unrolled so that the loads of
// all of them are in flight together; NPC = N + 1 fixed at compile time
// (0: any order).
template <typename T, int RPB, int NPC>
__global__ void __launch_bounds__(kBS)
update_kernel(const CgState *__restrict__ st, const T *__restrict__ w, T *__restrict__ x, T *__restrict__ r,
              const T *__restrict__ p, const T *__restrict__ dinv, Lattice L, double *__restrict__ part)
{
    if (st->done) return;
    const T alpha = (T)st->alpha;
    double acc[2] = {0.0, 0.0};
    const int nrows = (int)(L.ny * L.nz), row0 = (int)blockIdx.x * RPB, ny = (int)L.ny, nx = (int)L.nx;
    for (int gi = threadIdx.x; gi < nx; gi += kBS) {
        T d[RPB], xg[RPB], pg[RPB], rg0[RPB], wg[RPB];
        int64_t g[RPB];
#pragma unroll
        for (int q = 0; q < RPB; ++q) {
            const int row = row0 + q < nrows ? row0 + q : nrows - 1;   // clamped rows are not stored
            g[q] = gi + (int64_t)nx * row;
            d[q] = dinv[g[q]];
            xg[q] = x[g[q]];
            pg[q] = p[g[q]];
            rg0[q] = r[g[q]];
            wg[q] = node_assemble_rows<NPC>(L, w, gi, row % ny, row / ny);
        }
#pragma unroll
        for (int q = 0; q < RPB; ++q) {
            if (row0 + q >= nrows || d[q] == T(0)) continue;   // Dirichlet node: r, p, x stay zero
            x[g[q]] = xg[q] + alpha * pg[q];
            const T rg = rg0[q] - alpha * wg[q];
            r[g[q]] = rg;
            acc[0] += (double)rg * (double)rg;
            acc[1] += (double)rg * (double)(d[q] * rg);
        }
    }
    block_store<2>(acc, part, gridDim.x);
}

// (r, r) and (r, z) from nb partials each (per workgroup, or the stage
// sums): iteration count, convergence test and beta
__global__ void __launch_bounds__(kWide) beta_direct_kernel(CgState *st, const double *__restrict__ part, int nb,
                                                             double *hist)
{
    double rr, rz;
    wide_sum2(part, part + nb, nb, rr, rz);
    if (threadIdx.x == 0 && !st->done) beta_finalize(st, rr, rz, hist);
}

template <typename T>
__global__ void __launch_bounds__(kBS)
p_kernel(const CgState *__restrict__ st, T *__restrict__ p, const T *__restrict__ r, const T *__restrict__ dinv, int64_t ng)
{
    if (st->done) return;
    const T beta = (T)st->beta;
    GRID_STRIDE(g, ng) p[g] = dinv[g] * r[g] + beta * p[g];
}

// r = b - Q^T w (w in the row layout; 0 on Dirichlet nodes); partial (r, r)
template <typename T>
__global__ void __launch_bounds__(kBS)
resid_kernel(const T *__restrict__ b, const T *__restrict__ w, T *__restrict__ r, const T *__restrict__ dinv, Lattice L,
             double *__restrict__ part)
{
    double acc[1] = {0.0};
    SEM_FOR_EACH_NODE(L, gi, gj, gk, g)
    {
        const T d = dinv[g], bg = b[g];
        const T wg = node_assemble_rows<0>(L, w, gi, gj, gk);
        const T rg = d != T(0) ? bg - wg : T(0);
        r[g] = rg;
        acc[0] += (double)rg * (double)rg;
    }
    block_store<1>(acc, part, gridDim.x);
}

__global__ void __launch_bounds__(kBS) resid_finalize(CgState *st, const double *__restrict__ part, int nb)
{
    const double rr = block_sum(part, nb);
    if (threadIdx.x == 0) st->true_rr = rr;
}

// restart from the residual in r: p = dinv r; partials (r,r), (r,z)
template <typename T>
__global__ void __launch_bounds__(kBS)
restart_kernel(const T *__restrict__ r, T *__restrict__ p, const T *__restrict__ dinv, int64_t ng, double *__restrict__ part)
{
    double acc[2] = {0.0, 0.0};
    GRID_STRIDE(g, ng)
    {
        const T rg = r[g], z = dinv[g] * rg;
        p[g] = z;
        acc[0] += (double)rg * (double)rg;
        acc[1] += (double)rg * (double)z;
    }
    block_store<2>(acc, part, gridDim.x);
}

__global__ void __launch_bounds__(kBS) restart_finalize(CgState *st, const double *__restrict__ part, int nb)
{
    const double rr = block_sum(part, nb);
    const double rz = block_sum(part + nb, nb);
    if (threadIdx.x == 0) {
        st->rr = rr;
        st->rz = rz;
        st->done = (rr <= st->tol2) ? 1 : (st->it >= st->max_it ? 3 : 0);
    }
}

// Residual replacement (reliable update) of a low-precision CG: r = inv_sigma
// * r64 (the FP64 true residual), x = 0.  mode = kReplaceFirst starts a run
// (p = dinv r, iteration count and |b| reset); kReplaceRestart sets
// p = dinv r but keeps the counters (used when the low-precision run had
// converged, so its last direction update was never made); kReplaceKeep
// keeps the search direction but swaps its preconditioned-residual part: the
// last direction update was p = dinv r_old + beta p_prev, so
// p + dinv (r_new - r_old) is the direction the new residual would have
// produced; p_scale = sigma_old / sigma_new converts to the new units.
// Partials (r, r), (r, dinv r).
template <typename T>
__global__ void __launch_bounds__(kBS)
replace_kernel(const double *__restrict__ r64, T *__restrict__ x, T *__restrict__ r, T *__restrict__ p,
               const T *__restrict__ dinv, double inv_sigma, double p_scale, int mode, int64_t ng,
               double *__restrict__ part)
{
    double acc[2] = {0.0, 0.0};
    GRID_STRIDE(g, ng)
    {
        const T d = dinv[g];
        const T rg = d == T(0) ? T(0) : (T)(inv_sigma * r64[g]);
        const T z = d * rg;
        x[g] = T(0);
        if (mode != kReplaceKeep) {
            p[g] = z;
        } else {
            const double r_old = (double)r[g];
            p[g] = (T)(p_scale * (double)p[g] + (double)d * ((double)rg - p_scale * r_old));
        }
        r[g] = rg;
        acc[0] += (double)rg * (double)rg;
        acc[1] += (double)rg * (double)z;
    }
    block_store<2>(acc, part, gridDim.x);
}

__global__ void __launch_bounds__(kBS) replace_finalize(CgState *st, const double *__restrict__ part, int nb, double tol2,
                                                         int mode)
{
    const double rr = block_sum(part, nb);
    const double rz = block_sum(part + nb, nb);
    if (threadIdx.x == 0) {
        if (mode == kReplaceFirst) {
            st->it = 0;
            st->bb = rr;
        }
        st->rr = rr;
        st->rz = rz;
        st->tol2 = tol2;
        st->status = 0;
        st->done = (rr <= tol2) ? 1 : (st->it >= st->max_it ? 3 : 0);
    }
}

// ---------------------------------------------------------------- single-reduction CG
//
// Chronopoulos & Gear (1989) form of preconditioned CG: with u = dinv r,
// w = S u, gamma = (r, u) and delta = (u, w) from ONE reduction phase,
//   beta = gamma / gamma_old, alpha = gamma / (delta - beta gamma / alpha_old),
//   p = u + beta p, s = w + beta s (s = S p), x += alpha p, r -= alpha s.
// One pass updates every vector (cg1_vec_kernel), the operator is applied to
// u (its per-element partials give delta), and one finalize computes the
// scalars: four launches per iteration instead of seven.

// x = 0 (unless keep_x), r = b (or r as given when keep_x), u = dinv r,
// p = s = 0; partials (r, u), (r, r)
__global__ void __launch_bounds__(kBS)
cg1_init_kernel(const double *__restrict__ b, double *__restrict__ x, double *__restrict__ r, double *__restrict__ u,
                double *__restrict__ p, double *__restrict__ sv, const double *__restrict__ dinv, int keep_x,
                int64_t ng, double *__restrict__ part)
{
    double acc[2] = {0.0, 0.0};
    GRID_STRIDE(g, ng)
    {
        const double d = dinv[g];
        const double rg = d == 0.0 ? 0.0 : (keep_x ? r[g] : b[g]);
        if (!keep_x) x[g] = 0.0;
        r[g] = rg;
        const double ug = d * rg;
        u[g] = ug;
        p[g] = 0.0;
        sv[g] = 0.0;
        acc[0] += rg * ug;
        acc[1] += rg * rg;
    }
    block_store<2>(acc, part, gridDim.x);
}

// after the operator on u: gamma, delta, (r, r); first = 1 starts a run
// (alpha = gamma / delta, beta = 0, bb and tol2 when fresh = 1)
__global__ void __launch_bounds__(kBS)
cg1_finalize(CgState *st, const double *__restrict__ stage_v, const double *__restrict__ stage_e, int first, int fresh,
             double tol, double *hist)
{
    if (st->done && !first) return;
    const double gamma = block_sum(stage_v, kStage);
    const double rr = block_sum(stage_v + kStage, kStage);
    const double delta = block_sum(stage_e, kStage);
    if (threadIdx.x != 0) return;
    if (first) {
        if (fresh) {
            st->bb = rr;
            st->tol2 = tol * tol * rr;
            st->it = 0;
            if (hist && st->hist_len > 0) hist[0] = 1.0;
        }
        st->status = 0;
        st->rr = rr;
        st->rz = gamma;
        st->beta = 0.0;
        st->done = rr == 0.0 || rr <= st->tol2 ? 1 : 0;
        if (!st->done) {
            if (!(delta > 0.0) || !isfinite(delta) || !isfinite(gamma)) {
                st->done = 2;
                st->status = SEM_ERR_BREAKDOWN;
            } else {
                st->alpha = gamma / delta;
            }
        }
        return;
    }
    const int it = st->it + 1;
    st->it = it;
    st->rr = rr;
    if (hist && it < st->hist_len) hist[it] = sqrt(rr / st->bb);
    if (!isfinite(rr) || !isfinite(gamma) || !isfinite(delta)) {
        st->done = 2;
        st->status = SEM_ERR_BREAKDOWN;
        return;
    }
    if (rr <= st->tol2) {
        st->done = 1;
        return;
    }
    if (it >= st->max_it) {
        st->done = 3;
        return;
    }
    const double beta = gamma / st->rz;
    const double den = delta - beta * gamma / st->alpha;
    if (!(den > 0.0)) {
        st->done = 2;
        st->status = SEM_ERR_BREAKDOWN;
        return;
    }
    st->beta = beta;
    st->alpha = gamma / den;
    st->rz = gamma;
}

// s = Q^T w + beta s; p = dinv r + beta p; x += alpha p; r -= alpha s;
// u = dinv r; partials (r, u), (r, r).  w in the row layout.
template <int RPB, int NPC>
__global__ void __launch_bounds__(kBS)
cg1_vec_kernel(const CgState *__restrict__ st, const double *__restrict__ w, double *__restrict__ x,
               double *__restrict__ r, double *__restrict__ p, double *__restrict__ sv, double *__restrict__ u,
               const double *__restrict__ dinv, Lattice L, double *__restrict__ part)
{
    if (st->done) return;
    const double alpha = st->alpha, beta = st->beta;
    double acc[2] = {0.0, 0.0};
    const int nrows = (int)(L.ny * L.nz), row0 = (int)blockIdx.x * RPB, ny = (int)L.ny, nx = (int)L.nx;
    for (int gi = threadIdx.x; gi < nx; gi += kBS) {
        double d[RPB], xg[RPB], pg[RPB], rg[RPB], sg[RPB], wg[RPB];
        int64_t g[RPB];
#pragma unroll
        for (int q = 0; q < RPB; ++q) {
            const int row = row0 + q < nrows ? row0 + q : nrows - 1;   // clamped rows are not stored
            g[q] = gi + (int64_t)nx * row;
            d[q] = dinv[g[q]];
            xg[q] = x[g[q]];
            pg[q] = p[g[q]];
            rg[q] = r[g[q]];
            sg[q] = sv[g[q]];
            wg[q] = node_assemble_rows<NPC>(L, w, gi, row % ny, row / ny);
        }
#pragma unroll
        for (int q = 0; q < RPB; ++q) {
            if (row0 + q >= nrows || d[q] == 0.0) continue;   // Dirichlet node: every vector stays zero
            const double sn = wg[q] + beta * sg[q];
            const double pn = d[q] * rg[q] + beta * pg[q];
            const double rn = rg[q] - alpha * sn;
            const double un = d[q] * rn;
            sv[g[q]] = sn;
            p[g[q]] = pn;
            x[g[q]] = xg[q] + alpha * pn;
            r[g[q]] = rn;
            u[g[q]] = un;
            acc[0] += rn * un;
            acc[1] += rn * rn;
        }
    }
    block_store<2>(acc, part, gridDim.x);
}

// y += s * (double)d   (defect correction: x64 += scale * d32)
template <typename T>
__global__ void __launch_bounds__(kBS) axpy_kernel(double *__restrict__ y, const T *__restrict__ d, double s, int64_t ng)
{
    GRID_STRIDE(g, ng) y[g] += s * (double)d[g];
}

__global__ void __launch_bounds__(kBS) rsub_kernel(const double *__restrict__ x, double *__restrict__ e, int64_t ng)
{
    GRID_STRIDE(g, ng) e[g] = x[g] - e[g];
}

// out = (T)(s * in)
template <typename T>
__global__ void __launch_bounds__(kBS) scale_kernel(const double *__restrict__ in, T *__restrict__ out, double s, int64_t ng)
{
    GRID_STRIDE(g, ng) out[g] = (T)(s * in[g]);
}

}  // namespace cg

// ---------------------------------------------------------------- launchers

int cg_blocks(int64_t n)
{
    const int64_t b = (n + kBS - 1) / kBS;
    return (int)std::max<int64_t>(1, std::min<int64_t>(b, kMaxVecBlocks));
}

#define L3(k, n) hipLaunchKernelGGL(k, dim3(cg_blocks(n)), dim3(kBS), 0, s,

template <typename T>
hipError_t cg_gather(const Mesh &m, const double *u, T *ug, hipStream_t s)
{
    hipLaunchKernelGGL((cg::gather_kernel<double, T>), dim3(node_grid(m.lat)), dim3(kBS), 0, s, u, ug, m.lat);
    return hipGetLastError();
}

template <typename T>
hipError_t cg_scatter(const Mesh &m, const T *ug, double *u, hipStream_t s)
{
    L3((cg::scatter_kernel<T, double>), m.nl) ug, u, m.lat, m.nl);
    return hipGetLastError();
}

template <typename T>
hipError_t cg_dinv(const Mesh &m, const double *diag_local, T *dinv, hipStream_t s)
{
    hipLaunchKernelGGL((cg::dinv_kernel<T>), dim3(node_grid(m.lat)), dim3(kBS), 0, s, diag_local, dinv, m.lat);
    return hipGetLastError();
}

template <typename T>
hipError_t cg_init(const Mesh &m, const CgVecs<T> &v, const T *b, CgState *st, double tol, double *hist, hipStream_t s)
{
    const int nb = cg_blocks(m.ng);
    L3((cg::init_kernel<T>), m.ng) b, v.x, v.r, v.p, v.dinv, m.ng, v.part_b);
    hipLaunchKernelGGL(cg::init_finalize, dim3(1), dim3(kBS), 0, s, st, v.part_b, nb, tol, hist);
    return hipGetLastError();
}

template <typename T>
hipError_t cg_step_after_ax(const Mesh &m, const CgVecs<T> &v, CgState *st, double *hist, hipStream_t s)
{
    const unsigned nb = row_grid(m.lat, update_rpb<T>());
    hipError_t e = cg_alpha(m, v.part_e, v.stage, st, s);
    if (e != hipSuccess) return e;
    constexpr int RPB = update_rpb<T>();
    if (m.lat.NP == 8)
        hipLaunchKernelGGL((cg::update_kernel<T, RPB, 8>), dim3(nb), dim3(kBS), 0, s, st, v.w, v.x, v.r, v.p, v.dinv,
                           m.lat, v.part_b);
    else
        hipLaunchKernelGGL((cg::update_kernel<T, RPB, 0>), dim3(nb), dim3(kBS), 0, s, st, v.w, v.x, v.r, v.p, v.dinv,
                           m.lat, v.part_b);
    const double *in = v.part_b;
    int64_t n = nb;
    if ((e = finalize_input(v.part_b, n, 2, v.stage, s, &in)) != hipSuccess) return e;
    hipLaunchKernelGGL(cg::beta_direct_kernel, dim3(1), dim3(kWide), 0, s, st, in, (int)n, hist);
    L3((cg::p_kernel<T>), m.ng) st, v.p, v.r, v.dinv, m.ng);
    return hipGetLastError();
}

template <typename T>
hipError_t cg_resid(const Mesh &m, const CgVecs<T> &v, const T *b, T *r, CgState *st, hipStream_t s)
{
    const int64_t rows = node_grid(m.lat);
    hipLaunchKernelGGL((cg::resid_kernel<T>), dim3((unsigned)rows), dim3(kBS), 0, s, b, v.w, r, v.dinv, m.lat, v.part_b);
    hipError_t e = cg_reduce(v.part_b, rows, 1, v.stage, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(cg::resid_finalize, dim3(1), dim3(kBS), 0, s, st, v.stage, kStage);
    return hipGetLastError();
}

template <typename T>
hipError_t cg_restart(const Mesh &m, const CgVecs<T> &v, CgState *st, hipStream_t s)
{
    const int nb = cg_blocks(m.ng);
    L3((cg::restart_kernel<T>), m.ng) v.r, v.p, v.dinv, m.ng, v.part_b);
    hipLaunchKernelGGL(cg::restart_finalize, dim3(1), dim3(kBS), 0, s, st, v.part_b, nb);
    return hipGetLastError();
}

template <typename T>
hipError_t cg_replace(const Mesh &m, const CgVecs<T> &v, const double *r64, CgState *st, double inv_sigma,
                      double p_scale, int mode, double tol2, hipStream_t s)
{
    const int nb = cg_blocks(m.ng);
    L3((cg::replace_kernel<T>), m.ng) r64, v.x, v.r, v.p, v.dinv, inv_sigma, p_scale, mode, m.ng, v.part_b);
    hipLaunchKernelGGL(cg::replace_finalize, dim3(1), dim3(kBS), 0, s, st, v.part_b, nb, tol2, mode);
    return hipGetLastError();
}

hipError_t cg1_init(const Mesh &m, const CgVecs<double> &v, const double *b, double *u, double *sv, int keep_x,
                    hipStream_t s)
{
    const int nb = cg_blocks(m.ng);
    hipLaunchKernelGGL(cg::cg1_init_kernel, dim3(nb), dim3(kBS), 0, s, b, v.x, v.r, u, v.p, sv, v.dinv, keep_x, m.ng,
                       v.part_b);
    return cg_reduce(v.part_b, nb, 2, v.stage, s);
}

hipError_t cg1_vec(const Mesh &m, const CgVecs<double> &v, double *u, double *sv, CgState *st, hipStream_t s)
{
    const int64_t rows = row_grid(m.lat, 1);
    if (m.lat.NP == 8)
        hipLaunchKernelGGL((cg::cg1_vec_kernel<1, 8>), dim3((unsigned)rows), dim3(kBS), 0, s, st, v.w, v.x, v.r, v.p,
                           sv, u, v.dinv, m.lat, v.part_b);
    else
        hipLaunchKernelGGL((cg::cg1_vec_kernel<1, 0>), dim3((unsigned)rows), dim3(kBS), 0, s, st, v.w, v.x, v.r, v.p,
                           sv, u, v.dinv, m.lat, v.part_b);
    return cg_reduce(v.part_b, rows, 2, v.stage, s);
}

hipError_t cg1_finalize(const Mesh &m, const CgVecs<double> &v, CgState *st, int first, int fresh, double tol,
                        double *hist, hipStream_t s)
{
    hipError_t e = cg_reduce(v.part_e, m.E, 1, v.stage + 2 * kStage, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(cg::cg1_finalize, dim3(1), dim3(kBS), 0, s, st, v.stage, v.stage + 2 * kStage, first, fresh,
                       tol, hist);
    return hipGetLastError();
}

template <typename T>
hipError_t cg_axpy(const Mesh &m, double *y, const T *d, double scale, hipStream_t s)
{
    L3((cg::axpy_kernel<T>), m.ng) y, d, scale, m.ng);
    return hipGetLastError();
}

template <typename T>
hipError_t cg_scale(const Mesh &m, const double *in, T *out, double scale, hipStream_t s)
{
    L3((cg::scale_kernel<T>), m.ng) in, out, scale, m.ng);
    return hipGetLastError();
}

hipError_t cg_reduce(const double *part, int64_t n, int nv, double *stage, hipStream_t s)
{
    hipLaunchKernelGGL(cg::reduce_stage_kernel, dim3(kStage), dim3(kBS), 0, s, part, n, nv, stage);
    return hipGetLastError();
}

hipError_t finalize_input(const double *part, int64_t &n, int nv, double *stage, hipStream_t s, const double **in)
{
    *in = part;
    if (n <= kDirectMax) return hipSuccess;
    hipError_t e = cg_reduce(part, n, nv, stage, s);
    *in = stage;
    n = kStage;
    return e;
}

hipError_t cg_alpha(const Mesh &m, const double *part_e, double *stage, CgState *st, hipStream_t s)
{
    const double *in = part_e;
    int64_t n = m.E;
    hipError_t e = finalize_input(part_e, n, 1, stage, s, &in);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(cg::alpha_direct_kernel, dim3(1), dim3(kWide), 0, s, st, in, n);
    return hipGetLastError();
}

hipError_t cg_rsub(const Mesh &m, const double *x, double *e, hipStream_t s)
{
    L3(cg::rsub_kernel, m.ng) x, e, m.ng);
    return hipGetLastError();
}

#define INST(T)                                                                                              \
    template hipError_t cg_gather<T>(const Mesh &, const double *, T *, hipStream_t);                        \
    template hipError_t cg_scatter<T>(const Mesh &, const T *, double *, hipStream_t);                       \
    template hipError_t cg_dinv<T>(const Mesh &, const double *, T *, hipStream_t);                          \
    template hipError_t cg_init<T>(const Mesh &, const CgVecs<T> &, const T *, CgState *, double, double *,  \
                                   hipStream_t);                                                             \
    template hipError_t cg_step_after_ax<T>(const Mesh &, const CgVecs<T> &, CgState *, double *, hipStream_t); \
    template hipError_t cg_resid<T>(const Mesh &, const CgVecs<T> &, const T *, T *, CgState *, hipStream_t); \
    template hipError_t cg_restart<T>(const Mesh &, const CgVecs<T> &, CgState *, hipStream_t);              \
    template hipError_t cg_replace<T>(const Mesh &, const CgVecs<T> &, const double *, CgState *, double,     \
                                      double, int, double, hipStream_t);                                     \
    template hipError_t cg_axpy<T>(const Mesh &, double *, const T *, double, hipStream_t);                  \
    template hipError_t cg_scale<T>(const Mesh &, const double *, T *, double, hipStream_t);
INST(double)
INST(float)

}  // namespace sem
