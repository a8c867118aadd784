// learned.hip -- learned-smoother entry points: creation and weights,
// training pairs from Jacobi-PCG snapshots, one training step of the A-norm
// loss, and flexible CG with the learned smoother and a Jacobi-PCG fallback.
//
// Flexible CG (Notay 2000; Golub & Ye 1999): CG with z_k = M(r_k), which is
// neither linear nor symmetric, and the Polak-Ribiere coefficient
//   beta_k = (z_k, r_k - r_{k-1}) / (z_{k-1}, r_{k-1}) = -alpha (z_k, S p) / rz.
// Fallback ("judge"): a non-finite value or (r, z) <= 0 rejects the smoother
// output; a residual reduction over `window` iterations worse than
// rate^window (rate: plain Jacobi-PCG's per-iteration reduction) counts as a
// stall.  Either switches the solve, from the current iterate, to Jacobi-PCG.
// The FP64 true residual decides convergence in every case.
#include <chrono>
#include <cmath>
#include <cstring>
#include <random>

#include "cg.hpp"
#include "nn.hpp"

#define SEM_TRY(x)                   \
    do {                             \
        sem_status _s = (x);         \
        if (_s != SEM_OK) return _s; \
    } while (0)

namespace sem {
namespace lk {

#define GRID_STRIDE(g, n) for (int64_t g = (int64_t)blockIdx.x * kBS + threadIdx.x; g < (n); g += (int64_t)gridDim.x * kBS)

// Q^T w at one node for an operator output w in the row layout
__device__ __forceinline__ double assemble_at(const Lattice &L, const double *__restrict__ w, int gi, int gj, int gk,
                                              bool &masked)
{
    masked = lattice_masked(L, gi, gj, gk);
    return node_assemble_rows<0>(L, w, gi, gj, gk);
}

template <int NV>
__device__ __forceinline__ void block_store(double (&v)[NV], double *out, int stride)
{
    __shared__ double red[NV][kBS];
#pragma unroll
    for (int q = 0; q < NV; ++q) red[q][threadIdx.x] = v[q];
    __syncthreads();
    for (int w = kBS / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
#pragma unroll
            for (int q = 0; q < NV; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < NV; ++q) out[q * stride + blockIdx.x] = red[q][0];
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

// ------------------------------------------------------------ training step

__global__ void f32_to_f64_kernel(const float *__restrict__ a, double *__restrict__ b, int64_t n)
{
    GRID_STRIDE(g, n) b[g] = (double)a[g];
}

// out = Q^T w (0 on Dirichlet nodes); partial (u, out)
__global__ void __launch_bounds__(kBS)
assemble_dot_kernel(const double *__restrict__ w, const double *__restrict__ u, double *__restrict__ out, Lattice L,
                    double *__restrict__ part)
{
    double acc[1] = {0.0};
    SEM_FOR_EACH_NODE(L, gi, gj, gk, g)
    {
        bool msk;
        const double v = assemble_at(L, w, gi, gj, gk, msk);
        const double o = msk ? 0.0 : v;
        out[g] = o;
        acc[0] += u[g] * o;
    }
    block_store<1>(acc, part, gridDim.x);
}

__global__ void sub_kernel(const double *__restrict__ a, const double *__restrict__ b, double *__restrict__ c, int64_t n)
{
    GRID_STRIDE(g, n) c[g] = a[g] - b[g];
}

// scal[0] = |e|_S^2 (from part_a), scal[1] = |d|_S^2 / |e|_S^2 (from part_b)
__global__ void __launch_bounds__(kBS) loss_finalize(const double *__restrict__ pa, const double *__restrict__ pb, int nb,
                                                     double *__restrict__ scal)
{
    const double en = block_sum(pa, nb);
    const double dd = block_sum(pb, nb);
    if (threadIdx.x == 0) {
        scal[0] = en;
        scal[1] = en > 0.0 ? dd / en : 0.0;
    }
}

__global__ void gz_kernel(const double *__restrict__ sd, const double *__restrict__ scal, double *__restrict__ gz, int64_t n)
{
    const double en = scal[0];
    const double f = en > 0.0 ? -2.0 / en : 0.0;
    GRID_STRIDE(g, n) gz[g] = f * sd[g];
}

// ------------------------------------------------------------ flexible CG

// wg = Q^T w; x += alpha p; r -= alpha wg; q = wg; partial (r, r)
__global__ void __launch_bounds__(kBS)
fcg_update_kernel(const CgState *__restrict__ st, const double *__restrict__ w, double *__restrict__ x,
                  double *__restrict__ r, const double *__restrict__ p, const double *__restrict__ dinv,
                  double *__restrict__ q, Lattice L, double *__restrict__ part)
{
    if (st->done) return;
    const double alpha = st->alpha;
    double acc[1] = {0.0};
    SEM_FOR_EACH_NODE(L, gi, gj, gk, g)
    {
        if (dinv[g] == 0.0) { q[g] = 0.0; continue; }
        bool msk;
        const double wg = assemble_at(L, w, gi, gj, gk, msk);
        x[g] += alpha * p[g];
        const double rg = r[g] - alpha * wg;
        r[g] = rg;
        q[g] = wg;
        acc[0] += rg * rg;
    }
    block_store<1>(acc, part, gridDim.x);
}

// iteration count, convergence, stall test
__global__ void __launch_bounds__(kBS)
fcg_check_kernel(CgState *st, const double *__restrict__ part, int nb, double *hist, int window, double rate)
{
    if (st->done) return;
    const double rr = block_sum(part, nb);
    if (threadIdx.x == 0) {
        const int it = st->it + 1;
        st->it = it;
        st->rr = rr;
        const double rel = sqrt(rr / st->bb);
        if (hist && it < st->hist_len) hist[it] = rel;
        if (!isfinite(rr)) {
            st->done = 2;
            st->status = SEM_ERR_BREAKDOWN;
        } else if (rr <= st->tol2) {
            st->done = 1;
        } else if (it >= st->max_it) {
            st->done = 3;
        } else if (st->learned && rate > 0.0 && hist && it >= window && it < st->hist_len &&
                   rel > hist[it - window] * pow(rate, (double)window)) {
            st->learned = 0;   // stall: continue as Jacobi-PCG
            st->fallback_at = it;
        }
        st->nn_skip = (st->done || !st->learned) ? 1 : 0;
    }
}

// z = dinv r + (learned ? Q^T(c / mult) + zp : 0), zp (optional) the
// learned multigrid's coarser-level part; partials (r, z), (z, q)
__global__ void __launch_bounds__(kBS)
fcg_z_kernel(const CgState *__restrict__ st, const double *__restrict__ r, const double *__restrict__ dinv,
             const float *__restrict__ c, const double *__restrict__ q, double *__restrict__ z, Lattice L,
             double *__restrict__ part, const double *__restrict__ zp)
{
    if (st->done) return;
    const bool with_c = st->learned != 0;
    double acc[2] = {0.0, 0.0};
    SEM_FOR_EACH_NODE(L, gi, gj, gk, g)
    {
        const double d = dinv[g];
        double zz = 0.0;
        if (d != 0.0) {
            zz = d * r[g];
            if (with_c) {
                int loc[8];
                bool msk;
                const int n = node_locals(L, gi, gj, gk, loc, msk);
                float s = 0.f;
                for (int k = 0; k < n; ++k) s += c[loc[k]];
                zz += (double)s / n;
                if (zp) zz += zp[g];
            }
        }
        z[g] = zz;
        acc[0] += r[g] * zz;
        acc[1] += zz * (q ? q[g] : 0.0);
    }
    block_store<2>(acc, part, gridDim.x);
}

// rz_new, beta (Polak-Ribiere while learned, Fletcher-Reeves after fallback)
__global__ void __launch_bounds__(kBS) fcg_beta_kernel(CgState *st, const double *__restrict__ part, int nb, int first)
{
    if (st->done) return;
    const double rz = block_sum(part, nb);
    const double zq = block_sum(part + nb, nb);
    if (threadIdx.x == 0) {
        const bool bad = !(rz > 0.0) || !isfinite(rz) || !isfinite(zq);
        if (st->learned && bad) {
            st->learned = 0;
            st->redo = 1;   // p restarts from dinv r; rz from the restart partials
            st->fallback_at = st->it;
            st->beta = 0.0;
        } else if (bad) {
            st->done = 2;
            st->status = SEM_ERR_BREAKDOWN;
        } else if (first || st->fallback_at == st->it) {
            st->beta = 0.0;   // first direction, or first after a stall fallback
            st->rz = rz;
        } else if (st->learned) {
            st->beta = -st->alpha * zq / st->rz;
            st->rz = rz;
        } else {
            st->beta = rz / st->rz;
            st->rz = rz;
        }
        st->nn_skip = (st->done || !st->learned) ? 1 : 0;
    }
}

// p = z + beta p, or p = dinv r after a rejected smoother output (partial (r, p))
__global__ void __launch_bounds__(kBS)
fcg_p_kernel(const CgState *__restrict__ st, double *__restrict__ p, const double *__restrict__ z,
             const double *__restrict__ r, const double *__restrict__ dinv, int64_t ng, double *__restrict__ part)
{
    if (st->done) return;
    const bool redo = st->redo != 0;
    const double beta = st->beta;
    double acc[1] = {0.0};
    GRID_STRIDE(g, ng)
    {
        if (redo) {
            const double pz = dinv[g] * r[g];
            p[g] = pz;
            acc[0] += r[g] * pz;
        } else {
            p[g] = z[g] + beta * p[g];
        }
    }
    if (redo) block_store<1>(acc, part, gridDim.x);
}

__global__ void __launch_bounds__(kBS) fcg_redo_finalize(CgState *st, const double *__restrict__ part, int nb)
{
    if (st->done || !st->redo) return;
    const double rz = block_sum(part, nb);
    if (threadIdx.x == 0) {
        st->rz = rz;
        st->redo = 0;
    }
}

// ------------------------------------------------------------ nested solver

// b32 = r / |r| rounded to FP32 (outer residual norm from the device state)
__global__ void __launch_bounds__(kBS)
scale_defect_kernel(const CgState *__restrict__ st, const double *__restrict__ r, float *__restrict__ b32, int64_t ng)
{
    if (st->done || !st->learned) return;
    const double s = st->rr > 0.0 ? 1.0 / sqrt(st->rr) : 0.0;
    GRID_STRIDE(g, ng) b32[g] = (float)(s * r[g]);
}

// z = |r| x32 (inner solution) while the inner solver is active, else
// dinv r; accumulates the inner iteration count; partials (r, z), (z, q)
__global__ void __launch_bounds__(kBS)
nested_z_kernel(CgState *st, const CgState *__restrict__ st_in, const float *__restrict__ x32,
                const double *__restrict__ r, const double *__restrict__ dinv, const double *__restrict__ q,
                double *__restrict__ z, int64_t ng, double *__restrict__ part)
{
    if (st->done) return;
    const bool inner = st->learned != 0;
    const double s = sqrt(st->rr);
    double acc[2] = {0.0, 0.0};
    GRID_STRIDE(g, ng)
    {
        const double zz = inner ? s * (double)x32[g] : dinv[g] * r[g];
        z[g] = zz;
        acc[0] += r[g] * zz;
        acc[1] += zz * (q ? q[g] : 0.0);
    }
    block_store<2>(acc, part, gridDim.x);
    if (blockIdx.x == 0 && threadIdx.x == 0 && inner) st->inner_its += st_in->it;
}

__global__ void zero_kernel(double *__restrict__ a, int64_t n)
{
    GRID_STRIDE(g, n) a[g] = 0.0;
}

}  // namespace lk

namespace {

inline size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

inline int node_blocks(const Mesh &m) { return (int)node_grid(m.lat); }

sem_status read_state(CgState &h, const CgState *d, hipStream_t s)
{
    SEM_HIP_TRY(hipMemcpyAsync(&h, d, sizeof(CgState), hipMemcpyDeviceToHost, s));
    SEM_HIP_TRY(hipStreamSynchronize(s));
    return SEM_OK;
}

// He-normal initialisation of layers 1 and 2, zero layer 3 (a zero last
// layer makes the initial smoother exactly Jacobi).
void he_init(std::vector<float> &w, uint32_t seed)
{
    std::mt19937_64 rng(seed);
    std::normal_distribution<double> nd(0.0, 1.0);
    const double s1 = std::sqrt(2.0 / (27.0 * 2)), s2 = std::sqrt(2.0 / (27.0 * kChannels));
    for (int q = 0; q < kW1; ++q) w[q] = (float)(s1 * nd(rng));
    for (int q = 0; q < kW2; ++q) w[kW1 + q] = (float)(s2 * nd(rng));
    for (int q = 0; q < kW3; ++q) w[kW1 + kW2 + q] = 0.f;
}

// training buffers: e, r, z, d, sd, dinv (6 ng) and w (nl)
struct TrainBufs {
    double *e, *r, *z, *d, *sd, *dinv, *w;
};
TrainBufs train_bufs(const Smoother &sm)
{
    TrainBufs t;
    t.e = sm.buf;
    t.r = t.e + sm.ng;
    t.z = t.r + sm.ng;
    t.d = t.z + sm.ng;
    t.sd = t.d + sm.ng;
    t.dinv = t.sd + sm.ng;
    t.w = t.dinv + sm.ng;
    return t;
}


// dinv (assembled, 0 on Dirichlet nodes) into t.dinv, using t.w as scratch,
// unless the buffer already holds it for this mesh and h1, h2 (force = true
// always rebuilds); records what the buffer now holds
hipError_t make_dinv(const Smoother &sm, const Mesh &m, double h1, double h2, const TrainBufs &t, hipStream_t s,
                     bool force)
{
    if (!force && sm.dinv_serial == m.serial && sm.dinv_h1 == h1 && sm.dinv_h2 == h2) return hipSuccess;
    sm.dinv_serial = 0;
    hipError_t e = launch_diag(m, h1, h2, t.w, s);
    if (e != hipSuccess) return e;
    e = cg_dinv<double>(m, t.w, t.dinv, s);
    if (e != hipSuccess) return e;
    sm.dinv_serial = m.serial;
    sm.dinv_h1 = h1;
    sm.dinv_h2 = h2;
    return hipSuccess;
}

// loss L(e) and dL/dz in t.sd -> gz (in t.d), leaves |e|_S^2 and L in sm.scal
sem_status loss_forward(const Smoother &sm, const Mesh &m, double h1, double h2, const TrainBufs &t, hipStream_t s)
{
    const int nb = cg_blocks(m.ng);
    const int nbn = node_blocks(m);
    // r = S e, partial (e, S e)
    SEM_HIP_TRY(launch_ax_f64_gather(m, h1, h2, t.e, t.w, nullptr, s));
    hipLaunchKernelGGL(lk::assemble_dot_kernel, dim3(nbn), dim3(kBS), 0, s, t.w, t.e, t.r, m.lat, sm.part);
    // z = M(r) (FP32 network), plus the coarser levels' part C(r) when
    // training in the context of the learned multigrid
    if (sm.mg_context) SEM_HIP_TRY(hsmg_coarse_part(m, h1, h2, t.r, sm.mg, kWeightAvg, s));
    SEM_HIP_TRY(nn_infer32(sm, m, t.r, t.dinv, sm.c_local, s, sm.act));
    SEM_HIP_TRY(nn_assemble_z<double>(m, t.r, t.dinv, sm.c_local, t.z, s, nullptr, sm.mg_context ? sm.mg.zp : nullptr));
    // d = e - z, sd = S d, partial (d, S d)
    hipLaunchKernelGGL(lk::sub_kernel, dim3(nb), dim3(kBS), 0, s, t.e, t.z, t.d, m.ng);
    SEM_HIP_TRY(launch_ax_f64_gather(m, h1, h2, t.d, t.w, nullptr, s));
    const int64_t cap = part_capacity(m.lat, m.E);
    hipLaunchKernelGGL(lk::assemble_dot_kernel, dim3(nbn), dim3(kBS), 0, s, t.w, t.d, t.sd, m.lat, sm.part + cap);
    SEM_HIP_TRY(cg_reduce(sm.part, nbn, 1, sm.stage, s));
    SEM_HIP_TRY(cg_reduce(sm.part + cap, nbn, 1, sm.stage + kStage, s));
    hipLaunchKernelGGL(lk::loss_finalize, dim3(1), dim3(kBS), 0, s, sm.stage, sm.stage + kStage, kStage, sm.scal);
    hipLaunchKernelGGL(lk::gz_kernel, dim3(nb), dim3(kBS), 0, s, t.sd, sm.scal, t.d, m.ng);
    SEM_HIP_TRY(hipGetLastError());
    return SEM_OK;
}

sem_status gather_local(const Mesh &m, const double *u_local, double *ug, hipStream_t s)
{
    SEM_HIP_TRY(cg_gather<double>(m, u_local, ug, s));
    return SEM_OK;
}

}  // namespace

sem_status check_pair(const Smoother &sm, const Mesh &m)
{
    if (m.N != 7) return fail(SEM_ERR_UNSUPPORTED, "the learned smoother needs order N = 7");
    if (sm.E != m.E || sm.ng != m.ng) return fail(SEM_ERR_INVALID_ARG, "smoother was created for another mesh");
    if (sm.mg_context && !m.hsmg)
        return fail(SEM_ERR_INVALID_ARG, "a smoother trained in the multigrid context needs a mesh created with "
                                         "SEM_PREP_HSMG");
    return SEM_OK;
}

// the learned multigrid's coarser-level part of r into mg->zp, queued on the
// mesh's side stream so that it runs beside the network (mg null: plain
// learned smoother); fcg_join makes s wait for it before z is formed
static sem_status fcg_coarse(const Mesh &m, const sem_solve_opts &o, const CgVecs<double> &v, const HsmgBufs *mg,
                             hipStream_t s)
{
    if (mg) SEM_HIP_TRY(hsmg_coarse_part_fork(m, o.h1, o.h2, v.r, *mg, kWeightAvg, s));
    return SEM_OK;
}
static sem_status fcg_join(const Mesh &m, const HsmgBufs *mg, hipStream_t s)
{
    if (mg) SEM_HIP_TRY(hsmg_coarse_part_join(m, s));
    return SEM_OK;
}

// queue the flexible-CG direction update after r changed (initial, restart)
static sem_status fcg_direction(const Mesh &m, const sem_solve_opts &o, const Smoother &sm, const CgVecs<double> &v,
                                double *z, CgState *st, int first, const HsmgBufs *mg, hipStream_t s)
{
    const int nb = cg_blocks(m.ng);
    const int nbn = node_blocks(m);
    SEM_TRY(fcg_coarse(m, o, v, mg, s));
    SEM_HIP_TRY(nn_infer<double>(sm, m, v.r, v.dinv, sm.c_local, s, &st->nn_skip));
    SEM_TRY(fcg_join(m, mg, s));
    hipLaunchKernelGGL(lk::fcg_z_kernel, dim3(nbn), dim3(kBS), 0, s, st, v.r, v.dinv, sm.c_local,
                       (const double *)nullptr, z, m.lat, v.part_b, mg ? (const double *)mg->zp : nullptr);
    SEM_HIP_TRY(cg_reduce(v.part_b, nbn, 2, v.stage, s));
    hipLaunchKernelGGL(lk::fcg_beta_kernel, dim3(1), dim3(kBS), 0, s, st, v.stage, kStage, first);
    hipLaunchKernelGGL(lk::fcg_p_kernel, dim3(nb), dim3(kBS), 0, s, st, v.p, z, v.r, v.dinv, m.ng, v.part_b);
    hipLaunchKernelGGL(lk::fcg_redo_finalize, dim3(1), dim3(kBS), 0, s, st, v.part_b, nb);
    SEM_HIP_TRY(hipGetLastError());
    return SEM_OK;
}

sem_status solve_fcg(const Mesh &m, const Smoother &sm, const sem_solve_opts &o, const CgVecs<double> &v,
                     const double *b64, double *z, double *q, CgState *st, double *hist, int hist_len,
                     int check_every, hipStream_t s, sem_solve_report *rep, CgState &h, const HsmgBufs *mg)
{
    SEM_TRY(check_pair(sm, m));
    const int nb = cg_blocks(m.ng);
    const int nbn = node_blocks(m);
    CgState init{};
    init.max_it = o.max_iter;
    init.hist_len = hist_len;
    init.learned = 1;
    init.fallback_at = -1;
    SEM_HIP_TRY(hipMemcpyAsync(st, &init, sizeof(CgState), hipMemcpyHostToDevice, s));
    SEM_HIP_TRY(cg_init<double>(m, v, b64, st, o.rel_tol, hist, s));
    hipLaunchKernelGGL(lk::zero_kernel, dim3(nb), dim3(kBS), 0, s, v.p, m.ng);
    SEM_TRY(fcg_direction(m, o, sm, v, z, st, 1, mg, s));
    int restarts = 0;
    PollPlan plan;
    for (;;) {
        for (;;) {
            SEM_TRY(read_state(h, st, s));
            if (h.done) break;
            const int nq = plan.next(h, check_every);
            for (int it = 0; it < nq; ++it) {
                SEM_HIP_TRY(launch_ax_f64_gather(m, o.h1, o.h2, v.p, v.w, v.part_e, s, &st->done));
                SEM_HIP_TRY(cg_alpha(m, v.part_e, v.stage, st, s));
                hipLaunchKernelGGL(lk::fcg_update_kernel, dim3(nbn), dim3(kBS), 0, s, st, v.w, v.x, v.r, v.p, v.dinv,
                                   q, m.lat, v.part_b);
                SEM_HIP_TRY(cg_reduce(v.part_b, nbn, 1, v.stage, s));
                hipLaunchKernelGGL(lk::fcg_check_kernel, dim3(1), dim3(kBS), 0, s, st, v.stage, kStage, hist,
                                   sm.stall_window, sm.stall_rate);
                SEM_TRY(fcg_coarse(m, o, v, mg, s));
                SEM_HIP_TRY(nn_infer<double>(sm, m, v.r, v.dinv, sm.c_local, s, &st->nn_skip));
                SEM_TRY(fcg_join(m, mg, s));
                hipLaunchKernelGGL(lk::fcg_z_kernel, dim3(nbn), dim3(kBS), 0, s, st, v.r, v.dinv, sm.c_local,
                                   (const double *)q, z, m.lat, v.part_b, mg ? (const double *)mg->zp : nullptr);
                SEM_HIP_TRY(cg_reduce(v.part_b, nbn, 2, v.stage, s));
                hipLaunchKernelGGL(lk::fcg_beta_kernel, dim3(1), dim3(kBS), 0, s, st, v.stage, kStage, 0);
                hipLaunchKernelGGL(lk::fcg_p_kernel, dim3(nb), dim3(kBS), 0, s, st, v.p, z, v.r, v.dinv, m.ng,
                                   v.part_b);
                hipLaunchKernelGGL(lk::fcg_redo_finalize, dim3(1), dim3(kBS), 0, s, st, v.part_b, nb);
            }
            SEM_HIP_TRY(hipGetLastError());
        }
        if (h.done != 1 || h.bb == 0.0) break;
        // FP64 true residual decides
        SEM_HIP_TRY(launch_ax_f64_gather(m, o.h1, o.h2, v.x, v.w, nullptr, s));
        SEM_HIP_TRY(cg_resid<double>(m, v, b64, v.r, st, s));
        SEM_TRY(read_state(h, st, s));
        if (h.true_rr <= h.tol2 || restarts == 3 || h.it >= h.max_it) break;
        ++restarts;
        // restart the search direction from the true residual (keeps the mode)
        CgState patch = h;
        patch.done = 0;
        patch.rr = h.true_rr;
        patch.nn_skip = h.learned ? 0 : 1;
        SEM_HIP_TRY(hipMemcpyAsync(st, &patch, sizeof(CgState), hipMemcpyHostToDevice, s));
        SEM_TRY(fcg_direction(m, o, sm, v, z, st, 1, mg, s));
    }
    if (h.done != 1 && h.bb > 0.0) {
        SEM_HIP_TRY(launch_ax_f64_gather(m, o.h1, o.h2, v.x, v.w, nullptr, s));
        SEM_HIP_TRY(cg_resid<double>(m, v, b64, v.r, st, s));
        SEM_TRY(read_state(h, st, s));
    }
    rep->iterations = h.it;
    rep->restarts = restarts;
    rep->fallback_used = h.fallback_at >= 0 ? 1 : 0;
    return SEM_OK;
}

// queue one preconditioner application: z = |r| * (inner_iters steps of
// low-precision Jacobi-PCG on r / |r|), then the partials (r, z), (z, q)
static sem_status nested_precondition(const Mesh &m, const sem_solve_opts &o, const CgVecs<double> &v,
                                      const CgVecs<float> &v32, float *b32, double *z, const double *q,
                                      CgState *st, CgState *st32, bool bf16, bool inner_active, hipStream_t s)
{
    const int nb = cg_blocks(m.ng);
    if (inner_active) {
        hipLaunchKernelGGL(lk::scale_defect_kernel, dim3(nb), dim3(kBS), 0, s, st, v.r, b32, m.ng);
        SEM_HIP_TRY(cg_init<float>(m, v32, b32, st32, o.inner_tol, nullptr, s));
        for (int k = 0; k < o.inner_iters; ++k) {
            if (bf16)
                SEM_HIP_TRY(launch_ax_bf16_gather(m, (float)o.h1, (float)o.h2, v32.p, v32.w, v32.part_e, s, &st32->done));
            else
                SEM_HIP_TRY(launch_ax_f32_gather(m, (float)o.h1, (float)o.h2, v32.p, v32.w, v32.part_e, s, &st32->done));
            SEM_HIP_TRY(cg_step_after_ax<float>(m, v32, st32, nullptr, s));
        }
    }
    hipLaunchKernelGGL(lk::nested_z_kernel, dim3(nb), dim3(kBS), 0, s, st, st32, v32.x, v.r, v.dinv, q, z, m.ng,
                       v.part_b);
    SEM_HIP_TRY(hipGetLastError());
    return SEM_OK;
}

sem_status solve_fcg_nested(const Mesh &m, const sem_solve_opts &o, const CgVecs<double> &v, const CgVecs<float> &v32,
                            float *b32, const double *b64, double *z, double *q, CgState *st, CgState *st32,
                            double *hist, int hist_len, int check_every, bool bf16, hipStream_t s,
                            sem_solve_report *rep, CgState &h)
{
    const int nb = cg_blocks(m.ng);
    const int nbn = node_blocks(m);
    CgState init{};
    init.max_it = o.max_iter;
    init.hist_len = hist_len;
    init.learned = 1;
    init.fallback_at = -1;
    SEM_HIP_TRY(hipMemcpyAsync(st, &init, sizeof(CgState), hipMemcpyHostToDevice, s));
    CgState init32{};
    init32.max_it = o.inner_iters;
    SEM_HIP_TRY(hipMemcpyAsync(st32, &init32, sizeof(CgState), hipMemcpyHostToDevice, s));
    SEM_HIP_TRY(cg_init<double>(m, v, b64, st, o.rel_tol, hist, s));
    hipLaunchKernelGGL(lk::zero_kernel, dim3(nb), dim3(kBS), 0, s, v.p, m.ng);
    bool inner_active = true;
    auto direction = [&](int first) -> sem_status {
        SEM_TRY(nested_precondition(m, o, v, v32, b32, z, first ? nullptr : q, st, st32, bf16, inner_active, s));
        hipLaunchKernelGGL(lk::fcg_beta_kernel, dim3(1), dim3(kBS), 0, s, st, v.part_b, nb, first);
        hipLaunchKernelGGL(lk::fcg_p_kernel, dim3(nb), dim3(kBS), 0, s, st, v.p, z, v.r, v.dinv, m.ng, v.part_b);
        hipLaunchKernelGGL(lk::fcg_redo_finalize, dim3(1), dim3(kBS), 0, s, st, v.part_b, nb);
        SEM_HIP_TRY(hipGetLastError());
        return SEM_OK;
    };
    SEM_TRY(direction(1));
    int restarts = 0;
    for (;;) {
        for (;;) {
            SEM_TRY(read_state(h, st, s));
            if (h.done) break;
            inner_active = h.learned != 0;
            for (int it = 0; it < check_every; ++it) {
                SEM_HIP_TRY(launch_ax_f64_gather(m, o.h1, o.h2, v.p, v.w, v.part_e, s, &st->done));
                SEM_HIP_TRY(cg_alpha(m, v.part_e, v.stage, st, s));
                hipLaunchKernelGGL(lk::fcg_update_kernel, dim3(nbn), dim3(kBS), 0, s, st, v.w, v.x, v.r, v.p, v.dinv,
                                   q, m.lat, v.part_b);
                SEM_HIP_TRY(cg_reduce(v.part_b, nbn, 1, v.stage, s));
                hipLaunchKernelGGL(lk::fcg_check_kernel, dim3(1), dim3(kBS), 0, s, st, v.stage, kStage, hist, 25, 0.0);
                SEM_TRY(direction(0));
            }
        }
        if (h.done != 1 || h.bb == 0.0) break;
        SEM_HIP_TRY(launch_ax_f64_gather(m, o.h1, o.h2, v.x, v.w, nullptr, s));
        SEM_HIP_TRY(cg_resid<double>(m, v, b64, v.r, st, s));
        SEM_TRY(read_state(h, st, s));
        if (h.true_rr <= h.tol2 || restarts == 3 || h.it >= h.max_it) break;
        ++restarts;
        CgState patch = h;
        patch.done = 0;
        patch.rr = h.true_rr;
        SEM_HIP_TRY(hipMemcpyAsync(st, &patch, sizeof(CgState), hipMemcpyHostToDevice, s));
        inner_active = h.learned != 0;
        SEM_TRY(direction(1));
    }
    if (h.done != 1 && h.bb > 0.0) {
        SEM_HIP_TRY(launch_ax_f64_gather(m, o.h1, o.h2, v.x, v.w, nullptr, s));
        SEM_HIP_TRY(cg_resid<double>(m, v, b64, v.r, st, s));
        SEM_TRY(read_state(h, st, s));
    }
    rep->iterations = h.inner_its;
    rep->outer_iterations = h.it;
    rep->restarts = restarts;
    rep->fallback_used = h.fallback_at >= 0 ? 1 : 0;
    return SEM_OK;
}

}  // namespace sem

using namespace sem;

extern "C" {

sem_status sem_smoother_create(const sem_mesh *mesh, const sem_smoother_desc *desc, sem_smoother **out)
{
    if (!mesh || !out) return fail(SEM_ERR_INVALID_ARG, "null mesh or out");
    *out = nullptr;
    const Mesh &m = mesh->m;
    if (m.N != 7) return fail(SEM_ERR_UNSUPPORTED, "the learned smoother needs order N = 7");
    sem_smoother *h = new (std::nothrow) sem_smoother();
    if (!h) return fail(SEM_ERR_OUT_OF_MEMORY, "host allocation");
    Smoother &sm = h->s;
    sm.E = m.E;
    sm.ng = m.ng;
    sm.nl = m.nl;
    uint32_t seed = 0;
    if (desc) {
        seed = desc->seed;
        if (desc->lr > 0) sm.lr = desc->lr;
        if (desc->beta1 > 0) sm.b1 = desc->beta1;
        if (desc->beta2 > 0) sm.b2 = desc->beta2;
        if (desc->eps > 0) sm.eps = desc->eps;
        if (desc->stall_window > 0) sm.stall_window = desc->stall_window;
        sm.stall_rate = desc->stall_rate;
        sm.mg_context = desc->mg_context != 0;
    }
    if (sm.mg_context && !m.hsmg) {
        delete h;
        return fail(SEM_ERR_INVALID_ARG, "mg_context needs a mesh created with SEM_PREP_HSMG");
    }
    struct Alloc { void **p; size_t bytes; } allocs[] = {
        {(void **)&sm.W, kParams * 4}, {(void **)&sm.m, kParams * 4}, {(void **)&sm.v, kParams * 4},
        {(void **)&sm.grad, kParams * 4}, {(void **)&sm.W2b, kWeightOperands * 2}, {(void **)&sm.Wt, kWtFloats * 4},
        {(void **)&sm.dW_elem, (size_t)m.E * kParams * 4}, {(void **)&sm.gpart, (size_t)kGradChunks * kParams * 8},
        {(void **)&sm.act, (size_t)m.E * 32 * 512 * 4},
        {(void **)&sm.c_local, (size_t)m.nl * 4},
        {(void **)&sm.buf, (size_t)(6 * m.ng + m.nl) * 8},
        {(void **)&sm.part, (size_t)part_capacity(m.lat, m.E) * 2 * 8}, {(void **)&sm.stage, (size_t)kStage * 2 * 8},
        {(void **)&sm.scal, 64}, {(void **)&sm.mg_ws, sm.mg_context ? hsmg_bufs_bytes(m) : 0}};
    for (auto &a : allocs) {
        if (a.bytes == 0) continue;
        if (hipMalloc(a.p, a.bytes) != hipSuccess) {
            sem_smoother_destroy(h);
            return fail(SEM_ERR_OUT_OF_MEMORY, "hipMalloc for the smoother");
        }
        sm.device_bytes += a.bytes;
    }
    if (sm.mg_context) sm.mg = hsmg_bufs_carve(m, sm.mg_ws);
    std::vector<float> w(kParams);
    he_init(w, seed);
    sem_status st = sem_smoother_set_weights(h, w.data(), kParams);
    if (st != SEM_OK) {
        sem_smoother_destroy(h);
        return st;
    }
    *out = h;
    return SEM_OK;
}

sem_status sem_smoother_destroy(sem_smoother *sm)
{
    if (!sm) return SEM_OK;
    Smoother &s = sm->s;
    void *ps[] = {s.W, s.m, s.v, s.grad, s.W2b, s.Wt, s.dW_elem, s.gpart, s.act, s.c_local, s.buf, s.part, s.stage, s.scal, s.mg_ws};
    for (void *p : ps)
        if (p) (void)hipFree(p);
    delete sm;
    return SEM_OK;
}

sem_status sem_smoother_set_weights(sem_smoother *sm, const float *host, size_t n)
{
    if (!sm || !host) return fail(SEM_ERR_INVALID_ARG, "null smoother or weights");
    if (n != (size_t)kParams) return fail(SEM_ERR_INVALID_ARG, "expected " + std::to_string(kParams) + " weights");
    Smoother &s = sm->s;
    SEM_HIP_TRY(hipMemcpy(s.W, host, kParams * 4, hipMemcpyHostToDevice));
    SEM_HIP_TRY(hipMemset(s.m, 0, kParams * 4));
    SEM_HIP_TRY(hipMemset(s.v, 0, kParams * 4));
    s.step = 0;
    s.dinv_serial = 0;
    SEM_HIP_TRY(nn_pack(s, nullptr));
    SEM_HIP_TRY(hipDeviceSynchronize());
    return SEM_OK;
}

sem_status sem_smoother_get_weights(const sem_smoother *sm, float *host, size_t n)
{
    if (!sm || !host) return fail(SEM_ERR_INVALID_ARG, "null smoother or weights");
    if (n != (size_t)kParams) return fail(SEM_ERR_INVALID_ARG, "expected " + std::to_string(kParams) + " weights");
    SEM_HIP_TRY(hipMemcpy(host, sm->s.W, kParams * 4, hipMemcpyDeviceToHost));
    return SEM_OK;
}

sem_status sem_smoother_get_state(const sem_smoother *sm, float *weights, float *adam_m, float *adam_v, size_t n,
                                  int32_t *step)
{
    if (!sm || !weights || !adam_m || !adam_v || !step) return fail(SEM_ERR_INVALID_ARG, "null argument");
    if (n != (size_t)kParams) return fail(SEM_ERR_INVALID_ARG, "expected " + std::to_string(kParams) + " values");
    const Smoother &s = sm->s;
    SEM_HIP_TRY(hipDeviceSynchronize());
    SEM_HIP_TRY(hipMemcpy(weights, s.W, kParams * 4, hipMemcpyDeviceToHost));
    SEM_HIP_TRY(hipMemcpy(adam_m, s.m, kParams * 4, hipMemcpyDeviceToHost));
    SEM_HIP_TRY(hipMemcpy(adam_v, s.v, kParams * 4, hipMemcpyDeviceToHost));
    *step = s.step;
    return SEM_OK;
}

sem_status sem_smoother_set_state(sem_smoother *sm, const float *weights, const float *adam_m, const float *adam_v,
                                  size_t n, int32_t step)
{
    if (!sm || !weights || !adam_m || !adam_v) return fail(SEM_ERR_INVALID_ARG, "null argument");
    if (n != (size_t)kParams) return fail(SEM_ERR_INVALID_ARG, "expected " + std::to_string(kParams) + " values");
    if (step < 0) return fail(SEM_ERR_INVALID_ARG, "negative Adam step count");
    Smoother &s = sm->s;
    SEM_HIP_TRY(hipDeviceSynchronize());
    SEM_HIP_TRY(hipMemcpy(s.W, weights, kParams * 4, hipMemcpyHostToDevice));
    SEM_HIP_TRY(hipMemcpy(s.m, adam_m, kParams * 4, hipMemcpyHostToDevice));
    SEM_HIP_TRY(hipMemcpy(s.v, adam_v, kParams * 4, hipMemcpyHostToDevice));
    s.step = step;
    SEM_HIP_TRY(nn_pack(s, nullptr));
    SEM_HIP_TRY(hipDeviceSynchronize());
    return SEM_OK;
}

sem_status sem_smoother_apply(const sem_smoother *sm, const sem_mesh *mesh, double h1, double h2, int fp32,
                              const double *r_local, double *z_local, void *stream)
{
    if (!sm || !mesh || !r_local || !z_local) return fail(SEM_ERR_INVALID_ARG, "null argument");
    const Smoother &s = sm->s;
    const Mesh &m = mesh->m;
    SEM_TRY(check_pair(s, m));
    hipStream_t st = (hipStream_t)stream;
    TrainBufs t = train_bufs(s);
    SEM_HIP_TRY(make_dinv(s, m, h1, h2, t, st, true));
    SEM_TRY(gather_local(m, r_local, t.r, st));
    if (fp32)
        SEM_HIP_TRY(nn_infer32(s, m, t.r, t.dinv, s.c_local, st));
    else
        SEM_HIP_TRY(nn_infer<double>(s, m, t.r, t.dinv, s.c_local, st, nullptr));
    SEM_HIP_TRY(nn_assemble_z<double>(m, t.r, t.dinv, s.c_local, t.z, st, nullptr));
    SEM_HIP_TRY(cg_scatter<double>(m, t.z, z_local, st));
    return SEM_OK;
}

sem_status sem_smoother_mg_apply(const sem_smoother *sm, const sem_mesh *mesh, double h1, double h2, int fp32,
                                 const double *r_local, double *z_local, void *workspace, size_t ws_bytes,
                                 void *stream)
{
    if (!sm || !mesh || !r_local || !z_local || !workspace) return fail(SEM_ERR_INVALID_ARG, "null argument");
    const Smoother &s = sm->s;
    const Mesh &m = mesh->m;
    SEM_TRY(check_pair(s, m));
    if (!m.hsmg) return fail(SEM_ERR_INVALID_ARG, "the learned multigrid needs a mesh created with SEM_PREP_HSMG");
    if (!(h1 > 0.0) || !(h2 >= 0.0) || !std::isfinite(h1) || !std::isfinite(h2))
        return fail(SEM_ERR_INVALID_ARG, "the learned multigrid needs h1 > 0 and h2 >= 0");
    if (ws_bytes < hsmg_bufs_bytes(m))
        return fail(SEM_ERR_INVALID_ARG, "workspace too small: need " + std::to_string(hsmg_bufs_bytes(m)) + " bytes");
    hipStream_t st = (hipStream_t)stream;
    TrainBufs t = train_bufs(s);
    const HsmgBufs hb = hsmg_bufs_carve(m, (char *)workspace);
    SEM_HIP_TRY(make_dinv(s, m, h1, h2, t, st, true));
    SEM_TRY(gather_local(m, r_local, t.r, st));
    const FineHook hook{&s, t.dinv, s.c_local, fp32 ? 1 : 0};
    SEM_HIP_TRY(hsmg_apply(m, h1, h2, t.r, t.z, hb, 3, kWeightAvg, st, &hook));
    SEM_HIP_TRY(cg_scatter<double>(m, t.z, z_local, st));
    return SEM_OK;
}

sem_status sem_smoother_loss_grad(sem_smoother *sm, const sem_mesh *mesh, double h1, double h2, const double *e_local,
                                  double *loss_host, float *grad_host, void *stream)
{
    if (!sm || !mesh || !e_local || !loss_host || !grad_host) return fail(SEM_ERR_INVALID_ARG, "null argument");
    Smoother &s = sm->s;
    const Mesh &m = mesh->m;
    SEM_TRY(check_pair(s, m));
    hipStream_t st = (hipStream_t)stream;
    TrainBufs t = train_bufs(s);
    SEM_HIP_TRY(make_dinv(s, m, h1, h2, t, st, true));
    SEM_TRY(gather_local(m, e_local, t.e, st));
    SEM_TRY(loss_forward(s, m, h1, h2, t, st));
    SEM_HIP_TRY(nn_grad(s, m, t.r, t.dinv, t.d, s.dW_elem, 1.0, s.grad, st, s.act));
    double scal[2];
    SEM_HIP_TRY(hipMemcpyAsync(scal, s.scal, 16, hipMemcpyDeviceToHost, st));
    SEM_HIP_TRY(hipMemcpyAsync(grad_host, s.grad, kParams * 4, hipMemcpyDeviceToHost, st));
    SEM_HIP_TRY(hipStreamSynchronize(st));
    *loss_host = scal[1];
    return SEM_OK;
}

sem_status sem_smoother_train_step(sem_smoother *sm, const sem_mesh *mesh, double h1, double h2, const float *e_global,
                                   double *loss_dev, void *stream)
{
    if (!sm || !mesh || !e_global) return fail(SEM_ERR_INVALID_ARG, "null argument");
    Smoother &s = sm->s;
    const Mesh &m = mesh->m;
    SEM_TRY(check_pair(s, m));
    hipStream_t st = (hipStream_t)stream;
    TrainBufs t = train_bufs(s);
    SEM_HIP_TRY(make_dinv(s, m, h1, h2, t, st, false));
    hipLaunchKernelGGL(lk::f32_to_f64_kernel, dim3(cg_blocks(m.ng)), dim3(kBS), 0, st, e_global, t.e, m.ng);
    SEM_TRY(loss_forward(s, m, h1, h2, t, st));
    SEM_HIP_TRY(nn_grad(s, m, t.r, t.dinv, t.d, s.dW_elem, 1.0, s.grad, st, s.act));
    SEM_HIP_TRY(nn_adam(s, s.grad, st));
    if (loss_dev) SEM_HIP_TRY(hipMemcpyAsync(loss_dev, s.scal + 1, 8, hipMemcpyDeviceToDevice, st));
    return SEM_OK;
}

}  // extern "C"
