// solve.hip -- the solve drivers (paper section 3.1: a preconditioned Krylov
// solve of Ax = b every time step) and the operator entry points of the C ABI.
//
// FP64 Jacobi-PCG (Hestenes & Stiefel 1952; z = dinv o r) on assembled
// vectors, one iteration =
//   1. w = A_L p          operator, p read through the numbering, per-element
//                         partial of p.w (= (p, S p) for a continuous p)
//   2. alpha = rz / pw    one-block finalize
//   3. Q^T w, x += a p, r -= a Q^T w, partials of (r,r), (r,z)
//   4. beta, convergence test (one block);  5. p = dinv r + beta p.
// The host only polls the device convergence flag every check_every
// iterations; kernels queued after convergence exit at once.
//
// FP32 defect correction (Wilkinson-style iterative refinement): the FP64
// true residual r = b - S x is scaled to unit norm, rounded to FP32, an FP32
// PCG on the FP32 operator (DC_BF16: the split-BF16 matrix-core operator)
// solves S d = r to inner_tol, and x += |r| d in FP64.  FP64 is kept for the outer residual, every inner product and the
// convergence tests.  The reliable-update forms keep one low-precision Krylov
// process and replace its residual instead (solve_reliable); the
// single-reduction form is solve_pcg1.
#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>

#include "cg.hpp"
#include "hsmg.hpp"
#include "nn.hpp"
#include "sem_internal.hpp"

#define SEM_TRY(x)                   \
    do {                             \
        sem_status _s = (x);         \
        if (_s != SEM_OK) return _s; \
    } while (0)

namespace sem {
namespace {

inline size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

struct Workspace {
    CgVecs<double> v64;      // x, r, p, dinv (assembled), w (local)
    double *b64;             // assembled right-hand side
    CgVecs<float> v32;       // inner FP32 vectors (DC form)
    float *b32;
    double *z, *q;           // flexible CG: smoother output and S p (assembled)
    CgState *st64, *st32;
    double *hist;
    GmresBufs gm;            // flexible GMRES with the multigrid preconditioner
    HsmgBufs hb;             // block-Jacobi preconditioner buffers
    size_t bytes;
};

bool uses_f32(int form)
{
    return form == SEM_FORM_DC_FP32 || form == SEM_FORM_DC_BF16 || form == SEM_FORM_FCG_INNER_FP32 ||
           form == SEM_FORM_FCG_INNER_BF16 || form == SEM_FORM_RELIABLE_FP32 || form == SEM_FORM_RELIABLE_BF16;
}
bool uses_fcg(int form)
{
    return form == SEM_FORM_FCG_LEARNED || form == SEM_FORM_FCG_INNER_FP32 || form == SEM_FORM_FCG_INNER_BF16 ||
           form == SEM_FORM_FCG_LEARNED_MG;
}
// forms that need the two extra assembled FP64 vectors z and q
bool uses_zq(int form)
{
    return uses_fcg(form) || form == SEM_FORM_PCG_1RED || form == SEM_FORM_PCG_BLOCK_JACOBI || form == SEM_FORM_PCG_HSMG;
}
int gmres_restart(const sem_solve_opts &o) { return o.restart > 0 ? std::min(o.restart, kGmresMaxRestart) : kGmresMaxRestart; }

Workspace carve(const Mesh &m, const sem_solve_opts &o, int hist_len, char *base)
{
    const int form = o.form;
    Workspace ws{};
    size_t off = 0;
    auto take = [&](size_t bytes) -> char * {
        char *p = base ? base + off : nullptr;
        off += align256(bytes);
        return p;
    };
    const size_t nl = (size_t)m.nl, ng = (size_t)m.ng;
    ws.v64.x = (double *)take(ng * 8);
    ws.v64.r = (double *)take(ng * 8);
    ws.v64.p = (double *)take(ng * 8);
    ws.v64.dinv = (double *)take(ng * 8);
    ws.b64 = (double *)take(ng * 8);
    ws.v64.w = (double *)take(nl * 8);
    ws.v64.part_e = (double *)take((size_t)std::max<int64_t>(m.E, 1) * 8);
    ws.v64.part_b = (double *)take((size_t)part_capacity(m.lat, m.E) * 3 * 8);
    ws.v64.stage = (double *)take((size_t)kStage * 3 * 8);
    ws.st64 = (CgState *)take(sizeof(CgState));
    ws.st32 = (CgState *)take(sizeof(CgState));
    ws.hist = (double *)take((size_t)std::max(hist_len, 1) * 8);
    if (uses_zq(form)) {
        ws.z = (double *)take(ng * 8);
        ws.q = (double *)take(ng * 8);
    }
    if (uses_f32(form)) {
        ws.v32.x = (float *)take(ng * 4);
        ws.v32.r = (float *)take(ng * 4);
        ws.v32.p = (float *)take(ng * 4);
        ws.v32.dinv = (float *)take(ng * 4);
        ws.b32 = (float *)take(ng * 4);
        ws.v32.w = (float *)take(nl * 4);
        ws.v32.part_e = ws.v64.part_e;
        ws.v32.part_b = ws.v64.part_b;
        ws.v32.stage = ws.v64.stage;
    }
    if (form == SEM_FORM_GMRES_HSMG || form == SEM_FORM_GMRES_LEARNED_MG) {
        const int mres = gmres_restart(o);
        char *p = take(gmres_bufs_bytes(m, mres));
        if (base) ws.gm = gmres_bufs_carve(m, mres, p);
    }
    if (form == SEM_FORM_PCG_BLOCK_JACOBI || form == SEM_FORM_PCG_HSMG || form == SEM_FORM_FCG_LEARNED_MG) {
        char *p = take(hsmg_bufs_bytes(m));
        if (base) ws.hb = hsmg_bufs_carve(m, p);
    }
    ws.bytes = off;
    return ws;
}

int hist_len_for(const sem_solve_opts &o) { return o.max_iter + 1; }

sem_status check_opts(const Mesh &m, const sem_solve_opts *o)
{
    if (!o) return fail(SEM_ERR_INVALID_ARG, "null opts");
    if (o->max_iter < 1) return fail(SEM_ERR_INVALID_ARG, "max_iter must be >= 1");
    if (!(o->rel_tol > 0.0) || !std::isfinite(o->rel_tol))
        return fail(SEM_ERR_INVALID_ARG, "rel_tol must be a positive finite number");
    if (!std::isfinite(o->h1) || !std::isfinite(o->h2)) return fail(SEM_ERR_INVALID_ARG, "non-finite h1/h2");
    switch (o->form) {
    case SEM_FORM_JACOBI_PCG:
    case SEM_FORM_PCG_1RED:
        return SEM_OK;
    case SEM_FORM_DC_FP32:
    case SEM_FORM_DC_BF16:
        if (o->form == SEM_FORM_DC_FP32 && !m.d_G32)
            return fail(SEM_ERR_INVALID_ARG, "SEM_FORM_DC_FP32 needs a mesh created with SEM_PREP_F32");
        if (o->form == SEM_FORM_DC_BF16 && !m.d_Gh)
            return fail(SEM_ERR_INVALID_ARG, "SEM_FORM_DC_BF16 needs a mesh created with SEM_PREP_BF16");
        if (o->form == SEM_FORM_DC_BF16 && m.N != 7)
            return fail(SEM_ERR_UNSUPPORTED, "the bf16 operator needs order N = 7");
        if (!(o->inner_tol > 0.0 && o->inner_tol < 1.0))
            return fail(SEM_ERR_INVALID_ARG, "inner_tol must be in (0, 1)");
        if (o->max_outer < 1) return fail(SEM_ERR_INVALID_ARG, "max_outer must be >= 1");
        return SEM_OK;
    case SEM_FORM_FCG_INNER_FP32:
    case SEM_FORM_FCG_INNER_BF16:
        if (o->form == SEM_FORM_FCG_INNER_FP32 && !m.d_G32)
            return fail(SEM_ERR_INVALID_ARG, "SEM_FORM_FCG_INNER_FP32 needs a mesh created with SEM_PREP_F32");
        if (o->form == SEM_FORM_FCG_INNER_BF16 && !m.d_Gbf)
            return fail(SEM_ERR_INVALID_ARG, "SEM_FORM_FCG_INNER_BF16 needs a mesh created with SEM_PREP_BF16");
        if (o->form == SEM_FORM_FCG_INNER_BF16 && m.N != 7)
            return fail(SEM_ERR_UNSUPPORTED, "the bf16 operator needs order N = 7");
        if (o->inner_iters < 1 || o->inner_iters > 10000) return fail(SEM_ERR_INVALID_ARG, "inner_iters must be in 1..10000");
        if (!(o->inner_tol >= 0.0 && o->inner_tol < 1.0)) return fail(SEM_ERR_INVALID_ARG, "inner_tol must be in [0, 1)");
        return SEM_OK;
    case SEM_FORM_RELIABLE_FP32:
    case SEM_FORM_RELIABLE_BF16:
        if (o->form == SEM_FORM_RELIABLE_FP32 && !m.d_G32)
            return fail(SEM_ERR_INVALID_ARG, "SEM_FORM_RELIABLE_FP32 needs a mesh created with SEM_PREP_F32");
        if (o->form == SEM_FORM_RELIABLE_BF16 && !m.d_Gbf)
            return fail(SEM_ERR_INVALID_ARG, "SEM_FORM_RELIABLE_BF16 needs a mesh created with SEM_PREP_BF16");
        if (o->form == SEM_FORM_RELIABLE_BF16 && m.N != 7)
            return fail(SEM_ERR_UNSUPPORTED, "the bf16 operator needs order N = 7");
        if (!(o->inner_tol > 0.0 && o->inner_tol < 1.0))
            return fail(SEM_ERR_INVALID_ARG, "inner_tol (the replacement threshold) must be in (0, 1)");
        return SEM_OK;
    case SEM_FORM_GMRES_HSMG:
    case SEM_FORM_PCG_BLOCK_JACOBI:
    case SEM_FORM_PCG_HSMG:
        if (!m.hsmg) return fail(SEM_ERR_INVALID_ARG, "this form needs a mesh created with SEM_PREP_HSMG");
        if (!(o->h1 > 0.0)) return fail(SEM_ERR_INVALID_ARG, "the multigrid and block-Jacobi forms need h1 > 0");
        if (o->h2 < 0.0) return fail(SEM_ERR_INVALID_ARG, "h2 must be >= 0");
        if (o->restart < 0 || o->restart > kGmresMaxRestart)
            return fail(SEM_ERR_INVALID_ARG, "restart must be in 0.." + std::to_string(kGmresMaxRestart));
        return SEM_OK;
    case SEM_FORM_FCG_LEARNED:
        if (!o->smoother) return fail(SEM_ERR_INVALID_ARG, "SEM_FORM_FCG_LEARNED needs opts.smoother");
        if (m.N != 7) return fail(SEM_ERR_UNSUPPORTED, "the learned smoother needs order N = 7");
        return SEM_OK;
    case SEM_FORM_GMRES_LEARNED_MG:
    case SEM_FORM_FCG_LEARNED_MG:
        if (!o->smoother) return fail(SEM_ERR_INVALID_ARG, "the learned multigrid forms need opts.smoother");
        if (m.N != 7) return fail(SEM_ERR_UNSUPPORTED, "the learned smoother needs order N = 7");
        if (!m.hsmg) return fail(SEM_ERR_INVALID_ARG, "this form needs a mesh created with SEM_PREP_HSMG");
        if (!(o->h1 > 0.0)) return fail(SEM_ERR_INVALID_ARG, "the multigrid forms need h1 > 0");
        if (o->h2 < 0.0) return fail(SEM_ERR_INVALID_ARG, "h2 must be >= 0");
        if (o->restart < 0 || o->restart > kGmresMaxRestart)
            return fail(SEM_ERR_INVALID_ARG, "restart must be in 0.." + std::to_string(kGmresMaxRestart));
        return SEM_OK;
    default:
        return fail(SEM_ERR_UNSUPPORTED, "solver form " + std::to_string(o->form) + " not available");
    }
}

sem_status read_state(CgState &h, const CgState *d, hipStream_t s)
{
    SEM_HIP_TRY(hipMemcpyAsync(&h, d, sizeof(CgState), hipMemcpyDeviceToHost, s));
    SEM_HIP_TRY(hipStreamSynchronize(s));
    return SEM_OK;
}

sem_status reset_state(CgState *d, int max_it, int hist_len, hipStream_t s)
{
    CgState init{};
    init.max_it = max_it;
    init.hist_len = hist_len;
    SEM_HIP_TRY(hipMemcpyAsync(d, &init, sizeof(CgState), hipMemcpyHostToDevice, s));
    return SEM_OK;
}

// Low-precision operators of the float solves.
enum LowOp { kOpF32 = 0, kOpBf16 = 1, kOpBf16Split = 2 };

// Iterate until the device flag says done; returns the final host state.
// op: the operator of a float solve (FP32, plain BF16 or split BF16).
template <typename T>
sem_status iterate(const Mesh &m, double h1, double h2, const CgVecs<T> &v, CgState *st, double *hist,
                   int check_every, hipStream_t s, CgState &h, int op = kOpF32)
{
    for (;;) {
        SEM_TRY(read_state(h, st, s));
        if (h.done) return SEM_OK;
        for (int q = 0; q < check_every; ++q) {
            if constexpr (sizeof(T) == 8) {
                SEM_HIP_TRY(launch_ax_f64_gather(m, h1, h2, v.p, v.w, v.part_e, s, &st->done));
            } else {
                if (op == kOpBf16)
                    SEM_HIP_TRY(launch_ax_bf16_gather(m, (float)h1, (float)h2, v.p, v.w, v.part_e, s, &st->done));
                else if (op == kOpBf16Split)
                    SEM_HIP_TRY(launch_ax_bf16s(m, (float)h1, (float)h2, v.p, v.w, v.part_e, s, &st->done, true));
                else
                    SEM_HIP_TRY(launch_ax_f32_gather(m, (float)h1, (float)h2, v.p, v.w, v.part_e, s, &st->done));
            }
            SEM_HIP_TRY(cg_step_after_ax<T>(m, v, st, hist, s));
        }
    }
}

// FP64 true residual of the assembled x: v.r = b - S x, returns (r, r) in h.true_rr
sem_status true_residual(const Mesh &m, double h1, double h2, const Workspace &ws, hipStream_t s, CgState &h)
{
    SEM_HIP_TRY(launch_ax_f64_gather(m, h1, h2, ws.v64.x, ws.v64.w, nullptr, s));
    SEM_HIP_TRY(cg_resid<double>(m, ws.v64, ws.b64, ws.v64.r, ws.st64, s));
    return read_state(h, ws.st64, s);
}

sem_status solve_pcg64(const Mesh &m, const sem_solve_opts &o, const Workspace &ws, int hist_len, hipStream_t s,
                       int check_every, sem_solve_report *rep, CgState &h)
{
    SEM_TRY(reset_state(ws.st64, o.max_iter, hist_len, s));
    SEM_HIP_TRY(cg_init<double>(m, ws.v64, ws.b64, ws.st64, o.rel_tol, ws.hist, s));
    int restarts = 0;
    for (;;) {
        SEM_TRY(iterate<double>(m, o.h1, o.h2, ws.v64, ws.st64, ws.hist, check_every, s, h));
        if (h.done != 1 || h.bb == 0.0) break;
        SEM_TRY(true_residual(m, o.h1, o.h2, ws, s, h));
        if (h.true_rr <= h.tol2 || restarts == 3 || h.it >= h.max_it) break;
        ++restarts;   // recursive residual drifted: restart CG from x
        SEM_HIP_TRY(cg_restart<double>(m, ws.v64, ws.st64, s));
    }
    if (h.done != 1 && h.bb > 0.0) SEM_TRY(true_residual(m, o.h1, o.h2, ws, s, h));
    rep->iterations = h.it;
    rep->restarts = restarts;
    return SEM_OK;
}

// Single-reduction Jacobi-PCG (Chronopoulos & Gear 1989; a
// communication-reducing CG): per iteration one vector pass, the operator on
// u = dinv r, and one finalize that forms alpha and beta from the three inner
// products of the same reduction phase.  Same convergence test and
// true-residual restarts as solve_pcg64.
sem_status solve_pcg1(const Mesh &m, const sem_solve_opts &o, const Workspace &ws, int hist_len, hipStream_t s,
                      int check_every, sem_solve_report *rep, CgState &h)
{
    double *u = ws.z, *sv = ws.q;
    SEM_TRY(reset_state(ws.st64, o.max_iter, hist_len, s));
    SEM_HIP_TRY(cg1_init(m, ws.v64, ws.b64, u, sv, 0, s));
    SEM_HIP_TRY(launch_ax_f64_gather(m, o.h1, o.h2, u, ws.v64.w, ws.v64.part_e, s));
    SEM_HIP_TRY(cg1_finalize(m, ws.v64, ws.st64, 1, 1, o.rel_tol, ws.hist, s));
    int restarts = 0;
    for (;;) {
        for (;;) {
            SEM_TRY(read_state(h, ws.st64, s));
            if (h.done) break;
            for (int q = 0; q < check_every; ++q) {
                SEM_HIP_TRY(cg1_vec(m, ws.v64, u, sv, ws.st64, s));
                SEM_HIP_TRY(launch_ax_f64_gather(m, o.h1, o.h2, u, ws.v64.w, ws.v64.part_e, s, &ws.st64->done));
                SEM_HIP_TRY(cg1_finalize(m, ws.v64, ws.st64, 0, 0, o.rel_tol, ws.hist, s));
            }
        }
        if (h.done != 1 || h.bb == 0.0) break;
        SEM_TRY(true_residual(m, o.h1, o.h2, ws, s, h));
        if (h.true_rr <= h.tol2 || restarts == 3 || h.it >= h.max_it) break;
        ++restarts;   // recursive residual drifted: restart from x with the true residual
        SEM_HIP_TRY(cg1_init(m, ws.v64, ws.b64, u, sv, 1, s));
        SEM_HIP_TRY(launch_ax_f64_gather(m, o.h1, o.h2, u, ws.v64.w, ws.v64.part_e, s));
        SEM_HIP_TRY(cg1_finalize(m, ws.v64, ws.st64, 1, 0, o.rel_tol, ws.hist, s));
    }
    if (h.done != 1 && h.bb > 0.0) SEM_TRY(true_residual(m, o.h1, o.h2, ws, s, h));
    rep->iterations = h.it;
    rep->restarts = restarts;
    return SEM_OK;
}

sem_status solve_dc32(const Mesh &m, const sem_solve_opts &o, const Workspace &ws, int hist_len, hipStream_t s,
                      int check_every, sem_solve_report *rep, CgState &h)
{
    // (b, b) and tol2 through the FP64 init (x = 0, r = b)
    SEM_TRY(reset_state(ws.st64, o.max_iter, hist_len, s));
    SEM_HIP_TRY(cg_init<double>(m, ws.v64, ws.b64, ws.st64, o.rel_tol, ws.hist, s));
    SEM_TRY(read_state(h, ws.st64, s));
    if (h.bb == 0.0) return SEM_OK;
    CgState hi{};
    int total = 0, outer = 0;
    double prev = h.bb;
    h.true_rr = h.bb;
    h.done = 0;
    while (outer < o.max_outer) {
        if (outer > 0) {
            SEM_TRY(true_residual(m, o.h1, o.h2, ws, s, h));
            if (h.true_rr <= h.tol2) { h.done = 1; break; }
            if (!std::isfinite(h.true_rr)) { h.done = 2; break; }
            if (!(h.true_rr < prev)) { h.done = kDoneStalled; break; }   // refinement stalled
            prev = h.true_rr;
        } else {
            // first outer step: r = b, already in v64.r
        }
        if (total >= o.max_iter) { h.done = 3; break; }
        const double rn = std::sqrt(h.true_rr);
        SEM_HIP_TRY(cg_scale<float>(m, ws.v64.r, ws.b32, 1.0 / rn, s));
        SEM_TRY(reset_state(ws.st32, o.max_iter - total, 0, s));
        SEM_HIP_TRY(cg_init<float>(m, ws.v32, ws.b32, ws.st32, o.inner_tol, nullptr, s));
        SEM_TRY(iterate<float>(m, o.h1, o.h2, ws.v32, ws.st32, nullptr, check_every, s, hi,
                               o.form == SEM_FORM_DC_BF16 ? kOpBf16Split : kOpF32));
        total += hi.it;
        SEM_HIP_TRY(cg_axpy<float>(m, ws.v64.x, ws.v32.x, rn, s));
        ++outer;
    }
    if (h.done == 0) {
        SEM_TRY(true_residual(m, o.h1, o.h2, ws, s, h));
        h.done = h.true_rr <= h.tol2 ? 1 : 3;
    }
    h.rr = h.true_rr;
    h.it = total;
    rep->iterations = total;
    rep->outer_iterations = outer;
    return SEM_OK;
}

// Low-precision CG with reliable updates (residual replacement after
// Sleijpen & van der Vorst 1996 and van der Vorst & Ye 2000): the Krylov
// recursion runs with FP32 vectors and the FP32 or split-BF16 operator on a
// residual scaled to unit norm; the solution is accumulated in FP64.
// Whenever the low-precision residual has fallen by delta = inner_tol below
// its largest value since the last replacement (or meets the tolerance), the
// host queues x64 += sigma x32, the FP64 true residual r64 = b - S x64, and
// restarts the low-precision residual from r64 / |r64| while the search
// direction is kept (rescaled, its dinv r part swapped for the new
// residual's), so the Krylov process is not restarted.
sem_status solve_reliable(const Mesh &m, const sem_solve_opts &o, const Workspace &ws, int hist_len, hipStream_t s,
                          int check_every, sem_solve_report *rep, CgState &h)
{
    const bool bf16 = o.form == SEM_FORM_RELIABLE_BF16;
    SEM_TRY(reset_state(ws.st64, o.max_iter, hist_len, s));
    SEM_HIP_TRY(cg_init<double>(m, ws.v64, ws.b64, ws.st64, o.rel_tol, nullptr, s));
    SEM_TRY(read_state(h, ws.st64, s));
    if (h.bb == 0.0) return SEM_OK;
    h.true_rr = h.bb;
    SEM_TRY(reset_state(ws.st32, o.max_iter, 0, s));
    double sigma = std::sqrt(h.bb);
    SEM_HIP_TRY(cg_replace<float>(m, ws.v32, ws.v64.r, ws.st32, 1.0 / sigma, 0.0, kReplaceFirst, h.tol2 / h.bb, s));
    const double delta2 = o.inner_tol * o.inner_tol;
    double rmax = 1.0, best = h.bb;
    int updates = 0, stalls = 0;
    CgState lo{};
    for (;;) {
        SEM_TRY(read_state(lo, ws.st32, s));
        if (lo.done >= 2) {
            h.done = lo.done;
            // iteration cap: x64 takes the last iterate; after a breakdown the
            // low-precision solution may be non-finite and is dropped
            if (lo.done == 3) SEM_HIP_TRY(cg_axpy<float>(m, ws.v64.x, ws.v32.x, sigma, s));
            break;
        }
        rmax = std::max(rmax, lo.rr);
        if (lo.done == 1 || lo.rr < delta2 * rmax) {
            // reliable update: fold the low-precision solution into x64 and
            // replace the residual by the FP64 true residual
            SEM_HIP_TRY(cg_axpy<float>(m, ws.v64.x, ws.v32.x, sigma, s));
            SEM_TRY(true_residual(m, o.h1, o.h2, ws, s, h));
            ++updates;
            if (h.true_rr <= h.tol2) { h.done = 1; break; }
            if (!std::isfinite(h.true_rr)) { h.done = 2; break; }
            if (h.true_rr < best) {
                best = h.true_rr;
                stalls = 0;
            } else if (++stalls >= 3) {
                h.done = kDoneStalled;   // the true residual stopped decreasing
                break;
            }
            if (lo.it >= o.max_iter) { h.done = 3; break; }
            const double sn = std::sqrt(h.true_rr);
            // after a converged low-precision run the last direction update
            // was skipped, so the direction restarts from dinv r
            const int mode = lo.done == 1 ? kReplaceRestart : kReplaceKeep;
            SEM_HIP_TRY(cg_replace<float>(m, ws.v32, ws.v64.r, ws.st32, 1.0 / sn, sigma / sn, mode, h.tol2 / h.true_rr, s));
            sigma = sn;
            rmax = 1.0;
        }
        for (int q = 0; q < check_every; ++q) {
            if (bf16)
                SEM_HIP_TRY(launch_ax_bf16s(m, (float)o.h1, (float)o.h2, ws.v32.p, ws.v32.w, ws.v32.part_e, s,
                                            &ws.st32->done, true));
            else
                SEM_HIP_TRY(launch_ax_f32_gather(m, (float)o.h1, (float)o.h2, ws.v32.p, ws.v32.w, ws.v32.part_e, s,
                                                 &ws.st32->done));
            SEM_HIP_TRY(cg_step_after_ax<float>(m, ws.v32, ws.st32, nullptr, s));
        }
    }
    if (h.done != 1) {
        // report the FP64 true residual of what x64 holds
        SEM_TRY(true_residual(m, o.h1, o.h2, ws, s, h));
    }
    h.rr = h.true_rr;
    h.it = lo.it;
    rep->iterations = lo.it;
    rep->outer_iterations = updates;
    return SEM_OK;
}

}  // namespace
}  // namespace sem

using namespace sem;

extern "C" {

sem_status sem_ax(const sem_mesh *mesh, double h1, double h2, sem_dtype in, const void *u, void *w,
                  void *stream)
{
    if (!mesh || !u || !w) return fail(SEM_ERR_INVALID_ARG, "null mesh, u or w");
    const Mesh &m = mesh->m;
    hipStream_t s = (hipStream_t)stream;
    switch (in) {
    case SEM_F64:
        SEM_HIP_TRY(launch_ax_f64(m, h1, h2, (const double *)u, (double *)w, nullptr, s));
        return SEM_OK;
    case SEM_F32:
        if (!m.d_G32) return fail(SEM_ERR_INVALID_ARG, "mesh was created without SEM_PREP_F32");
        SEM_HIP_TRY(launch_ax_f32(m, (float)h1, (float)h2, (const float *)u, (float *)w, nullptr, s));
        return SEM_OK;
    case SEM_BF16:
        if (!m.d_Gbf) return fail(SEM_ERR_INVALID_ARG, "mesh was created without SEM_PREP_BF16");
        if (m.N != 7) return fail(SEM_ERR_UNSUPPORTED, "the bf16 operator needs order N = 7");
        SEM_HIP_TRY(launch_ax_bf16(m, (float)h1, (float)h2, (const uint16_t *)u, (float *)w, s));
        return SEM_OK;
    case SEM_BF16_SPLIT:
        if (!m.d_Gbf) return fail(SEM_ERR_INVALID_ARG, "mesh was created without SEM_PREP_BF16");
        if (m.N != 7) return fail(SEM_ERR_UNSUPPORTED, "the bf16 operator needs order N = 7");
        SEM_HIP_TRY(launch_ax_bf16s(m, (float)h1, (float)h2, (const float *)u, (float *)w, nullptr, s, nullptr, false));
        return SEM_OK;
    default:
        return fail(SEM_ERR_INVALID_ARG, "unknown dtype");
    }
}

sem_status sem_dssum(const sem_mesh *mesh, sem_dtype dt, void *u, int apply_mask, void *stream)
{
    if (!mesh || !u) return fail(SEM_ERR_INVALID_ARG, "null mesh or u");
    hipStream_t s = (hipStream_t)stream;
    if (dt == SEM_F64) {
        SEM_HIP_TRY(launch_dssum_f64(mesh->m, (double *)u, apply_mask, s));
        return SEM_OK;
    }
    if (dt == SEM_F32) {
        SEM_HIP_TRY(launch_dssum_f32(mesh->m, (float *)u, apply_mask, s));
        return SEM_OK;
    }
    return fail(SEM_ERR_INVALID_ARG, "dssum supports SEM_F64 and SEM_F32");
}

sem_status sem_rhs(const sem_mesh *mesh, const double *f, double *b, void *stream)
{
    if (!mesh || !f || !b) return fail(SEM_ERR_INVALID_ARG, "null mesh, f or b");
    hipStream_t s = (hipStream_t)stream;
    SEM_HIP_TRY(launch_scale_by_B(mesh->m, f, b, s));
    SEM_HIP_TRY(launch_dssum_f64(mesh->m, b, 1, s));
    return SEM_OK;
}

sem_status sem_jacobi(const sem_mesh *mesh, double h1, double h2, double *dinv, void *stream)
{
    if (!mesh || !dinv) return fail(SEM_ERR_INVALID_ARG, "null mesh or dinv");
    hipStream_t s = (hipStream_t)stream;
    SEM_HIP_TRY(launch_diag(mesh->m, h1, h2, dinv, s));
    SEM_HIP_TRY(launch_dssum_f64(mesh->m, dinv, 0, s));
    SEM_HIP_TRY(launch_jacobi_finish(mesh->m, dinv, s));
    return SEM_OK;
}

sem_status sem_dot(const sem_mesh *mesh, const double *u, const double *v, double *result, void *stream)
{
    if (!mesh || !u || !v || !result) return fail(SEM_ERR_INVALID_ARG, "null argument");
    const Mesh &m = mesh->m;
    SEM_HIP_TRY(launch_dot(m, u, v, m.d_scratch, m.scratch_len - 1, result, (hipStream_t)stream));
    return SEM_OK;
}

sem_status sem_solve_workspace_bytes(const sem_mesh *mesh, const sem_solve_opts *opts, size_t *bytes)
{
    if (!mesh || !bytes) return fail(SEM_ERR_INVALID_ARG, "null mesh or bytes");
    SEM_TRY(check_opts(mesh->m, opts));
    *bytes = carve(mesh->m, *opts, hist_len_for(*opts), nullptr).bytes;
    return SEM_OK;
}

sem_status sem_pcg_solve(const sem_mesh *mesh, const sem_solve_opts *opts, const double *b, double *x,
                         void *workspace, size_t ws_bytes, sem_solve_report *rep, void *stream)
{
    const auto t0 = std::chrono::steady_clock::now();
    if (!mesh || !b || !x || !workspace || !rep) return fail(SEM_ERR_INVALID_ARG, "null argument");
    const Mesh &m = mesh->m;
    SEM_TRY(check_opts(m, opts));
    std::memset(rep, 0, sizeof(*rep));
    const int hist_len = hist_len_for(*opts);
    Workspace ws = carve(m, *opts, hist_len, (char *)workspace);
    if (ws_bytes < ws.bytes)
        return fail(SEM_ERR_INVALID_ARG, "workspace too small: need " + std::to_string(ws.bytes) + " bytes");
    hipStream_t s = (hipStream_t)stream;
    const int check_every = std::max(1, opts->check_every > 0 ? opts->check_every : 16);

    // preconditioner (0 on Dirichlet nodes) and the assembled right-hand side
    SEM_HIP_TRY(launch_diag(m, opts->h1, opts->h2, ws.v64.w, s));
    SEM_HIP_TRY(cg_dinv<double>(m, ws.v64.w, ws.v64.dinv, s));
    if (uses_f32(opts->form)) SEM_HIP_TRY(cg_dinv<float>(m, ws.v64.w, ws.v32.dinv, s));
    SEM_HIP_TRY(cg_gather<double>(m, b, ws.b64, s));

    CgState h{};
    if (opts->form == SEM_FORM_DC_FP32 || opts->form == SEM_FORM_DC_BF16)
        SEM_TRY(solve_dc32(m, *opts, ws, hist_len, s, check_every, rep, h));
    else if (opts->form == SEM_FORM_FCG_INNER_FP32 || opts->form == SEM_FORM_FCG_INNER_BF16)
        SEM_TRY(solve_fcg_nested(m, *opts, ws.v64, ws.v32, ws.b32, ws.b64, ws.z, ws.q, ws.st64, ws.st32, ws.hist,
                                 hist_len, std::max(1, std::min(check_every, 4)),
                                 opts->form == SEM_FORM_FCG_INNER_BF16, s, rep, h));
    else if (opts->form == SEM_FORM_PCG_1RED)
        SEM_TRY(solve_pcg1(m, *opts, ws, hist_len, s, check_every, rep, h));
    else if (opts->form == SEM_FORM_RELIABLE_FP32 || opts->form == SEM_FORM_RELIABLE_BF16)
        SEM_TRY(solve_reliable(m, *opts, ws, hist_len, s, check_every, rep, h));
    else if (opts->form == SEM_FORM_GMRES_HSMG)
        SEM_TRY(solve_gmres_hsmg(m, *opts, ws.v64, ws.b64, ws.st64, ws.gm, s, rep, h));
    else if (opts->form == SEM_FORM_GMRES_LEARNED_MG) {
        const Smoother &sm = opts->smoother->s;
        SEM_TRY(check_pair(sm, m));
        const FineHook hook{&sm, ws.v64.dinv, sm.c_local, 0};
        SEM_TRY(solve_gmres_hsmg(m, *opts, ws.v64, ws.b64, ws.st64, ws.gm, s, rep, h, &hook));
    }
    else if (opts->form == SEM_FORM_PCG_BLOCK_JACOBI || opts->form == SEM_FORM_PCG_HSMG)
        SEM_TRY(solve_pcg_precond(m, *opts, ws.v64, ws.b64, ws.z, ws.st64, ws.hb,
                                  opts->form == SEM_FORM_PCG_HSMG ? 3 : 1, ws.hist, hist_len, check_every, s, rep, h));
    else if (opts->form == SEM_FORM_FCG_LEARNED)
        SEM_TRY(solve_fcg(m, opts->smoother->s, *opts, ws.v64, ws.b64, ws.z, ws.q, ws.st64, ws.hist, hist_len,
                          check_every, s, rep, h));
    else if (opts->form == SEM_FORM_FCG_LEARNED_MG)
        SEM_TRY(solve_fcg(m, opts->smoother->s, *opts, ws.v64, ws.b64, ws.z, ws.q, ws.st64, ws.hist, hist_len,
                          check_every, s, rep, h, &ws.hb));
    else
        SEM_TRY(solve_pcg64(m, *opts, ws, hist_len, s, check_every, rep, h));
    SEM_HIP_TRY(cg_scatter<double>(m, ws.v64.x, x, s));

    rep->rel_res = h.bb > 0 ? std::sqrt(h.rr / h.bb) : 0.0;
    rep->true_rel_res = h.bb > 0 ? std::sqrt(h.true_rr / h.bb) : 0.0;
    if (opts->history && opts->history_len > 0 &&
        (opts->form == SEM_FORM_JACOBI_PCG || opts->form == SEM_FORM_PCG_1RED || opts->form == SEM_FORM_PCG_BLOCK_JACOBI ||
         opts->form == SEM_FORM_PCG_HSMG || uses_fcg(opts->form))) {
        const int n = std::min(opts->history_len, std::min(h.it + 1, hist_len));
        SEM_HIP_TRY(hipMemcpyAsync(opts->history, ws.hist, sizeof(double) * n, hipMemcpyDeviceToHost, s));
        SEM_HIP_TRY(hipStreamSynchronize(s));
        rep->history_written = n;
    } else {
        SEM_HIP_TRY(hipStreamSynchronize(s));
    }
    const auto t1 = std::chrono::steady_clock::now();
    rep->elapsed_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
    if (h.done == 2) {
        rep->status = SEM_ERR_BREAKDOWN;
        return fail(SEM_ERR_BREAKDOWN, "CG breakdown: (p, S p) <= 0 or a non-finite value");
    }
    if (h.done == kDoneStalled) {
        rep->status = SEM_ERR_NOT_CONVERGED;
        return fail(SEM_ERR_NOT_CONVERGED, "refinement stalled: the FP64 true residual stopped decreasing at " +
                                               std::to_string(rep->true_rel_res) + " relative");
    }
    if (h.bb > 0.0 && !(h.true_rr <= h.tol2)) {
        rep->status = SEM_ERR_NOT_CONVERGED;
        return fail(SEM_ERR_NOT_CONVERGED, "relative residual above rel_tol after " +
                                               std::to_string(rep->iterations) + " iterations");
    }
    rep->status = SEM_OK;
    return SEM_OK;
}

sem_status sem_pcg_snapshots(const sem_mesh *mesh, const sem_solve_opts *opts, const double *b, const int32_t *iters,
                             int32_t n_iters, double *e_out, void *workspace, size_t ws_bytes, sem_solve_report *rep,
                             void *stream)
{
    if (!mesh || !opts || !b || !workspace || !rep || (n_iters > 0 && (!iters || !e_out)))
        return fail(SEM_ERR_INVALID_ARG, "null argument");
    const Mesh &m = mesh->m;
    sem_solve_opts o = *opts;
    o.form = SEM_FORM_JACOBI_PCG;
    SEM_TRY(check_opts(m, &o));
    for (int q = 0; q < n_iters; ++q)
        if (iters[q] < 0 || (q > 0 && iters[q] < iters[q - 1]))
            return fail(SEM_ERR_INVALID_ARG, "iters must be non-negative and ascending");
    std::memset(rep, 0, sizeof(*rep));
    const int hist_len = hist_len_for(o);
    Workspace ws = carve(m, o, hist_len, (char *)workspace);
    if (ws_bytes < ws.bytes)
        return fail(SEM_ERR_INVALID_ARG, "workspace too small: need " + std::to_string(ws.bytes) + " bytes");
    hipStream_t s = (hipStream_t)stream;
    const int check_every = std::max(1, o.check_every > 0 ? o.check_every : 16);
    SEM_HIP_TRY(launch_diag(m, o.h1, o.h2, ws.v64.w, s));
    SEM_HIP_TRY(cg_dinv<double>(m, ws.v64.w, ws.v64.dinv, s));
    SEM_HIP_TRY(cg_gather<double>(m, b, ws.b64, s));
    SEM_TRY(reset_state(ws.st64, o.max_iter, hist_len, s));
    SEM_HIP_TRY(cg_init<double>(m, ws.v64, ws.b64, ws.st64, o.rel_tol, ws.hist, s));
    CgState h{};
    for (int q = 0; q < n_iters; ++q) {
        // advance exactly to iteration iters[q] (or to convergence)
        for (;;) {
            SEM_TRY(read_state(h, ws.st64, s));
            if (h.done || h.it >= iters[q]) break;
            const int n = std::min(check_every, iters[q] - h.it);
            for (int k = 0; k < n; ++k) {
                SEM_HIP_TRY(launch_ax_f64_gather(m, o.h1, o.h2, ws.v64.p, ws.v64.w, ws.v64.part_e, s, &ws.st64->done));
                SEM_HIP_TRY(cg_step_after_ax<double>(m, ws.v64, ws.st64, ws.hist, s));
            }
        }
        SEM_HIP_TRY(hipMemcpyAsync(e_out + (size_t)q * m.ng, ws.v64.x, (size_t)m.ng * 8, hipMemcpyDeviceToDevice, s));
    }
    SEM_TRY(iterate<double>(m, o.h1, o.h2, ws.v64, ws.st64, ws.hist, check_every, s, h));
    for (int q = 0; q < n_iters; ++q) SEM_HIP_TRY(cg_rsub(m, ws.v64.x, e_out + (size_t)q * m.ng, s));
    if (h.bb > 0.0) SEM_TRY(true_residual(m, o.h1, o.h2, ws, s, h));
    rep->iterations = h.it;
    rep->rel_res = h.bb > 0 ? std::sqrt(h.rr / h.bb) : 0.0;
    rep->true_rel_res = h.bb > 0 ? std::sqrt(h.true_rr / h.bb) : 0.0;
    rep->status = (h.bb == 0.0 || h.true_rr <= h.tol2) ? SEM_OK : SEM_ERR_NOT_CONVERGED;
    SEM_HIP_TRY(hipStreamSynchronize(s));
    if (rep->status != SEM_OK) return fail((sem_status)rep->status, "snapshot solve did not converge");
    return SEM_OK;
}


static Workspace carve_batched(const Mesh &m, int nrhs, int form, char *base, std::vector<CgVecs<double>> &vc,
                               CgState **states, double **b64)
{
    Workspace ws{};
    size_t off = 0;
    auto take = [&](size_t bytes) -> char * {
        char *p = base ? base + off : nullptr;
        off += align256(bytes);
        return p;
    };
    const size_t nl = (size_t)m.nl, ng = (size_t)m.ng;
    double *X = (double *)take(nrhs * ng * 8), *R = (double *)take(nrhs * ng * 8), *Pp = (double *)take(nrhs * ng * 8);
    double *dinv = (double *)take(ng * 8);
    *b64 = (double *)take(nrhs * ng * 8);
    double *W = (double *)take(nrhs * nl * 8);
    double *PE = (double *)take((size_t)nrhs * std::max<int64_t>(m.E, 1) * 8);
    double *PB = (double *)take((size_t)part_capacity(m.lat, m.E) * 3 * 8);
    double *ST = (double *)take((size_t)kStage * 3 * 8);
    *states = (CgState *)take(sizeof(CgState) * nrhs);
    if (form == SEM_FORM_PCG_BLOCK_JACOBI && m.hsmg) {
        // block-Jacobi: one z per field and one set of preconditioner buffers
        ws.z = (double *)take(nrhs * ng * 8);
        char *hbase = take(hsmg_bufs_bytes(m));
        if (base) ws.hb = hsmg_bufs_carve(m, hbase);
    }
    vc.resize(nrhs);
    for (int c = 0; c < nrhs; ++c) {
        vc[c].x = X + c * ng;
        vc[c].r = R + c * ng;
        vc[c].p = Pp + c * ng;
        vc[c].dinv = dinv;
        vc[c].w = W + c * nl;
        vc[c].part_e = PE + c * m.E;
        vc[c].part_b = PB;
        vc[c].stage = ST;
    }
    ws.bytes = off;
    return ws;
}

sem_status sem_solve_workspace_bytes_batched(const sem_mesh *mesh, const sem_solve_opts *opts, int32_t nrhs,
                                             size_t *bytes)
{
    if (!mesh || !bytes || !opts) return fail(SEM_ERR_INVALID_ARG, "null argument");
    if (nrhs < 1 || nrhs > 4) return fail(SEM_ERR_INVALID_ARG, "nrhs must be in 1..4");
    std::vector<CgVecs<double>> vc;
    CgState *st;
    double *b64;
    *bytes = carve_batched(mesh->m, nrhs, opts->form, nullptr, vc, &st, &b64).bytes;
    return SEM_OK;
}

sem_status sem_pcg_solve_batched(const sem_mesh *mesh, const sem_solve_opts *opts, int32_t nrhs, const double *b,
                                 double *x, void *workspace, size_t ws_bytes, sem_solve_report *reps, void *stream)
{
    const auto t0 = std::chrono::steady_clock::now();
    if (!mesh || !opts || !b || !x || !workspace || !reps) return fail(SEM_ERR_INVALID_ARG, "null argument");
    if (nrhs < 1 || nrhs > 4) return fail(SEM_ERR_INVALID_ARG, "nrhs must be in 1..4");
    const Mesh &m = mesh->m;
    if (m.N != 7) return fail(SEM_ERR_UNSUPPORTED, "batched solves need order N = 7");
    if (opts->form != SEM_FORM_JACOBI_PCG && opts->form != SEM_FORM_PCG_BLOCK_JACOBI)
        return fail(SEM_ERR_UNSUPPORTED, "batched solves use SEM_FORM_JACOBI_PCG or SEM_FORM_PCG_BLOCK_JACOBI");
    SEM_TRY(check_opts(m, opts));
    std::vector<CgVecs<double>> vc;
    CgState *st;
    double *b64;
    Workspace ws = carve_batched(m, nrhs, opts->form, (char *)workspace, vc, &st, &b64);
    if (ws_bytes < ws.bytes)
        return fail(SEM_ERR_INVALID_ARG, "workspace too small: need " + std::to_string(ws.bytes) + " bytes");
    hipStream_t s = (hipStream_t)stream;
    const int check_every = std::max(1, opts->check_every > 0 ? opts->check_every : 16);
    const sem_solve_opts &o = *opts;
    SEM_HIP_TRY(launch_diag(m, o.h1, o.h2, vc[0].w, s));
    SEM_HIP_TRY(cg_dinv<double>(m, vc[0].w, vc[0].dinv, s));
    if (o.form == SEM_FORM_PCG_BLOCK_JACOBI) {
        // the velocity solves' method: CG with the element block-Jacobi
        // preconditioner, the operator batched over the fields
        for (int c = 0; c < nrhs; ++c)
            SEM_HIP_TRY(cg_gather<double>(m, b + (size_t)c * m.nl, b64 + (size_t)c * m.ng, s));
        std::vector<CgState> hb(nrhs);
        std::vector<sem_solve_report> rb(nrhs);
        for (auto &r : rb) std::memset(&r, 0, sizeof(r));
        SEM_TRY(solve_pcg_precond_batched(m, o, nrhs, vc.data(), b64, ws.z, st, ws.hb, 1, check_every, s, rb.data(),
                                          hb.data()));
        sem_status worst = SEM_OK;
        for (int c = 0; c < nrhs; ++c) {
            SEM_HIP_TRY(cg_scatter<double>(m, vc[c].x, x + (size_t)c * m.nl, s));
            const CgState &hc = hb[c];
            sem_solve_report &r = reps[c];
            r = rb[c];
            r.rel_res = hc.bb > 0 ? std::sqrt(hc.rr / hc.bb) : 0.0;
            r.true_rel_res = hc.bb > 0 ? std::sqrt(hc.true_rr / hc.bb) : 0.0;
            r.status = hc.done == 2 ? SEM_ERR_BREAKDOWN
                                    : ((hc.bb > 0.0 && !(hc.true_rr <= hc.tol2)) ? SEM_ERR_NOT_CONVERGED : SEM_OK);
            if (r.status != SEM_OK && worst == SEM_OK) worst = (sem_status)r.status;
        }
        SEM_HIP_TRY(hipStreamSynchronize(s));
        const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        for (int c = 0; c < nrhs; ++c) reps[c].elapsed_ms = ms;
        if (worst != SEM_OK) return fail(worst, "a batched field did not converge");
        return SEM_OK;
    }
    for (int c = 0; c < nrhs; ++c) {
        SEM_HIP_TRY(cg_gather<double>(m, b + (size_t)c * m.nl, b64 + (size_t)c * m.ng, s));
        SEM_TRY(reset_state(st + c, o.max_iter, 0, s));
        SEM_HIP_TRY(cg_init<double>(m, vc[c], b64 + (size_t)c * m.ng, st + c, o.rel_tol, nullptr, s));
    }
    std::vector<CgState> h(nrhs);
    for (;;) {
        bool all = true;
        for (int c = 0; c < nrhs; ++c) {
            SEM_TRY(read_state(h[c], st + c, s));
            all = all && h[c].done != 0;
        }
        if (all) break;
        for (int q = 0; q < check_every; ++q) {
            SEM_HIP_TRY(launch_ax_f64_gather_batched(m, nrhs, o.h1, o.h2, vc[0].p, m.ng, vc[0].w, vc[0].part_e,
                                                     &st->done, (int)(sizeof(CgState) / sizeof(int32_t)), s));
            for (int c = 0; c < nrhs; ++c) SEM_HIP_TRY(cg_step_after_ax<double>(m, vc[c], st + c, nullptr, s));
        }
    }
    // FP64 true residual per field; a drifted field restarts on its own
    sem_status worst = SEM_OK;
    for (int c = 0; c < nrhs; ++c) {
        Workspace one{};
        one.v64 = vc[c];
        one.b64 = b64 + (size_t)c * m.ng;
        one.st64 = st + c;
        int restarts = 0;
        CgState &hc = h[c];
        while (hc.bb > 0.0) {
            SEM_TRY(true_residual(m, o.h1, o.h2, one, s, hc));
            if (hc.true_rr <= hc.tol2 || hc.done != 1 || restarts == 3 || hc.it >= hc.max_it) break;
            ++restarts;
            SEM_HIP_TRY(cg_restart<double>(m, vc[c], st + c, s));
            SEM_TRY(iterate<double>(m, o.h1, o.h2, vc[c], st + c, nullptr, check_every, s, hc));
        }
        SEM_HIP_TRY(cg_scatter<double>(m, vc[c].x, x + (size_t)c * m.nl, s));
        sem_solve_report &r = reps[c];
        std::memset(&r, 0, sizeof(r));
        r.iterations = hc.it;
        r.restarts = restarts;
        r.rel_res = hc.bb > 0 ? std::sqrt(hc.rr / hc.bb) : 0.0;
        r.true_rel_res = hc.bb > 0 ? std::sqrt(hc.true_rr / hc.bb) : 0.0;
        r.status = hc.done == 2 ? SEM_ERR_BREAKDOWN
                                : ((hc.bb > 0.0 && !(hc.true_rr <= hc.tol2)) ? SEM_ERR_NOT_CONVERGED : SEM_OK);
        if (r.status != SEM_OK && worst == SEM_OK) worst = (sem_status)r.status;
    }
    SEM_HIP_TRY(hipStreamSynchronize(s));
    const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    for (int c = 0; c < nrhs; ++c) reps[c].elapsed_ms = ms;
    if (worst != SEM_OK) return fail(worst, "a batched field did not converge");
    return SEM_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Allocation-free solve: the workspace lives in a file-scope device array.
// Each device that loads the library holds its own copy until the process
// ends; the host never passes the array's name to a kernel (in host code it
// is only a stand-in symbol) but the device address that
// hipGetSymbolAddress returns for the current device.

namespace sem {
namespace {

constexpr size_t kNoAllocScratchBytes = SEM_NOALLOC_SCRATCH_BYTES;
static_assert(kNoAllocScratchBytes % 256 == 0, "scratch size");
constexpr int kNoAllocMaxDevices = 64;

static __device__ __align__(256) char scratch[kNoAllocScratchBytes];

std::mutex g_scratch_mutex;
void *g_scratch_ptr[kNoAllocMaxDevices] = {};

// Device address of `scratch` on the current device (looked up once per
// device, with that device current).
sem_status scratch_address(void **out)
{
    int dev = 0;
    SEM_HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kNoAllocMaxDevices) return fail(SEM_ERR_UNSUPPORTED, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        SEM_HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) return fail(SEM_ERR_HIP, "hipGetSymbolAddress returned a null address for the scratch array");
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return SEM_OK;
}

}  // namespace
}  // namespace sem

extern "C" {

sem_status sem_pcg_solve_noalloc(const sem_mesh *mesh, const sem_solve_opts *opts, const double *b, double *x,
                                 sem_solve_report *rep, void *stream)
{
    if (!mesh || !opts || !b || !x || !rep) return fail(SEM_ERR_INVALID_ARG, "null argument");
    const Mesh &m = mesh->m;
    SEM_TRY(check_opts(m, opts));
    int dev = 0;
    SEM_HIP_TRY(hipGetDevice(&dev));
    if (dev != m.device) return fail(SEM_ERR_INVALID_ARG, "the mesh lives on another device than the current one");
    const size_t need = carve(m, *opts, hist_len_for(*opts), nullptr).bytes;
    if (need > kNoAllocScratchBytes)
        return fail(SEM_ERR_INVALID_ARG, "solve needs " + std::to_string(need) + " bytes of workspace, more than the " +
                                             std::to_string(kNoAllocScratchBytes) + "-byte static scratch");
    void *ptr = nullptr;
    SEM_TRY(scratch_address(&ptr));
    return sem_pcg_solve(mesh, opts, b, x, ptr, kNoAllocScratchBytes, rep, stream);
}

}  // extern "C"
