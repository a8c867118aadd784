// cg.hpp -- internal interface of the assembled-vector Krylov kernels.
#pragma once
#include <algorithm>
#include <cmath>

#include "sem_internal.hpp"

namespace sem {

constexpr int kBS = 256;             // threads per block of the vector kernels
constexpr int kMaxVecBlocks = 4096;  // grid cap of the flat vector kernels
constexpr int kStage = 256;          // second-stage partial sums

// Grid of the per-node kernels: one workgroup per lattice row (gj, gk).
inline unsigned node_grid(const Lattice &L) { return (unsigned)(L.ny * L.nz); }
// Rows per workgroup of the CG update (a measured choice: the per-workgroup
// prologue is a chain of scalar loads, and FP32 rows carry half the bytes, so
// FP32 takes four rows per workgroup and FP64 two).
template <typename T> constexpr int update_rpb() { return sizeof(T) == 4 ? 4 : 2; }
inline unsigned row_grid(const Lattice &L, int rpb) { return (unsigned)((L.ny * L.nz + rpb - 1) / rpb); }
// Partial-sum capacity per quantity for any kernel of a mesh.
inline int64_t part_capacity(const Lattice &L, int64_t E)
{
    return std::max<int64_t>(std::max<int64_t>(L.ny * L.nz, kMaxVecBlocks), E);
}

// Device-resident scalars of one CG run.
struct CgState {
    double rz, pw, rr, bb, alpha, beta, tol2, true_rr;
    int32_t it, done, status, max_it;
    int32_t hist_len, learned, redo, fallback_at;
    int32_t nn_skip, inner_its, pad1, pad2;
};
// done: 0 running, 1 converged (recursive residual), 2 breakdown, 3 max_iter,
// kDoneStalled: a refinement loop's FP64 true residual stopped decreasing
constexpr int32_t kDoneStalled = 4;
// flexible CG: learned = 1 while the learned smoother is in use, redo = 1 when
// the last smoother output was rejected (p restarts from dinv r),
// fallback_at = iteration of the switch to Jacobi (-1: none), nn_skip =
// done || !learned

// Iterations to queue before the next host poll of a CG run: check_every,
// or fewer once the contraction of the recursive residual observed between
// polls says convergence is nearer.  The kernels of a converged run return
// at once, but a multigrid or network preconditioner queued after
// convergence still runs, so over-queueing there costs whole applications.
struct PollPlan {
    double rr0 = -1.0;
    int it0 = 0;
    int next(const CgState &h, int check_every)
    {
        int n = check_every;
        if (rr0 > 0.0 && h.it > it0 && h.rr > h.tol2 && h.rr < rr0 && h.tol2 > 0.0) {
            const double per_it = std::log(h.rr / rr0) / (double)(h.it - it0);   // < 0
            const double need = std::log(h.tol2 / h.rr) / per_it;                // > 0
            if (need < (double)check_every) n = std::max(1, (int)std::ceil(need));
        }
        rr0 = h.rr;
        it0 = h.it;
        return n;
    }
};

// Vectors of one CG run: x, r, p, dinv are assembled (n_global); w is local
// (n_local, the unassembled operator output); part_e has n_elem entries,
// part_b 3 * part_capacity, stage 3 * kStage.
template <typename T>
struct CgVecs {
    T *x, *r, *p, *dinv, *w;
    double *part_e, *part_b, *stage;
};

// stage[q * kStage + b] = fixed-order sum of chunk b of part[q * n .. q * n + n)
// for q < nv (deterministic first stage of a two-stage reduction).
hipError_t cg_reduce(const double *part, int64_t n, int nv, double *stage, hipStream_t s);

int cg_blocks(int64_t n);

template <typename T> hipError_t cg_gather(const Mesh &m, const double *u, T *ug, hipStream_t s);
template <typename T> hipError_t cg_scatter(const Mesh &m, const T *ug, double *u, hipStream_t s);
template <typename T> hipError_t cg_dinv(const Mesh &m, const double *diag_local, T *dinv, hipStream_t s);
template <typename T>
hipError_t cg_init(const Mesh &m, const CgVecs<T> &v, const T *b, CgState *st, double tol, double *hist, hipStream_t s);
// after the operator has written v.w = A_L p and v.part_e = per-element p.w:
// alpha, update (with assembly), beta / convergence test, p update
template <typename T>
hipError_t cg_step_after_ax(const Mesh &m, const CgVecs<T> &v, CgState *st, double *hist, hipStream_t s);
// r = b - Q^T v.w (Dirichlet nodes 0), st->true_rr = (r, r)
template <typename T>
hipError_t cg_resid(const Mesh &m, const CgVecs<T> &v, const T *b, T *r, CgState *st, hipStream_t s);
template <typename T> hipError_t cg_restart(const Mesh &m, const CgVecs<T> &v, CgState *st, hipStream_t s);
// alpha from the per-element partials of (p, S p) (reduces them first)
// Input of a one-workgroup finalize over nv quantities of n partials each
// (part[q * n + b]): the partials themselves when n <= kDirectMax, else the
// kStage sums of a queued two-stage reduction (then n = kStage).
hipError_t finalize_input(const double *part, int64_t &n, int nv, double *stage, hipStream_t s, const double **in);
hipError_t cg_alpha(const Mesh &m, const double *part_e, double *stage, CgState *st, hipStream_t s);
// e = x - e on assembled vectors
hipError_t cg_rsub(const Mesh &m, const double *x, double *e, hipStream_t s);
// residual replacement of a low-precision run: r = inv_sigma * r64, x = 0;
// p = dinv r (kReplaceFirst, kReplaceRestart) or p_scale * p with its dinv r
// part swapped (kReplaceKeep); st: rr, rz, tol2 (kReplaceFirst also it = 0,
// bb = rr)
enum { kReplaceKeep = 0, kReplaceFirst = 1, kReplaceRestart = 2 };
template <typename T>
hipError_t cg_replace(const Mesh &m, const CgVecs<T> &v, const double *r64, CgState *st, double inv_sigma,
                      double p_scale, int mode, double tol2, hipStream_t s);
// single-reduction (Chronopoulos-Gear) CG on FP64 vectors, u and sv extra
// assembled vectors: init (x = 0 unless keep_x; partials of (r,u), (r,r)
// reduced into v.stage), vector pass (partials reduced into v.stage), and the
// finalize after the operator on u has left its per-element partials in
// v.part_e (first = 1 starts a run; fresh = 1 also sets bb and tol2)
hipError_t cg1_init(const Mesh &m, const CgVecs<double> &v, const double *b, double *u, double *sv, int keep_x,
                    hipStream_t s);
hipError_t cg1_vec(const Mesh &m, const CgVecs<double> &v, double *u, double *sv, CgState *st, hipStream_t s);
hipError_t cg1_finalize(const Mesh &m, const CgVecs<double> &v, CgState *st, int first, int fresh, double tol,
                        double *hist, hipStream_t s);
template <typename T> hipError_t cg_axpy(const Mesh &m, double *y, const T *d, double scale, hipStream_t s);
template <typename T> hipError_t cg_scale(const Mesh &m, const double *in, T *out, double scale, hipStream_t s);

}  // namespace sem
