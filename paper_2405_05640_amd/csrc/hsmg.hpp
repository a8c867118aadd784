// hsmg.hpp -- internal interface of the hybrid Schwarz multigrid
// preconditioner and the flexible GMRES solver (the paper's pressure solver,
// section 3.1: restarted GMRES with a hybrid-Schwarz multigrid
// preconditioner; CG with block-Jacobi for the velocity solves).
#pragma once

#include "cg.hpp"
#include "sem_internal.hpp"

namespace sem {

constexpr int kHsmgMidOrder = 3;      // p-multigrid levels N -> 3 -> 1
constexpr int kGmresMaxRestart = 30;  // upper bound on the restart length m

// Device data of the preconditioner (built by SEM_PREP_HSMG).
//  - fdm_f, fdm_m: per element the separable local solver of the fine and
//    mid levels, [E][3 * NP * NP + 3 * NP] doubles: S_x, S_y, S_z (row a =
//    node, column q = mode; B-orthonormal columns) then the eigenvalues
//    l_x, l_y, l_z.  A node on a Dirichlet face has a zero row and its mode
//    slot a zero column with eigenvalue +inf (its inverse is 0).
//  - Jfm [(N+1) x 4], Jmc [4 x 2]: GLL-to-GLL interpolation, row = fine node.
//  - coarse (order 1): per axis S [n x n] and eigenvalues of the global
//    separable operator, same conventions; n = nodes of the order-1 lattice.
struct Hsmg {
    int Nm = kHsmgMidOrder;
    Lattice lat_m{}, lat_c{};     // mid and coarse lattices (closed form, no tables)
    int64_t ng_m = 0, ng_c = 0;
    double *d_fdm_f = nullptr, *d_fdm_m = nullptr;
    double *d_Jfm = nullptr, *d_Jmc = nullptr;
    double *d_cS[3] = {nullptr, nullptr, nullptr};
    double *d_clam[3] = {nullptr, nullptr, nullptr};
    int cn[3] = {0, 0, 0};
    size_t bytes = 0;
    // GMRES stop flags read one iteration behind (pinned host words, two
    // slots) and the events that mark their copies; made at setup so that a
    // solve allocates nothing
    int *h_flag = nullptr;
    hipEvent_t ev[2] = {nullptr, nullptr};
    // side stream (default priority) on which the learned multigrid's
    // coarser levels run beside the network, and its fork / join events
    hipStream_t side = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
};

// host setup from the mesh description (vertices) and the built mesh
sem_status hsmg_setup(const sem_mesh_desc &d, Mesh &m);
void hsmg_release(Mesh &m);

// Work buffers of one preconditioner application.
struct HsmgBufs {
    double *rows_f;   // fine local rows (n_local): Schwarz corrections
    double *rows_m;   // mid local rows (E * 64): restricted residual, then Schwarz corrections
    double *rm;       // mid assembled residual (ng_m)
    double *zm;       // mid assembled correction (ng_m)
    double *rows_c;   // coarse local rows (E * 8)
    double *rc;       // coarse assembled residual (ng_c)
    double *tc;       // coarse scratch (ng_c)
    double *zp;       // fine assembled prolongation of the mid correction (n_global)
};
size_t hsmg_bufs_bytes(const Mesh &m);
HsmgBufs hsmg_bufs_carve(const Mesh &m, char *base);

// Weighting of the Schwarz corrections over node copies: none (sum), the
// average (1/mult after the sum), or symmetric (1/sqrt(mult) on the residual
// before the local solves and on the sum after them).
enum { kWeightNone = 0, kWeightAvg = 1, kWeightSym = 2 };

struct Smoother;

// The learned multigrid's fine level: the learned smoother M(r) = dinv o r
// + mask(Q^T (c / mult)) of the network sm (BF16 inference, or the FP32
// network if fp32), with c_local the element-output buffer and dinv the
// assembled Jacobi inverse (0 on Dirichlet nodes).
struct FineHook {
    const Smoother *sm;
    const double *dinv;
    float *c_local;
    int fp32;
};

// z = M r on assembled fine vectors (z and r distinct; both zero on
// Dirichlet nodes).  levels: 1 = fine Schwarz only, 3 = the full
// three-level cycle; weight applies to the fine and mid levels.  fine (not
// null): the three-level cycle with the learned smoother in place of the
// fine Schwarz level (levels is then ignored).  part_rz (not null, and fine
// null): block partials of (r, z), one per workgroup of the last kernel
// (ceil(ny nz / 4) of them, lattice rows of the fine level).
hipError_t hsmg_apply(const Mesh &m, double h1, double h2, const double *r, double *z, const HsmgBufs &b,
                      int levels, int weight, hipStream_t s, const FineHook *fine = nullptr,
                      double *part_rz = nullptr);

// The mid and coarse levels' part alone: b.zp = P_01 [Sw_1(R_10 r) +
// P_12 C^-1 R_21 R_10 r] (what the cycle adds to its fine level).
hipError_t hsmg_coarse_part(const Mesh &m, double h1, double h2, const double *r, const HsmgBufs &b, int weight,
                            hipStream_t s);
// The same part queued on the mesh's side stream after the work queued so
// far on s (fork), and s made to wait for it (join): the learned
// multigrid's network and coarser levels are independent terms of z.
hipError_t hsmg_coarse_part_fork(const Mesh &m, double h1, double h2, const double *r, const HsmgBufs &b, int weight,
                                 hipStream_t s);
hipError_t hsmg_coarse_part_join(const Mesh &m, hipStream_t s);

// Flexible GMRES work buffers: V [(m+1) ng], Z [m ng], block partials,
// reduction stage, device vectors of inner products and of y.
struct GmresDev;   // device-resident state of one restart cycle
struct GmresBufs {
    double *V, *Z, *part, *stage, *hdev, *h2dev, *ydev;
    GmresDev *gd;
    HsmgBufs hb;
};
size_t gmres_bufs_bytes(const Mesh &m, int mres);
GmresBufs gmres_bufs_carve(const Mesh &m, int mres, char *base);

// Flexible GMRES(m) with the hybrid Schwarz multigrid preconditioner on
// S x = b (assembled b; x from zero).  v: x, r (assembled), w (row-layout
// operator output), dinv, part_b, stage of the caller's workspace; st: a
// device CgState used for the true residual.  Fills h (bb, tol2, rr,
// true_rr, done) and rep (iterations, restarts, history).  fine: the
// learned multigrid in place of the hybrid Schwarz multigrid.
sem_status solve_gmres_hsmg(const Mesh &m, const sem_solve_opts &o, const CgVecs<double> &v, const double *b,
                            CgState *st, const GmresBufs &gb, hipStream_t s, sem_solve_report *rep, CgState &h,
                            const FineHook *fine = nullptr);

// CG with a symmetric positive definite preconditioner: levels = 1 is the
// block-Jacobi one (unweighted element-local separable solves), levels = 3
// the hybrid Schwarz multigrid with symmetric weighting; z: assembled
// scratch vector; same conventions as the FP64 Jacobi-PCG (device scalars,
// host polls every check_every iterations, true-residual restarts).
sem_status solve_pcg_precond(const Mesh &m, const sem_solve_opts &o, const CgVecs<double> &v, const double *b,
                             double *z, CgState *st, const HsmgBufs &hb, int levels, double *hist, int hist_len,
                             int check_every, hipStream_t s, sem_solve_report *rep, CgState &h);
// The same for nrhs fields that share the operator and h1/h2 (fields c at
// v[c], b + c ng, z + c ng, st + c): one batched operator launch per
// iteration, every other step per field; each field then gets its own true
// residual check (and restarts) as in the single-field solve.
sem_status solve_pcg_precond_batched(const Mesh &m, const sem_solve_opts &o, int nrhs, const CgVecs<double> *v,
                                     const double *b, double *z, CgState *st, const HsmgBufs &hb, int levels,
                                     int check_every, hipStream_t s, sem_solve_report *reps, CgState *h);

}  // namespace sem
