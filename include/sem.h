/*
 * sem.h -- C ABI of libsem: the spectral-element pressure-solve hot path on
 * one AMD Instinct MI355X (gfx950).
 *
 * The method (paper, section 3.1 "Neko"): the domain is split into E
 * non-overlapping hexahedral elements carrying order-N polynomials on the
 * Gauss-Lobatto-Legendre (GLL) points; operators are applied element by
 * element without assembling a matrix; the elements are coupled only by a
 * unit-depth gather-scatter; each time step solves A x = b with a
 * preconditioned Krylov method.  The spectral-element definitions are the
 * textbook ones the paper cites (Deville, Fischer & Mund 2002).
 *
 * Conventions shared by every entry point
 *  - Meshes are structured boxes of nelx*nely*nelz hexahedra given by their
 *    vertex lattice.  Element e = ex + nelx*(ey + nely*ez).
 *  - A "local" field is a contiguous device array [E][N+1][N+1][N+1] with the
 *    last index (i, the r direction) fastest: one value per element node.
 *    Shared nodes appear once per element that holds them.
 *  - Device pointers are plain HIP device addresses (e.g. torch tensors'
 *    data_ptr()); host pointers are marked HOST.  The library never frees or
 *    reallocates caller memory.  Streams are hipStream_t passed as void*
 *    (NULL = the null stream).  Calls marked "async" only enqueue work.
 *  - Every function returns a sem_status and never throws; on failure
 *    sem_last_error() describes the problem (thread-local string, valid until
 *    the next call on the same thread).
 *  - The library allocates device memory only in sem_mesh_create and
 *    sem_smoother_create; hot calls allocate nothing.  Concurrent calls on one
 *    mesh are safe when their output buffers and workspaces are distinct
 *    (exceptions: sem_dot; the smoother's apply, loss and training calls
 *    share the smoother's buffers).
 */
#ifndef SEM_H
#define SEM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SEM_OK = 0,
    SEM_ERR_INVALID_ARG = 1,   /* null pointer, bad size/dtype/order, inverted element */
    SEM_ERR_OUT_OF_MEMORY = 2, /* device or host allocation failed */
    SEM_ERR_HIP = 3,           /* a HIP runtime call failed */
    SEM_ERR_NOT_CONVERGED = 4, /* max_iter reached, or a refinement form's FP64 true residual
                                  stopped decreasing; x holds the last iterate */
    SEM_ERR_BREAKDOWN = 5,     /* non-finite value or (p, S p) <= 0 in CG */
    SEM_ERR_UNSUPPORTED = 6    /* valid request the library does not provide */
} sem_status;

typedef enum { SEM_F64 = 0, SEM_F32 = 1, SEM_BF16 = 2, SEM_BF16_SPLIT = 3 } sem_dtype;

typedef struct sem_mesh sem_mesh;           /* opaque, immutable after create */
typedef struct sem_smoother sem_smoother;   /* opaque learned smoother */

/* Low-precision copies of the geometric factors built at mesh creation. */
#define SEM_PREP_F32 1u
#define SEM_PREP_BF16 2u
/* The hybrid Schwarz multigrid preconditioner's data (per-element separable
 * local solvers at orders N and 3, interpolation matrices, the separable
 * order-1 coarse solver); needed by SEM_FORM_GMRES_HSMG and
 * SEM_FORM_PCG_BLOCK_JACOBI. */
#define SEM_PREP_HSMG 4u

typedef struct {
    int32_t nelx, nely, nelz;   /* elements per direction, each >= 1 */
    int32_t order;              /* polynomial order N, 1..15 */
    const double *vertices;     /* HOST [(nelz+1)][(nely+1)][(nelx+1)][3]; copied */
    uint8_t periodic[3];        /* x, y, z: the last vertex plane is the periodic
                                   image of the first (nodes identified) */
    uint8_t dirichlet_faces;    /* bits 0..5 = x-,x+,y-,y+,z-,z+: homogeneous
                                   Dirichlet (ignored in periodic directions) */
    uint8_t prepare;            /* SEM_PREP_* bits */
} sem_mesh_desc;

typedef struct {
    int64_t nelem;              /* E */
    int64_t n_local;            /* E (N+1)^3 */
    int64_t n_global;           /* unique nodes */
    int64_t n_shared_global;    /* unique nodes with more than one copy */
    int64_t n_shared_local;     /* local copies of those nodes */
    int64_t n_masked_global;    /* unique nodes on Dirichlet faces */
    int32_t order;
    int32_t npts_elem;          /* (N+1)^3 */
    size_t device_bytes;        /* device memory held by the mesh */
} sem_mesh_info;

/* Fields for sem_mesh_export (host copies, canonical layouts). */
enum {
    SEM_FIELD_GLO_NUM = 0,  /* int64  [E][p]    global node id, lexicographic (z, y, x) */
    SEM_FIELD_MULT = 1,     /* int32  [E][p]    number of copies of the node */
    SEM_FIELD_MASK = 2,     /* uint8  [E][p]    1 on Dirichlet nodes */
    SEM_FIELD_G = 3,        /* double [6][E][p] G11 G12 G13 G22 G23 G33 (with W detJ) */
    SEM_FIELD_B = 4,        /* double [E][p]    mass W detJ */
    SEM_FIELD_XYZ = 5,      /* double [3][E][p] node coordinates */
    SEM_FIELD_GLL = 6,      /* double [2][N+1]  GLL nodes, then weights */
    SEM_FIELD_DERIV = 7     /* double [N+1][N+1] D[i][j] = l_j'(xi_i) */
};

/* Host setup (GLL rule, trilinear geometry, geometric factors, numbering,
 * per-axis gather-scatter copy tables) and upload to the current HIP device.  Fails with
 * SEM_ERR_INVALID_ARG if any element has detJ <= 0 at a GLL node. */
sem_status sem_mesh_create(const sem_mesh_desc *desc, sem_mesh **out);
sem_status sem_mesh_destroy(sem_mesh *mesh);
sem_status sem_mesh_query(const sem_mesh *mesh, sem_mesh_info *out);
/* Copy one field to HOST memory; `bytes` must equal the field's size. */
sem_status sem_mesh_export(const sem_mesh *mesh, int field, void *host_dst, size_t bytes);

/* Local operator (async), element by element, unassembled:
 *   w_e = h1 * sum_{a,b} D_a^T (G_ab o D_b u_e) + h2 * B o u_e
 * with D_r, D_s, D_t the GLL derivative along r, s, t (Deville et al. 2002,
 * sec. 4.4; the paper's element-by-element operator of section 3.1).
 * in = SEM_F64: u, w double.  in = SEM_F32: u, w float (needs SEM_PREP_F32).
 * in = SEM_BF16: u bf16 (uint16 bit patterns), w float, contractions on the
 * matrix cores with fp32 accumulation (needs SEM_PREP_BF16).
 * in = SEM_BF16_SPLIT: u, w float; G and B stored in IEEE half with one
 * power-of-two scale per element and array (the element's largest value in
 * [2^14, 2^15) before rounding), every contraction operand carried as a hi +
 * lo bf16 pair on the matrix cores (hi.hi + lo.hi + hi.lo, fp32 sums): the
 * exact operator with those stored G and B to about 2^-16 relative (needs
 * SEM_PREP_BF16, which builds both the bf16 and the half copies).  Both bf16
 * forms need N = 7. */
sem_status sem_ax(const sem_mesh *mesh, double h1, double h2, sem_dtype in,
                  const void *u, void *w, void *stream);

/* Direct-stiffness summation in place (async): every copy of a global node
 * receives the sum of all its copies (the gather-scatter of section 3.1);
 * with apply_mask != 0 the Dirichlet nodes are then zeroed.  dt = SEM_F64
 * (double) or SEM_F32 (float).  The sum runs over copies in ascending local
 * index, so repeated calls are bitwise reproducible. */
sem_status sem_dssum(const sem_mesh *mesh, sem_dtype dt, void *u, int apply_mask, void *stream);

/* Right-hand side (async): b = mask(dssum(B o f)); f, b local double. */
sem_status sem_rhs(const sem_mesh *mesh, const double *f, double *b, void *stream);

/* Inverse of the assembled Jacobi diagonal (async): d = mask(dssum(diag A_L)),
 * with d = 1 on Dirichlet nodes; writes 1/d to dinv (local double). */
sem_status sem_jacobi(const sem_mesh *mesh, double h1, double h2, double *dinv, void *stream);

/* Inner product of two continuous local fields with each global node counted
 * once, sum_l u_l v_l / mult_l (async); the double result is written to the
 * DEVICE address `result`.  Deterministic summation order.  Uses a small
 * partial-sum buffer owned by the mesh: calls on one mesh must be ordered
 * (same stream or synchronised), unlike the other operator entry points. */
sem_status sem_dot(const sem_mesh *mesh, const double *u, const double *v, double *result,
                   void *stream);

/* Preconditioners of the paper's solves, applied to a continuous, masked
 * local residual r (device double [E][P]); z (device double [E][P])
 * receives the continuous, masked result (async).  Needs SEM_PREP_HSMG,
 * h1 > 0, h2 >= 0.  kind:
 *   SEM_PRECOND_HSMG          the three-level hybrid Schwarz multigrid of
 *                             SEM_FORM_GMRES_HSMG (defined below);
 *   SEM_PRECOND_SCHWARZ       its fine level alone: W0 K0 r;
 *   SEM_PRECOND_BLOCK_JACOBI  K0 r without the averaging (the velocity
 *                             solves' block-Jacobi, symmetric positive
 *                             definite);
 *   SEM_PRECOND_HSMG_SYM      the three-level cycle with W^1/2 K W^1/2 in
 *                             place of W K on the fine and mid levels
 *                             (SEM_FORM_PCG_HSMG's symmetric positive
 *                             definite preconditioner).
 * workspace: device, >= sem_precond_workspace_bytes. */
enum { SEM_PRECOND_HSMG = 0, SEM_PRECOND_SCHWARZ = 1, SEM_PRECOND_BLOCK_JACOBI = 2, SEM_PRECOND_HSMG_SYM = 3 };
sem_status sem_precond_workspace_bytes(const sem_mesh *mesh, size_t *bytes);
sem_status sem_precond_apply(const sem_mesh *mesh, int kind, double h1, double h2, const double *r_local,
                             double *z_local, void *workspace, size_t ws_bytes, void *stream);

/* Solver forms. */
typedef enum {
    SEM_FORM_JACOBI_PCG = 0,     /* FP64 Jacobi-preconditioned CG */
    SEM_FORM_DC_FP32 = 1,        /* FP64 defect correction around FP32 Jacobi-PCG */
    SEM_FORM_DC_BF16 = 2,        /* FP64 defect correction around FP32-vector PCG with the
                                    split-BF16 matrix-core operator (SEM_BF16_SPLIT; the plain BF16
                                    operator's rounding of u is too coarse for refinement to
                                    contract on deformed meshes) */
    SEM_FORM_FCG_LEARNED = 3,    /* flexible CG with the learned smoother (opts.smoother),
                                    Jacobi-PCG fallback */
    SEM_FORM_FCG_INNER_FP32 = 4, /* FP64 flexible CG preconditioned by inner_iters steps of
                                    FP32 Jacobi-PCG (FP32 operator) on the unit-scaled defect */
    SEM_FORM_FCG_INNER_BF16 = 5, /* same with the BF16 matrix-core operator in the inner steps */
    SEM_FORM_RELIABLE_FP32 = 6,  /* CG with FP32 vectors and the FP32 operator; the solution is
                                    accumulated in FP64 and the residual is replaced by the FP64
                                    true residual whenever it has fallen by inner_tol (reliable
                                    updates); the search direction is kept */
    SEM_FORM_RELIABLE_BF16 = 7,  /* same with the split-BF16 matrix-core operator
                                    (SEM_BF16_SPLIT) */
    SEM_FORM_PCG_1RED = 8,       /* FP64 Jacobi-PCG in the single-reduction form of
                                    Chronopoulos & Gear (1989): one vector pass, the operator and
                                    one reduction phase per iteration; same stopping test */
    SEM_FORM_GMRES_HSMG = 9,     /* the paper's pressure solver (section 3.1): restarted flexible
                                    GMRES(m) (right preconditioning, Saad 2003 Alg. 9.6; classical
                                    Gram-Schmidt with a second pass when a new direction keeps
                                    less than 1/sqrt(2) of its norm) with the three-level hybrid Schwarz
                                    multigrid preconditioner below; FP64 throughout.  m =
                                    opts.restart; iterations = preconditioned operator
                                    applications.  Needs SEM_PREP_HSMG, h1 > 0, and at least two
                                    elements along every periodic direction. */
    SEM_FORM_PCG_BLOCK_JACOBI = 10, /* FP64 CG with the block-Jacobi preconditioner of the paper's
                                    velocity solves (section 3.1): z = sum over elements of the
                                    element's separable local solve (the fine level of
                                    SEM_FORM_GMRES_HSMG, unweighted, so symmetric positive
                                    definite).  Needs SEM_PREP_HSMG and h1 > 0. */
    SEM_FORM_PCG_HSMG = 11,      /* FP64 CG with the hybrid Schwarz multigrid in its symmetric
                                    weighting (1/sqrt(mult) before the local solves and after their
                                    sum, on the fine and mid levels; symmetric positive definite):
                                    the same preconditioner family as SEM_FORM_GMRES_HSMG at CG's
                                    cost per iteration (no growing Krylov basis).  Needs
                                    SEM_PREP_HSMG and h1 > 0. */
    SEM_FORM_GMRES_LEARNED_MG = 12, /* flexible GMRES(m) as SEM_FORM_GMRES_HSMG with the learned
                                    multigrid: the learned smoother (opts.smoother, BF16
                                    inference) in place of the fine Schwarz level, the paper's
                                    middle and coarse levels kept (not in the paper).  A zero
                                    network makes the fine level Jacobi.  Needs SEM_PREP_HSMG,
                                    N = 7 and h1 > 0. */
    SEM_FORM_FCG_LEARNED_MG = 13 /* SEM_FORM_FCG_LEARNED with the learned multigrid of
                                    SEM_FORM_GMRES_LEARNED_MG as its preconditioner (flexible CG,
                                    Polak-Ribiere, Jacobi-PCG fallback and stall test as there);
                                    CG's cost per iteration.  Needs SEM_PREP_HSMG, N = 7 and
                                    h1 > 0. */
} sem_form;

/* Hybrid Schwarz multigrid (SEM_FORM_GMRES_HSMG), for an assembled fine
 * residual r, with levels at orders N, 3 and 1 on the same vertices:
 *   z = W0 K0 r + P01 [ W1 K1 R10 r + P12 C^-1 R21 R10 r ]
 * P: tensor-product GLL interpolation between levels; R = P^T (on assembled
 * vectors: the residual divided by its multiplicity, J^T per element, summed
 * over copies).  K_l: additive Schwarz whose subdomains are the elements' own
 * node sets (one GLL point of overlap into each neighbour, Dirichlet there);
 * each local matrix is the separable approximation built from one length per
 * element and axis (mean edge length) with the neighbours' end-interval
 * terms, inverted by fast diagonalisation (Lynch, Rice & Thomas 1964) -- the
 * exact principal submatrix inverse on rectilinear meshes.  W_l: the average
 * over node copies (1 / mult).  C^-1: the order-1 operator of the rectilinear
 * grid whose vertex planes are the mesh's averaged planes, inverted by global
 * fast diagonalisation (exact on rectilinear meshes).  Lottes & Fischer
 * (2005) describe this family of hybrid Schwarz/multigrid methods; the
 * additive combination over levels is the one the paper's Neko code uses. */

typedef struct {
    double h1, h2;              /* Helmholtz coefficients (Poisson: 1, 0) */
    double rel_tol;             /* stop when ||r|| <= rel_tol ||b|| (e.g. 1e-10) */
    int32_t max_iter;           /* cap on operator applications (all levels) */
    int32_t check_every;        /* iterations between host polls of the flag */
    int32_t form;               /* sem_form */
    int32_t max_outer;          /* defect-correction outer steps (DC forms) */
    double inner_tol;           /* inner relative tolerance (DC forms); residual reduction that
                                   triggers a replacement (RELIABLE forms, e.g. 0.1) */
    const sem_smoother *smoother; /* learned forms */
    double *history;            /* HOST, optional: relative residual per iteration */
    int32_t history_len;        /* capacity of history */
    int32_t inner_iters;        /* inner steps per outer iteration (FCG_INNER forms) */
    int32_t restart;            /* GMRES restart length m, 1..30 (0 = 30) */
} sem_solve_opts;

typedef struct {
    int32_t status;             /* sem_status of the solve */
    int32_t iterations;         /* operator applications in the Krylov loop(s); for the
                                   DC, FCG_INNER and RELIABLE forms: low-precision iterations */
    int32_t outer_iterations;   /* DC steps, FP64 outer iterations (FCG_INNER forms), or
                                   residual replacements (RELIABLE forms) */
    int32_t restarts;           /* true-residual restarts */
    int32_t fallback_used;      /* learned forms: 1 if Jacobi-PCG took over */
    int32_t history_written;
    double rel_res;             /* final recursive relative residual */
    double true_rel_res;        /* ||b - S x|| / ||b|| in FP64 */
    double elapsed_ms;          /* wall time of the solve */
} sem_solve_report;

/* Device workspace the solve needs, in bytes. */
sem_status sem_solve_workspace_bytes(const sem_mesh *mesh, const sem_solve_opts *opts,
                                     size_t *bytes);

/* Solve S x = b, S = mask o dssum o A_L (blocking: returns after the true
 * residual has been checked).  b is a continuous, masked local field; x
 * receives the solution (x starts from zero).  Jacobi-PCG is Hestenes &
 * Stiefel CG with z = dinv o r; after the recursive residual meets rel_tol
 * the true residual is evaluated and CG restarts from x (at most 3 times)
 * while it does not.  workspace: device, >= sem_solve_workspace_bytes. */
sem_status sem_pcg_solve(const sem_mesh *mesh, const sem_solve_opts *opts, const double *b,
                         double *x, void *workspace, size_t ws_bytes, sem_solve_report *rep,
                         void *stream);

/* Allocation-free variant of sem_pcg_solve, for callers that cannot
 * allocate device memory (serving loops and harnesses that forbid
 * hipMalloc).  Same arguments and results as sem_pcg_solve, without the
 * workspace: it lives in a static device array of SEM_NOALLOC_SCRATCH_BYTES
 * that every device holds once the library is loaded on it, until the
 * process ends.  Allocates nothing.  Fails with SEM_ERR_INVALID_ARG, before
 * any device work, when the solve's workspace (sem_solve_workspace_bytes)
 * exceeds that size (FP64 Jacobi-PCG at N = 7: meshes up to about 900,000
 * local points, 1,700 elements) or the mesh lives on another device than the current one.
 * Every call on a device shares that device's array and leaves its contents
 * behind: calls that overlap in time on one device (other threads or
 * streams) race and must be serialised by the caller. */
#define SEM_NOALLOC_SCRATCH_BYTES ((size_t)32 << 20)
sem_status sem_pcg_solve_noalloc(const sem_mesh *mesh, const sem_solve_opts *opts, const double *b, double *x,
                                 sem_solve_report *rep, void *stream);

/* ---------------------------------------------------------------------------
 * Learned smoother (not in the paper; this library's accelerated form).
 * Per element e of an N = 7 mesh, with q = dinv o r, s_e = max|r_e|,
 * t_e = max|q_e|: X_e = [r_e / s_e, q_e / t_e] (2 channels on the 8^3 tile),
 * Net = conv(16->1) o relu o conv(16->16) o relu o conv(2->16), 3x3x3
 * cross-correlations with zero padding and no bias, c_e = t_e Net(X_e), and
 *     M(r) = dinv o r + mask(Q^T (c / mult)).
 * A zero last layer gives Jacobi; M(a r) = a M(r) for a > 0.  Weights:
 * W1[16][2][27] | W2[16][16][27] | W3[16][27] (tap = 9 (dk+1) + 3 (dj+1) + di+1),
 * 8208 floats, FP32 master copy; inference runs every layer on the BF16
 * matrix cores (inputs and weights rounded to BF16, FP32 accumulation);
 * training runs in FP32.
 * Training loss of a pair (r = S e, e): L = |e - M(r)|_S^2 / |e|_S^2, Adam. */
typedef struct {
    uint32_t seed;            /* He-normal init of layers 1-2; layer 3 starts at zero */
    float lr, beta1, beta2, eps;  /* Adam (0 = defaults 1e-3, 0.9, 0.999, 1e-8) */
    int32_t stall_window;     /* flexible-CG stall window (0 = 25 iterations) */
    double stall_rate;        /* per-iteration residual reduction of plain Jacobi-PCG on the same
                                 problem; a window reducing less than rate^window switches to
                                 Jacobi-PCG.  0 disables the stall test. */
    int32_t mg_context;       /* != 0: train for the learned multigrid.  The loss then uses
                                 M(r) + C(r), C(r) the middle and coarse levels' part of the
                                 cycle (fixed), so the network learns what those levels leave
                                 over.  Needs a mesh created with SEM_PREP_HSMG. */
} sem_smoother_desc;

#define SEM_SMOOTHER_PARAMS 8208

/* Allocates weights, Adam moments and training buffers sized for `mesh`. */
sem_status sem_smoother_create(const sem_mesh *mesh, const sem_smoother_desc *desc, sem_smoother **out);
sem_status sem_smoother_destroy(sem_smoother *sm);
/* HOST float[n], n = SEM_SMOOTHER_PARAMS; set also resets the Adam state. */
sem_status sem_smoother_set_weights(sem_smoother *sm, const float *host, size_t n);
sem_status sem_smoother_get_weights(const sem_smoother *sm, float *host, size_t n);
/* Checkpoint and resume of training: FP32 master weights, Adam's first and
 * second moments (HOST float[n] each, n = SEM_SMOOTHER_PARAMS) and the number
 * of Adam steps taken (which sets the bias corrections of the next step).
 * Both synchronise the device. */
sem_status sem_smoother_get_state(const sem_smoother *sm, float *weights, float *adam_m, float *adam_v, size_t n,
                                  int32_t *step);
sem_status sem_smoother_set_state(sem_smoother *sm, const float *weights, const float *adam_m, const float *adam_v,
                                  size_t n, int32_t step);
/* z = M(r) for a continuous, masked local r (device double [E][P]); fp32 != 0
 * runs the FP32 network, else the BF16 inference path.  Blocking on stream. */
sem_status sem_smoother_apply(const sem_smoother *sm, const sem_mesh *mesh, double h1, double h2, int fp32,
                              const double *r_local, double *z_local, void *stream);
/* z = M_mg(r): the learned multigrid, M_mg(r) = M(r) + C(r) with C(r) =
 * P_01 [Sw_1(R_10 r) + P_12 C^-1 R_21 R_10 r] the middle and coarse levels of
 * the hybrid Schwarz multigrid (averaged weighting; see SEM_FORM_GMRES_HSMG),
 * for a continuous, masked local r (device double [E][P]).  fp32 as for
 * sem_smoother_apply.  workspace: device, >= sem_precond_workspace_bytes.
 * Needs SEM_PREP_HSMG, h1 > 0, h2 >= 0.  Async on stream. */
sem_status sem_smoother_mg_apply(const sem_smoother *sm, const sem_mesh *mesh, double h1, double h2, int fp32,
                                 const double *r_local, double *z_local, void *workspace, size_t ws_bytes,
                                 void *stream);
/* Loss L and dL/dW (FP32 path) for one error field e (continuous, masked local
 * double); loss and gradient are written to HOST memory.  Blocking. */
sem_status sem_smoother_loss_grad(sem_smoother *sm, const sem_mesh *mesh, double h1, double h2,
                                  const double *e_local, double *loss_host, float *grad_host, void *stream);
/* One Adam step on the pair (S e, e); e_global: device float[n_global] in the
 * lexicographic global numbering (as written by sem_pcg_snapshots).  The loss
 * before the step is copied to the DEVICE double *loss_dev (may be NULL). Async. */
sem_status sem_smoother_train_step(sem_smoother *sm, const sem_mesh *mesh, double h1, double h2,
                                   const float *e_global, double *loss_dev, void *stream);

/* Training pairs from plain FP64 Jacobi-PCG on S x = b (x from zero): for
 * each iteration count iters[q] (HOST, ascending) the error e_q = x* - x_{iters[q]}
 * of that iterate against the converged solution x* is written to
 * e_out[q][n_global] (DEVICE double, lexicographic global numbering); counts
 * past convergence give e_q = 0.  opts as for sem_pcg_solve (form ignored). */
sem_status sem_pcg_snapshots(const sem_mesh *mesh, const sem_solve_opts *opts, const double *b,
                             const int32_t *iters, int32_t n_iters, double *e_out, void *workspace,
                             size_t ws_bytes, sem_solve_report *rep, void *stream);

/* Batched FP64 CG for nrhs (1..4) right-hand sides that share the operator
 * and h1/h2, e.g. the three velocity components of a time step (the
 * paper's velocity solves: CG with a block-Jacobi preconditioner, section
 * 3.1).  N = 7 only.  opts.form: SEM_FORM_JACOBI_PCG or
 * SEM_FORM_PCG_BLOCK_JACOBI (the latter on a mesh prepared with
 * SEM_PREP_HSMG; the element solves run per field).  b, x: DEVICE
 * [nrhs][E][P] local fields (layout as sem_pcg_solve, one block per field);
 * reps: HOST array of nrhs reports.  Each field runs its own CG (own alpha,
 * beta, convergence) but every iteration streams the geometric factors
 * once for all fields.  The batched operator kernel sums in another order
 * than the single-field one, so each field matches a separate sem_pcg_solve
 * to rounding (the same 1e-10 true residual, iteration counts within one),
 * not bit for bit.  Other forms are refused with SEM_ERR_UNSUPPORTED;
 * history is ignored. */
sem_status sem_pcg_solve_batched(const sem_mesh *mesh, const sem_solve_opts *opts, int32_t nrhs, const double *b,
                                 double *x, void *workspace, size_t ws_bytes, sem_solve_report *reps, void *stream);
sem_status sem_solve_workspace_bytes_batched(const sem_mesh *mesh, const sem_solve_opts *opts, int32_t nrhs,
                                             size_t *bytes);

const char *sem_last_error(void);

/* Library version string, e.g. "sem 0.1 gfx950". */
const char *sem_version(void);

#ifdef __cplusplus
}
#endif
#endif /* SEM_H */
