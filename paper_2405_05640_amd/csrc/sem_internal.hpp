// sem_internal.hpp -- internal declarations of libsem (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/sem.h"
#include "lattice.hpp"

namespace sem {

// Thread-local error text for sem_last_error().
void set_error(const std::string &msg);
sem_status fail(sem_status st, const std::string &msg);

#define SEM_HIP_TRY(expr)                                                                   \
    do {                                                                                    \
        hipError_t _e = (expr);                                                             \
        if (_e != hipSuccess)                                                               \
            return ::sem::fail(SEM_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(_e)); \
    } while (0)

constexpr int kMaxOrder = 15;

struct Hsmg;

// GLL rule and derivative matrix of the library (mesh.cpp)
void gll_rule(int N, std::vector<double> &x, std::vector<double> &w);
std::vector<double> deriv_matrix(const std::vector<double> &x);

// Device-resident mesh.  Local fields are [E][NP][NP][NP], i fastest.
struct Mesh {
    int nelx = 0, nely = 0, nelz = 0, N = 0, NP = 0;
    int64_t E = 0, P = 0, nl = 0, ng = 0;
    uint8_t periodic[3] = {0, 0, 0};
    uint8_t dirichlet = 0;
    int64_t n_shared_global = 0, n_shared_local = 0, n_masked_global = 0;
    int device = 0;

    std::vector<double> xi, wq, D;      // host reference element

    // device data
    double *d_D = nullptr;     // [NP][NP]
    float *d_D32 = nullptr;
    uint16_t *d_Dbf = nullptr; // bf16 bits: D rounded (P2 values), then the remainders D - hi
    double *d_G = nullptr;     // [E][6][P] element-blocked geometric factors
    double *d_B = nullptr;     // [E][P]
    double *d_xyz = nullptr;   // [3][E][P]
    uint8_t *d_wcode = nullptr;  // per local node: 0 masked, else 1 + log2(mult)
    uint8_t *d_mult = nullptr;   // per local node: mult
    Lattice lat{};               // closed-form numbering used by the kernels
    int2 *d_tab = nullptr;       // axis copy tables (x, y, z concatenated)
    float *d_G32 = nullptr, *d_B32 = nullptr;          // [E][6][P], [E][P]
    uint16_t *d_Gbf = nullptr, *d_Bbf = nullptr;       // bf16 copies
    // half copies for the split-BF16 operator: value = half(a / 2^k) 2^k with
    // one k per element and array; d_hscale[2 e] = 2^k of G, [2 e + 1] of B
    uint16_t *d_Gh = nullptr, *d_Bh = nullptr;
    float *d_hscale = nullptr;
    double *d_scratch = nullptr;  // small device scratch for sem_dot partials
    int32_t scratch_len = 0;
    Hsmg *hsmg = nullptr;         // multigrid preconditioner (SEM_PREP_HSMG)
    size_t device_bytes = 0;
    uint64_t serial = 0;          // unique per created mesh (process-wide counter)

    int64_t glo(int64_t e, int i, int j, int k) const;
};

// ---- kernel launchers (defined in the .hip files) ----
// partial_uw (optional): per-element sum of u*w, written to partial_uw[e].
// skip (optional device flag): when *skip != 0 the launch does nothing.
hipError_t launch_ax_f64(const Mesh &m, double h1, double h2, const double *u, double *w,
                         double *partial_uw, hipStream_t s, const int32_t *skip = nullptr);
hipError_t launch_ax_f32(const Mesh &m, float h1, float h2, const float *u, float *w,
                         double *partial_uw, hipStream_t s, const int32_t *skip = nullptr);
// same, with u an assembled vector (one value per global node)
hipError_t launch_ax_f64_gather(const Mesh &m, double h1, double h2, const double *ug, double *w,
                                double *partial_uw, hipStream_t s, const int32_t *skip = nullptr);
hipError_t launch_ax_f32_gather(const Mesh &m, float h1, float h2, const float *ug, float *w,
                                double *partial_uw, hipStream_t s, const int32_t *skip = nullptr);
// nc (1..4) assembled fields through one pass over G (N = 7): field c at
// ug + c * ustride, output w + c * n_local, partials partial[c * E + e];
// skipped when every done_flags[c * done_stride] is set.
hipError_t launch_ax_f64_gather_batched(const Mesh &m, int nc, double h1, double h2, const double *ug, int64_t ustride,
                                        double *w, double *partial, const int32_t *done_flags, int done_stride,
                                        hipStream_t s);
// BF16 operator on the matrix cores (N = 7): u local bf16 bits, or (gather)
// an assembled float vector rounded to bf16 on load; w float local.
hipError_t launch_ax_bf16(const Mesh &m, float h1, float h2, const uint16_t *u, float *w, hipStream_t s);
// split-BF16 operator: FP32 u (local, or assembled when gather), FP32 w, optional per-element u.w
hipError_t launch_ax_bf16s(const Mesh &m, float h1, float h2, const float *u, float *w, double *partial,
                           hipStream_t s, const int32_t *skip, bool gather);
hipError_t launch_ax_bf16_gather(const Mesh &m, float h1, float h2, const float *ug, float *w, double *partial_uw,
                                 hipStream_t s, const int32_t *skip = nullptr);
hipError_t launch_diag(const Mesh &m, double h1, double h2, double *d, hipStream_t s);
hipError_t launch_dssum_f64(const Mesh &m, double *u, int apply_mask, hipStream_t s,
                           const int32_t *skip = nullptr);
hipError_t launch_dssum_f32(const Mesh &m, float *u, int apply_mask, hipStream_t s,
                           const int32_t *skip = nullptr);
hipError_t launch_scale_by_B(const Mesh &m, const double *f, double *b, hipStream_t s);
hipError_t launch_jacobi_finish(const Mesh &m, double *d, hipStream_t s);
hipError_t launch_dot(const Mesh &m, const double *u, const double *v, double *partials,
                      int nblocks, double *result, hipStream_t s);
int dot_blocks(const Mesh &m);

}  // namespace sem

struct sem_mesh {
    sem::Mesh m;
};
