// nn.hpp -- internal interface of the learned smoother.
#pragma once

#include "cg.hpp"
#include "hsmg.hpp"
#include "sem_internal.hpp"

namespace sem {

constexpr int kChannels = 16;
constexpr int kW1 = kChannels * 2 * 27;          // layer 1: [o][c][tap]
constexpr int kW2 = kChannels * kChannels * 27;  // layer 2: [o][c][tap]
constexpr int kW3 = kChannels * 27;              // layer 3: [c][tap]
constexpr int kParams = kW1 + kW2 + kW3;         // 8208
constexpr int kWtFloats = kW1 + 2 * kW2;        // FP32 weight layouts of the training loops
constexpr int kGradChunks = 64;                  // first-stage chunks of the gradient sum over elements
constexpr int kWeightOperands = 28 * 256 + 28 * 16 + 16 * 64;   // BF16 operands of layers 2, 3, 1

struct Smoother {
    int64_t E = 0, ng = 0, nl = 0;
    float *W = nullptr;             // FP32 master weights [W1 | W2 | W3]
    float *m = nullptr, *v = nullptr;  // Adam moments
    float *grad = nullptr;          // reduced gradient
    unsigned short *W2b = nullptr;  // BF16 matrix-core operands of the inference (kWeightOperands)
    float *Wt = nullptr;            // FP32 weights in the training loops' layouts (kWtFloats)
    float *dW_elem = nullptr;       // [E][kParams] per-element gradients
    double *gpart = nullptr;        // [kGradChunks][kParams] chunk sums of the gradient
    float *act = nullptr;           // [E][32][512] forward activations (Y1, Y2) kept from the loss for the backward
    float *c_local = nullptr;       // [nl] element outputs
    double *buf = nullptr;          // training vectors: e, r, z, d, sd (5 x ng), w (nl)
    double *part = nullptr;         // partial sums (2 x part_capacity)
    double *stage = nullptr;        // second-stage sums (2 x kStage)
    double *scal = nullptr;         // device scalars: |e|_S^2, loss, ...
    int step = 0;
    float lr = 1e-3f, b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    int stall_window = 25;
    double stall_rate = 0.0;        // 0: stall test off
    // what the dinv in the training buffers was built for: mesh serial and
    // h1, h2 (every call that rebuilds it updates the key)
    mutable uint64_t dinv_serial = 0;
    mutable double dinv_h1 = -1.0, dinv_h2 = -1.0;
    // training in the context of the learned multigrid: the loss adds the
    // coarser levels' part of the cycle to the smoother output (work
    // buffers of one cycle in mg_ws)
    int mg_context = 0;
    char *mg_ws = nullptr;
    HsmgBufs mg{};
    size_t device_bytes = 0;
};

// the smoother was created for a mesh of this size and order N = 7 (and,
// if trained in the multigrid context, the mesh has SEM_PREP_HSMG)
sem_status check_pair(const Smoother &sm, const Mesh &m);

// flexible CG with the learned smoother (learned.hip)
// v: x, r, p, dinv (assembled), w (local); z, q: assembled scratch; the
// smoother's c_local buffer holds the element outputs.  mg (not null): the
// learned multigrid, whose coarser-level part (averaged weighting) is added
// to the smoother output while the network is in use.
sem_status solve_fcg(const Mesh &m, const Smoother &sm, const sem_solve_opts &o, const CgVecs<double> &v,
                     const double *b64, double *z, double *q, CgState *st, double *hist, int hist_len,
                     int check_every, hipStream_t s, sem_solve_report *rep, CgState &h,
                     const HsmgBufs *mg = nullptr);

// FP64 flexible CG preconditioned by inner_iters steps of FP32-vector
// Jacobi-PCG with the FP32 or BF16 operator (learned.hip)
sem_status solve_fcg_nested(const Mesh &m, const sem_solve_opts &o, const CgVecs<double> &v, const CgVecs<float> &v32,
                            float *b32, const double *b64, double *z, double *q, CgState *st, CgState *st32,
                            double *hist, int hist_len, int check_every, bool bf16, hipStream_t s,
                            sem_solve_report *rep, CgState &h);

template <typename TR>
hipError_t nn_infer(const Smoother &sm, const Mesh &m, const TR *rg, const TR *dinvg, float *c_local, hipStream_t s,
                    const int32_t *skip);
template <typename TR>
hipError_t nn_assemble_z(const Mesh &m, const TR *rg, const TR *dinvg, const float *c_local, TR *z, hipStream_t s,
                         const int32_t *use_c, const TR *zp = nullptr);
hipError_t nn_grad(const Smoother &sm, const Mesh &m, const double *rg, const double *dinvg, const double *gz,
                   float *dW_elem, double scale, float *grad, hipStream_t s,
                   const float *act = nullptr);
hipError_t nn_adam(Smoother &sm, const float *grad, hipStream_t s);
hipError_t nn_pack(Smoother &sm, hipStream_t s);
hipError_t nn_infer32(const Smoother &sm, const Mesh &m, const double *rg, const double *dinvg, float *c_local,
                      hipStream_t s,
                      float *act = nullptr);

}  // namespace sem

struct sem_smoother {
    sem::Smoother s;
};
