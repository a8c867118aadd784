// nn.hip -- the learned per-element smoother: inference (BF16 matrix cores),
// FP32 training (forward + backward), Adam, and the assembled smoother.
//
// Not in the paper (which uses Jacobi-type and multigrid preconditioners in
// its Krylov solves, section 3.1); the definition is this project's:
//   X_e = [r_e / s_e, q_e / t_e],  q = dinv o r,  s_e = max|r_e|, t_e = max|q_e|
//   c_e = t_e Net(X_e),  Net = conv3(relu(conv2(relu(conv1(X)))))
//   conv: 3x3x3 cross-correlation, zero padding 1, no bias; 2 -> 16 -> 16 -> 1
//   M(r) = dinv o r + mask(Q^T (c / mult))
// Only N = 7 (8^3 tiles) is supported.
//
// Inference layout (one element per 512-thread workgroup, thread = position):
//  - layer 1 (2 -> 16, 54 MACs per output) and layer 3 (16 -> 1) on the FP32
//    vector units, weights read as wave-uniform (scalar) loads;
//  - layer 2 (16 -> 16, 27 taps) on the matrix cores: for each tap a
//    16x16x16 BF16 MFMA multiplies 16 positions x 16 input channels by the
//    tap's 16 x 16 weight block, FP32 accumulation.  Activations sit in LDS
//    channel-last with a zero halo (10^3 x 16 BF16 = 32 KB), so every A
//    operand is one 8-byte LDS read; the 27 B operands stay in registers.
// Training keeps everything in FP32 (the accuracy reference of the BF16
// inference path); per-element weight gradients are reduced over elements
// in a fixed order.
#include "cg.hpp"
#include "nn.hpp"

namespace sem {
namespace nn {

typedef __attribute__((__vector_size__(4 * sizeof(short)))) short bf16x4;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f4;

constexpr int NP = 8, P3 = 512, PD = 10, PD3 = 1000;

__device__ __forceinline__ unsigned short f2bf(float f)
{
    unsigned u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (unsigned short)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
    u += 0x7fffu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf2f(unsigned short b) { return __uint_as_float(((unsigned)b) << 16); }

__device__ __forceinline__ int pidx(int k, int j, int i) { return ((k + 1) * PD + (j + 1)) * PD + (i + 1); }

// block-wide max of a non-negative value (512 threads)
__device__ float block_max512(float v, float *red)
{
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
    const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
    __syncthreads();
    if (lane == 0) red[wid] = v;
    __syncthreads();
    float m = red[0];
#pragma unroll
    for (int q = 1; q < 8; ++q) m = fmaxf(m, red[q]);
    return m;
}

// Features of element e from assembled r and dinv: Xs[2][PD3] (zero halo
// must already be in place).  Returns t_e and whether the element is live.
template <typename TR>
__device__ void load_features(const TR *__restrict__ rg, const TR *__restrict__ dinvg, const Lattice &L,
                              int64_t e, float *Xs, float *red, float &t_out, bool &live)
{
    const int p = threadIdx.x, i = p & 7, j = (p >> 3) & 7, k = p >> 6;
    const int64_t g = lattice_glo(L, e, i, j, k);
    const double r = (double)rg[g];
    const double q = (double)dinvg[g] * r;
    const float s = block_max512((float)fabs(r), red);
    const float t = block_max512((float)fabs(q), red);
    live = (s > 0.f) && (t > 0.f);
    if (live) {
        Xs[pidx(k, j, i)] = (float)(r / (double)s);
        Xs[PD3 + pidx(k, j, i)] = (float)(q / (double)t);
    }
    t_out = t;
}

__device__ __forceinline__ int tap_off(int tap)
{
    const int dk = tap / 9 - 1, dj = (tap / 3) % 3 - 1, di = tap % 3 - 1;
    return (dk * PD + dj) * PD + di;
}

// ---------------------------------------------------------------- inference

template <typename TR>
__global__ void __launch_bounds__(512)
infer_kernel(const TR *__restrict__ rg, const TR *__restrict__ dinvg, Lattice L, const float *__restrict__ W1,
             const unsigned short *__restrict__ W2b, const float *__restrict__ W3, float *__restrict__ c_out,
             const int32_t *__restrict__ skip)
{
    if (skip && *skip) return;
    __shared__ float Xs[2 * PD3];
    __shared__ __attribute__((aligned(16))) unsigned short Ys[PD3 * 16];
    __shared__ float red[8];
    const int p = threadIdx.x, i = p & 7, j = (p >> 3) & 7, k = p >> 6;
    const int64_t e = xcd_block();
    for (int q = p; q < 2 * PD3; q += 512) Xs[q] = 0.f;
    for (int q = p; q < PD3 * 8; q += 512) ((unsigned *)Ys)[q] = 0u;
    float t;
    bool live;
    __syncthreads();
    load_features(rg, dinvg, L, e, Xs, red, t, live);
    if (!live) {   // uniform across the block
        c_out[e * P3 + p] = 0.f;
        return;
    }
    __syncthreads();
    // layer 1: 2 -> 16, FP32
    {
        float acc[16];
#pragma unroll
        for (int o = 0; o < 16; ++o) acc[o] = 0.f;
        const int base = pidx(k, j, i);
        for (int c = 0; c < 2; ++c)
            for (int tap = 0; tap < 27; ++tap) {
                const float x = Xs[c * PD3 + base + tap_off(tap)];
#pragma unroll
                for (int o = 0; o < 16; ++o) acc[o] += W1[(o * 2 + c) * 27 + tap] * x;
            }
        unsigned pk[8];
#pragma unroll
        for (int o = 0; o < 8; ++o)
            pk[o] = (unsigned)f2bf(fmaxf(acc[2 * o], 0.f)) | ((unsigned)f2bf(fmaxf(acc[2 * o + 1], 0.f)) << 16);
        uint4 *dst = (uint4 *)&Ys[base * 16];
        dst[0] = make_uint4(pk[0], pk[1], pk[2], pk[3]);
        dst[1] = make_uint4(pk[4], pk[5], pk[6], pk[7]);
    }
    __syncthreads();
    // layer 2: 16 -> 16 on the matrix cores
    const int lane = p & 63, wave = p >> 6;
    const int mrow = lane & 15, kq = lane >> 4;   // A: row m, channels 4kq..4kq+3
    f4 acc[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[b] = f4{0.f, 0.f, 0.f, 0.f};
    int abase[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const int pos = (wave * 4 + b) * 16 + mrow;
        abase[b] = pidx(pos >> 6, (pos >> 3) & 7, pos & 7) * 16 + 4 * kq;
    }
    for (int tap = 0; tap < 27; ++tap) {
        const bf16x4 bop = *(const bf16x4 *)&W2b[(tap * 16 + (lane & 15)) * 16 + 4 * kq];
        const int off = tap_off(tap) * 16;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const bf16x4 aop = *(const bf16x4 *)&Ys[abase[b] + off];
            acc[b] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(aop, bop, acc[b], 0, 0, 0);
        }
    }
    __syncthreads();   // every wave has finished reading layer-1 activations
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int pos = (wave * 4 + b) * 16 + 4 * kq + q;   // C: row 4kq+q, column = out channel
            Ys[pidx(pos >> 6, (pos >> 3) & 7, pos & 7) * 16 + (lane & 15)] = f2bf(fmaxf(acc[b][q], 0.f));
        }
    __syncthreads();
    // layer 3: 16 -> 1, FP32
    float y = 0.f;
    const int base = pidx(k, j, i);
    for (int tap = 0; tap < 27; ++tap) {
        const unsigned short *yp = &Ys[(base + tap_off(tap)) * 16];
#pragma unroll
        for (int c = 0; c < 16; ++c) y += W3[c * 27 + tap] * bf2f(yp[c]);
    }
    c_out[e * P3 + p] = t * y;
}

// ---------------------------------------------------------------- training (FP32)

// Forward of element e in FP32; keeps X (Xs), Y1 (Y1s, channel-major padded)
// and Y2 (Y2s) in LDS.  Returns y3 at this thread's position.
__device__ float fwd32(const float *__restrict__ W1, const float *__restrict__ W2, const float *__restrict__ W3,
                       const float *Xs, float *Y1s, float *Y2s)
{
    const int p = threadIdx.x, i = p & 7, j = (p >> 3) & 7, k = p >> 6;
    const int base = pidx(k, j, i);
    float acc[16];
#pragma unroll
    for (int o = 0; o < 16; ++o) acc[o] = 0.f;
    for (int c = 0; c < 2; ++c)
        for (int tap = 0; tap < 27; ++tap) {
            const float x = Xs[c * PD3 + base + tap_off(tap)];
#pragma unroll
            for (int o = 0; o < 16; ++o) acc[o] += W1[(o * 2 + c) * 27 + tap] * x;
        }
#pragma unroll
    for (int o = 0; o < 16; ++o) Y1s[o * PD3 + base] = fmaxf(acc[o], 0.f);
    __syncthreads();
#pragma unroll
    for (int o = 0; o < 16; ++o) acc[o] = 0.f;
    for (int c = 0; c < 16; ++c)
        for (int tap = 0; tap < 27; ++tap) {
            const float x = Y1s[c * PD3 + base + tap_off(tap)];
#pragma unroll
            for (int o = 0; o < 16; ++o) acc[o] += W2[(o * 16 + c) * 27 + tap] * x;
        }
#pragma unroll
    for (int o = 0; o < 16; ++o) Y2s[o * PD3 + base] = fmaxf(acc[o], 0.f);
    __syncthreads();
    float y = 0.f;
    for (int c = 0; c < 16; ++c)
        for (int tap = 0; tap < 27; ++tap) y += W3[c * 27 + tap] * Y2s[c * PD3 + base + tap_off(tap)];
    return y;
}

// One element of the loss gradient.  gz: dL/dz on assembled nodes; the
// element's output gradient is g3 = t_e gz[glo] / mult (0 on Dirichlet nodes).
// Writes the element's weight gradient (kParams floats) to dW[e].
template <typename TR>
__global__ void __launch_bounds__(512)
train_kernel(const TR *__restrict__ rg, const TR *__restrict__ dinvg, const double *__restrict__ gz, Lattice L,
             const float *__restrict__ W1, const float *__restrict__ W2, const float *__restrict__ W3,
             float *__restrict__ dW)
{
    __shared__ float Xs[2 * PD3];
    __shared__ float Y1s[16 * PD3];
    __shared__ float Bs[16 * PD3];   // Y2, then g2, then g1
    __shared__ float g3s[PD3];
    __shared__ float red[8];
    const int p = threadIdx.x, i = p & 7, j = (p >> 3) & 7, k = p >> 6;
    const int base = pidx(k, j, i);
    const int64_t e = xcd_block();
    float *dWe = dW + e * kParams;
    for (int q = p; q < 2 * PD3; q += 512) Xs[q] = 0.f;
    for (int q = p; q < 16 * PD3; q += 512) { Y1s[q] = 0.f; Bs[q] = 0.f; }
    for (int q = p; q < PD3; q += 512) g3s[q] = 0.f;
    float t;
    bool live;
    __syncthreads();
    load_features(rg, dinvg, L, e, Xs, red, t, live);
    if (!live) {
        for (int q = p; q < kParams; q += 512) dWe[q] = 0.f;
        return;
    }
    __syncthreads();
    fwd32(W1, W2, W3, Xs, Y1s, Bs);
    // output gradient
    {
        int ex, ey, ez;
        elem_coords(L, e, ex, ey, ez);
        int gi = (int)(ex * L.N + i), gj = (int)(ey * L.N + j), gk = (int)(ez * L.N + k);
        if (gi >= L.nx) gi -= (int)L.nx;
        if (gj >= L.ny) gj -= (int)L.ny;
        if (gk >= L.nz) gk -= (int)L.nz;
        const int64_t g = gi + L.nx * (gj + L.ny * gk);
        int loc[8];
        bool msk;
        const int n = node_locals(L, gi, gj, gk, loc, msk);
        g3s[base] = msk ? 0.f : (float)(t * gz[g] / n);
    }
    __syncthreads();
    // dW3[c][tap] = sum_pos g3[pos] Y2[c][pos+tap]
    for (int w = p; w < 16 * 27; w += 512) {
        const int c = w / 27, off = tap_off(w % 27);
        float s = 0.f;
        for (int q = 0; q < P3; ++q) {
            const int b = pidx(q >> 6, (q >> 3) & 7, q & 7);
            s += g3s[b] * Bs[c * PD3 + b + off];
        }
        dWe[kW1 + kW2 + w] = s;
    }
    // g2[c][pos] = (sum_tap W3[c][tap] g3[pos - tap]) * (Y2 > 0)
    float g2v[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) {
        float s = 0.f;
        for (int tap = 0; tap < 27; ++tap) s += W3[c * 27 + tap] * g3s[base - tap_off(tap)];
        g2v[c] = Bs[c * PD3 + base] > 0.f ? s : 0.f;
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 16; ++c) Bs[c * PD3 + base] = g2v[c];
    __syncthreads();
    // dW2[o][c][tap] = sum_pos g2[o][pos] Y1[c][pos+tap]
    for (int w = p; w < 16 * 16 * 27; w += 512) {
        const int o = w / (16 * 27), c = (w / 27) % 16, off = tap_off(w % 27);
        float s = 0.f;
        for (int q = 0; q < P3; ++q) {
            const int b = pidx(q >> 6, (q >> 3) & 7, q & 7);
            s += Bs[o * PD3 + b] * Y1s[c * PD3 + b + off];
        }
        dWe[kW1 + w] = s;
    }
    // g1[c][pos] = (sum_o sum_tap W2[o][c][tap] g2[o][pos - tap]) * (Y1 > 0)
    float g1v[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) g1v[c] = 0.f;
    for (int o = 0; o < 16; ++o)
        for (int tap = 0; tap < 27; ++tap) {
            const float gv = Bs[o * PD3 + base - tap_off(tap)];
#pragma unroll
            for (int c = 0; c < 16; ++c) g1v[c] += W2[(o * 16 + c) * 27 + tap] * gv;
        }
#pragma unroll
    for (int c = 0; c < 16; ++c) g1v[c] = Y1s[c * PD3 + base] > 0.f ? g1v[c] : 0.f;
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 16; ++c) Bs[c * PD3 + base] = g1v[c];
    __syncthreads();
    // dW1[o][c][tap] = sum_pos g1[o][pos] X[c][pos+tap]
    for (int w = p; w < kW1; w += 512) {
        const int o = w / 54, c = (w / 27) % 2, off = tap_off(w % 27);
        float s = 0.f;
        for (int q = 0; q < P3; ++q) {
            const int b = pidx(q >> 6, (q >> 3) & 7, q & 7);
            s += Bs[o * PD3 + b] * Xs[c * PD3 + b + off];
        }
        dWe[w] = s;
    }
}

// FP32 forward writing c = t y3 (the training-path smoother output)
template <typename TR>
__global__ void __launch_bounds__(512)
infer32_kernel(const TR *__restrict__ rg, const TR *__restrict__ dinvg, Lattice L, const float *__restrict__ W1,
               const float *__restrict__ W2, const float *__restrict__ W3, float *__restrict__ c_out)
{
    __shared__ float Xs[2 * PD3];
    __shared__ float Y1s[16 * PD3];
    __shared__ float Y2s[16 * PD3];
    __shared__ float red[8];
    const int p = threadIdx.x;
    const int64_t e = xcd_block();
    for (int q = p; q < 2 * PD3; q += 512) Xs[q] = 0.f;
    for (int q = p; q < 16 * PD3; q += 512) { Y1s[q] = 0.f; Y2s[q] = 0.f; }
    float t;
    bool live;
    __syncthreads();
    load_features(rg, dinvg, L, e, Xs, red, t, live);
    if (!live) {
        c_out[e * P3 + p] = 0.f;
        return;
    }
    __syncthreads();
    const float y = fwd32(W1, W2, W3, Xs, Y1s, Y2s);
    c_out[e * P3 + p] = t * y;
}

// out[w] = scale * sum_e dW[e][w] (fixed order)
__global__ void reduce_grad_kernel(const float *__restrict__ dW, int64_t E, double scale, float *__restrict__ out)
{
    const int w = blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= kParams) return;
    double s = 0.0;
    for (int64_t e = 0; e < E; ++e) s += (double)dW[e * kParams + w];
    out[w] = (float)(s * scale);
}

__global__ void adam_kernel(float *__restrict__ W, float *__restrict__ m, float *__restrict__ v,
                            const float *__restrict__ g, float lr, float b1, float b2, float eps, float c1, float c2)
{
    const int w = blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= kParams) return;
    const float gw = g[w];
    const float mw = b1 * m[w] + (1.f - b1) * gw;
    const float vw = b2 * v[w] + (1.f - b2) * gw * gw;
    m[w] = mw;
    v[w] = vw;
    W[w] -= lr * (mw / c1) / (sqrtf(vw / c2) + eps);
}

// W2 (FP32 [o][c][tap]) -> BF16 matrix-core operands [tap][o][c]
__global__ void pack_w2_kernel(const float *__restrict__ W, unsigned short *__restrict__ W2b)
{
    const int w = blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= kW2) return;
    const int o = w / (16 * 27), c = (w / 27) % 16, tap = w % 27;
    W2b[(tap * 16 + o) * 16 + c] = f2bf(W[kW1 + w]);
}

// z = dinv r + sum_copies c / mult (+ zp[g] if zp: the learned multigrid's
// coarser-level part), 0 on Dirichlet nodes, assembled
template <typename TR>
__global__ void __launch_bounds__(kBS)
assemble_z_kernel(const TR *__restrict__ rg, const TR *__restrict__ dinvg, const float *__restrict__ c, Lattice L,
                  TR *__restrict__ z, const int32_t *__restrict__ use_c, const TR *__restrict__ zp)
{
    const bool with_c = !use_c || *use_c;
    SEM_FOR_EACH_NODE(L, gi, gj, gk, g)
    {
        const TR d = dinvg[g];
        if (d == TR(0)) { z[g] = TR(0); continue; }
        double zz = (double)d * (double)rg[g];
        if (with_c) {
            int loc[8];
            bool msk;
            const int n = node_locals(L, gi, gj, gk, loc, msk);
            float s = 0.f;
            for (int q = 0; q < n; ++q) s += c[loc[q]];
            zz += (double)s / n;
        }
        if (zp) zz += (double)zp[g];
        z[g] = (TR)zz;
    }
}

}  // namespace nn

// ---------------------------------------------------------------- launchers

template <typename TR>
hipError_t nn_infer(const Smoother &sm, const Mesh &m, const TR *rg, const TR *dinvg, float *c_local, hipStream_t s,
                    const int32_t *skip)
{
    hipLaunchKernelGGL((nn::infer_kernel<TR>), dim3((unsigned)m.E), dim3(512), 0, s, rg, dinvg, m.lat, sm.W,
                       sm.W2b, sm.W + kW1 + kW2, c_local, skip);
    return hipGetLastError();
}

template <typename TR>
hipError_t nn_assemble_z(const Mesh &m, const TR *rg, const TR *dinvg, const float *c_local, TR *z, hipStream_t s,
                         const int32_t *use_c, const TR *zp)
{
    hipLaunchKernelGGL((nn::assemble_z_kernel<TR>), dim3(node_grid(m.lat)), dim3(kBS), 0, s, rg, dinvg, c_local,
                       m.lat, z, use_c, zp);
    return hipGetLastError();
}

hipError_t nn_grad(const Smoother &sm, const Mesh &m, const double *rg, const double *dinvg, const double *gz,
                   float *dW_elem, double scale, float *grad, hipStream_t s)
{
    hipLaunchKernelGGL((nn::train_kernel<double>), dim3((unsigned)m.E), dim3(512), 0, s, rg, dinvg, gz, m.lat, sm.W,
                       sm.W + kW1, sm.W + kW1 + kW2, dW_elem);
    hipLaunchKernelGGL(nn::reduce_grad_kernel, dim3((kParams + 255) / 256), dim3(256), 0, s, dW_elem, m.E, scale,
                       grad);
    return hipGetLastError();
}

hipError_t nn_adam(Smoother &sm, const float *grad, hipStream_t s)
{
    sm.step += 1;
    // bias corrections 1 - beta^t in FP64 (in FP32, 1 - 0.999^t loses about
    // 15 bits to cancellation at small t), then rounded once
    const float c1 = (float)(1.0 - std::pow((double)sm.b1, (double)sm.step));
    const float c2 = (float)(1.0 - std::pow((double)sm.b2, (double)sm.step));
    hipLaunchKernelGGL(nn::adam_kernel, dim3((kParams + 255) / 256), dim3(256), 0, s, sm.W, sm.m, sm.v, grad, sm.lr,
                       sm.b1, sm.b2, sm.eps, c1, c2);
    return nn_pack(sm, s);
}

hipError_t nn_pack(Smoother &sm, hipStream_t s)
{
    hipLaunchKernelGGL(nn::pack_w2_kernel, dim3((kW2 + 255) / 256), dim3(256), 0, s, sm.W, sm.W2b);
    return hipGetLastError();
}

hipError_t nn_infer32(const Smoother &sm, const Mesh &m, const double *rg, const double *dinvg, float *c_local,
                      hipStream_t s)
{
    hipLaunchKernelGGL((nn::infer32_kernel<double>), dim3((unsigned)m.E), dim3(512), 0, s, rg, dinvg, m.lat, sm.W,
                       sm.W + kW1, sm.W + kW1 + kW2, c_local);
    return hipGetLastError();
}

template hipError_t nn_infer<double>(const Smoother &, const Mesh &, const double *, const double *, float *,
                                     hipStream_t, const int32_t *);
template hipError_t nn_assemble_z<double>(const Mesh &, const double *, const double *, const float *, double *,
                                          hipStream_t, const int32_t *, const double *);

}  // namespace sem
