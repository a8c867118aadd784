// ax_bf16.hip -- the local operator with BF16 inputs on the matrix cores
// (FP32 accumulation), for the mixed-precision solve.
//
//   w_e = h1 sum_a D_a^T (sum_b G_ab (D_b u_e)) + h2 B o u_e      (N = 7 only)
//
// Rounding (mirrored by the oracle's emulation): u, D, G, B are BF16; the
// derivative contractions accumulate in FP32 on the matrix cores; the
// G-combination runs in FP32 and its three results are rounded to BF16
// before the transposed contractions; those accumulate in FP32 and the r, s,
// t contributions are added in that order; the Helmholtz term is FP32.
//
// Matrix-core mapping (one wavefront per element): a directional
// contraction is a (64 lines x 8) x (8 x 8) product.  A 16x16x16 BF16 MFMA
// takes two lines per A row (K = 2 x 8) against B = blockdiag(D^T, D^T), so
// no K padding is wasted: two MFMAs per direction and element.  Lines along
// r are contiguous in the element tile (one 8-byte LDS read per operand);
// lines along s and t are gathered from LDS with strides 8 and 64.
#include "sem_internal.hpp"

namespace sem {
namespace {

typedef __attribute__((__vector_size__(4 * sizeof(short)))) short bf16x4;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f4;

__device__ __forceinline__ unsigned short f2bf(float f)
{
    unsigned u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (unsigned short)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
    u += 0x7fffu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf2f(unsigned short b) { return __uint_as_float(((unsigned)b) << 16); }

// point index of entry c (0..7) of line L along direction dir (0 = r, 1 = s, 2 = t)
__device__ __forceinline__ int line_point(int dir, int L, int c)
{
    if (dir == 0) return L * 8 + c;                          // L = 8k + j, c = i
    if (dir == 1) return (L >> 3) * 64 + c * 8 + (L & 7);    // L = 8k + i, c = j
    return c * 64 + L;                                       // L = 8j + i, c = k
}

// One directional contraction of the 512-point tile src (BF16 in LDS):
// out[line][n] = sum_c src[line][c] Bop[c][n]; the 64 lines are processed as
// 32 line pairs in two MFMAs.  Results go to dst (FP32 in LDS), added when acc.
__device__ __forceinline__ void contract(int dir, const unsigned short *src, float *dst, bf16x4 bop, bool acc)
{
    const int lane = threadIdx.x & 63;
    const int m = lane & 15, kq = lane >> 4;
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        // A operand: row m of this MFMA = line pair (2 (16 t + m), +1); K
        // entries 4 kq .. 4 kq + 3 = line (kq >> 1), entries 4 (kq & 1) + q
        const int Lpair = 16 * t + m;
        const int L = 2 * Lpair + (kq >> 1);
        const int c0 = 4 * (kq & 1);
        bf16x4 a;
        if (dir == 0) {
            a = *(const bf16x4 *)&src[line_point(0, L, c0)];
        } else {
#pragma unroll
            for (int q = 0; q < 4; ++q) a[q] = (short)src[line_point(dir, L, c0 + q)];
        }
        f4 c = {0.f, 0.f, 0.f, 0.f};
        c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, bop, c, 0, 0, 0);
        // C: column n = lane & 15 -> line (n >> 3), entry n & 7; rows 4 kq + q -> line pairs
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int pair = 16 * t + 4 * kq + q;
            const int n = lane & 15;
            const int p = line_point(dir, 2 * pair + (n >> 3), n & 7);
            if (acc)
                dst[p] += c[q];
            else
                dst[p] = c[q];
        }
    }
}

template <bool GATHER, bool HELM>
__global__ void __launch_bounds__(64)
ax_bf16_kernel(const void *__restrict__ uin, float *__restrict__ w, const unsigned short *__restrict__ G,
               const unsigned short *__restrict__ Bm, const unsigned short *__restrict__ Dbf, float h1, float h2,
               double *__restrict__ partial, const int32_t *__restrict__ skip, Lattice L)
{
    if (skip && *skip) return;
    __shared__ __attribute__((aligned(16))) unsigned short su[512];
    __shared__ __attribute__((aligned(16))) unsigned short sw[3][512];
    __shared__ float sd[3][512];
    __shared__ unsigned short sD[64];
    const int lane = threadIdx.x;
    const int64_t e = blockIdx.x;
    sD[lane] = Dbf[lane];
    // u tile (BF16) into LDS: each lane 8 consecutive points
    if (GATHER) {
        const float *ug = (const float *)uin;
        const int64_t ex = e % L.nelx, ey = (e / L.nelx) % L.nely, ez = e / ((int64_t)L.nelx * L.nely);
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int p = lane * 8 + q, i = p & 7, j = (p >> 3) & 7, k = p >> 6;
            int64_t gi = ex * 7 + i, gj = ey * 7 + j, gk = ez * 7 + k;
            if (gi >= L.nx) gi -= L.nx;
            if (gj >= L.ny) gj -= L.ny;
            if (gk >= L.nz) gk -= L.nz;
            su[p] = f2bf(ug[gi + L.nx * (gj + L.ny * gk)]);
        }
    } else {
        const uint4 v = ((const uint4 *)((const unsigned short *)uin + e * 512))[lane];
        ((uint4 *)su)[lane] = v;
    }
    __syncthreads();
    // B operands: lane holds B[4 kq + q][n], n = lane & 15
    const int n = lane & 15, kq = lane >> 4;
    bf16x4 bT, bD;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int kk = 4 * kq + q;
        const bool blk = (kk >> 3) == (n >> 3);
        const int a = kk & 7, b = n & 7;
        bT[q] = blk ? (short)sD[b * 8 + a] : (short)0;   // D^T[a][b] = D[b][a]
        bD[q] = blk ? (short)sD[a * 8 + b] : (short)0;   // D[a][b]
    }
    contract(0, su, sd[0], bT, false);
    contract(1, su, sd[1], bT, false);
    contract(2, su, sd[2], bT, false);
    __syncthreads();
    // G-combination, FP32, rounded to BF16
    const unsigned short *Ge = G + e * 6 * 512;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int p = lane + 64 * q;
        const float ur = sd[0][p], us = sd[1][p], ut = sd[2][p];
        const float g11 = bf2f(Ge[p]), g12 = bf2f(Ge[512 + p]), g13 = bf2f(Ge[1024 + p]);
        const float g22 = bf2f(Ge[1536 + p]), g23 = bf2f(Ge[2048 + p]), g33 = bf2f(Ge[2560 + p]);
        sw[0][p] = f2bf(g11 * ur + g12 * us + g13 * ut);
        sw[1][p] = f2bf(g12 * ur + g22 * us + g23 * ut);
        sw[2][p] = f2bf(g13 * ur + g23 * us + g33 * ut);
    }
    __syncthreads();
    // transposed contractions, accumulated r, s, t into sd[0]
    contract(0, sw[0], sd[0], bD, false);
    __syncthreads();
    contract(1, sw[1], sd[0], bD, true);
    __syncthreads();
    contract(2, sw[2], sd[0], bD, true);
    __syncthreads();
    double dot = 0.0;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int p = lane + 64 * q;
        float v = h1 * sd[0][p];
        const float uu = bf2f(su[p]);
        if (HELM) v += h2 * bf2f(Bm[e * 512 + p]) * uu;
        w[e * 512 + p] = v;
        if (partial) dot += (double)uu * (double)v;
    }
    if (partial) {
        for (int o = 32; o > 0; o >>= 1) dot += __shfl_xor(dot, o);
        if (lane == 0) partial[e] = dot;
    }
}

}  // namespace

static hipError_t launch_bf16(const Mesh &m, float h1, float h2, const void *u, float *w, double *partial,
                              hipStream_t s, const int32_t *skip, bool gather)
{
    if (m.E == 0) return hipSuccess;
    if (m.N != 7) return hipErrorInvalidValue;
    const bool helm = h2 != 0.f;
    const dim3 grid((unsigned)m.E), block(64);
    if (gather) {
        if (helm)
            hipLaunchKernelGGL((ax_bf16_kernel<true, true>), grid, block, 0, s, u, w, m.d_Gbf, m.d_Bbf, m.d_Dbf, h1, h2, partial, skip, m.lat);
        else
            hipLaunchKernelGGL((ax_bf16_kernel<true, false>), grid, block, 0, s, u, w, m.d_Gbf, m.d_Bbf, m.d_Dbf, h1, h2, partial, skip, m.lat);
    } else {
        if (helm)
            hipLaunchKernelGGL((ax_bf16_kernel<false, true>), grid, block, 0, s, u, w, m.d_Gbf, m.d_Bbf, m.d_Dbf, h1, h2, partial, skip, m.lat);
        else
            hipLaunchKernelGGL((ax_bf16_kernel<false, false>), grid, block, 0, s, u, w, m.d_Gbf, m.d_Bbf, m.d_Dbf, h1, h2, partial, skip, m.lat);
    }
    return hipGetLastError();
}

hipError_t launch_ax_bf16(const Mesh &m, float h1, float h2, const uint16_t *u, float *w, hipStream_t s)
{
    return launch_bf16(m, h1, h2, u, w, nullptr, s, nullptr, false);
}

hipError_t launch_ax_bf16_gather(const Mesh &m, float h1, float h2, const float *ug, float *w, double *partial_uw,
                                 hipStream_t s, const int32_t *skip)
{
    return launch_bf16(m, h1, h2, ug, w, partial_uw, s, skip, true);
}

}  // namespace sem
