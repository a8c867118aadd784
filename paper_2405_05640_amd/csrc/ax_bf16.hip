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
typedef __attribute__((__vector_size__(4 * sizeof(unsigned)))) unsigned u32x4;

// FP32 -> BF16, round to nearest even (the gfx950 conversion instruction)
__device__ __forceinline__ unsigned short f2bf(float f) { return __builtin_bit_cast(unsigned short, (__bf16)f); }
__device__ __forceinline__ float bf2f(unsigned short b) { return __uint_as_float(((unsigned)b) << 16); }
// BF16 number q (0..7) of a 16-byte vector, widened to FP32
__device__ __forceinline__ float bf_at(const u32x4 &v, int q)
{
    const unsigned w = v[q >> 1];
    return __uint_as_float((q & 1) ? (w & 0xffff0000u) : (w << 16));
}

// half-precision entry q (0..7) of a 16-byte vector, widened to float (exact)
__device__ __forceinline__ float h_at(const u32x4 &v, int q)
{
    const unsigned w = v[q >> 1];
    return (float)__builtin_bit_cast(_Float16, (unsigned short)((q & 1) ? (w >> 16) : (w & 0xffffu)));
}

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
    const int64_t e = xcd_block();
    int ex = 0, ey = 0, ez = 0;   // element coordinates (gather mode)
    if (GATHER) elem_coords(L, e, ex, ey, ez);
    // Issue every streaming load of the element first (G: six 16-byte
    // vectors per lane, each lane owning the contiguous 8-point row 8 lane ..
    // 8 lane + 7; B likewise) so that their latency overlaps the u gather and
    // the first contractions.
    const unsigned short *Ge = G + e * 6 * 512;
    u32x4 gq[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) gq[c] = __builtin_nontemporal_load((const u32x4 *)(Ge + c * 512) + lane);
    u32x4 bq = {0u, 0u, 0u, 0u};
    if (HELM) bq = __builtin_nontemporal_load((const u32x4 *)(Bm + e * 512) + lane);
    sD[lane] = Dbf[lane];
    // u tile (BF16) into LDS; gathered in point order (lane = i + 8 j within
    // k-plane q), so a load instruction spans 8 runs of 8 consecutive global
    // nodes
    if (GATHER) {
        const float *ug = (const float *)uin;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int p = 64 * q + lane, i = p & 7, j = (p >> 3) & 7, k = p >> 6;
            su[p] = f2bf(ug[gather_index32(L, ex, ey, ez, i, j, k)]);
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
    // G-combination, FP32, rounded to BF16 (lane: points 8 lane .. 8 lane + 7)
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int p = 8 * lane + q;
        const float ur = sd[0][p], us = sd[1][p], ut = sd[2][p];
        const float g11 = bf_at(gq[0], q), g12 = bf_at(gq[1], q), g13 = bf_at(gq[2], q);
        const float g22 = bf_at(gq[3], q), g23 = bf_at(gq[4], q), g33 = bf_at(gq[5], q);
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
    float out[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int p = 8 * lane + q;
        float v = h1 * sd[0][p];
        const float uu = bf2f(su[p]);
        if (HELM) v += h2 * bf_at(bq, q) * uu;
        out[q] = v;
        if (partial) dot += (double)uu * (double)v;
    }
    float4 *wo = (float4 *)(w + (GATHER ? (int64_t)rows_index32(L, ex, ey, ez, 0, lane & 7, lane >> 3) : e * 512 + 8 * lane));
    wo[0] = make_float4(out[0], out[1], out[2], out[3]);
    wo[1] = make_float4(out[4], out[5], out[6], out[7]);
    if (partial) {
        for (int o = 32; o > 0; o >>= 1) dot += __shfl_xor(dot, o);
        if (lane == 0) partial[e] = dot;
    }
}

// ---------------------------------------------------------------------------
// Split-BF16 operator: FP32 u through the BF16 matrix cores.  Every operand x
// of a contraction (u, D, the fluxes, D^T) is carried as a pair of BF16
// numbers x = hi + lo (hi = bf16(x), lo = bf16(x - hi): 16 significant bits),
// and a contraction sums hi.Dhi + lo.Dhi + hi.Dlo in FP32 (the lo.lo product,
// about 2^-18 relative, is dropped).  The hi/lo split of u and of the
// fluxes is made once per value, into LDS.  G and B are IEEE half storage
// with one power-of-two scale per element and array (11 significant bits,
// the largest value of an element in the top half binade), so the operator
// reproduces the exact operator with those stored G and B to about 2^-16
// relative while streaming 12 + 2 bytes of geometry per point.
//
// One 16x16x32 MFMA handles 16 lines of a direction: A row m = line
// (K = [hi(8) | lo(8) | hi(8) | 0(8)]), B = [Dhi^T; Dhi^T; Dlo^T; 0] in output
// columns 0..7 (columns 8..15 are zero), four MFMAs per direction.
typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(8 * sizeof(short)))) short s16x8;

// hi and lo BF16 parts of eight FP32 values
__device__ __forceinline__ void split8(const float (&v)[8], s16x8 &h, s16x8 &l)
{
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const unsigned short hb = f2bf(v[q]);
        h[q] = (short)hb;
        l[q] = (short)f2bf(v[q] - bf2f(hb));
    }
}

// The BF16 hi and lo tiles in LDS are padded: point p = i + 8 j + 64 k sits
// at halfword p + 8 k, so each k-plane (72 halfwords) starts 4 banks after the
// previous one, and a lo tile starts kHalfTile halfwords (16 banks mod 32)
// after its hi tile.  The s- and t-direction operand reads of hi and lo then
// fall in distinct banks, and rows stay 16-byte aligned.
constexpr int kHalfTile = 608;   // 512 + 8 * 8 padding + 32 bank offset
__device__ __forceinline__ int hpad(int p) { return p + ((p >> 6) << 3); }
// FP32 tiles (derivatives, accumulator): 4 floats of padding per 32, which
// spreads the scattered MFMA result writes over more banks while each 8-value
// row stays contiguous and 16-byte aligned; a tile spans kFloatTile floats.
constexpr int kFloatTile = 608;
__device__ __forceinline__ int fpad(int p) { return p + ((p >> 5) << 2); }

// One directional contraction of a 512-point tile whose values were split
// once into hi and lo BF16 tiles (LDS, padded as above): four MFMAs, 16
// lines each.
__device__ __forceinline__ void contract_split(int dir, const unsigned short *hi, const unsigned short *lo, float *dst,
                                               bf16x8 bop, bool acc)
{
    const int lane = threadIdx.x & 63;
    const int m = lane & 15, g = lane >> 4, n = lane & 15;
    const unsigned short *src = g == 1 ? lo : hi;   // K groups: hi | lo | hi | (zero)
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int L = 16 * t + m;
        s16x8 a;
        if (dir == 0) {
            a = *(const s16x8 *)&src[hpad(L * 8)];
        } else {
#pragma unroll
            for (int q = 0; q < 8; ++q) a[q] = (short)src[hpad(line_point(dir, L, q))];
        }
        if (g == 3) a = s16x8{0, 0, 0, 0, 0, 0, 0, 0};
        f4 c = {0.f, 0.f, 0.f, 0.f};
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), bop, c, 0, 0, 0);
        // C: column n = entry (n < 8), rows 4 g + q = lines 16 t + 4 g + q
        if (n < 8) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int p = fpad(line_point(dir, 16 * t + 4 * g + q, n));
                if (acc)
                    dst[p] += c[q];
                else
                    dst[p] = c[q];
            }
        }
    }
}

template <bool GATHER, bool HELM>
__global__ void __launch_bounds__(64)
ax_bf16s_kernel(const float *__restrict__ uin, float *__restrict__ w, const unsigned short *__restrict__ G,
                const unsigned short *__restrict__ Bm, const float *__restrict__ scale,
                const unsigned short *__restrict__ Dhl, float h1, float h2, double *__restrict__ partial,
                const int32_t *__restrict__ skip, Lattice L)
{
    // G and B are half-precision values of one element, each array with its
    // own power-of-two scale; the scales multiply h1 and h2 (exact).
    if (skip && *skip) return;
    // LDS: u as padded hi | lo BF16 tiles (later the FP32 accumulator), the
    // FP32 derivatives (later the fluxes as padded hi | lo BF16 tiles), D hi | lo
    __shared__ __attribute__((aligned(16))) unsigned short suh[2 * kHalfTile];
    __shared__ __attribute__((aligned(16))) float sd[3 * kFloatTile];   // 3 FP32 tiles, or 6 BF16 tiles
    __shared__ unsigned short sD[128];
    static_assert(2 * kHalfTile * 2 >= kFloatTile * 4, "the accumulator fits the u tiles");
    static_assert(3 * kFloatTile * 4 >= 6 * kHalfTile * 2, "the flux tiles fit the derivative tiles");
    float *acc = (float *)&suh[0];
    unsigned short *sf = (unsigned short *)&sd[0];   // 6 tiles: flux a hi, lo at (2 a), (2 a + 1) kHalfTile
    const int lane = threadIdx.x;
    const int64_t e = xcd_block();
    int ex = 0, ey = 0, ez = 0;   // element coordinates (gather mode)
    if (GATHER) elem_coords(L, e, ex, ey, ez);
    const unsigned short *Ge = G + e * 6 * 512;
    u32x4 gq[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) gq[c] = __builtin_nontemporal_load((const u32x4 *)(Ge + c * 512) + lane);
    u32x4 bq = {0u, 0u, 0u, 0u};
    if (HELM) bq = __builtin_nontemporal_load((const u32x4 *)(Bm + e * 512) + lane);
    const float2 sc = ((const float2 *)scale)[e];
    sD[lane] = Dhl[lane];
    sD[64 + lane] = Dhl[64 + lane];
    // lane owns the 8-point row p = 8 lane + q: i = q, j = lane & 7, k = lane >> 3
    float uu[8];
    if (GATHER) {
        // gathered in point order (lane = i + 8 j within k-plane q, so a load
        // instruction spans 8 runs of 8 consecutive global nodes), then
        // turned into rows through the (still unused) derivative tile
        float ug[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) ug[q] = uin[gather_index32(L, ex, ey, ez, lane & 7, lane >> 3, q)];
#pragma unroll
        for (int q = 0; q < 8; ++q) sd[fpad(64 * q + lane)] = ug[q];
        __syncthreads();
        const float4 r0 = *(const float4 *)&sd[fpad(8 * lane)], r1 = *(const float4 *)&sd[fpad(8 * lane) + 4];
        uu[0] = r0.x; uu[1] = r0.y; uu[2] = r0.z; uu[3] = r0.w;
        uu[4] = r1.x; uu[5] = r1.y; uu[6] = r1.z; uu[7] = r1.w;
    } else {
        const float4 v0 = ((const float4 *)(uin + e * 512))[2 * lane], v1 = ((const float4 *)(uin + e * 512))[2 * lane + 1];
        uu[0] = v0.x; uu[1] = v0.y; uu[2] = v0.z; uu[3] = v0.w;
        uu[4] = v1.x; uu[5] = v1.y; uu[6] = v1.z; uu[7] = v1.w;
    }
    {
        s16x8 h, l;
        split8(uu, h, l);
        *(s16x8 *)&suh[hpad(8 * lane)] = h;
        *(s16x8 *)&suh[kHalfTile + hpad(8 * lane)] = l;
    }
    __syncthreads();
    // B operands (lane: column n, K rows 8 g + q)
    const int n = lane & 15, g = lane >> 4;
    s16x8 bFs = {0, 0, 0, 0, 0, 0, 0, 0}, bTs = {0, 0, 0, 0, 0, 0, 0, 0};
    if (n < 8 && g < 3) {
        const int off = g == 2 ? 64 : 0;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            bFs[q] = (short)sD[off + n * 8 + q];   // forward: out[n] = sum_c in[c] D[n][c]
            bTs[q] = (short)sD[off + q * 8 + n];   // transposed: out[n] = sum_c in[c] D[c][n]
        }
    }
    const bf16x8 bF = __builtin_bit_cast(bf16x8, bFs), bT = __builtin_bit_cast(bf16x8, bTs);
    contract_split(0, suh, suh + kHalfTile, sd, bF, false);
    contract_split(1, suh, suh + kHalfTile, sd + kFloatTile, bF, false);
    contract_split(2, suh, suh + kHalfTile, sd + 2 * kFloatTile, bF, false);
    __syncthreads();
    // G-combination in FP32; the fluxes are split once into hi | lo BF16
    float fl[3][8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int p = 8 * lane + q;
        const float ur = sd[fpad(p)], us = sd[kFloatTile + fpad(p)], ut = sd[2 * kFloatTile + fpad(p)];
        const float g11 = h_at(gq[0], q), g12 = h_at(gq[1], q), g13 = h_at(gq[2], q);
        const float g22 = h_at(gq[3], q), g23 = h_at(gq[4], q), g33 = h_at(gq[5], q);
        fl[0][q] = g11 * ur + g12 * us + g13 * ut;
        fl[1][q] = g12 * ur + g22 * us + g23 * ut;
        fl[2][q] = g13 * ur + g23 * us + g33 * ut;
    }
    __syncthreads();
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        s16x8 h, l;
        split8(fl[a], h, l);
        *(s16x8 *)&sf[(2 * a) * kHalfTile + hpad(8 * lane)] = h;
        *(s16x8 *)&sf[(2 * a + 1) * kHalfTile + hpad(8 * lane)] = l;
    }
    __syncthreads();
    // transposed contractions accumulated r, s, t (u itself is in registers)
    contract_split(0, sf + 0 * kHalfTile, sf + 1 * kHalfTile, acc, bT, false);
    __syncthreads();
    contract_split(1, sf + 2 * kHalfTile, sf + 3 * kHalfTile, acc, bT, true);
    __syncthreads();
    contract_split(2, sf + 4 * kHalfTile, sf + 5 * kHalfTile, acc, bT, true);
    __syncthreads();
    const float h1s = h1 * sc.x, h2s = h2 * sc.y;
    double dot = 0.0;
    float out[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        float v = h1s * acc[fpad(8 * lane + q)];
        if (HELM) v += h2s * h_at(bq, q) * uu[q];
        out[q] = v;
        if (partial) dot += (double)uu[q] * (double)v;
    }
    float4 *wo = (float4 *)(w + (GATHER ? (int64_t)rows_index32(L, ex, ey, ez, 0, lane & 7, lane >> 3) : e * 512 + 8 * lane));
    wo[0] = make_float4(out[0], out[1], out[2], out[3]);
    wo[1] = make_float4(out[4], out[5], out[6], out[7]);
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

hipError_t launch_ax_bf16s(const Mesh &m, float h1, float h2, const float *u, float *w, double *partial,
                           hipStream_t s, const int32_t *skip, bool gather)
{
    if (m.E == 0) return hipSuccess;
    if (m.N != 7) return hipErrorInvalidValue;
    const bool helm = h2 != 0.f;
    const dim3 grid((unsigned)m.E), block(64);
#define SEM_BF16S(G_, H_)                                                                                     \
    hipLaunchKernelGGL((ax_bf16s_kernel<G_, H_>), grid, block, 0, s, u, w, m.d_Gh, m.d_Bh, m.d_hscale, m.d_Dbf, \
                       h1, h2, partial, skip, m.lat)
    if (gather) {
        if (helm) SEM_BF16S(true, true);
        else SEM_BF16S(true, false);
    } else {
        if (helm) SEM_BF16S(false, true);
        else SEM_BF16S(false, false);
    }
#undef SEM_BF16S
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
