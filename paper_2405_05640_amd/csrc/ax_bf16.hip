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
// (K = [hi(8) | lo(8) | hi(8) | hi(8)]), B = [Dhi^T; Dhi^T; Dlo^T; 0] in output
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

// The BF16 hi and lo tiles in LDS are padded: slot p (0..511) sits at
// halfword p + 8 (p / 64), so each group of 8 lines (72 halfwords) starts 4
// banks after the previous one, and a lo tile starts kHalfTile halfwords (16
// banks mod 32) after its hi tile.  The scattered 16-bit stores of the s- and
// t-line-major tiles (lane (j, k) writes slots 64 k + 8 i + j or 64 j + 8 i +
// k) then hit 32 distinct banks per instruction, and lines stay 16-byte
// aligned.
constexpr int kHalfTile = 608;   // 512 + 8 * 8 padding + 32 bank offset
__device__ __forceinline__ int hpad(int p) { return p + ((p >> 6) << 3); }
// FP32 tiles (derivatives, accumulator): 4 floats of padding per 32, which
// spreads the scattered MFMA result writes over more banks while each 8-value
// row stays contiguous and 16-byte aligned; a tile spans kFloatTile floats.
constexpr int kFloatTile = 608;
__device__ __forceinline__ int fpad(int p) { return p + ((p >> 5) << 2); }

// Line-major BF16 tiles: a direction's tile stores each of its 64 lines as
// 8 contiguous halfwords (line L at hpad(8 L)), so every MFMA operand is one
// 16-byte LDS read.  Lines: r: L = j + 8 k (entries i), the point layout
// itself; s: L = i + 8 k (entries j); t: L = i + 8 j (entries k).
__device__ __forceinline__ int line_slot(int dir, int i, int j, int k)
{
    if (dir == 0) return hpad(i + 8 * j + 64 * k);
    if (dir == 1) return hpad(8 * (i + 8 * k) + j);
    return hpad(8 * (i + 8 * j) + k);
}

// Store a lane's row (j, k) of eight values (i = 0..7), split into hi | lo,
// into the line-major hi and lo tiles of direction dir.
__device__ __forceinline__ void store_split(int dir, const float (&v)[8], unsigned short *hi, unsigned short *lo,
                                            int j, int k)
{
    s16x8 h, l;
    split8(v, h, l);
    if (dir == 0) {
        *(s16x8 *)&hi[line_slot(0, 0, j, k)] = h;
        *(s16x8 *)&lo[line_slot(0, 0, j, k)] = l;
    } else {
        // entry i of the s- and t-lines through (j, k) sits 8 i halfwords
        // after entry 0 (the padding is per 64, and 8 i + j, 8 i + k < 64)
        unsigned short *ph = hi + line_slot(dir, 0, j, k), *pl = lo + line_slot(dir, 0, j, k);
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            ph[8 * i] = (unsigned short)h[i];
            pl[8 * i] = (unsigned short)l[i];
        }
    }
}

// fpad(line_point(dir, 16 t + 4 g + q, n)) for n < 8, g < 4, t < 4, q < 4,
// split into a lane part and a compile-time part (the padding's shifts do not
// carry across the two here, which the compiler cannot see by itself)
__device__ __forceinline__ int out_base(int dir, int g, int n)
{
    if (dir == 0) return 36 * g + n;
    if (dir == 1) return 72 * (g >> 1) + 8 * n + 4 * (n >> 2) + 4 * (g & 1);
    return 72 * n + 4 * g;
}
__device__ __forceinline__ int out_offset(int dir, int t, int q)
{
    if (dir == 0) return 144 * t + 8 * q;
    if (dir == 1) return 144 * t + q;
    return 16 * t + 4 * (t >> 1) + q;
}

// One directional contraction of a 512-point tile held as line-major hi and
// lo BF16 tiles: four MFMAs, 16 lines each.  Results (FP32) go to dst in the
// padded point layout, added when acc.  Every operand read is issued before
// the first result write, so dst may be the region that holds the source
// tiles (a wavefront's LDS operations complete in issue order).
__device__ __forceinline__ void contract_split(int dir, const unsigned short *hi, const unsigned short *lo, float *dst,
                                               bf16x8 bop, bool acc)
{
    const int lane = threadIdx.x & 63;
    const int m = lane & 15, g = lane >> 4, n = lane & 15;
    // K groups hi | lo | hi | hi; the B rows of the last group are zero, so
    // what it reads (finite tile values) does not contribute
    const unsigned short *src = g == 1 ? lo : hi;
    s16x8 a[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) a[t] = *(const s16x8 *)&src[hpad(8 * (16 * t + m))];
    f4 c[4];
#pragma unroll
    for (int t = 0; t < 4; ++t)
        c[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a[t]), bop, f4{0.f, 0.f, 0.f, 0.f},
                                                        0, 0, 0);
    __asm__ volatile("" ::: "memory");   // keep the writes after the reads
    // C: column n = entry (n < 8), rows 4 g + q = lines 16 t + 4 g + q
    const int base = out_base(dir, g, n);
    if (n < 8) {
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int p = base + out_offset(dir, t, q);
                if (acc)
                    dst[p] += c[t][q];
                else
                    dst[p] = c[t][q];
            }
    }
}

// The global loads of one element: G and B (half precision, 16 bytes per
// lane and array), the scales, and u (eight values per lane: in gather mode
// in point order, lane = i + 8 j within k-plane q, so a load instruction
// spans 8 runs of 8 consecutive global nodes; otherwise the lane's row).
template <bool GATHER, bool HELM>
struct SplitLoads {
    u32x4 gq[6];
    u32x4 bq;
    float2 sc;
    float u[8];
};

template <bool GATHER, bool HELM>
__device__ __forceinline__ void split_load(SplitLoads<GATHER, HELM> &ld, int64_t e, const float *__restrict__ uin,
                                           const unsigned short *__restrict__ G,
                                           const unsigned short *__restrict__ Bm, const float *__restrict__ scale,
                                           const Lattice &L, int lane)
{
    const unsigned short *Ge = G + e * 6 * 512;
#pragma unroll
    for (int c = 0; c < 6; ++c) ld.gq[c] = __builtin_nontemporal_load((const u32x4 *)(Ge + c * 512) + lane);
    ld.bq = u32x4{0u, 0u, 0u, 0u};
    if (HELM) ld.bq = __builtin_nontemporal_load((const u32x4 *)(Bm + e * 512) + lane);
    ld.sc = ((const float2 *)scale)[e];
    if (GATHER) {
        int ex, ey, ez;
        elem_coords(L, e, ex, ey, ez);
#pragma unroll
        for (int q = 0; q < 8; ++q) ld.u[q] = uin[gather_index32(L, ex, ey, ez, lane & 7, lane >> 3, q)];
    } else {
        const float4 v0 = ((const float4 *)(uin + e * 512))[2 * lane], v1 = ((const float4 *)(uin + e * 512))[2 * lane + 1];
        ld.u[0] = v0.x; ld.u[1] = v0.y; ld.u[2] = v0.z; ld.u[3] = v0.w;
        ld.u[4] = v1.x; ld.u[5] = v1.y; ld.u[6] = v1.z; ld.u[7] = v1.w;
    }
}

// One wavefront per element.  At most 96 VGPRs (five wavefronts per SIMD, as
// many as the 7.4 KB of LDS per wavefront allows).  Measured on the 32^3
// mesh: the same access pattern without the arithmetic streams in 53 us, the
// kernel takes about 72 us; neither fewer instructions (this layout issues
// about 540 VALU and 180 LDS instructions per element, against 930 and 240
// for strided operand gathers from one point-layout tile) nor more
// wavefronts per SIMD (4 -> 5) changed that, and two or four elements per
// wavefront with the next element's loads issued early were slower (fewer
// wavefronts, more registers).
template <bool GATHER, bool HELM>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(5)))
ax_bf16s_kernel(const float *__restrict__ uin, float *__restrict__ w, const unsigned short *__restrict__ G,
                const unsigned short *__restrict__ Bm, const float *__restrict__ scale,
                const unsigned short *__restrict__ Dhl, float h1, float h2, double *__restrict__ partial,
                const int32_t *__restrict__ skip, Lattice L)
{
    // G and B are half-precision values of one element, each array with its
    // own power-of-two scale; the scales multiply h1 and h2 (exact).
    if (skip && *skip) return;
    // LDS: three regions, one per direction, each one FP32 tile or a hi | lo
    // pair of BF16 tiles, reused through the phases (u tiles -> derivatives
    // -> flux tiles -> accumulator), plus D hi | lo: 7.4 KB per wavefront
    __shared__ __attribute__((aligned(16))) float lds[3 * kFloatTile];
    __shared__ unsigned short sD[128];
    static_assert(kFloatTile * 4 >= 2 * kHalfTile * 2, "a hi | lo tile pair fits a region");
    float *R[3] = {lds, lds + kFloatTile, lds + 2 * kFloatTile};
    auto hiT = [&](int q) { return (unsigned short *)R[q]; };
    auto loT = [&](int q) { return (unsigned short *)R[q] + kHalfTile; };
    const int lane = threadIdx.x & 63;   // (the mask lets the compiler fold lane-constant address terms)
    const int j = lane & 7, k = lane >> 3;   // lane owns the 8-point row (j, k), i = 0..7
    const int64_t e = xcd_block();
    SplitLoads<GATHER, HELM> cur;
    split_load(cur, e, uin, G, Bm, scale, L, lane);
    sD[lane] = Dhl[lane];
    sD[64 + lane] = Dhl[64 + lane];
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
    {
        int ex = 0, ey = 0, ez = 0;   // element coordinates (gather mode)
        if (GATHER) elem_coords(L, e, ex, ey, ez);
        float uu[8];
        if (GATHER) {
            // the point-order gather turned into rows through region 0
#pragma unroll
            for (int q = 0; q < 8; ++q) R[0][fpad(lane) + 72 * q] = cur.u[q];   // = fpad(64 q + lane)
            __syncthreads();
            const float4 r0 = *(const float4 *)&R[0][fpad(8 * lane)], r1 = *(const float4 *)&R[0][fpad(8 * lane) + 4];
            uu[0] = r0.x; uu[1] = r0.y; uu[2] = r0.z; uu[3] = r0.w;
            uu[4] = r1.x; uu[5] = r1.y; uu[6] = r1.z; uu[7] = r1.w;
            __syncthreads();   // the rows are read before region 0 takes the u tiles
        } else {
#pragma unroll
            for (int q = 0; q < 8; ++q) uu[q] = cur.u[q];
        }
        // u split once, stored line-major per direction d in region d
        store_split(0, uu, hiT(0), loT(0), j, k);
        store_split(1, uu, hiT(1), loT(1), j, k);
        store_split(2, uu, hiT(2), loT(2), j, k);
        __syncthreads();
        // derivative d replaces the u tiles of direction d in region d
        contract_split(0, hiT(0), loT(0), R[0], bF, false);
        contract_split(1, hiT(1), loT(1), R[1], bF, false);
        contract_split(2, hiT(2), loT(2), R[2], bF, false);
        __syncthreads();
        // G-combination in FP32
        float fl[3][8];
        const int rowp = 8 * lane + 4 * (lane >> 2);   // fpad(8 lane + q) = rowp + q
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int p = rowp + q;
            const float ur = R[0][p], us = R[1][p], ut = R[2][p];
            const float g11 = h_at(cur.gq[0], q), g12 = h_at(cur.gq[1], q), g13 = h_at(cur.gq[2], q);
            const float g22 = h_at(cur.gq[3], q), g23 = h_at(cur.gq[4], q), g33 = h_at(cur.gq[5], q);
            fl[0][q] = g11 * ur + g12 * us + g13 * ut;
            fl[1][q] = g12 * ur + g22 * us + g23 * ut;
            fl[2][q] = g13 * ur + g23 * us + g33 * ut;
        }
        __syncthreads();
        // fluxes split once, line-major for their own direction d, in region d
        store_split(0, fl[0], hiT(0), loT(0), j, k);
        store_split(1, fl[1], hiT(1), loT(1), j, k);
        store_split(2, fl[2], hiT(2), loT(2), j, k);
        __syncthreads();
        // transposed contractions accumulated r, s, t into region 0 (u itself is
        // in registers)
        float *acc = R[0];
        contract_split(0, hiT(0), loT(0), acc, bT, false);
        __syncthreads();
        contract_split(1, hiT(1), loT(1), acc, bT, true);
        __syncthreads();
        contract_split(2, hiT(2), loT(2), acc, bT, true);
        __syncthreads();
        const float h1s = h1 * cur.sc.x, h2s = h2 * cur.sc.y;
        double dot = 0.0;
        float out[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            float v = h1s * acc[rowp + q];
            if (HELM) v += h2s * h_at(cur.bq, q) * uu[q];
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
