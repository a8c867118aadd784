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
// Inference layout (one element per 512-thread workgroup; every layer on
// the BF16 matrix cores with FP32 accumulation, each wavefront owning four
// blocks of 16 positions, inputs and weights rounded to BF16):
//  - layer 1 (2 -> 16): K = (channel, tap) = 54 terms padded to 64, two
//    16x16x32 MFMAs per block;
//  - layer 2 (16 -> 16, 27 taps): K = (tap, channel) = 432 padded to 448,
//    fourteen 16x16x32 MFMAs per block, two taps of 16 channels each.
//    Activations sit in LDS channel-last with a zero halo (10^3 positions x
//    16 BF16, 48-byte pitch = 48 KB), so every A operand is one 16-byte LDS
//    read and every activation store one 32-bit word;
//  - layer 3 (16 -> 1): the same A operands against a B whose column 0 holds
//    W3 (15 of 16 columns idle, still far fewer cycles than 432 vector FMAs
//    per position).
// (Layers 1 and 3 on the vector units, 16-bit activation stores into a
// 32-byte pitch and 16x16x16 MFMAs took 178 us per launch on the 16^3
// channel; rocprofv3 counted 4.8e7 LDS bank-conflict cycles against 1.4e7
// active LDS cycles.)
// Training keeps everything in FP32 (the accuracy reference of the BF16
// inference path); per-element weight gradients are reduced over elements
// in a fixed order.
#include "cg.hpp"
#include "nn.hpp"

namespace sem {
namespace nn {

typedef __attribute__((__vector_size__(4 * sizeof(short)))) short bf16x4;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f4;
typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(8 * sizeof(short)))) short s16x8;
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __attribute__((__vector_size__(4 * sizeof(unsigned)))) unsigned u32x4;

constexpr int NP = 8, P3 = 512, PD = 10, PD3 = 1000;
// channel stride of the FP32 channel-major activation tiles of the training
// path: 1001 floats, so that 16 channels at one position fall on 16
// different banks (with 1000, channels 4 apart share a bank)
constexpr int CS = 1001;

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

// The two features at this thread's point of element e from assembled r and
// dinv (r / max|r| and dinv r / max|dinv r| over the element), t_e, and
// whether the element is live (both maxima positive).
template <typename TR>
__device__ void feature_values(const TR *__restrict__ rg, const TR *__restrict__ dinvg, const Lattice &L, int64_t e,
                               float *red, float &x0, float &x1, float &t_out, bool &live)
{
    const int p = threadIdx.x, i = p & 7, j = (p >> 3) & 7, k = p >> 6;
    const int64_t g = lattice_glo(L, e, i, j, k);
    const double r = (double)rg[g];
    const double q = (double)dinvg[g] * r;
    const float s = block_max512((float)fabs(r), red);
    const float t = block_max512((float)fabs(q), red);
    live = (s > 0.f) && (t > 0.f);
    x0 = live ? (float)(r / (double)s) : 0.f;
    x1 = live ? (float)(q / (double)t) : 0.f;
    t_out = t;
}

// Features of element e into Xs[2][PD3] (zero halo must already be in place).
template <typename TR>
__device__ void load_features(const TR *__restrict__ rg, const TR *__restrict__ dinvg, const Lattice &L,
                              int64_t e, float *Xs, float *red, float &t_out, bool &live)
{
    const int p = threadIdx.x, i = p & 7, j = (p >> 3) & 7, k = p >> 6;
    float x0, x1;
    feature_values(rg, dinvg, L, e, red, x0, x1, t_out, live);
    if (live) {
        Xs[pidx(k, j, i)] = x0;
        Xs[PD3 + pidx(k, j, i)] = x1;
    }
}

__device__ __forceinline__ int tap_off(int tap)
{
    const int dk = tap / 9 - 1, dj = (tap / 3) % 3 - 1, di = tap % 3 - 1;
    return (dk * PD + dj) * PD + di;
}

// ---------------------------------------------------------------- inference

// value of the neighbouring lane (lane ^ 1), a DPP move (no LDS traffic)
__device__ __forceinline__ float lane_xor1(float v)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1, 0xF, 0xF, false));
}

// two floats -> packed BF16 pair (round to nearest even, one instruction)
__device__ __forceinline__ unsigned pack_bf16(float lo, float hi)
{
    return __builtin_bit_cast(unsigned, __builtin_convertvector((f32x2){lo, hi}, bf16x2));
}

// LDS row of one position of the BF16 activation tile: 16 channels plus 8
// halfwords of padding.  The 48-byte pitch keeps the 16-byte operand reads
// aligned and puts positions 4 apart (the rows a C tile's lanes write
// together) on different banks; a 32-byte pitch put them on the same eight.
constexpr int YS = 24;
// matrix-core weight operands (BF16, built from the FP32 master weights):
//   layer 2 [tap 0..27][o][c] (tap 27 zero), layer 3 [tap 0..27][c],
//   layer 1 [o][k], k = 2 tap + c (k = 54..63 zero)
constexpr int kW2B = 28 * 256, kW3B = 28 * 16, kW1B = 16 * 64;

// Point (i + 8 j + 64 k) of MFMA row pos of the inference tiles.  A block of
// 16 rows is i = 0..7 on two lines j0 and j0 + 4 of one k-plane (not two
// adjacent lines): with the 48-byte pitch, the 16 operand reads of a lane
// group then cover 64 distinct banks, where lines j0 and j0 + 1 overlap on
// two rows.
__device__ __forceinline__ int row_point(int pos)
{
    const int bl = pos >> 4, m = pos & 15;
    return (m & 7) + 8 * ((bl & 3) + 4 * (m >> 3)) + 64 * (bl >> 2);
}
__device__ __forceinline__ int row_pidx(int pos)
{
    const int pt = row_point(pos);
    return pidx(pt >> 6, (pt >> 3) & 7, pt & 7);
}

// Padded-tile index of halo position h (0..487): the k = 0 and k = 9 planes,
// then per interior plane the j = 0 and j = 9 lines and the i = 0, 9 ends of
// the interior lines.
constexpr int kHalo = PD3 - P3;
__device__ __forceinline__ int halo_index(int h)
{
    if (h < PD * PD) return h;
    if (h < 2 * PD * PD) return (PD - 1) * PD * PD + (h - PD * PD);
    const int q = h - 2 * PD * PD, k = 1 + q / 36, r = q % 36;
    int j, i;
    if (r < PD) {
        j = 0; i = r;
    } else if (r < 2 * PD) {
        j = PD - 1; i = r - PD;
    } else {
        j = 1 + ((r - 2 * PD) >> 1); i = ((r - 2 * PD) & 1) * (PD - 1);
    }
    return (k * PD + j) * PD + i;
}

// Activation store from an MFMA C tile (lane (kq, n): rows 4 kq + q, column
// n = channel): each even lane packs channels (n, n + 1) of rows q = 0, 1,
// each odd lane channels (n - 1, n) of rows q = 2, 3, so every store is one
// 32-bit word (ReLU, then BF16).
__device__ __forceinline__ void store_tile(unsigned short *Ys, const f4 &acc, int row0, int kq, int n16)
{
    float x[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) x[q] = lane_xor1(acc[q]);
    const bool odd = n16 & 1;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int q = odd ? 2 + h : h;
        const float own = fmaxf(acc[q], 0.f), other = fmaxf(x[q], 0.f);
        const int at = row_pidx(row0 + 4 * kq + q) * YS + (n16 & ~1);
        *(unsigned *)&Ys[at] = odd ? pack_bf16(other, own) : pack_bf16(own, other);
    }
}

// 16 x 16 x 432 contraction of a layer with 16 input channels over the 27
// taps: 14 MFMAs of K = 32 (two taps of 16 channels; the 28th tap is zero).
// Lane (g, m): A row m = position pb[b], K group g = tap 2 st + g / 2,
// channels 8 (g % 2) .. + 7.
__device__ __forceinline__ void conv16(const unsigned short *Ys, const int (&pb)[4], int g, const bf16x8 (&bop)[14],
                                       f4 (&acc)[4])
{
#pragma unroll
    for (int st = 0; st < 14; ++st) {
        const int tap = 2 * st + (g >> 1);
        const int off = (tap < 27 ? tap_off(tap) : 0) * YS + 8 * (g & 1);
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            s16x8 a = *(const s16x8 *)&Ys[pb[b] * YS + off];
            if (tap >= 27) a = s16x8{0, 0, 0, 0, 0, 0, 0, 0};
            acc[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), bop[st], acc[b], 0, 0, 0);
        }
    }
}

template <typename TR>
__global__ void __launch_bounds__(512)
infer_kernel(const TR *__restrict__ rg, const TR *__restrict__ dinvg, Lattice L, const unsigned short *__restrict__ Wb,
             float *__restrict__ c_out, const int32_t *__restrict__ skip)
{
    if (skip && *skip) return;
    // features as BF16 pairs (x0 in the low half), one word per position
    __shared__ unsigned Xp[PD3];
    __shared__ __attribute__((aligned(16))) unsigned short Ys[PD3 * YS];
    __shared__ float red[8];
    const int p = threadIdx.x;
    const int64_t e = xcd_block();
    // zero halo (the interior is written before it is read: features here,
    // every activation channel by store_tile)
    if (p < kHalo) {
        const int h = halo_index(p);
        Xp[h] = 0u;
        u32x4 *y = (u32x4 *)&Ys[h * YS];   // channels 0..15 (the 8 padding halfwords are never read)
        y[0] = u32x4{0u, 0u, 0u, 0u};
        y[1] = u32x4{0u, 0u, 0u, 0u};
    }
    float t, x0, x1;
    bool live;
    __syncthreads();
    feature_values(rg, dinvg, L, e, red, x0, x1, t, live);
    if (!live) {   // uniform across the block
        c_out[e * P3 + p] = 0.f;
        return;
    }
    Xp[pidx(p >> 6, (p >> 3) & 7, p & 7)] = pack_bf16(x0, x1);
    __syncthreads();
    // Each wavefront owns four blocks of 16 positions (rows of the MFMA
    // tiles); lane = (g, n): A row / C column n = lane & 15, K group g.
    const int lane = p & 63, wave = p >> 6;
    const int n16 = lane & 15, g = lane >> 4;
    const unsigned short *W2b = Wb, *W3b = Wb + kW2B, *W1b = Wb + kW2B + kW3B;
    int pb[4];   // padded-tile index of this lane's A row in each block
#pragma unroll
    for (int b = 0; b < 4; ++b) pb[b] = row_pidx((wave * 4 + b) * 16 + n16);
    // layer 1: 2 -> 16, K = (tap, channel) = 54 terms padded to 64, two
    // 16x16x32 BF16 MFMAs per block: the lane's K entries 8 g .. 8 g + 7 of
    // step st are taps 16 st + 4 g + h (h < 4), each one feature word.  The
    // padding taps (27..31) read tap 0 again; their weights are zero.
    {
        int koff[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int tap = 16 * (q >> 2) + 4 * g + (q & 3);
            koff[q] = tap_off(tap < 27 ? tap : 0);
        }
        f4 acc[4];
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[b] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int st = 0; st < 2; ++st) {
            const bf16x8 bop = *(const bf16x8 *)&W1b[n16 * 64 + 32 * st + 8 * g];
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                unsigned w[4];
#pragma unroll
                for (int h = 0; h < 4; ++h) w[h] = Xp[pb[b] + koff[4 * st + h]];
                const bf16x8 aop = __builtin_bit_cast(bf16x8, (u32x4){w[0], w[1], w[2], w[3]});
                acc[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aop, bop, acc[b], 0, 0, 0);
            }
        }
#pragma unroll
        for (int b = 0; b < 4; ++b) store_tile(Ys, acc[b], (wave * 4 + b) * 16, g, n16);
    }
    __syncthreads();
    // layer 2: 16 -> 16 (B: the tap's 16 x 16 block, output channel n16)
    f4 acc[4];
    {
        bf16x8 bop[14];
#pragma unroll
        for (int st = 0; st < 14; ++st)
            bop[st] = *(const bf16x8 *)&W2b[((2 * st + (g >> 1)) * 16 + n16) * 16 + 8 * (g & 1)];
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[b] = f4{0.f, 0.f, 0.f, 0.f};
        conv16(Ys, pb, g, bop, acc);
    }
    __syncthreads();   // every wave has finished reading layer-1 activations
#pragma unroll
    for (int b = 0; b < 4; ++b) store_tile(Ys, acc[b], (wave * 4 + b) * 16, g, n16);
    __syncthreads();
    // layer 3: 16 -> 1 as a 16 -> 16 layer whose B has only column 0 (W3)
    {
        bf16x8 bop[14];
#pragma unroll
        for (int st = 0; st < 14; ++st) {
            bop[st] = *(const bf16x8 *)&W3b[(2 * st + (g >> 1)) * 16 + 8 * (g & 1)];
            if (n16 != 0) bop[st] = __builtin_bit_cast(bf16x8, s16x8{0, 0, 0, 0, 0, 0, 0, 0});
        }
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[b] = f4{0.f, 0.f, 0.f, 0.f};
        conv16(Ys, pb, g, bop, acc);
    }
    // column 0 lives in lanes n16 == 0; stage through LDS (the feature tile
    // is free) so that the output store is coalesced
    float *Xo = (float *)Xp;
    if (n16 == 0) {
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
            for (int q = 0; q < 4; ++q) Xo[row_point((wave * 4 + b) * 16 + 4 * g + q)] = acc[b][q];
    }
    __syncthreads();
    c_out[e * P3 + p] = t * Xo[p];
}

// ---------------------------------------------------------------- training (FP32)

// Forward of element e in FP32; keeps X (Xs), Y1 (Y1s, channel-major padded)
// and Y2 (Y2s) in LDS.  Returns y3 at this thread's position.  W1t, W2t:
// layers 1 and 2 as [c][tap][o], so that the 16 output-channel weights of an
// (input channel, tap) pair are one contiguous wave-uniform load.
__device__ float fwd32(const float *__restrict__ W1t, const float *__restrict__ W2t, const float *__restrict__ W3,
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
            for (int o = 0; o < 16; ++o) acc[o] += W1t[(c * 27 + tap) * 16 + o] * x;
        }
#pragma unroll
    for (int o = 0; o < 16; ++o) Y1s[o * CS + base] = fmaxf(acc[o], 0.f);
    __syncthreads();
#pragma unroll
    for (int o = 0; o < 16; ++o) acc[o] = 0.f;
    for (int c = 0; c < 16; ++c)
        for (int tap = 0; tap < 27; ++tap) {
            const float x = Y1s[c * CS + base + tap_off(tap)];
#pragma unroll
            for (int o = 0; o < 16; ++o) acc[o] += W2t[(c * 27 + tap) * 16 + o] * x;
        }
#pragma unroll
    for (int o = 0; o < 16; ++o) Y2s[o * CS + base] = fmaxf(acc[o], 0.f);
    __syncthreads();
    float y = 0.f;
    for (int c = 0; c < 16; ++c)
        for (int tap = 0; tap < 27; ++tap) y += W3[c * 27 + tap] * Y2s[c * CS + base + tap_off(tap)];
    return y;
}

// One element of the loss gradient.  gz: dL/dz on assembled nodes; the
// element's output gradient is g3 = t_e gz[glo] / mult (0 on Dirichlet nodes).
// Writes the element's weight gradient (kParams floats) to dW[e].
template <typename TR>
__global__ void __launch_bounds__(512)
train_kernel(const TR *__restrict__ rg, const TR *__restrict__ dinvg, const double *__restrict__ gz, Lattice L,
             const float *__restrict__ W1t, const float *__restrict__ W2t, const float *__restrict__ W3,
             const float *__restrict__ W2u, float *__restrict__ dW, const float *__restrict__ act)
{
    __shared__ float Xs[2 * PD3];
    __shared__ float Y1s[16 * CS];
    __shared__ float Bs[16 * CS];   // Y2, then g2, then g1
    __shared__ float g3s[PD3];
    __shared__ float red[8];
    const int p = threadIdx.x, i = p & 7, j = (p >> 3) & 7, k = p >> 6;
    const int base = pidx(k, j, i);
    const int64_t e = xcd_block();
    float *dWe = dW + e * kParams;
    for (int q = p; q < 2 * PD3; q += 512) Xs[q] = 0.f;
    for (int q = p; q < 16 * CS; q += 512) { Y1s[q] = 0.f; Bs[q] = 0.f; }
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
    if (act) {   // the forward activations the loss's forward pass stored
        const float *a = act + e * (32 * P3);
#pragma unroll
        for (int c = 0; c < 16; ++c) {
            Y1s[c * CS + base] = a[c * P3 + p];
            Bs[c * CS + base] = a[(16 + c) * P3 + p];
        }
        __syncthreads();
    } else {
        fwd32(W1t, W2t, W3, Xs, Y1s, Bs);
    }
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
            s += g3s[b] * Bs[c * CS + b + off];
        }
        dWe[kW1 + kW2 + w] = s;
    }
    // g2[c][pos] = (sum_tap W3[c][tap] g3[pos - tap]) * (Y2 > 0)
    float g2v[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) {
        float s = 0.f;
        for (int tap = 0; tap < 27; ++tap) s += W3[c * 27 + tap] * g3s[base - tap_off(tap)];
        g2v[c] = Bs[c * CS + base] > 0.f ? s : 0.f;
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 16; ++c) Bs[c * CS + base] = g2v[c];
    __syncthreads();
    // dW2[o][c][tap] = sum_pos g2[o][pos] Y1[c][pos+tap] on the FP32 matrix
    // cores: per tap a 16 x 16 x 512 product, 128 16x16x4 MFMAs (A = g2:
    // row o, K = position; B = the shifted Y1: K = position, column c); wave
    // w takes taps w, w + 8, ... (the per-weight loop over 512 positions it
    // replaces issued 13,824 LDS reads per thread)
    {
        const int lane = p & 63, wave = p >> 6, n16 = lane & 15, kq = lane >> 4;
        for (int tap = wave; tap < 27; tap += 8) {
            const int off = tap_off(tap);
            f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll 4
            for (int st = 0; st < 128; ++st) {
                const int pos = 4 * st + kq;
                const int b = pidx(pos >> 6, (pos >> 3) & 7, pos & 7);
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(Bs[n16 * CS + b], Y1s[n16 * CS + b + off], acc, 0, 0, 0);
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) dWe[kW1 + ((4 * kq + q) * 16 + n16) * 27 + tap] = acc[q];
        }
    }
    // g1[c][pos] = (sum_o sum_tap W2[o][c][tap] g2[o][pos - tap]) * (Y1 > 0)
    float g1v[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) g1v[c] = 0.f;
    for (int o = 0; o < 16; ++o)
        for (int tap = 0; tap < 27; ++tap) {
            const float gv = Bs[o * CS + base - tap_off(tap)];
#pragma unroll
            for (int c = 0; c < 16; ++c) g1v[c] += W2u[(o * 27 + tap) * 16 + c] * gv;
        }
#pragma unroll
    for (int c = 0; c < 16; ++c) g1v[c] = Y1s[c * CS + base] > 0.f ? g1v[c] : 0.f;
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 16; ++c) Bs[c * CS + base] = g1v[c];
    __syncthreads();
    // dW1[o][c][tap] = sum_pos g1[o][pos] X[c][pos+tap]
    for (int w = p; w < kW1; w += 512) {
        const int o = w / 54, c = (w / 27) % 2, off = tap_off(w % 27);
        float s = 0.f;
        for (int q = 0; q < P3; ++q) {
            const int b = pidx(q >> 6, (q >> 3) & 7, q & 7);
            s += Bs[o * CS + b] * Xs[c * PD3 + b + off];
        }
        dWe[w] = s;
    }
}

// FP32 forward writing c = t y3 (the training-path smoother output)
template <typename TR>
__global__ void __launch_bounds__(512)
infer32_kernel(const TR *__restrict__ rg, const TR *__restrict__ dinvg, Lattice L, const float *__restrict__ W1t,
               const float *__restrict__ W2t, const float *__restrict__ W3, float *__restrict__ c_out,
               float *__restrict__ act)
{
    __shared__ float Xs[2 * PD3];
    __shared__ float Y1s[16 * CS];
    __shared__ float Y2s[16 * CS];
    __shared__ float red[8];
    const int p = threadIdx.x;
    const int64_t e = xcd_block();
    for (int q = p; q < 2 * PD3; q += 512) Xs[q] = 0.f;
    for (int q = p; q < 16 * CS; q += 512) { Y1s[q] = 0.f; Y2s[q] = 0.f; }
    float t;
    bool live;
    __syncthreads();
    load_features(rg, dinvg, L, e, Xs, red, t, live);
    if (!live) {
        c_out[e * P3 + p] = 0.f;
        return;
    }
    __syncthreads();
    const float y = fwd32(W1t, W2t, W3, Xs, Y1s, Y2s);
    c_out[e * P3 + p] = t * y;
    if (act) {   // Y1 and Y2 at this thread's position, for the training kernel
        const int base = pidx(p >> 6, (p >> 3) & 7, p & 7);
        float *a = act + e * (32 * P3);
#pragma unroll
        for (int c = 0; c < 16; ++c) {
            a[c * P3 + p] = Y1s[c * CS + base];
            a[(16 + c) * P3 + p] = Y2s[c * CS + base];
        }
    }
}

// Weight gradient summed over elements in two fixed-order stages: stage 1
// sums chunk blockIdx.y of the elements for every weight (coalesced rows of
// dW), stage 2 the kGradChunks chunk sums.  (One thread per weight looping
// over all elements took 1.06 ms per training step on the 16^3 channel.)
__global__ void __launch_bounds__(256)
grad_chunks_kernel(const float *__restrict__ dW, int64_t E, double *__restrict__ part)
{
    const int w = blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= kParams) return;
    const int64_t chunk = (E + kGradChunks - 1) / kGradChunks;
    const int64_t lo = blockIdx.y * chunk, hi = lo + chunk < E ? lo + chunk : E;
    double s = 0.0;
    for (int64_t e = lo; e < hi; ++e) s += (double)dW[e * kParams + w];
    part[(int64_t)blockIdx.y * kParams + w] = s;
}

// out[w] = scale * sum over chunks of part[chunk][w] (fixed order)
__global__ void __launch_bounds__(256)
grad_finish_kernel(const double *__restrict__ part, double scale, float *__restrict__ out)
{
    const int w = blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= kParams) return;
    double s = 0.0;
    for (int c = 0; c < kGradChunks; ++c) s += part[(int64_t)c * kParams + w];
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

// FP32 master weights -> the BF16 matrix-core operands of the inference
// kernel (layouts at kW2B): W2 [o][c][tap] -> [tap][o][c], W3 [c][tap] ->
// [tap][c], W1 [o][c][tap] -> [o][27 c + tap]; padding entries are zero
__global__ void pack_w2_kernel(const float *__restrict__ W, unsigned short *__restrict__ Wb)
{
    const int w = blockIdx.x * blockDim.x + threadIdx.x;
    if (w < kW2B) {
        const int tap = w / 256, o = (w / 16) % 16, c = w % 16;
        Wb[w] = tap < 27 ? f2bf(W[kW1 + (o * 16 + c) * 27 + tap]) : 0;
    } else if (w < kW2B + kW3B) {
        const int v = w - kW2B, tap = v / 16, c = v % 16;
        Wb[w] = tap < 27 ? f2bf(W[kW1 + kW2 + c * 27 + tap]) : 0;
    } else if (w < kW2B + kW3B + kW1B) {
        const int v = w - kW2B - kW3B, o = v / 64, k = v % 64;
        Wb[w] = k < 54 ? f2bf(W[o * 54 + 27 * (k & 1) + (k >> 1)]) : 0;
    }
}

// FP32 master weights -> the FP32 layouts of the training loops (at Wt):
// W1t, W2t [c][tap][o] (the forward's output channels contiguous), W2u
// [o][tap][c] (the backward's input channels contiguous)
__global__ void pack_t_kernel(const float *__restrict__ W, float *__restrict__ Wt)
{
    const int w = blockIdx.x * blockDim.x + threadIdx.x;
    if (w < kW1) {
        const int c = w / (27 * 16), tap = (w / 16) % 27, o = w % 16;
        Wt[w] = W[(o * 2 + c) * 27 + tap];
    } else if (w < kW1 + kW2) {
        const int v = w - kW1, c = v / (27 * 16), tap = (v / 16) % 27, o = v % 16;
        Wt[w] = W[kW1 + (o * 16 + c) * 27 + tap];
    } else if (w < kW1 + 2 * kW2) {
        const int v = w - kW1 - kW2, o = v / (27 * 16), tap = (v / 16) % 27, c = v % 16;
        Wt[w] = W[kW1 + (o * 16 + c) * 27 + tap];
    }
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
    hipLaunchKernelGGL((nn::infer_kernel<TR>), dim3((unsigned)m.E), dim3(512), 0, s, rg, dinvg, m.lat, sm.W2b,
                       c_local, skip);
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
                   float *dW_elem, double scale, float *grad, hipStream_t s, const float *act)
{
    hipLaunchKernelGGL((nn::train_kernel<double>), dim3((unsigned)m.E), dim3(512), 0, s, rg, dinvg, gz, m.lat, sm.Wt,
                       sm.Wt + kW1, sm.W + kW1 + kW2, sm.Wt + kW1 + kW2, dW_elem, act);
    hipLaunchKernelGGL(nn::grad_chunks_kernel, dim3((kParams + 255) / 256, kGradChunks), dim3(256), 0, s, dW_elem,
                       m.E, sm.gpart);
    hipLaunchKernelGGL(nn::grad_finish_kernel, dim3((kParams + 255) / 256), dim3(256), 0, s, sm.gpart, scale, grad);
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
    hipLaunchKernelGGL(nn::pack_w2_kernel, dim3((nn::kW2B + nn::kW3B + nn::kW1B + 255) / 256), dim3(256), 0, s, sm.W,
                       sm.W2b);
    hipLaunchKernelGGL(nn::pack_t_kernel, dim3((kWtFloats + 255) / 256), dim3(256), 0, s, sm.W, sm.Wt);
    return hipGetLastError();
}

hipError_t nn_infer32(const Smoother &sm, const Mesh &m, const double *rg, const double *dinvg, float *c_local,
                      hipStream_t s, float *act)
{
    hipLaunchKernelGGL((nn::infer32_kernel<double>), dim3((unsigned)m.E), dim3(512), 0, s, rg, dinvg, m.lat, sm.Wt,
                       sm.Wt + kW1, sm.W + kW1 + kW2, c_local, act);
    return hipGetLastError();
}

template hipError_t nn_infer<double>(const Smoother &, const Mesh &, const double *, const double *, float *,
                                     hipStream_t, const int32_t *);
template hipError_t nn_assemble_z<double>(const Mesh &, const double *, const double *, const float *, double *,
                                          hipStream_t, const int32_t *, const double *);

}  // namespace sem
