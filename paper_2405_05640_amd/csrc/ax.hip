// ax.hip -- matrix-free local spectral-element operator for gfx950.
//
//   w_e = h1 * sum_{a,b in {r,s,t}} D_a^T (G_ab o D_b u_e) + h2 * B o u_e
//
// (Deville, Fischer & Mund 2002, sec. 4.4; the paper's element-by-element,
// matrix-free operator of section 3.1, which the paper's section 4.2 notes is
// memory bound).
//
// Three designs: thread-per-point kernels for N <= 7 (one point per thread in
// FP64; in FP32 at N = 7, several points per thread sharing an (i, j) pencil),
// and for higher orders the k-pencil kernel (one (N+1)x(N+1) workgroup per
// element):
//  - the workgroup is the (N+1)x(N+1) "i,j" plane of an element: lane (i,j)
//    owns the k-pencil u(i,j,0..N) and w(i,j,0..N) in registers;
//  - each k-slice of u is staged once in LDS; the r and s derivatives read
//    the slice from LDS, the t derivative is a register contraction over the
//    pencil; the same holds for the transposed contractions;
//  - every global access is a whole (N+1)^2 slice: at N = 7 one wave reads
//    512 contiguous bytes per field per slice (fully coalesced), so u, the six
//    geometric factors, B and w each stream from HBM exactly once;
//  - the geometric factors of slice k+1 are requested before slice k is
//    computed, so HBM latency overlaps the LDS/FMA work.
#include "sem_internal.hpp"

namespace sem {
namespace {


// GATHER: u is an assembled vector (one value per global node) read through
// the closed-form numbering and w is written in the row layout; otherwise u
// and w are local [E][P].
template <typename T, int NP, bool HELM, bool DOT, bool GATHER>
__global__ void __launch_bounds__(NP * NP)
ax_kernel(const T *__restrict__ u, T *__restrict__ w, const T *__restrict__ G,
          const T *__restrict__ Bm, const T *__restrict__ Dg, T h1, T h2,
          double *__restrict__ partial, const int32_t *__restrict__ skip, Lattice L)
{
    if (skip && *skip) return;   // uniform across the grid
    constexpr int P2 = NP * NP;
    constexpr int P3 = NP * NP * NP;
    __shared__ T sD[P2];
    __shared__ T su[P2];
    __shared__ T sr[P2];
    __shared__ T ss[P2];

    const int t = threadIdx.x;
    const int i = t % NP;
    const int j = t / NP;
    const int64_t e = xcd_block();
    int ex = 0, ey = 0, ez = 0;   // element coordinates (gather mode)
    if (GATHER) elem_coords(L, e, ex, ey, ez);
    const T *Ge = G + e * (6 * P3);

    sD[t] = Dg[t];

    T ru[NP], rw[NP];
    if (GATHER) {
        int64_t gi = ex * (NP - 1) + i, gj = ey * (NP - 1) + j;
        if (gi >= L.nx) gi -= L.nx;
        if (gj >= L.ny) gj -= L.ny;
        const int64_t base = gi + L.nx * gj, plane = L.nx * L.ny;
#pragma unroll
        for (int k = 0; k < NP; ++k) {
            int64_t gk = ez * (NP - 1) + k;
            if (gk >= L.nz) gk -= L.nz;
            ru[k] = u[base + plane * gk];
            rw[k] = T(0);
        }
    } else {
        const T *ue = u + e * P3;
#pragma unroll
        for (int k = 0; k < NP; ++k) {
            ru[k] = ue[k * P2 + t];
            rw[k] = T(0);
        }
    }
    T g[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) g[q] = Ge[q * P3 + t];

    __syncthreads();
    T Di[NP], Dj[NP], DiT[NP], DjT[NP];
#pragma unroll
    for (int m = 0; m < NP; ++m) {
        Di[m] = sD[i * NP + m];
        Dj[m] = sD[j * NP + m];
        DiT[m] = sD[m * NP + i];
        DjT[m] = sD[m * NP + j];
    }

#pragma unroll
    for (int k = 0; k < NP; ++k) {
        // prefetch the next slice's geometric factors
        T gn[6];
        if (k + 1 < NP) {
#pragma unroll
            for (int q = 0; q < 6; ++q) gn[q] = Ge[q * P3 + (k + 1) * P2 + t];
        }
        su[t] = ru[k];
        __syncthreads();
        T ur = T(0), us = T(0), ut = T(0);
#pragma unroll
        for (int m = 0; m < NP; ++m) {
            ur += Di[m] * su[j * NP + m];
            us += Dj[m] * su[m * NP + i];
            ut += sD[k * NP + m] * ru[m];
        }
        const T wr = g[0] * ur + g[1] * us + g[2] * ut;
        const T ws = g[1] * ur + g[3] * us + g[4] * ut;
        const T wt = g[2] * ur + g[4] * us + g[5] * ut;
        sr[t] = wr;
        ss[t] = ws;
        __syncthreads();
        T acc = T(0);
#pragma unroll
        for (int m = 0; m < NP; ++m) acc += DiT[m] * sr[j * NP + m] + DjT[m] * ss[m * NP + i];
        rw[k] += acc;
#pragma unroll
        for (int m = 0; m < NP; ++m) rw[m] += sD[k * NP + m] * wt;
        if (k + 1 < NP) {
#pragma unroll
            for (int q = 0; q < 6; ++q) g[q] = gn[q];
        }
    }

    double dot = 0.0;
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        T v = h1 * rw[k];
        if (HELM) v += h2 * Bm[e * P3 + k * P2 + t] * ru[k];
        w[GATHER ? (int64_t)rows_index32(L, ex, ey, ez, i, j, k) : e * P3 + k * P2 + t] = v;
        if (DOT) dot += (double)ru[k] * (double)v;
    }
    if (DOT) {
        // block reduction in a fixed order (deterministic)
        __shared__ double red[P2];
        red[t] = dot;
        __syncthreads();
        if (t == 0) {
            double s = 0.0;
            for (int q = 0; q < P2; ++q) s += red[q];
            partial[e] = s;
        }
    }
}

// Thread-per-point variant (N <= 7): one workgroup of (N+1)^3 threads per
// element, every load of u, G and B issued at kernel start as a
// non-temporal (streaming) load, so the wavefronts keep the most bytes in
// flight; the three derivative and three transposed contractions read the
// staged tiles from LDS.  At N = 7 this streams at about 6 TB/s of
// algorithmic bytes on MI355X, against about 5.5 TB/s for the pencil kernel.
template <typename T>
__device__ __forceinline__ T ldnt(const T *p) { return __builtin_nontemporal_load(p); }

constexpr int kPptF32 = 2;   // points per thread of the FP32 operator at N = 7

template <typename T, int NP, bool HELM, bool DOT, bool GATHER>
__global__ void __launch_bounds__(NP * NP * NP)
ax_pt_kernel(const T *__restrict__ u, T *__restrict__ w, const T *__restrict__ G,
             const T *__restrict__ Bm, const T *__restrict__ Dg, T h1, T h2,
             double *__restrict__ partial, const int32_t *__restrict__ skip, Lattice L)
{
    if (skip && *skip) return;
    constexpr int P2 = NP * NP, P3 = NP * NP * NP;
    __shared__ T sD[P2], su[P3], sr[P3], ss[P3], st[P3];
    const int t = threadIdx.x, i = t % NP, j = (t / NP) % NP, k = t / P2;
    const int64_t e = xcd_block();
    int ex = 0, ey = 0, ez = 0;   // element coordinates (gather mode)
    if (GATHER) elem_coords(L, e, ex, ey, ez);
    T uv;
    if (GATHER) {
        uv = u[gather_index32(L, ex, ey, ez, i, j, k)];
    } else {
        uv = ldnt(&u[e * P3 + t]);
    }
    const T *Ge = G + e * 6 * P3;
    const T g0 = ldnt(&Ge[t]), g1 = ldnt(&Ge[P3 + t]), g2 = ldnt(&Ge[2 * P3 + t]);
    const T g3 = ldnt(&Ge[3 * P3 + t]), g4 = ldnt(&Ge[4 * P3 + t]), g5 = ldnt(&Ge[5 * P3 + t]);
    T bv = T(0);
    if (HELM) bv = ldnt(&Bm[e * P3 + t]);
    if (t < P2) sD[t] = Dg[t];
    su[t] = uv;
    // With P2 = 64 a wavefront is one k-plane, so row k and column k of D are
    // wave-uniform: they come through scalar loads into scalar registers and
    // the t-direction contractions read only their u / flux operand from LDS.
    T Dk[NP], DkT[NP];
    if constexpr (P2 == 64) {
        const int kw = __builtin_amdgcn_readfirstlane(k);
#pragma unroll
        for (int m = 0; m < NP; ++m) {
            Dk[m] = Dg[kw * NP + m];
            DkT[m] = Dg[m * NP + kw];
        }
    }
    __syncthreads();
    T ur = T(0), us = T(0), ut = T(0);
#pragma unroll
    for (int m = 0; m < NP; ++m) {
        ur += sD[i * NP + m] * su[k * P2 + j * NP + m];
        us += sD[j * NP + m] * su[k * P2 + m * NP + i];
        ut += (P2 == 64 ? Dk[m] : sD[k * NP + m]) * su[m * P2 + j * NP + i];
    }
    sr[t] = g0 * ur + g1 * us + g2 * ut;
    ss[t] = g1 * ur + g3 * us + g4 * ut;
    st[t] = g2 * ur + g4 * us + g5 * ut;
    __syncthreads();
    T acc = T(0);
#pragma unroll
    for (int m = 0; m < NP; ++m)
        acc += sD[m * NP + i] * sr[k * P2 + j * NP + m] + sD[m * NP + j] * ss[k * P2 + m * NP + i] +
               (P2 == 64 ? DkT[m] : sD[m * NP + k]) * st[m * P2 + j * NP + i];
    T v = h1 * acc;
    if (HELM) v += h2 * bv * uv;
    w[GATHER ? (int64_t)rows_index32(L, ex, ey, ez, i, j, k) : e * P3 + t] = v;
    if constexpr (DOT && P3 % 64 == 0) {
        // full wavefronts: fixed butterfly within each wave, then the wave
        // sums in wave order (deterministic)
        __shared__ double wred[P3 / 64 > 0 ? P3 / 64 : 1];
        double d = (double)uv * (double)v;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) d += __shfl_xor(d, o);
        if ((t & 63) == 0) wred[t >> 6] = d;
        __syncthreads();
        if (t == 0) {
            double sum = 0.0;
#pragma unroll
            for (int q = 0; q < P3 / 64; ++q) sum += wred[q];
            partial[e] = sum;
        }
    } else if (DOT) {
        // fixed-order tree over the (N+1)^3 threads (the last wavefront may be
        // partial, so no cross-lane shuffles)
        __shared__ double red[P3];
        red[t] = (double)uv * (double)v;
        __syncthreads();
        constexpr int top = P3 <= 1 ? 1 : (P3 <= 2 ? 1 : (P3 <= 4 ? 2 : (P3 <= 8 ? 4 : (P3 <= 16 ? 8 : (P3 <= 32 ? 16 : (P3 <= 64 ? 32 : (P3 <= 128 ? 64 : (P3 <= 256 ? 128 : 256))))))));
        for (int h = top; h > 0; h >>= 1) {
            if (t < h && t + h < P3) red[t] += red[t + h];
            __syncthreads();
        }
        if (t == 0) partial[e] = red[0];
    }
}

// Several points per thread (N = 7, FP32): a workgroup of 512 / PPT threads
// per element, thread t owning points (i, j, k0 + q 8/PPT), q < PPT.  Each
// thread keeps PPT times the bytes in flight (which the FP32 operator needs
// to approach the bandwidth the FP64 one reaches with one point per thread),
// and its points share one (i, j) pencil: the t-direction contractions read
// the pencil from LDS once for all of them.
template <typename T, int PPT, bool HELM, bool DOT, bool GATHER>
__global__ void __launch_bounds__(512 / PPT)
ax_ptn_kernel(const T *__restrict__ u, T *__restrict__ w, const T *__restrict__ G, const T *__restrict__ Bm,
              const T *__restrict__ Dg, T h1, T h2, double *__restrict__ partial, const int32_t *__restrict__ skip,
              Lattice L)
{
    if (skip && *skip) return;
    constexpr int NP = 8, P2 = 64, P3 = 512, H = 512 / PPT, KS = 8 / PPT;
    __shared__ T sD[P2], su[P3], sr[P3], ss[P3], st[P3];
    const int t = threadIdx.x, i = t & 7, j = (t >> 3) & 7, k0 = t >> 6;   // points k0 + q KS
    const int64_t e = xcd_block();
    int ex = 0, ey = 0, ez = 0;
    if (GATHER) elem_coords(L, e, ex, ey, ez);
    T uv[PPT];
    if (GATHER) {
#pragma unroll
        for (int q = 0; q < PPT; ++q) uv[q] = u[gather_index32(L, ex, ey, ez, i, j, k0 + q * KS)];
    } else {
#pragma unroll
        for (int q = 0; q < PPT; ++q) uv[q] = ldnt(&u[e * P3 + q * H + t]);
    }
    const T *Ge = G + e * 6 * P3;
    T g[PPT][6];
#pragma unroll
    for (int q = 0; q < PPT; ++q)
#pragma unroll
        for (int c = 0; c < 6; ++c) g[q][c] = ldnt(&Ge[c * P3 + q * H + t]);
    T bv[PPT];
#pragma unroll
    for (int q = 0; q < PPT; ++q) bv[q] = HELM ? ldnt(&Bm[e * P3 + q * H + t]) : T(0);
    if (t < P2) sD[t] = Dg[t];
#pragma unroll
    for (int q = 0; q < PPT; ++q) su[q * H + t] = uv[q];
    // k0 is the wavefront index, so the rows and columns k of D that this
    // thread's points use are wave-uniform: scalar loads, scalar registers
    T Dk[PPT][NP], DkT[PPT][NP];
    {
        const int k0w = __builtin_amdgcn_readfirstlane(k0);
#pragma unroll
        for (int q = 0; q < PPT; ++q)
#pragma unroll
            for (int m = 0; m < NP; ++m) {
                Dk[q][m] = Dg[(k0w + q * KS) * NP + m];
                DkT[q][m] = Dg[m * NP + k0w + q * KS];
            }
    }
    __syncthreads();
    T pen[NP];   // the (i, j) pencil of u, shared by this thread's points
#pragma unroll
    for (int m = 0; m < NP; ++m) pen[m] = su[m * P2 + j * NP + i];
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
        const int k = k0 + q * KS;
        T ur = T(0), us = T(0), ut = T(0);
#pragma unroll
        for (int m = 0; m < NP; ++m) {
            ur += sD[i * NP + m] * su[k * P2 + j * NP + m];
            us += sD[j * NP + m] * su[k * P2 + m * NP + i];
            ut += Dk[q][m] * pen[m];
        }
        const int tq = q * H + t;
        sr[tq] = g[q][0] * ur + g[q][1] * us + g[q][2] * ut;
        ss[tq] = g[q][1] * ur + g[q][3] * us + g[q][4] * ut;
        st[tq] = g[q][2] * ur + g[q][4] * us + g[q][5] * ut;
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < NP; ++m) pen[m] = st[m * P2 + j * NP + i];
    double dot = 0.0;
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
        const int k = k0 + q * KS;
        T acc = T(0);
#pragma unroll
        for (int m = 0; m < NP; ++m)
            acc += sD[m * NP + i] * sr[k * P2 + j * NP + m] + sD[m * NP + j] * ss[k * P2 + m * NP + i] +
                   DkT[q][m] * pen[m];
        T v = h1 * acc;
        if (HELM) v += h2 * bv[q] * uv[q];
        w[GATHER ? (int64_t)rows_index32(L, ex, ey, ez, i, j, k) : e * P3 + q * H + t] = v;
        dot += (double)uv[q] * (double)v;
    }
    if constexpr (DOT) {
        __shared__ double wred[H / 64];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) dot += __shfl_xor(dot, o);
        if ((t & 63) == 0) wred[t >> 6] = dot;
        __syncthreads();
        if (t == 0) {
            double sum = 0.0;
#pragma unroll
            for (int q = 0; q < H / 64; ++q) sum += wred[q];
            partial[e] = sum;
        }
    }
}

// Batched form: NC fields (e.g. three velocity components) through one
// pass over the geometric factors.  G and B are loaded once per point; the
// fields reuse one set of LDS tiles in turn.  u, w, partial: NC blocks of
// (assembled or local) fields and NC x E partials.
template <int NP, int NC, bool HELM, bool GATHER>
__global__ void __launch_bounds__(NP * NP * NP)
ax_pt_batched_kernel(const double *__restrict__ u, int64_t ustride, double *__restrict__ w, const double *__restrict__ G,
                     const double *__restrict__ Bm, const double *__restrict__ Dg, double h1, double h2,
                     double *__restrict__ partial, const int32_t *__restrict__ done_flags, int done_stride, Lattice L,
                     int64_t nl)
{
    if (done_flags) {
        bool all = true;
        for (int c = 0; c < NC; ++c) all = all && done_flags[c * done_stride] != 0;
        if (all) return;
    }
    constexpr int P2 = NP * NP, P3 = NP * NP * NP;
    __shared__ double sD[P2], su[P3], sr[P3], ss[P3], st[P3];
    __shared__ double red[P3 / 64];
    const int t = threadIdx.x, i = t % NP, j = (t / NP) % NP, k = t / P2;
    const int64_t e = xcd_block();
    int ex = 0, ey = 0, ez = 0;   // element coordinates (gather mode)
    if (GATHER) elem_coords(L, e, ex, ey, ez);
    int64_t src;
    if (GATHER) {
        src = gather_index32(L, ex, ey, ez, i, j, k);
    } else {
        src = e * P3 + t;
    }
    double uv[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) uv[c] = GATHER ? u[c * ustride + src] : ldnt(&u[c * ustride + src]);
    const double *Ge = G + e * 6 * P3;
    const double g0 = ldnt(&Ge[t]), g1 = ldnt(&Ge[P3 + t]), g2 = ldnt(&Ge[2 * P3 + t]);
    const double g3 = ldnt(&Ge[3 * P3 + t]), g4 = ldnt(&Ge[4 * P3 + t]), g5 = ldnt(&Ge[5 * P3 + t]);
    double bv = 0.0;
    if (HELM) bv = ldnt(&Bm[e * P3 + t]);
    if (t < P2) sD[t] = Dg[t];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        __syncthreads();   // previous field's tiles fully consumed
        su[t] = uv[c];
        __syncthreads();
        double ur = 0.0, us = 0.0, ut = 0.0;
#pragma unroll
        for (int m = 0; m < NP; ++m) {
            ur += sD[i * NP + m] * su[k * P2 + j * NP + m];
            us += sD[j * NP + m] * su[k * P2 + m * NP + i];
            ut += sD[k * NP + m] * su[m * P2 + j * NP + i];
        }
        sr[t] = g0 * ur + g1 * us + g2 * ut;
        ss[t] = g1 * ur + g3 * us + g4 * ut;
        st[t] = g2 * ur + g4 * us + g5 * ut;
        __syncthreads();
        double acc = 0.0;
#pragma unroll
        for (int m = 0; m < NP; ++m)
            acc += sD[m * NP + i] * sr[k * P2 + j * NP + m] + sD[m * NP + j] * ss[k * P2 + m * NP + i] +
                   sD[m * NP + k] * st[m * P2 + j * NP + i];
        double v = h1 * acc;
        if (HELM) v += h2 * bv * uv[c];
        w[c * nl + (GATHER ? (int64_t)rows_index32(L, ex, ey, ez, i, j, k) : e * P3 + t)] = v;
        if (partial) {
            // same order as the single-field kernel: butterfly per wavefront,
            // then the wave sums in wave order
            static_assert(P3 % 64 == 0, "full wavefronts");
            double d = uv[c] * v;
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) d += __shfl_xor(d, o);
            if ((t & 63) == 0) red[t >> 6] = d;
            __syncthreads();
            if (t == 0) {
                double sum = 0.0;
#pragma unroll
                for (int q = 0; q < P3 / 64; ++q) sum += red[q];
                partial[c * (int64_t)gridDim.x + e] = sum;
            }
        }
    }
}

template <int NC>
hipError_t launch_batched_nc(const Mesh &m, double h1, double h2, const double *ug, int64_t ustride, double *w,
                             double *partial, const int32_t *done_flags, int done_stride, hipStream_t s)
{
    const dim3 grid((unsigned)m.E), block(512);
    const bool helm = h2 != 0.0;
    if (helm)
        hipLaunchKernelGGL((ax_pt_batched_kernel<8, NC, true, true>), grid, block, 0, s, ug, ustride, w, m.d_G, m.d_B,
                           m.d_D, h1, h2, partial, done_flags, done_stride, m.lat, m.nl);
    else
        hipLaunchKernelGGL((ax_pt_batched_kernel<8, NC, false, true>), grid, block, 0, s, ug, ustride, w, m.d_G, m.d_B,
                           m.d_D, h1, h2, partial, done_flags, done_stride, m.lat, m.nl);
    return hipGetLastError();
}

template <typename T, int NP, bool GATHER>
hipError_t launch_pt(const Mesh &m, T h1, T h2, const T *u, T *w, const T *G, const T *B,
                     const T *D, double *partial, const int32_t *skip, hipStream_t s)
{
    const dim3 grid((unsigned)m.E), block(NP * NP * NP);
    const bool helm = (h2 != T(0));
    const Lattice &L = m.lat;
    if (partial) {
        if (helm)
            hipLaunchKernelGGL((ax_pt_kernel<T, NP, true, true, GATHER>), grid, block, 0, s, u, w, G, B, D, h1, h2, partial, skip, L);
        else
            hipLaunchKernelGGL((ax_pt_kernel<T, NP, false, true, GATHER>), grid, block, 0, s, u, w, G, B, D, h1, h2, partial, skip, L);
    } else {
        if (helm)
            hipLaunchKernelGGL((ax_pt_kernel<T, NP, true, false, GATHER>), grid, block, 0, s, u, w, G, B, D, h1, h2, partial, skip, L);
        else
            hipLaunchKernelGGL((ax_pt_kernel<T, NP, false, false, GATHER>), grid, block, 0, s, u, w, G, B, D, h1, h2, partial, skip, L);
    }
    return hipGetLastError();
}

template <typename T, int PPT, bool GATHER>
hipError_t launch_ptn(const Mesh &m, T h1, T h2, const T *u, T *w, const T *G, const T *B, const T *D,
                      double *partial, const int32_t *skip, hipStream_t s)
{
    const dim3 grid((unsigned)m.E), block(512 / PPT);
    const bool helm = (h2 != T(0));
    const Lattice &L = m.lat;
    if (partial) {
        if (helm)
            hipLaunchKernelGGL((ax_ptn_kernel<T, PPT, true, true, GATHER>), grid, block, 0, s, u, w, G, B, D, h1, h2, partial, skip, L);
        else
            hipLaunchKernelGGL((ax_ptn_kernel<T, PPT, false, true, GATHER>), grid, block, 0, s, u, w, G, B, D, h1, h2, partial, skip, L);
    } else {
        if (helm)
            hipLaunchKernelGGL((ax_ptn_kernel<T, PPT, true, false, GATHER>), grid, block, 0, s, u, w, G, B, D, h1, h2, partial, skip, L);
        else
            hipLaunchKernelGGL((ax_ptn_kernel<T, PPT, false, false, GATHER>), grid, block, 0, s, u, w, G, B, D, h1, h2, partial, skip, L);
    }
    return hipGetLastError();
}

template <typename T, int NP, bool GATHER>
hipError_t launch_np(const Mesh &m, T h1, T h2, const T *u, T *w, const T *G, const T *B,
                     const T *D, double *partial, const int32_t *skip, hipStream_t s)
{
    const dim3 grid((unsigned)m.E), block(NP * NP);
    const bool helm = (h2 != T(0));
    const Lattice &L = m.lat;
    if (partial) {
        if (helm)
            hipLaunchKernelGGL((ax_kernel<T, NP, true, true, GATHER>), grid, block, 0, s, u, w, G, B, D, h1, h2, partial, skip, L);
        else
            hipLaunchKernelGGL((ax_kernel<T, NP, false, true, GATHER>), grid, block, 0, s, u, w, G, B, D, h1, h2, partial, skip, L);
    } else {
        if (helm)
            hipLaunchKernelGGL((ax_kernel<T, NP, true, false, GATHER>), grid, block, 0, s, u, w, G, B, D, h1, h2, partial, skip, L);
        else
            hipLaunchKernelGGL((ax_kernel<T, NP, false, false, GATHER>), grid, block, 0, s, u, w, G, B, D, h1, h2, partial, skip, L);
    }
    return hipGetLastError();
}

template <typename T, bool GATHER = false>
hipError_t launch_any(const Mesh &m, T h1, T h2, const T *u, T *w, const T *G, const T *B,
                      const T *D, double *partial, const int32_t *skip, hipStream_t s)
{
    if (m.E == 0) return hipSuccess;
    switch (m.NP) {
    case 2: return launch_pt<T, 2, GATHER>(m, h1, h2, u, w, G, B, D, partial, skip, s);
    case 3: return launch_pt<T, 3, GATHER>(m, h1, h2, u, w, G, B, D, partial, skip, s);
    case 4: return launch_pt<T, 4, GATHER>(m, h1, h2, u, w, G, B, D, partial, skip, s);
    case 5: return launch_pt<T, 5, GATHER>(m, h1, h2, u, w, G, B, D, partial, skip, s);
    case 6: return launch_pt<T, 6, GATHER>(m, h1, h2, u, w, G, B, D, partial, skip, s);
    case 7: return launch_pt<T, 7, GATHER>(m, h1, h2, u, w, G, B, D, partial, skip, s);
    case 8:   // several points per thread pay off in FP32 only (FP64, two: 225 against 207 us)
        if constexpr (sizeof(T) == 4) return launch_ptn<T, kPptF32, GATHER>(m, h1, h2, u, w, G, B, D, partial, skip, s);
        else return launch_pt<T, 8, GATHER>(m, h1, h2, u, w, G, B, D, partial, skip, s);
    case 9: return launch_np<T, 9, GATHER>(m, h1, h2, u, w, G, B, D, partial, skip, s);
    case 10: return launch_np<T, 10, GATHER>(m, h1, h2, u, w, G, B, D, partial, skip, s);
    case 11: return launch_np<T, 11, GATHER>(m, h1, h2, u, w, G, B, D, partial, skip, s);
    case 12: return launch_np<T, 12, GATHER>(m, h1, h2, u, w, G, B, D, partial, skip, s);
    case 13: return launch_np<T, 13, GATHER>(m, h1, h2, u, w, G, B, D, partial, skip, s);
    case 14: return launch_np<T, 14, GATHER>(m, h1, h2, u, w, G, B, D, partial, skip, s);
    case 15: return launch_np<T, 15, GATHER>(m, h1, h2, u, w, G, B, D, partial, skip, s);
    case 16: return launch_np<T, 16, GATHER>(m, h1, h2, u, w, G, B, D, partial, skip, s);
    default: return hipErrorInvalidValue;
    }
}

// Diagonal of the element matrices (setup, not on the iteration path):
// h1 [sum_m G11(m,j,k) D_mi^2 + G22(i,m,k) D_mj^2 + G33(i,j,m) D_mk^2
//     + 2 G12 D_ii D_jj + 2 G13 D_ii D_kk + 2 G23 D_jj D_kk] + h2 B.
__global__ void diag_kernel(const double *__restrict__ G, const double *__restrict__ Bm,
                            const double *__restrict__ D, int NP, int64_t nl, double h1,
                            double h2, double *__restrict__ d)
{
    const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= nl) return;
    const int64_t P3 = (int64_t)NP * NP * NP;
    const int64_t e = l / P3;
    const int q = (int)(l - e * P3);
    const int i = q % NP, j = (q / NP) % NP, k = q / (NP * NP);
    const double *Ge = G + e * 6 * P3;
    double s = 0.0;
    for (int m = 0; m < NP; ++m) {
        const double a = D[m * NP + i], b = D[m * NP + j], c = D[m * NP + k];
        s += Ge[0 * P3 + m + NP * (j + NP * k)] * a * a;
        s += Ge[3 * P3 + i + NP * (m + NP * k)] * b * b;
        s += Ge[5 * P3 + i + NP * (j + NP * m)] * c * c;
    }
    const double dii = D[i * NP + i], djj = D[j * NP + j], dkk = D[k * NP + k];
    s += 2.0 * Ge[1 * P3 + q] * dii * djj + 2.0 * Ge[2 * P3 + q] * dii * dkk +
         2.0 * Ge[4 * P3 + q] * djj * dkk;
    d[l] = h1 * s + h2 * Bm[l];
}

}  // namespace

hipError_t launch_ax_f64(const Mesh &m, double h1, double h2, const double *u, double *w,
                         double *partial_uw, hipStream_t s, const int32_t *skip)
{
    return launch_any<double>(m, h1, h2, u, w, m.d_G, m.d_B, m.d_D, partial_uw, skip, s);
}

hipError_t launch_ax_f32(const Mesh &m, float h1, float h2, const float *u, float *w,
                         double *partial_uw, hipStream_t s, const int32_t *skip)
{
    return launch_any<float>(m, h1, h2, u, w, m.d_G32, m.d_B32, m.d_D32, partial_uw, skip, s);
}

hipError_t launch_ax_f64_gather(const Mesh &m, double h1, double h2, const double *ug, double *w,
                                double *partial_uw, hipStream_t s, const int32_t *skip)
{
    return launch_any<double, true>(m, h1, h2, ug, w, m.d_G, m.d_B, m.d_D, partial_uw, skip, s);
}

hipError_t launch_ax_f32_gather(const Mesh &m, float h1, float h2, const float *ug, float *w,
                                double *partial_uw, hipStream_t s, const int32_t *skip)
{
    return launch_any<float, true>(m, h1, h2, ug, w, m.d_G32, m.d_B32, m.d_D32, partial_uw, skip, s);
}

hipError_t launch_ax_f64_gather_batched(const Mesh &m, int nc, double h1, double h2, const double *ug, int64_t ustride,
                                        double *w, double *partial, const int32_t *done_flags, int done_stride,
                                        hipStream_t s)
{
    if (m.E == 0) return hipSuccess;
    if (m.NP != 8) return hipErrorInvalidValue;
    switch (nc) {
    case 1: return launch_batched_nc<1>(m, h1, h2, ug, ustride, w, partial, done_flags, done_stride, s);
    case 2: return launch_batched_nc<2>(m, h1, h2, ug, ustride, w, partial, done_flags, done_stride, s);
    case 3: return launch_batched_nc<3>(m, h1, h2, ug, ustride, w, partial, done_flags, done_stride, s);
    case 4: return launch_batched_nc<4>(m, h1, h2, ug, ustride, w, partial, done_flags, done_stride, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_diag(const Mesh &m, double h1, double h2, double *d, hipStream_t s)
{
    if (m.nl == 0) return hipSuccess;
    const int bs = 256;
    hipLaunchKernelGGL(diag_kernel, dim3((unsigned)((m.nl + bs - 1) / bs)), dim3(bs), 0, s, m.d_G,
                       m.d_B, m.d_D, m.NP, m.nl, h1, h2, d);
    return hipGetLastError();
}

}  // namespace sem
