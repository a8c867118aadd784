// ax.hip -- matrix-free local spectral-element operator for gfx950.
//
//   w_e = h1 * sum_{a,b in {r,s,t}} D_a^T (G_ab o D_b u_e) + h2 * B o u_e
//
// (Deville, Fischer & Mund 2002, sec. 4.4; the paper's element-by-element,
// matrix-free operator of section 3.1, which the paper's section 4.2 notes is
// memory bound).
//
// Design (one wavefront per element at N = 7):
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
// the closed-form numbering; otherwise u is local [E][P].
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
    const int64_t e = blockIdx.x;
    const T *Ge = G + e * (6 * P3);

    sD[t] = Dg[t];

    T ru[NP], rw[NP];
    if (GATHER) {
        const int64_t ex = e % L.nelx, ey = (e / L.nelx) % L.nely, ez = e / ((int64_t)L.nelx * L.nely);
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

    T *we = w + e * P3;
    double dot = 0.0;
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        T v = h1 * rw[k];
        if (HELM) v += h2 * Bm[e * P3 + k * P2 + t] * ru[k];
        we[k * P2 + t] = v;
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
    case 2: return launch_np<T, 2, GATHER>(m, h1, h2, u, w, G, B, D, partial, skip, s);
    case 3: return launch_np<T, 3, GATHER>(m, h1, h2, u, w, G, B, D, partial, skip, s);
    case 4: return launch_np<T, 4, GATHER>(m, h1, h2, u, w, G, B, D, partial, skip, s);
    case 5: return launch_np<T, 5, GATHER>(m, h1, h2, u, w, G, B, D, partial, skip, s);
    case 6: return launch_np<T, 6, GATHER>(m, h1, h2, u, w, G, B, D, partial, skip, s);
    case 7: return launch_np<T, 7, GATHER>(m, h1, h2, u, w, G, B, D, partial, skip, s);
    case 8: return launch_np<T, 8, GATHER>(m, h1, h2, u, w, G, B, D, partial, skip, s);
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

hipError_t launch_diag(const Mesh &m, double h1, double h2, double *d, hipStream_t s)
{
    if (m.nl == 0) return hipSuccess;
    const int bs = 256;
    hipLaunchKernelGGL(diag_kernel, dim3((unsigned)((m.nl + bs - 1) / bs)), dim3(bs), 0, s, m.d_G,
                       m.d_B, m.d_D, m.NP, m.nl, h1, h2, d);
    return hipGetLastError();
}

}  // namespace sem
