// gs.hip -- gather-scatter (direct-stiffness summation), mask, and the small
// vector kernels behind sem_rhs / sem_jacobi / sem_dot.
//
// The gather-scatter is the only coupling between elements (paper section
// 3.1) and the part the paper's section 4.2 identifies as the communication
// bottleneck.  Every global node receives the sum of its local copies, taken
// in ascending local index, and the sum is written back to every copy; the
// copies are found in closed form on the structured lattice (no index lists).
//
// Three implementations, chosen by shape:
// * N = 7, nelx <= 256 (the default): one or two lanes per element row
//   segment in every y/z copy of a global lattice row, x-face partners by
//   cross-lane shuffles or, for rows wider than a wavefront, LDS
//   (gs_seg_kernel);
// * other orders with nelx (N+1) <= 1024: whole lattice rows per workgroup,
//   x-face partners through LDS (gs_lattice_kernel);
// * otherwise two passes over disjoint nodes: rows on an element-face plane,
//   node by node, and the x-face nodes of all other rows (gs_rows_kernel,
//   gs_xface_kernel), with copies from three small per-axis tables.
// Every element row is fetched once per pass.
#include <type_traits>

#include "cg.hpp"
#include "lattice.hpp"
#include "sem_internal.hpp"

namespace sem {
namespace {

// Rows on an element-face plane (or, with the mask, on a Dirichlet plane):
// every node of the row is visited.
template <typename T, int MASK>
__global__ void __launch_bounds__(256)
gs_rows_kernel(T *__restrict__ u, Lattice L, const int32_t *__restrict__ skip)
{
    if (skip && *skip) return;
    const int gj = (int)(blockIdx.x % L.ny), gk = (int)(blockIdx.x / L.ny);   // one row per workgroup
    const int2 ay = L.tab[1][gj], az = L.tab[2][gk];
    const bool full = axis_count(ay) > 1 || axis_count(az) > 1 || (MASK && (axis_masked(ay) || axis_masked(az)));
    if (!full) return;   // uniform over the block
    for (int gi = threadIdx.x; gi < L.nx; gi += blockDim.x) {
        int loc[8];
        bool msk;
        const int n = node_locals(L, gi, gj, gk, loc, msk);
        const bool zero = MASK && msk;
        if (n == 1 && !zero) continue;
        T s = T(0);
        if (!zero)
            for (int c = 0; c < n; ++c) s += u[loc[c]];
        for (int c = 0; c < n; ++c) u[loc[c]] = s;
    }
}

// Every other row shares only its x-face nodes gi = m N: one thread per
// (x-face, row); lanes m and m+1 touch the two ends of one element row.
template <typename T, int MASK>
__global__ void __launch_bounds__(256)
gs_xface_kernel(T *__restrict__ u, Lattice L, int mx, const int32_t *__restrict__ skip)
{
    if (skip && *skip) return;
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= (int64_t)mx * L.ny * L.nz) return;
    const int64_t row = id / mx;
    const int m = (int)(id - row * mx);
    const int gj = (int)(row % L.ny), gk = (int)(row / L.ny);
    const int2 ay = L.tab[1][gj], az = L.tab[2][gk];
    if (axis_count(ay) > 1 || axis_count(az) > 1 || (MASK && (axis_masked(ay) || axis_masked(az)))) return;
    int loc[8];
    bool msk;
    const int n = node_locals(L, m * L.N, gj, gk, loc, msk);
    const bool zero = MASK && msk;
    if (n == 1 && !zero) return;
    T s = T(0);
    if (!zero)
        for (int c = 0; c < n; ++c) s += u[loc[c]];
    for (int c = 0; c < n; ++c) u[loc[c]] = s;
}

// Whole-row pass (the default): a workgroup of whole wavefronts per RPT
// global lattice rows (gj, gk).
// The row's copies in y and z are uniform over the workgroup (up to 2 x 2
// element rows), and thread X = ex (N+1) + i reads local point i of element
// ex in each of them.  Every 8-value element row of the field is read once, as
// a contiguous segment, by the workgroup of the global row it belongs to:
// the x-face copies, which share no segment with their partner in the
// [E][k][j][i] layout, then cost no extra sector traffic.  The values pass
// through LDS so that x-face partners (the neighbouring X) are summed in the
// same ascending-local-index order as the copy enumeration.  Nodes with a
// single copy are not written.  Needs nelx (N+1) <= 1024 and sorted axis
// tables (no periodic single-element axis).
template <typename T, int MASK, int RPT>
__global__ void __launch_bounds__(1024)
gs_lattice_kernel(T *__restrict__ u, Lattice L, const int32_t *__restrict__ skip)
{
    if (skip && *skip) return;
    extern __shared__ __attribute__((aligned(16))) unsigned char gs_smem[];
    const int NP = L.NP, P = (int)L.P, nxl = L.nelx * NP, nrows = (int)(L.ny * L.nz);
    const int X = (int)threadIdx.x;
    const int ex = X / NP, i = X - ex * NP;
    // every load of the thread's RPT rows first, then one barrier
    T own[RPT][4];
    int loc[RPT][4], cyz[RPT][2];
    bool mskyz[RPT];
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
        const int row = (int)blockIdx.x * RPT + r;
        const bool row_ok = row < nrows;
        const int gj = row_ok ? row % (int)L.ny : 0, gk = row_ok ? row / (int)L.ny : 0;
        const int2 ay = L.tab[1][gj], az = L.tab[2][gk];
        const int cy = row_ok ? axis_count(ay) : 0, cz = row_ok ? axis_count(az) : 0;
        cyz[r][0] = cy;
        cyz[r][1] = cz;
        mskyz[r] = MASK && (axis_masked(ay) || axis_masked(az));
        T *sv = (T *)gs_smem + (size_t)r * 4 * nxl;   // [4][nelx (N+1)] per row
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                const int q = c * 2 + b;
                if (X < nxl && c < cz && b < cy) {
                    const int e = ex + L.nelx * (axis_elem(ay, b) + L.nely * axis_elem(az, c));
                    loc[r][q] = e * P + i + NP * (axis_loc(ay, b) + NP * axis_loc(az, c));
                    own[r][q] = u[loc[r][q]];
                    sv[q * nxl + X] = own[r][q];
                }
            }
    }
    __syncthreads();
    if (X >= nxl) return;
    // x partner of this node: the neighbouring element's end point
    int part = -1;
    bool part_first = false;
    if (i == 0 && (ex > 0 || L.per[0])) {
        part = ex > 0 ? X - 1 : nxl - 1;
        part_first = ex > 0;   // the partner's element index is lower
    } else if (i == L.N && (ex < L.nelx - 1 || L.per[0])) {
        part = ex < L.nelx - 1 ? X + 1 : 0;
        part_first = ex == L.nelx - 1;
    }
    const int gi = ex * L.N + i;   // global x index (wrapped below when periodic)
    const bool msk_x = MASK && !L.per[0] && ((gi == 0 && (L.dir & 1)) || (gi == L.nelx * L.N && (L.dir & 2)));
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
        const int cy = cyz[r][0], cz = cyz[r][1];
        if (cy == 0) continue;   // past the last row
        const bool msk = msk_x || mskyz[r];
        if (cy * cz == 1 && part < 0 && !msk) continue;   // single copy: unchanged
        const T *sv = (const T *)gs_smem + (size_t)r * 4 * nxl;
        T s = T(0);
        if (!msk) {
#pragma unroll
            for (int c = 0; c < 2; ++c)
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    const int q = c * 2 + b;
                    if (c < cz && b < cy) {
                        if (part >= 0 && part_first) s += sv[q * nxl + part];
                        s += own[r][q];
                        if (part >= 0 && !part_first) s += sv[q * nxl + part];
                    }
                }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if ((q >> 1) < cz && (q & 1) < cy) u[loc[r][q]] = s;
    }
}

// Segment pass (N = 7, the default where it applies): the 8 values i = 0..7
// of one element row (j, k) form a 64-byte segment, and SPL lanes (1 or 2)
// own one, VPL = 8 / SPL values each, in every y/z copy of a global lattice
// row (gj, gk).  G lanes (a power of two >= SPL nelx, at most 256) serve
// one row, lane l = SPL ex + part owning points i = VPL part .. VPL part +
// VPL - 1 of element ex.  Loads are 16-byte vectors, so a wavefront keeps
// 4 KB per copy in flight.  The x-face node between elements ex and ex+1
// (gi = (ex+1) N) is summed by the lane holding i = N of ex from its own
// values and the next lane's i = 0 values, in ascending local index: copies
// in (z, y) order, and within a copy the lower element first (the
// partner's, across the periodic wrap).  The lane holding i = 0 of ex+1
// then takes that sum from its left neighbour.  Rows that fit a wavefront
// exchange these values by cross-lane shuffles (no LDS, no barrier); wider
// rows exchange them through LDS, with two barriers.
// Interior points sum their y/z copies; a node with a single copy keeps its
// value.  Every segment is written back whole.  Needs sorted axis tables (no
// periodic single-element axis) and SPL nelx <= 256.
template <typename T, int MASK, int G, int SPL>
__global__ void __launch_bounds__(256)
gs_seg_kernel(T *__restrict__ u, Lattice L, const int32_t *__restrict__ skip)
{
    if (skip && *skip) return;
    constexpr int NP = 8, N = 7, VPL = NP / SPL;
    typedef typename std::conditional<sizeof(T) == 8, double2, float4>::type V;   // 16 bytes
    constexpr int PV = 16 / (int)sizeof(T), NV = VPL / PV;
    static_assert(NV >= 1 && VPL % PV == 0, "a lane's values are whole 16-byte vectors");
    const int lane = (int)threadIdx.x & (G - 1);
    const int row = (int)((blockIdx.x * blockDim.x + threadIdx.x) / G);
    const int nelx = L.nelx, ny = (int)L.ny, nx = (int)L.nx, P = (int)L.P, nl = SPL * nelx;
    const bool active = lane < nl && row < (int)(L.ny * L.nz);
    const int ex = lane / SPL, i0 = (lane % SPL) * VPL;
    const bool has_left = i0 == 0, has_right = i0 + VPL == NP;   // holds i = 0 / i = N
    const int gj = active ? row % ny : 0, gk = active ? row / ny : 0;
    // copies in y and z computed in closed form (element * 8 + local), so
    // the segment loads wait on no table load
    int Y[2], Z[2];
    const int cy = active ? axis_copies_t<NP>(gj, L.nely, N, L.per[1] != 0, Y) : 0;
    const int cz = active ? axis_copies_t<NP>(gk, L.nelz, N, L.per[2] != 0, Z) : 0;
    const int n = cy * cz;
    const bool myz = MASK && (axis_dirichlet(L, 1, gj, L.nely) || axis_dirichlet(L, 2, gk, L.nelz));
    T v[4][VPL];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int m = 0; m < VPL; ++m) v[q][m] = T(0);   // absent copies (never summed)
    int base[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int c = q >> 1, b = q & 1;
        base[q] = -1;
        if (c < cz && b < cy) {
            const int e = ex + nelx * ((Y[b] >> 3) + L.nely * (Z[c] >> 3));
            base[q] = e * P + NP * ((Y[b] & 7) + NP * (Z[c] & 7)) + i0;
            const V *src = (const V *)(u + base[q]);
#pragma unroll
            for (int h = 0; h < NV; ++h) {
                const V x = src[h];
                const T *xs = (const T *)&x;
#pragma unroll
                for (int m = 0; m < PV; ++m) v[q][h * PV + m] = xs[m];
            }
        }
    }
    // the element's two end nodes along x: gi = (ex+1) N (wrapped) and ex N
    int giR = ex * N + N;
    if (giR >= nx) giR -= nx;
    int XR[2], XL[2];
    const int cxR = axis_copies_t<NP>(active ? giR : 0, nelx, N, L.per[0] != 0, XR);
    const int cxL = axis_copies_t<NP>(active ? ex * N : 0, nelx, N, L.per[0] != 0, XL);
    const bool mR = MASK && (myz || axis_dirichlet(L, 0, giR, nelx));
    const bool mL = MASK && (myz || axis_dirichlet(L, 0, ex * N, nelx));
    // the next lane's first values (i = 0 of element ex+1; lane 0 across the wrap)
    const int srcR = lane + 1 >= nl ? 0 : lane + 1, srcL = lane == 0 ? nl - 1 : lane - 1;   // both < G
    // rows wider than a wavefront exchange through LDS (two barriers)
    constexpr bool kLds = G > 64;
    __shared__ T xv[kLds ? 256 : 1][4], xs[kLds ? 256 : 1];
    const int rb = (int)threadIdx.x - lane;   // first thread of this row
    T pv[4];
    if constexpr (kLds) {
#pragma unroll
        for (int q = 0; q < 4; ++q) xv[threadIdx.x][q] = v[q][0];
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 4; ++q) pv[q] = xv[rb + srcR][q];
    } else {
#pragma unroll
        for (int q = 0; q < 4; ++q) pv[q] = __shfl(v[q][0], srcR, G);
    }
    // node gi = (ex+1) N, on the lane holding i = N: masked, shared with the
    // next element, or its own copies only
    T sR = v[0][VPL - 1];
    if (mR) {
        sR = T(0);
    } else if (cxR == 2) {
        const bool pfirst = (XR[0] >> 3) != ex;   // the neighbour holds the lower element
        sR = T(0);
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if ((q >> 1) < cz && (q & 1) < cy) {
                if (pfirst) {
                    sR += pv[q];
                    sR += v[q][VPL - 1];
                } else {
                    sR += v[q][VPL - 1];
                    sR += pv[q];
                }
            }
    } else if (n > 1) {
        sR = T(0);
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if ((q >> 1) < cz && (q & 1) < cy) sR += v[q][VPL - 1];
    }
    T fromL;
    if constexpr (kLds) {
        xs[threadIdx.x] = sR;
        __syncthreads();
        fromL = xs[rb + srcL];
    } else {
        fromL = __shfl(sR, srcL, G);
    }
    if (!active) return;
    T out[VPL];
#pragma unroll
    for (int m = 0; m < VPL; ++m) {
        const bool left = has_left && m == 0, right = has_right && m == VPL - 1;
        if (right) {
            out[m] = sR;
        } else if (left && cxL == 2) {
            out[m] = fromL;   // the previous element's sum for the shared node
        } else if (left ? mL : (MASK && myz)) {
            out[m] = T(0);
        } else if (n > 1) {
            T s = T(0);
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if ((q >> 1) < cz && (q & 1) < cy) s += v[q][m];
            out[m] = s;
        } else {
            out[m] = v[0][m];
        }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
        if (base[q] >= 0) {
            V *dst = (V *)(u + base[q]);
#pragma unroll
            for (int h = 0; h < NV; ++h) {
                V x;
                T *xs = (T *)&x;
#pragma unroll
                for (int m = 0; m < PV; ++m) xs[m] = out[h * PV + m];
                dst[h] = x;
            }
        }
}

template <typename T, int MASK, int SPL>
hipError_t launch_seg_spl(const Lattice &L, T *u, hipStream_t s, const int32_t *skip)
{
    const int64_t rows = L.ny * L.nz;
    int g = 4;
    while (g < SPL * L.nelx) g *= 2;
    const unsigned rpb = 256 / g;
    const dim3 grid((unsigned)((rows + rpb - 1) / rpb)), block(256);
    switch (g) {
    case 4: hipLaunchKernelGGL((gs_seg_kernel<T, MASK, 4, SPL>), grid, block, 0, s, u, L, skip); break;
    case 8: hipLaunchKernelGGL((gs_seg_kernel<T, MASK, 8, SPL>), grid, block, 0, s, u, L, skip); break;
    case 16: hipLaunchKernelGGL((gs_seg_kernel<T, MASK, 16, SPL>), grid, block, 0, s, u, L, skip); break;
    case 32: hipLaunchKernelGGL((gs_seg_kernel<T, MASK, 32, SPL>), grid, block, 0, s, u, L, skip); break;
    case 64: hipLaunchKernelGGL((gs_seg_kernel<T, MASK, 64, SPL>), grid, block, 0, s, u, L, skip); break;
    case 128: hipLaunchKernelGGL((gs_seg_kernel<T, MASK, 128, SPL>), grid, block, 0, s, u, L, skip); break;
    case 256: hipLaunchKernelGGL((gs_seg_kernel<T, MASK, 256, SPL>), grid, block, 0, s, u, L, skip); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// two lanes per segment while a row fits a workgroup that way (fewer
// registers per lane, more wavefronts in flight), else one (nelx <= 256)
template <typename T, int MASK>
hipError_t launch_seg(const Lattice &L, T *u, hipStream_t s, const int32_t *skip)
{
    return 2 * L.nelx <= 256 ? launch_seg_spl<T, MASK, 2>(L, u, s, skip) : launch_seg_spl<T, MASK, 1>(L, u, s, skip);
}

__global__ void scale_by_B_kernel(const double *__restrict__ f, const double *__restrict__ Bm,
                                  double *__restrict__ b, int64_t nl)
{
    const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (l < nl) b[l] = Bm[l] * f[l];
}

// d <- 1/d on free nodes, 1 on Dirichlet nodes (wcode == 0)
__global__ void jacobi_finish_kernel(double *__restrict__ d, const uint8_t *__restrict__ wcode,
                                     int64_t nl)
{
    const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (l < nl) d[l] = wcode[l] == 0 ? 1.0 : 1.0 / d[l];
}

constexpr int kDotBlock = 256;
constexpr int kDotMaxBlocks = 2048;

// partial[b] = sum over a grid-stride range of u v / mult, fixed order
__global__ void __launch_bounds__(kDotBlock)
dot_partial_kernel(const double *__restrict__ u, const double *__restrict__ v,
                   const uint8_t *__restrict__ mult, int64_t nl, double *__restrict__ partial)
{
    __shared__ double red[kDotBlock];
    double s = 0.0;
    for (int64_t l = (int64_t)blockIdx.x * kDotBlock + threadIdx.x; l < nl;
         l += (int64_t)gridDim.x * kDotBlock)
        s += u[l] * v[l] / (double)mult[l];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = kDotBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(kDotBlock)
sum_partials_kernel(const double *__restrict__ partial, int n, double *__restrict__ out)
{
    __shared__ double red[kDotBlock];
    double s = 0.0;
    for (int q = threadIdx.x; q < n; q += kDotBlock) s += partial[q];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = kDotBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0];
}

inline unsigned blocks_for(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

template <typename T>
hipError_t dssum_impl(const Mesh &m, T *u, int apply_mask, hipStream_t s, const int32_t *skip)
{
    const Lattice &L = m.lat;
    const int64_t rows = L.ny * L.nz;
    if (rows == 0) return hipSuccess;
    const int nxl = L.nelx * L.NP;
    if (!L.unsorted && L.NP == 8 && L.nelx <= 256)
        return apply_mask ? launch_seg<T, 1>(L, u, s, skip) : launch_seg<T, 0>(L, u, s, skip);
    if (!L.unsorted && nxl <= 1024) {
        // one workgroup of whole wavefronts per RPT rows, each thread taking
        // the same x position in every row with all its loads issued first
        // (measured at N = 7 on the 32^3 case, before the segment pass took
        // over there: 79 us with one row, 69 us with two or three, 78 with four)
        constexpr int RPT = 2;
        const int nxp = (nxl + 63) / 64 * 64;
        const dim3 block((unsigned)nxp), grid((unsigned)((rows + RPT - 1) / RPT));
        const size_t lds = (size_t)RPT * 4 * nxl * sizeof(T);
        if (apply_mask)
            hipLaunchKernelGGL((gs_lattice_kernel<T, 1, RPT>), grid, block, lds, s, u, L, skip);
        else
            hipLaunchKernelGGL((gs_lattice_kernel<T, 0, RPT>), grid, block, lds, s, u, L, skip);
        return hipGetLastError();
    }
    const unsigned g1 = (unsigned)rows;
    const int mx = L.per[0] ? L.nelx : L.nelx + 1;
    const unsigned g2 = (unsigned)((mx * rows + 255) / 256);
    if (apply_mask) {
        hipLaunchKernelGGL((gs_rows_kernel<T, 1>), dim3(g1), dim3(256), 0, s, u, L, skip);
        hipLaunchKernelGGL((gs_xface_kernel<T, 1>), dim3(g2), dim3(256), 0, s, u, L, mx, skip);
    } else {
        hipLaunchKernelGGL((gs_rows_kernel<T, 0>), dim3(g1), dim3(256), 0, s, u, L, skip);
        hipLaunchKernelGGL((gs_xface_kernel<T, 0>), dim3(g2), dim3(256), 0, s, u, L, mx, skip);
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_dssum_f64(const Mesh &m, double *u, int apply_mask, hipStream_t s,
                           const int32_t *skip)
{
    return dssum_impl<double>(m, u, apply_mask, s, skip);
}

hipError_t launch_dssum_f32(const Mesh &m, float *u, int apply_mask, hipStream_t s,
                           const int32_t *skip)
{
    return dssum_impl<float>(m, u, apply_mask, s, skip);
}

hipError_t launch_scale_by_B(const Mesh &m, const double *f, double *b, hipStream_t s)
{
    if (m.nl == 0) return hipSuccess;
    hipLaunchKernelGGL(scale_by_B_kernel, dim3(blocks_for(m.nl, 256)), dim3(256), 0, s, f, m.d_B, b, m.nl);
    return hipGetLastError();
}

hipError_t launch_jacobi_finish(const Mesh &m, double *d, hipStream_t s)
{
    if (m.nl == 0) return hipSuccess;
    hipLaunchKernelGGL(jacobi_finish_kernel, dim3(blocks_for(m.nl, 256)), dim3(256), 0, s, d, m.d_wcode, m.nl);
    return hipGetLastError();
}

int dot_blocks(const Mesh &m)
{
    const int64_t b = (m.nl + kDotBlock - 1) / kDotBlock;
    return (int)std::max<int64_t>(1, std::min<int64_t>(b, kDotMaxBlocks));
}

hipError_t launch_dot(const Mesh &m, const double *u, const double *v, double *partials,
                      int nblocks, double *result, hipStream_t s)
{
    hipLaunchKernelGGL(dot_partial_kernel, dim3(nblocks), dim3(kDotBlock), 0, s, u, v, m.d_mult, m.nl, partials);
    hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(kDotBlock), 0, s, partials, nblocks, result);
    return hipGetLastError();
}

}  // namespace sem
