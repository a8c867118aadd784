// hsmg.hip -- the paper's pressure preconditioner and Krylov method
// (section 3.1, "Neko": restarted GMRES with a hybrid-Schwarz multigrid
// preconditioner; CG with block-Jacobi for the velocity solves), on
// assembled vectors.
//
// One preconditioner application z = M r (three levels, orders N, 3, 1):
//   1. fine Schwarz: per element (one workgroup, one thread per node) gather
//      r_e, fast-diagonalisation solve (three forward contractions with the
//      element's S^T, division by h1 (lx + ly + lz) + h2, three backward
//      contractions with S) -> fine rows; in the same pass r_e / mult is
//      restricted to order 3 (J^T along r, s, t) -> mid rows
//   2. mid assembly: r_m = mask(sum of copies)
//   3. mid Schwarz (one wavefront per element at order 3) -> mid rows, and
//      restriction to order 1 -> coarse rows
//   4. coarse assembly; 5. coarse solve: six axis contractions with the
//      global separable factors on the order-1 lattice
//   6. z_m = mask(sum of copies / mult) + P z_c (node-wise interpolation)
//   7. per element: z_p = J (x) J (x) J z_m at the nodes the element owns
//   8. z = mask(sum of copies / mult) + z_p: the averaged fine Schwarz
//      correction plus the prolongated coarser levels.
// (In the symmetric weighting the averages are 1/sqrt(mult) on both sides
// of the local solves.)
// All sums run in a fixed order, so results are bitwise reproducible.
//
// Flexible GMRES(m) (Saad 2003, Algorithm 9.6) keeps V (m+1 vectors) and
// Z = M V (m vectors) on the device; the Hessenberg column and Givens
// rotations are handled on the host, which reads the (j+2) inner products
// of each Arnoldi step (one synchronisation per iteration).  The new
// direction's inner products with every V_i and its own norm come from one
// fused pass that also assembles S Z_j (wave-shuffle partial sums, fixed
// order); its norm after the projection follows from those (Pythagoras) and
// one more pass subtracts the projections and normalises.  When the
// direction keeps less than 1/sqrt(2) of its norm, classical Gram-Schmidt
// takes a second pass ("twice is enough"), whose inner products come from
// the same read of V as the first update: three passes over V instead of
// four.
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "hsmg.hpp"
#include "nn.hpp"
#include "reduce.hpp"

namespace sem {

// Device-resident state of one GMRES restart cycle: the Hessenberg matrix
// (row-major, row stride kGmresMaxRestart), the Givens rotations, the
// rotated right-hand side g, |g[j+1]| after each step, the coefficients the
// normalisation subtracts, and the flags the skipping kernels read.
struct GmresDev {
    double H[(kGmresMaxRestart + 1) * kGmresMaxRestart];
    double cs[kGmresMaxRestart], sn[kGmresMaxRestart], g[kGmresMaxRestart + 1];
    double res[kGmresMaxRestart];
    double coef[kGmresMaxRestart + 2];
    double beta2, inv_bj, tol_abs;
    int skip_re;   // no second Gram-Schmidt pass in this step (or stopped)
    int stop;      // 0 running; 1 converged, at max_it or lucky breakdown; 2 non-finite
    int k, it, max_it, pad;
};

namespace mg {

#define GRID_STRIDE(g, n) for (int64_t g = (int64_t)blockIdx.x * kBS + threadIdx.x; g < (n); g += (int64_t)gridDim.x * kBS)

constexpr int kRowsPerBlock = 4;   // lattice rows per workgroup of the row-blocked node kernels

__device__ __forceinline__ bool node_masked(const Lattice &L, int gi, int gj, int gk)
{
    return axis_dirichlet(L, 0, gi, L.nelx) || axis_dirichlet(L, 1, gj, L.nely) || axis_dirichlet(L, 2, gk, L.nelz);
}

template <int NPC = 0>
__device__ __forceinline__ int node_count(const Lattice &L, int gi, int gj, int gk)
{
    int X[2];
    return axis_copies_t<NPC>(gi, L.nelx, L.N, L.per[0] != 0, X) * axis_copies_t<NPC>(gj, L.nely, L.N, L.per[1] != 0, X) *
           axis_copies_t<NPC>(gk, L.nelz, L.N, L.per[2] != 0, X);
}

// Block partial sums of NV values per thread: wave butterfly, then the
// waves of the block in order (deterministic); part[q * nb + block].
template <int NV>
__device__ __forceinline__ void block_partials(double (&acc)[NV], int nv, double *__restrict__ part, int nb)
{
    __shared__ double red[kBS / 64][NV];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        if (q < nv) {
            double v = acc[q];
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
            if (lane == 0) red[wv][q] = v;
        }
    }
    __syncthreads();
    for (int q = threadIdx.x; q < nv; q += kBS) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < kBS / 64; ++w) s += red[w][q];
        part[(int64_t)q * nb + blockIdx.x] = s;
    }
}

// ---------------------------------------------------------------- level kernels

// Element Schwarz solve (and, NPC > 0, restriction of r / mult to the
// coarser level's NPC points per direction).  One workgroup of NP^3 threads
// per element, thread = node (i, j, k).
template <int NP, int NPC>
__global__ void __launch_bounds__(NP * NP * NP)
schwarz_kernel(const double *__restrict__ rg, Lattice L, const double *__restrict__ fdm, double h1, double h2,
               double *__restrict__ rows, const double *__restrict__ J, Lattice Lc, double *__restrict__ rows_c,
               int sym)
{
    constexpr int P2 = NP * NP, P3 = P2 * NP, NF = 3 * P2 + 3 * NP;
    constexpr int NJ = NPC > 0 ? NP * NPC : 1;
    __shared__ double sF[NF];
    __shared__ double sa[P3], sb[P3];
    __shared__ double sJ[NJ];
    const int t = threadIdx.x, i = t % NP, j = (t / NP) % NP, k = t / P2;
    const int64_t e = xcd_block();
    int ex, ey, ez;
    elem_coords(L, e, ex, ey, ez);
    const double r = rg[gather_index32(L, ex, ey, ez, i, j, k)];
    for (int q = t; q < NF; q += P3) sF[q] = fdm[e * NF + q];
    if constexpr (NPC > 0)
        for (int q = t; q < NJ; q += P3) sJ[q] = J[q];
    const int gi0 = ex * L.N + i, gj0 = ey * L.N + j, gk0 = ez * L.N + k;
    const int cnt = node_count(L, gi0 >= L.nx ? gi0 - (int)L.nx : gi0, gj0 >= L.ny ? gj0 - (int)L.ny : gj0,
                               gk0 >= L.nz ? gk0 - (int)L.nz : gk0);
    sa[t] = sym ? r / sqrt((double)cnt) : r;   // symmetric weighting: 1/sqrt(mult) on both sides
    __syncthreads();
    const double *Sx = sF, *Sy = sF + P2, *Sz = sF + 2 * P2;
    const double *lx = sF + 3 * P2, *ly = lx + NP, *lz = ly + NP;
    double v = 0.0;
#pragma unroll
    for (int a = 0; a < NP; ++a) v += Sx[a * NP + i] * sa[k * P2 + j * NP + a];   // modes along r
    sb[t] = v;
    __syncthreads();
    v = 0.0;
#pragma unroll
    for (int b = 0; b < NP; ++b) v += Sy[b * NP + j] * sb[k * P2 + b * NP + i];   // along s
    sa[t] = v;
    __syncthreads();
    v = 0.0;
#pragma unroll
    for (int c = 0; c < NP; ++c) v += Sz[c * NP + k] * sa[c * P2 + j * NP + i];   // along t
    const double d = h1 * (lx[i] + ly[j] + lz[k]) + h2;                         // +inf on unused modes
    sb[t] = d > 0.0 ? v / d : 0.0;
    __syncthreads();
    v = 0.0;
#pragma unroll
    for (int c = 0; c < NP; ++c) v += Sz[k * NP + c] * sb[c * P2 + j * NP + i];
    sa[t] = v;
    __syncthreads();
    v = 0.0;
#pragma unroll
    for (int b = 0; b < NP; ++b) v += Sy[j * NP + b] * sa[k * P2 + b * NP + i];
    sb[t] = v;
    __syncthreads();
    v = 0.0;
#pragma unroll
    for (int a = 0; a < NP; ++a) v += Sx[i * NP + a] * sb[k * P2 + j * NP + a];
    rows[rows_index32(L, ex, ey, ez, i, j, k)] = v;
    if constexpr (NPC > 0) {
        // restriction of r / mult: J^T along r, then s, then t
        __syncthreads();   // sa is free again
        sa[t] = r / cnt;
        __syncthreads();
        if (t < NPC * P2) {
            const int c = t % NPC, jj = (t / NPC) % NP, kk = t / (NPC * NP);
            double s = 0.0;
#pragma unroll
            for (int q = 0; q < NP; ++q) s += sJ[q * NPC + c] * sa[kk * P2 + jj * NP + q];
            sb[(kk * NP + jj) * NPC + c] = s;
        }
        __syncthreads();
        if (t < NPC * NPC * NP) {
            const int a = t % NPC, b = (t / NPC) % NPC, kk = t / (NPC * NPC);
            double s = 0.0;
#pragma unroll
            for (int q = 0; q < NP; ++q) s += sJ[q * NPC + b] * sb[(kk * NP + q) * NPC + a];
            sa[(kk * NPC + b) * NPC + a] = s;
        }
        __syncthreads();
        if (t < NPC * NPC * NPC) {
            const int a = t % NPC, b = (t / NPC) % NPC, c = t / (NPC * NPC);
            double s = 0.0;
#pragma unroll
            for (int q = 0; q < NP; ++q) s += sJ[q * NPC + c] * sa[(q * NPC + b) * NPC + a];
            rows_c[rows_index32(Lc, ex, ey, ez, a, b, c)] = s;
        }
    }
}

// Restriction alone (the learned multigrid, whose fine level is not a
// Schwarz solve): rows_c = J^T (x) J^T (x) J^T (r / mult) per element, NPC
// points per direction on the coarser level.  One workgroup of NP^3 threads
// per element, thread = node (i, j, k); the same contraction order as the
// Schwarz kernels' restriction.
template <int NP, int NPC>
__global__ void __launch_bounds__(NP * NP * NP)
restrict_kernel(const double *__restrict__ rg, Lattice L, const double *__restrict__ J, Lattice Lc,
                double *__restrict__ rows_c)
{
    constexpr int P2 = NP * NP;
    __shared__ double sa[P2 * NP], sb[P2 * NP];
    __shared__ double sJ[NP * NPC];
    const int t = threadIdx.x, i = t % NP, j = (t / NP) % NP, k = t / P2;
    const int64_t e = xcd_block();
    int ex, ey, ez;
    elem_coords(L, e, ex, ey, ez);
    const double r = rg[gather_index32(L, ex, ey, ez, i, j, k)];
    for (int q = t; q < NP * NPC; q += P2 * NP) sJ[q] = J[q];
    const int gi0 = ex * L.N + i, gj0 = ey * L.N + j, gk0 = ez * L.N + k;
    const int cnt = node_count(L, gi0 >= L.nx ? gi0 - (int)L.nx : gi0, gj0 >= L.ny ? gj0 - (int)L.ny : gj0,
                               gk0 >= L.nz ? gk0 - (int)L.nz : gk0);
    sa[t] = r / cnt;
    __syncthreads();
    if (t < NPC * P2) {
        const int c = t % NPC, jj = (t / NPC) % NP, kk = t / (NPC * NP);
        double v = 0.0;
#pragma unroll
        for (int q = 0; q < NP; ++q) v += sJ[q * NPC + c] * sa[kk * P2 + jj * NP + q];
        sb[(kk * NP + jj) * NPC + c] = v;
    }
    __syncthreads();
    if (t < NPC * NPC * NP) {
        const int a = t % NPC, b = (t / NPC) % NPC, kk = t / (NPC * NPC);
        double v = 0.0;
#pragma unroll
        for (int q = 0; q < NP; ++q) v += sJ[q * NPC + b] * sb[(kk * NP + q) * NPC + a];
        sa[(kk * NPC + b) * NPC + a] = v;
    }
    __syncthreads();
    if (t < NPC * NPC * NPC) {
        const int a = t % NPC, b = (t / NPC) % NPC, c = t / (NPC * NPC);
        double v = 0.0;
#pragma unroll
        for (int q = 0; q < NP; ++q) v += sJ[q * NPC + c] * sa[(q * NPC + b) * NPC + a];
        rows_c[rows_index32(Lc, ex, ey, ez, a, b, c)] = v;
    }
}

// The same element Schwarz solve at N = 7 with one wavefront per element and
// one x-pencil of 8 nodes per lane: every contraction runs on the 8 values a
// lane holds in registers, with the element's factors as wave-uniform
// (scalar) operands, and the pencils change direction through a padded LDS
// tile (four transposes per solve instead of six LDS-staged contractions of
// 512 threads).  (Staging the factors in LDS instead made the compiler hold
// all 64 entries of a matrix in vector registers: 210 VGPRs, or spills when
// capped.)  Lane t = (a, b) owns the pencil along the direction of the
// current phase; NPC > 0 also restricts r / mult to NPC points.
template <int NPC>
__global__ void __launch_bounds__(64)
schwarz_pencil_kernel(const double *__restrict__ rg, Lattice L, const double *__restrict__ fdm, double h1, double h2,
                      double *__restrict__ rows, const double *__restrict__ J, Lattice Lc, double *__restrict__ rows_c,
                      int sym)
{
    constexpr int NP = 8, P2 = 64, NF = 3 * P2 + 3 * NP, PAD = 9;
    __shared__ double T[NP * NP * PAD];   // [k][j][i] with a 9-double row pitch
    const int t = threadIdx.x, ta = t & 7, tb = t >> 3;
    const int64_t e = __builtin_amdgcn_readfirstlane((int)xcd_block());
    int ex, ey, ez;
    elem_coords(L, e, ex, ey, ez);
    const double *__restrict__ F = fdm + e * NF;   // wave-uniform: scalar loads
    const double *Sx = F, *Sy = F + P2, *Sz = F + 2 * P2, *lx = F + 3 * P2, *ly = lx + NP, *lz = ly + NP;
    auto T_at = [&](int k, int j, int i) -> double & { return T[(k * NP + j) * PAD + i]; };
    // x-pencils: lane (j, k) = (ta, tb)
    double r[NP], v[NP], o[NP];
    int cnt[NP];   // copies of each node of the pencil
#pragma unroll
    for (int i = 0; i < NP; ++i) r[i] = rg[gather_index32(L, ex, ey, ez, i, ta, tb)];
    {
        const int gj = ey * L.N + ta, gk = ez * L.N + tb;
        int X[2];
        const int cyz = axis_copies_t<NP>(gj >= L.ny ? gj - (int)L.ny : gj, L.nely, L.N, L.per[1] != 0, X) *
                        axis_copies_t<NP>(gk >= L.nz ? gk - (int)L.nz : gk, L.nelz, L.N, L.per[2] != 0, X);
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            int gi = ex * L.N + i;
            if (gi >= L.nx) gi -= (int)L.nx;
            cnt[i] = cyz * axis_copies_t<NP>(gi, L.nelx, L.N, L.per[0] != 0, X);
        }
    }
#pragma unroll
    for (int i = 0; i < NP; ++i) v[i] = sym ? r[i] / sqrt((double)cnt[i]) : r[i];   // symmetric weighting
#pragma unroll
    for (int q = 0; q < NP; ++q) o[q] = 0.0;
#pragma unroll
    for (int a = 0; a < NP; ++a)
#pragma unroll
        for (int q = 0; q < NP; ++q) o[q] += Sx[a * NP + q] * v[a];
#pragma unroll
    for (int q = 0; q < NP; ++q) T_at(tb, ta, q) = o[q];
    __syncthreads();
    // y-pencils: lane (i, k) = (ta, tb)
#pragma unroll
    for (int b = 0; b < NP; ++b) v[b] = T_at(tb, b, ta);
#pragma unroll
    for (int q = 0; q < NP; ++q) o[q] = 0.0;
#pragma unroll
    for (int b = 0; b < NP; ++b)
#pragma unroll
        for (int q = 0; q < NP; ++q) o[q] += Sy[b * NP + q] * v[b];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NP; ++q) T_at(tb, q, ta) = o[q];
    __syncthreads();
    // z-pencils: lane (i, j) = (ta, tb); forward, divide, backward in registers
#pragma unroll
    for (int c = 0; c < NP; ++c) v[c] = T_at(c, tb, ta);
#pragma unroll
    for (int q = 0; q < NP; ++q) o[q] = 0.0;
#pragma unroll
    for (int c = 0; c < NP; ++c)
#pragma unroll
        for (int q = 0; q < NP; ++q) o[q] += Sz[c * NP + q] * v[c];
    const double lxy = lx[ta] + ly[tb];
#pragma unroll
    for (int q = 0; q < NP; ++q) {
        const double d = h1 * (lxy + lz[q]) + h2;   // +inf on unused modes
        o[q] = d > 0.0 ? o[q] / d : 0.0;
    }
#pragma unroll
    for (int c = 0; c < NP; ++c) {
        double s = 0.0;
#pragma unroll
        for (int q = 0; q < NP; ++q) s += Sz[c * NP + q] * o[q];
        v[c] = s;
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < NP; ++c) T_at(c, tb, ta) = v[c];
    __syncthreads();
    // y-pencils again: lane (i, k)
#pragma unroll
    for (int q = 0; q < NP; ++q) o[q] = T_at(tb, q, ta);
#pragma unroll
    for (int b = 0; b < NP; ++b) {
        double s = 0.0;
#pragma unroll
        for (int q = 0; q < NP; ++q) s += Sy[b * NP + q] * o[q];
        v[b] = s;
    }
    __syncthreads();
#pragma unroll
    for (int b = 0; b < NP; ++b) T_at(tb, b, ta) = v[b];
    __syncthreads();
    // x-pencils again: lane (j, k)
#pragma unroll
    for (int q = 0; q < NP; ++q) o[q] = T_at(tb, ta, q);
#pragma unroll
    for (int a = 0; a < NP; ++a) {
        double s = 0.0;
#pragma unroll
        for (int q = 0; q < NP; ++q) s += Sx[a * NP + q] * o[q];
        rows[rows_index32(L, ex, ey, ez, a, ta, tb)] = s;
    }
    if constexpr (NPC > 0) {
        // restriction of r / mult (x-pencils still in r): J^T along x in
        // registers, then along y and z through the tile
        double s1[NPC];
#pragma unroll
        for (int c = 0; c < NPC; ++c) s1[c] = 0.0;
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            const double rr = r[i] / cnt[i];
#pragma unroll
            for (int c = 0; c < NPC; ++c) s1[c] += J[i * NPC + c] * rr;
        }
        __syncthreads();
#pragma unroll
        for (int c = 0; c < NPC; ++c) T_at(tb, ta, c) = s1[c];   // [k][j][a']
        __syncthreads();
        // lanes (a', k) with a' < NPC: along y
        double s2[NPC];
        if (ta < NPC) {
#pragma unroll
            for (int c = 0; c < NPC; ++c) s2[c] = 0.0;
#pragma unroll
            for (int j = 0; j < NP; ++j) {
                const double w = T_at(tb, j, ta);
#pragma unroll
                for (int c = 0; c < NPC; ++c) s2[c] += J[j * NPC + c] * w;
            }
        }
        __syncthreads();
        if (ta < NPC) {
#pragma unroll
            for (int c = 0; c < NPC; ++c) T_at(tb, c, ta) = s2[c];   // [k][b'][a']
        }
        __syncthreads();
        // lanes (a', b') with both < NPC: along z
        if (ta < NPC && tb < NPC) {
#pragma unroll
            for (int c = 0; c < NPC; ++c) {
                double s = 0.0;
#pragma unroll
                for (int k = 0; k < NP; ++k) s += J[k * NPC + c] * T_at(k, tb, ta);
                rows_c[rows_index32(Lc, ex, ey, ez, ta, tb, c)] = s;
            }
        }
    }
}

// Fine-level result: z[g] = mask(W (sum of the copies of rows at g)) +
// zp[g], W = 1, 1 / mult or 1 / sqrt(mult); zp (optional) is the
// prolongated coarser-level correction, one value per node.  kRowsPerBlock
// lattice rows per workgroup, every load issued before the arithmetic.
//
// part (optional): block partials of (r, out), for the CG that applies the
// preconditioner (saves its separate inner-product pass over r and z).
template <int NPC>
__global__ void __launch_bounds__(kBS)
assemble_fine_kernel(const double *__restrict__ rows, Lattice L, int weighted, const double *__restrict__ zp,
                     double *__restrict__ out, const double *__restrict__ r, double *__restrict__ part)
{
    const int nrows = (int)(L.ny * L.nz), ny = (int)L.ny, nx = (int)L.nx, row0 = (int)blockIdx.x * kRowsPerBlock;
    double acc[1] = {0.0};
    for (int gi = threadIdx.x; gi < nx; gi += kBS) {
        double v[kRowsPerBlock], a[kRowsPerBlock], rv[kRowsPerBlock];
        int64_t g[kRowsPerBlock];
        int gj[kRowsPerBlock], gk[kRowsPerBlock];
#pragma unroll
        for (int q = 0; q < kRowsPerBlock; ++q) {
            const int row = row0 + q < nrows ? row0 + q : nrows - 1;
            gj[q] = row % ny;
            gk[q] = row / ny;
            g[q] = gi + (int64_t)nx * row;
            v[q] = node_assemble_rows<NPC>(L, rows, gi, gj[q], gk[q]);
            a[q] = zp ? zp[g[q]] : 0.0;
            rv[q] = part ? r[g[q]] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < kRowsPerBlock; ++q) {
            if (row0 + q >= nrows) continue;
            double z = 0.0;
            if (!node_masked(L, gi, gj[q], gk[q])) {
                z = v[q];
                if (weighted == kWeightAvg) z /= node_count<NPC>(L, gi, gj[q], gk[q]);
                if (weighted == kWeightSym) z /= sqrt((double)node_count<NPC>(L, gi, gj[q], gk[q]));
                z += a[q];
            }
            out[g[q]] = z;
            acc[0] += rv[q] * z;
        }
    }
    if (part) block_partials<1>(acc, 1, part, gridDim.x);
}

// zp = J (x) J (x) J zm (the mid level's assembled correction interpolated
// to the fine nodes), one value per fine node: every element interpolates
// its nodes and writes those it owns (local index below N along each axis,
// or the last element along a non-periodic axis), so each node is written
// once
template <int NP, int NPM>
__global__ void __launch_bounds__(NP * NP * NP)
prolong_owned_kernel(const double *__restrict__ zm, Lattice Lm, const double *__restrict__ J, Lattice L,
                     double *__restrict__ zp)
{
    constexpr int P3 = NP * NP * NP;
    __shared__ double s0[NPM * NPM * NPM], s1[NP * NPM * NPM], s2[NP * NP * NPM];
    __shared__ double sJ[NP * NPM];
    const int t = threadIdx.x, i = t % NP, j = (t / NP) % NP, k = t / (NP * NP);
    const int64_t e = xcd_block();
    int ex, ey, ez;
    elem_coords(L, e, ex, ey, ez);
    if (t < NPM * NPM * NPM) {
        const int a = t % NPM, b = (t / NPM) % NPM, c = t / (NPM * NPM);
        s0[t] = zm[gather_index32(Lm, ex, ey, ez, a, b, c)];
    }
    for (int q = t; q < NP * NPM; q += P3) sJ[q] = J[q];
    __syncthreads();
    if (t < NP * NPM * NPM) {
        const int ii = t % NP, b = (t / NP) % NPM, c = t / (NP * NPM);
        double s = 0.0;
#pragma unroll
        for (int a = 0; a < NPM; ++a) s += sJ[ii * NPM + a] * s0[(c * NPM + b) * NPM + a];
        s1[t] = s;
    }
    __syncthreads();
    if (t < NP * NP * NPM) {
        const int ii = t % NP, jj = (t / NP) % NP, c = t / (NP * NP);
        double s = 0.0;
#pragma unroll
        for (int b = 0; b < NPM; ++b) s += sJ[jj * NPM + b] * s1[(c * NPM + b) * NP + ii];
        s2[t] = s;
    }
    __syncthreads();
    const int N = L.N;
    const bool own = (i < N || (ex == L.nelx - 1 && !L.per[0])) && (j < N || (ey == L.nely - 1 && !L.per[1])) &&
                     (k < N || (ez == L.nelz - 1 && !L.per[2]));
    if (!own) return;
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < NPM; ++c) s += sJ[k * NPM + c] * s2[(c * NP + j) * NP + i];
    zp[gather_index32(L, ex, ey, ez, i, j, k)] = s;
}

// N = 7 with the order-3 middle level: the same interpolation with one
// wavefront per element and the same sums in the same order.  The 64 lanes
// load the 4^3 middle values, each lane forms two of the 128 x-interpolated
// values, then lane (j, k) finishes the x-pencil zp(0..7, j, k) in registers
// and writes the nodes it owns (eight consecutive global nodes per lane).
__global__ void __launch_bounds__(64)
prolong_pencil_kernel(const double *__restrict__ zm, Lattice Lm, const double *__restrict__ J, Lattice L,
                      double *__restrict__ zp)
{
    constexpr int NP = 8, NPM = 4;
    __shared__ double s0[NPM * NPM * NPM], s1[NP * NPM * NPM], sJ[NP * NPM];
    const int t = threadIdx.x & 63;
    const int64_t e = xcd_block();
    int ex, ey, ez;
    elem_coords(L, e, ex, ey, ez);
    s0[t] = zm[gather_index32(Lm, ex, ey, ez, t % NPM, (t / NPM) % NPM, t / (NPM * NPM))];
    if (t < NP * NPM) sJ[t] = J[t];
    __syncthreads();
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int q = t + 64 * h, ii = q % NP, b = (q / NP) % NPM, c = q / (NP * NPM);
        double s = 0.0;
#pragma unroll
        for (int a = 0; a < NPM; ++a) s += sJ[ii * NPM + a] * s0[(c * NPM + b) * NPM + a];
        s1[q] = s;
    }
    __syncthreads();
    const int j = t % NP, k = t / NP;
    const int N = L.N;
    const bool own_jk = (j < N || (ey == L.nely - 1 && !L.per[1])) && (k < N || (ez == L.nelz - 1 && !L.per[2]));
    if (!own_jk) return;
    const bool last_x = ex == L.nelx - 1 && !L.per[0];
    double Jj[NPM], Jk[NPM];
#pragma unroll
    for (int b = 0; b < NPM; ++b) {
        Jj[b] = sJ[j * NPM + b];
        Jk[b] = sJ[k * NPM + b];
    }
    const int64_t g0 = gather_index32(L, ex, ey, ez, 0, j, k);   // the pencil's 8 nodes are consecutive
#pragma unroll 2
    for (int i = 0; i < NP; ++i) {
        if (i == N && !last_x) continue;
        double s = 0.0;
#pragma unroll
        for (int c = 0; c < NPM; ++c) {
            double s2 = 0.0;
#pragma unroll
            for (int b = 0; b < NPM; ++b) s2 += Jj[b] * s1[(c * NPM + b) * NP + i];
            s += Jk[c] * s2;
        }
        zp[g0 + i] = s;
    }
}

// out[g] = mask(sum of the copies of rows at g, times 1 / count
// (kWeightAvg) or 1 / sqrt(count) (kWeightSym)) + (zc != null: the order-1
// interpolant of zc at g); NPC = N + 1 of the level fixed at compile time
// (0: any)
template <int NPC>
__global__ void __launch_bounds__(kBS)
assemble_kernel(const double *__restrict__ rows, Lattice L, int weighted, double *__restrict__ out,
                const double *__restrict__ zc, Lattice Lc, const double *__restrict__ J)
{
    SEM_FOR_EACH_NODE(L, gi, gj, gk, g)
    {
        if (node_masked(L, gi, gj, gk)) {
            out[g] = 0.0;
            continue;
        }
        double v = node_assemble_rows<NPC>(L, rows, gi, gj, gk);
        if (weighted == kWeightAvg) v /= node_count<NPC>(L, gi, gj, gk);
        if (weighted == kWeightSym) v /= sqrt((double)node_count<NPC>(L, gi, gj, gk));
        if (zc) {
            const int N = L.N;
            int ex = gi / N, ey = gj / N, ez = gk / N;
            if (ex >= L.nelx) ex = L.nelx - 1;
            if (ey >= L.nely) ey = L.nely - 1;
            if (ez >= L.nelz) ez = L.nelz - 1;
            const int i = gi - ex * N, j = gj - ey * N, k = gk - ez * N;
            double s = 0.0;
            for (int c = 0; c < 2; ++c)
                for (int b = 0; b < 2; ++b)
                    for (int a = 0; a < 2; ++a)
                        s += J[i * 2 + a] * J[j * 2 + b] * J[k * 2 + c] * zc[gather_index32(Lc, ex, ey, ez, a, b, c)];
            v += s;
        }
        out[g] = v;
    }
}

// One axis of the global coarse solve on the (nz, ny, nx) order-1 lattice:
// forward out[.., q, ..] = sum_a S[a][q] in[.., a, ..] (then, scale != 0,
// divided by h1 (lx + ly + lz) + h2), backward out[.., a, ..] = sum_q S[a][q] in[.., q, ..].
__global__ void __launch_bounds__(kBS)
coarse_axis_kernel(const double *__restrict__ in, double *__restrict__ out, const double *__restrict__ S, int axis,
                   int fwd, int nx, int ny, int nz, const double *__restrict__ lx, const double *__restrict__ ly,
                   const double *__restrict__ lz, double h1, double h2, int scale)
{
    const int64_t ntot = (int64_t)nx * ny * nz;
    const int n = axis == 0 ? nx : (axis == 1 ? ny : nz);
    const int64_t stride = axis == 0 ? 1 : (axis == 1 ? nx : (int64_t)nx * ny);
    GRID_STRIDE(g, ntot)
    {
        const int i = (int)(g % nx), j = (int)((g / nx) % ny), k = (int)(g / ((int64_t)nx * ny));
        const int idx = axis == 0 ? i : (axis == 1 ? j : k);
        const int64_t base = g - idx * stride;
        double v = 0.0;
        if (fwd)
            for (int a = 0; a < n; ++a) v += S[a * n + idx] * in[base + a * stride];
        else
            for (int q = 0; q < n; ++q) v += S[idx * n + q] * in[base + q * stride];
        if (scale) {
            const double d = h1 * (lx[i] + ly[j] + lz[k]) + h2;
            v = d > 0.0 ? v / d : 0.0;
        }
        out[g] = v;
    }
}

// The coarse solve in three launches instead of six, same arithmetic order
// per output (bit-identical to coarse_axis_kernel's six passes):
//  - coarse_plane_kernel: one workgroup per z-plane, the plane in LDS; the
//    x then the y transform (forward), or y then x (backward), each output
//    computed into registers, then written back over the plane;
//  - coarse_column_kernel: whole z-columns in LDS, forward z transform,
//    division by the eigenvalue sum, backward z transform.
constexpr int kCoarsePlane = 4352;   // LDS plane capacity (doubles): up to 64 x 68 nodes
// 1024 threads per plane: at 32^3 the lattice has 33 planes of 1,089 nodes, so
// the grid is small and each thread's outputs (length-n dot products) are
// the critical path
constexpr int kPlaneThreads = 1024;
constexpr int kCoarsePer = (kCoarsePlane + kPlaneThreads - 1) / kPlaneThreads;
__global__ void __launch_bounds__(kPlaneThreads)
coarse_plane_kernel(double *__restrict__ u, const double *__restrict__ Sx, const double *__restrict__ Sy, int nx, int ny,
                    int fwd)
{
    __shared__ double T[kCoarsePlane];
    const int np = nx * ny;
    double *pl = u + (int64_t)blockIdx.x * np;
    for (int g = threadIdx.x; g < np; g += kPlaneThreads) T[g] = pl[g];
    __syncthreads();
    for (int ph = 0; ph < 2; ++ph) {
        // forward: x then y; backward: y then x
        const int ax = fwd ? ph : 1 - ph;
        const int n = ax == 0 ? nx : ny;
        const double *S = ax == 0 ? Sx : Sy;
        double v[kCoarsePer];
#pragma unroll
        for (int r = 0; r < kCoarsePer; ++r) {
            const int g = threadIdx.x + r * kPlaneThreads;
            v[r] = 0.0;
            if (g >= np) continue;
            const int i = g % nx, j = g / nx;
            const int idx = ax == 0 ? i : j;
            const int base = ax == 0 ? j * nx : i, stride = ax == 0 ? 1 : nx;
            double acc = 0.0;
            if (fwd)
                for (int a = 0; a < n; ++a) acc += S[a * n + idx] * T[base + a * stride];
            else
                for (int q = 0; q < n; ++q) acc += S[idx * n + q] * T[base + q * stride];
            v[r] = acc;
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < kCoarsePer; ++r) {
            const int g = threadIdx.x + r * kPlaneThreads;
            if (g < np) T[g] = v[r];
        }
        __syncthreads();
    }
    for (int g = threadIdx.x; g < np; g += kPlaneThreads) pl[g] = T[g];
}

// z-columns (i, j) of the coarse lattice, ncol = kBS / nz per workgroup:
// forward transform along z, divided by h1 (lx + ly + lz) + h2 (0 where that
// is not positive), backward transform
__global__ void __launch_bounds__(kBS)
coarse_column_kernel(double *__restrict__ u, const double *__restrict__ Sz, int nx, int ny, int nz,
                     const double *__restrict__ lx, const double *__restrict__ ly, const double *__restrict__ lz,
                     double h1, double h2)
{
    __shared__ double T[kBS];
    const int ncol = kBS / nz, c = threadIdx.x / nz, k = threadIdx.x % nz;
    const int64_t col = (int64_t)blockIdx.x * ncol + c;
    const int64_t plane = (int64_t)nx * ny;
    const bool on = c < ncol && col < plane;
    if (on) T[threadIdx.x] = u[col + k * plane];
    __syncthreads();
    double v = 0.0;
    if (on) {
        const double *t = T + c * nz;
        for (int a = 0; a < nz; ++a) v += Sz[a * nz + k] * t[a];
        const int i = (int)(col % nx), j = (int)(col / nx);
        const double d = h1 * (lx[i] + ly[j] + lz[k]) + h2;
        v = d > 0.0 ? v / d : 0.0;
    }
    __syncthreads();
    if (on) T[threadIdx.x] = v;
    __syncthreads();
    if (on) {
        const double *t = T + c * nz;
        double w = 0.0;
        for (int q = 0; q < nz; ++q) w += Sz[k * nz + q] * t[q];
        u[col + k * plane] = w;
    }
}

// ---------------------------------------------------------------- Krylov kernels

constexpr int kMaxDots = kGmresMaxRestart + 2;   // (V_i, w) for i <= j, plus (w, w)

// partials of (V_i, w), i <= j, and (w, w) for an assembled w
__global__ void __launch_bounds__(kBS)
dots_kernel(const double *__restrict__ w, const double *__restrict__ V, int64_t ng, int j, double *__restrict__ part)
{
    double acc[kMaxDots];
#pragma unroll
    for (int q = 0; q < kMaxDots; ++q) acc[q] = 0.0;
    GRID_STRIDE(g, ng)
    {
        const double wg = w[g];
#pragma unroll
        for (int q = 0; q < kMaxDots - 1; ++q)
            if (q <= j) acc[q] += V[q * ng + g] * wg;
        const double ww = wg * wg;
#pragma unroll
        for (int q = 0; q < kMaxDots; ++q)
            if (q == j + 1) acc[q] += ww;
    }
    block_partials<kMaxDots>(acc, j + 2, part, gridDim.x);
}

// h[q] = sum of stage[q * kStage ...] for q < nv
__global__ void __launch_bounds__(kBS) sums_finalize(const double *__restrict__ stage, int nv, double *__restrict__ h,
                                                     const int *__restrict__ skip = nullptr)
{
    if (skip && *skip) return;   // uniform across the block
    for (int q = 0; q < nv; ++q) {
        __shared__ double red[kBS];
        red[threadIdx.x] = stage[q * kStage + threadIdx.x];
        __syncthreads();
        for (int w = kBS / 2; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) h[q] = red[0];
        __syncthreads();
    }
}

// w = (w - sum_{i <= j} h_i V_i) * scale (scale from device memory)
__global__ void __launch_bounds__(kBS)
orth_kernel(double *__restrict__ w, const double *__restrict__ V, int64_t ng, int j, const double *__restrict__ h,
            const double *__restrict__ scale_p, const int *__restrict__ skip)
{
    if (*skip) return;   // uniform across the grid
    const double scale = *scale_p;
    double hq[kMaxDots];
#pragma unroll
    for (int q = 0; q < kMaxDots - 1; ++q) hq[q] = q <= j ? h[q] : 0.0;
    GRID_STRIDE(g, ng)
    {
        double v = w[g];
#pragma unroll
        for (int q = 0; q < kMaxDots - 1; ++q)
            if (q <= j) v -= hq[q] * V[q * ng + g];
        w[g] = v * scale;
    }
}

// s = w - sum_{i <= j} h_i V_i written back to w, and partials of (V_i, s),
// i <= j, and (s, s): the first update of a two-pass classical Gram-Schmidt
// with the second pass's inner products from the same read of V
__global__ void __launch_bounds__(kBS)
orth_dots_kernel(double *__restrict__ w, const double *__restrict__ V, int64_t ng, int j, const double *__restrict__ h,
                 double *__restrict__ part, const int *__restrict__ skip)
{
    if (*skip) return;   // uniform across the grid
    double hq[kMaxDots - 1], acc[kMaxDots];
#pragma unroll
    for (int q = 0; q < kMaxDots - 1; ++q) hq[q] = q <= j ? h[q] : 0.0;
#pragma unroll
    for (int q = 0; q < kMaxDots; ++q) acc[q] = 0.0;
    GRID_STRIDE(g, ng)
    {
        double vq[kMaxDots - 1];
        double v = w[g];
#pragma unroll
        for (int q = 0; q < kMaxDots - 1; ++q)
            if (q <= j) {
                vq[q] = V[q * ng + g];
                v -= hq[q] * vq[q];
            }
        w[g] = v;
#pragma unroll
        for (int q = 0; q < kMaxDots - 1; ++q)
            if (q <= j) acc[q] += vq[q] * v;
        const double ss = v * v;
#pragma unroll
        for (int q = 0; q < kMaxDots; ++q)
            if (q == j + 1) acc[q] += ss;
    }
    block_partials<kMaxDots>(acc, j + 2, part, gridDim.x);
}

// x += sum_{i < k} y_i Z_i
__global__ void __launch_bounds__(kBS)
combine_kernel(double *__restrict__ x, const double *__restrict__ Z, int64_t ng, int k, const double *__restrict__ y)
{
    double yq[kMaxDots];
#pragma unroll
    for (int q = 0; q < kMaxDots; ++q) yq[q] = q < k ? y[q] : 0.0;
    GRID_STRIDE(g, ng)
    {
        double v = x[g];
#pragma unroll
        for (int q = 0; q < kMaxDots; ++q)
            if (q < k) v += yq[q] * Z[q * ng + g];
        x[g] = v;
    }
}

__global__ void __launch_bounds__(kBS) scale_kernel(const double *__restrict__ in, double *__restrict__ out, int64_t ng,
                                                    double s)
{
    GRID_STRIDE(g, ng) out[g] = in[g] * s;
}

// GMRES cycle start: g = (beta, 0, ...), flags cleared
__global__ void gmres_start_kernel(GmresDev *d, double beta, double tol_abs, int it, int max_it)
{
    if (threadIdx.x != 0) return;
    for (int q = 0; q <= kGmresMaxRestart; ++q) d->g[q] = 0.0;
    d->g[0] = beta;
    d->tol_abs = tol_abs;
    d->it = it;
    d->max_it = max_it;
    d->k = 0;
    d->stop = 0;
    d->skip_re = 1;
}

// Step j, after the first pass's sums hv[0..j] = (V_i, w), hv[j+1] = (w, w):
// column j of H, ||w - V h||^2 = (w, w) - |h|^2, and whether a second
// classical Gram-Schmidt pass is needed ("twice is enough": the new
// direction kept less than 1/sqrt(2) of its norm)
__global__ void gmres_column_kernel(GmresDev *d, const double *__restrict__ hv, int j)
{
    if (threadIdx.x != 0) return;
    if (d->stop) {
        d->skip_re = 1;
        return;
    }
    const double ww = hv[j + 1];
    double hh = 0.0;
    for (int i = 0; i <= j; ++i) {
        d->H[i * kGmresMaxRestart + j] = hv[i];
        d->coef[i] = hv[i];
        hh += hv[i] * hv[i];
    }
    d->beta2 = ww - hh;
    d->skip_re = d->beta2 >= 0.5 * ww ? 1 : 0;
}

// Step j, after the optional second pass (h2v as hv): the column finished,
// the previous rotations applied to it, the new rotation, g rotated, and the
// stop test |g[j+1]| <= tol_abs, it >= max_it or a zero new direction
__global__ void gmres_givens_kernel(GmresDev *d, const double *__restrict__ h2v, int j)
{
    if (threadIdx.x != 0) return;
    if (d->stop) return;
    double *H = d->H;
    auto Hs = [&](int r, int c) -> double & { return H[r * kGmresMaxRestart + c]; };
    double beta2 = d->beta2;
    if (!d->skip_re) {
        double h2 = 0.0;
        for (int i = 0; i <= j; ++i) {
            Hs(i, j) += h2v[i];
            d->coef[i] = h2v[i];
            h2 += h2v[i] * h2v[i];
        }
        beta2 = h2v[j + 1] - h2;
    }
    if (!isfinite(beta2)) {
        d->stop = 2;
        return;
    }
    const double bj = beta2 > 0.0 ? sqrt(beta2) : 0.0;
    d->inv_bj = bj > 0.0 ? 1.0 / bj : 0.0;
    Hs(j + 1, j) = bj;
    for (int i = 0; i < j; ++i) {
        const double a = Hs(i, j), c = Hs(i + 1, j);
        Hs(i, j) = d->cs[i] * a + d->sn[i] * c;
        Hs(i + 1, j) = -d->sn[i] * a + d->cs[i] * c;
    }
    const double den = hypot(Hs(j, j), Hs(j + 1, j));
    d->cs[j] = Hs(j, j) / den;
    d->sn[j] = Hs(j + 1, j) / den;
    Hs(j, j) = den;
    Hs(j + 1, j) = 0.0;
    d->g[j + 1] = -d->sn[j] * d->g[j];
    d->g[j] = d->cs[j] * d->g[j];
    d->res[j] = fabs(d->g[j + 1]);
    d->it += 1;
    d->k = j + 1;
    if (fabs(d->g[j + 1]) <= d->tol_abs || d->it >= d->max_it || bj == 0.0) d->stop = 1;
}

// ---------------------------------------------------------------- block-Jacobi CG kernels

// x = 0, r = b (0 on Dirichlet nodes); partial (r, r)
__global__ void __launch_bounds__(kBS)
bj_init_kernel(const double *__restrict__ b, const double *__restrict__ dinv, double *__restrict__ x,
               double *__restrict__ r, int64_t ng, double *__restrict__ part)
{
    double acc[1] = {0.0};
    GRID_STRIDE(g, ng)
    {
        const double rg = dinv[g] == 0.0 ? 0.0 : b[g];
        x[g] = 0.0;
        r[g] = rg;
        acc[0] += rg * rg;
    }
    block_partials<1>(acc, 1, part, gridDim.x);
}

// (r, z) from nb partials (per workgroup, or the stage sums): beta = (r, z) / rz_old (0 on the
// first call), rz = (r, z); a breakdown if (r, z) is not positive
__global__ void __launch_bounds__(kWide) bj_rz_finalize(CgState *st, const double *__restrict__ part, int nb, int first)
{
    const double rz = wide_sum(part, nb);
    if (threadIdx.x != 0 || st->done) return;
    if (!(rz > 0.0) || !isfinite(rz)) {
        st->done = 2;
        st->status = SEM_ERR_BREAKDOWN;
        return;
    }
    st->beta = first ? 0.0 : rz / st->rz;
    st->rz = rz;
}

// first = 1: bb, tol2, rr from the (r, r) partials (run start)
__global__ void __launch_bounds__(kBS) bj_start_finalize(CgState *st, const double *__restrict__ part, int nb, double tol)
{
    __shared__ double red[kBS];
    double s = 0.0;
    for (int q = threadIdx.x; q < nb; q += kBS) s += part[q];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = kBS / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        st->bb = red[0];
        st->rr = red[0];
        st->tol2 = tol * tol * red[0];
        st->it = 0;
        st->status = 0;
        st->beta = 0.0;
        st->done = red[0] == 0.0 ? 1 : 0;
    }
}

// wg = Q^T rows; x += alpha p; r -= alpha wg; partial (r, r).  kRowsPerBlock
// lattice rows per workgroup with every load of a node issued before its
// arithmetic; NPC = N + 1 fixed at compile time (0: any order).
template <int NPC>
__global__ void __launch_bounds__(kBS)
bj_update_kernel(const CgState *__restrict__ st, const double *__restrict__ rows, double *__restrict__ x,
                 double *__restrict__ r, const double *__restrict__ p, const double *__restrict__ dinv, Lattice L,
                 double *__restrict__ part)
{
    if (st->done) return;
    const double alpha = st->alpha;
    double acc[1] = {0.0};
    const int nrows = (int)(L.ny * L.nz), ny = (int)L.ny, nx = (int)L.nx, row0 = (int)blockIdx.x * kRowsPerBlock;
    for (int gi = threadIdx.x; gi < nx; gi += kBS) {
        double d[kRowsPerBlock], xg[kRowsPerBlock], pg[kRowsPerBlock], rg0[kRowsPerBlock], wg[kRowsPerBlock];
        int64_t g[kRowsPerBlock];
#pragma unroll
        for (int q = 0; q < kRowsPerBlock; ++q) {
            const int row = row0 + q < nrows ? row0 + q : nrows - 1;   // clamped rows are not stored
            g[q] = gi + (int64_t)nx * row;
            d[q] = dinv[g[q]];
            xg[q] = x[g[q]];
            pg[q] = p[g[q]];
            rg0[q] = r[g[q]];
            wg[q] = node_assemble_rows<NPC>(L, rows, gi, row % ny, row / ny);
        }
#pragma unroll
        for (int q = 0; q < kRowsPerBlock; ++q) {
            if (row0 + q >= nrows || d[q] == 0.0) continue;
            x[g[q]] = xg[q] + alpha * pg[q];
            const double rg = rg0[q] - alpha * wg[q];
            r[g[q]] = rg;
            acc[0] += rg * rg;
        }
    }
    block_partials<1>(acc, 1, part, gridDim.x);
}

// (r, r) from nb partials (per workgroup, or the stage sums): iteration
// count, residual history, convergence test
__global__ void __launch_bounds__(kWide) bj_check_finalize(CgState *st, const double *__restrict__ part, int nb,
                                                           double *hist)
{
    const double rr = wide_sum(part, nb);
    if (threadIdx.x != 0 || st->done) return;
    const int it = st->it + 1;
    st->it = it;
    st->rr = rr;
    if (hist && it < st->hist_len) hist[it] = sqrt(rr / st->bb);
    if (!isfinite(rr)) {
        st->done = 2;
        st->status = SEM_ERR_BREAKDOWN;
    } else if (rr <= st->tol2) {
        st->done = 1;
    } else if (it >= st->max_it) {
        st->done = 3;
    }
}

// p = z + beta p
__global__ void __launch_bounds__(kBS) bj_p_kernel(const CgState *st, double *__restrict__ p,
                                                   const double *__restrict__ z, int64_t ng)
{
    if (st->done) return;
    const double beta = st->beta;
    GRID_STRIDE(g, ng) p[g] = z[g] + beta * p[g];
}

}  // namespace mg

// ---------------------------------------------------------------- preconditioner

size_t hsmg_bufs_bytes(const Mesh &m)
{
    const Hsmg &h = *m.hsmg;
    auto a = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t E = (size_t)m.E, Pm = (size_t)h.lat_m.P, Pc = 8;
    return a(m.nl * 8) + a(E * Pm * 8) + 2 * a(h.ng_m * 8) + a(E * Pc * 8) + 2 * a(h.ng_c * 8) + a(m.ng * 8);
}

HsmgBufs hsmg_bufs_carve(const Mesh &m, char *base)
{
    const Hsmg &h = *m.hsmg;
    auto a = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t E = (size_t)m.E, Pm = (size_t)h.lat_m.P, Pc = 8;
    HsmgBufs b{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        double *p = (double *)(base + off);
        off += a(bytes);
        return p;
    };
    b.rows_f = take(m.nl * 8);
    b.rows_m = take(E * Pm * 8);
    b.rm = take(h.ng_m * 8);
    b.zm = take(h.ng_m * 8);
    b.rows_c = take(E * Pc * 8);
    b.rc = take(h.ng_c * 8);
    b.tc = take(h.ng_c * 8);
    b.zp = take(m.ng * 8);
    return b;
}

namespace {

void launch_assemble_fine(const Lattice &L, const double *rows, int weighted, const double *zp, double *out,
                          hipStream_t s, const double *r = nullptr, double *part = nullptr)
{
    const dim3 grid((unsigned)((L.ny * L.nz + mg::kRowsPerBlock - 1) / mg::kRowsPerBlock)), block(kBS);
    if (L.NP == 8)
        hipLaunchKernelGGL(mg::assemble_fine_kernel<8>, grid, block, 0, s, rows, L, weighted, zp, out, r, part);
    else
        hipLaunchKernelGGL(mg::assemble_fine_kernel<0>, grid, block, 0, s, rows, L, weighted, zp, out, r, part);
}

void launch_assemble(const Lattice &L, const double *rows, int weighted, double *out, const double *zc,
                     const Lattice &Lc, const double *J, hipStream_t s)
{
    const dim3 grid(node_grid(L)), block(kBS);
    switch (L.NP) {
    case 2: hipLaunchKernelGGL(mg::assemble_kernel<2>, grid, block, 0, s, rows, L, weighted, out, zc, Lc, J); break;
    case 4: hipLaunchKernelGGL(mg::assemble_kernel<4>, grid, block, 0, s, rows, L, weighted, out, zc, Lc, J); break;
    case 8: hipLaunchKernelGGL(mg::assemble_kernel<8>, grid, block, 0, s, rows, L, weighted, out, zc, Lc, J); break;
    default: hipLaunchKernelGGL(mg::assemble_kernel<0>, grid, block, 0, s, rows, L, weighted, out, zc, Lc, J); break;
    }
}

template <int NP, int NPC>
void launch_schwarz(const Mesh &m, const Lattice &L, const double *r, const double *fdm, double h1, double h2,
                    double *rows, const double *J, const Lattice &Lc, double *rows_c, int sym, hipStream_t s)
{
    if constexpr (NP == 8)
        hipLaunchKernelGGL((mg::schwarz_pencil_kernel<NPC>), dim3((unsigned)m.E), dim3(64), 0, s, r, L, fdm, h1, h2,
                           rows, J, Lc, rows_c, sym);
    else
        hipLaunchKernelGGL((mg::schwarz_kernel<NP, NPC>), dim3((unsigned)m.E), dim3(NP * NP * NP), 0, s, r, L, fdm,
                           h1, h2, rows, J, Lc, rows_c, sym);
}

// fine Schwarz (+ restriction to the mid level when restrict_mid)
hipError_t fine_schwarz(const Mesh &m, const double *r, double h1, double h2, const HsmgBufs &b, bool restrict_mid,
                        int sym, hipStream_t s)
{
    const Hsmg &h = *m.hsmg;
#define SEM_FS(NP, NPM)                                                                                               \
    case NP:                                                                                                          \
        if (restrict_mid)                                                                                             \
            launch_schwarz<NP, NPM>(m, m.lat, r, h.d_fdm_f, h1, h2, b.rows_f, h.d_Jfm, h.lat_m, b.rows_m, sym, s);    \
        else                                                                                                          \
            launch_schwarz<NP, 0>(m, m.lat, r, h.d_fdm_f, h1, h2, b.rows_f, nullptr, h.lat_m, nullptr, sym, s);       \
        break;
    switch (m.NP) {
        SEM_FS(3, 2)
        SEM_FS(4, 3)
        SEM_FS(5, 4)
        SEM_FS(6, 4)
        SEM_FS(7, 4)
        SEM_FS(8, 4)
        SEM_FS(9, 4)
        SEM_FS(10, 4)
    default:
        return hipErrorInvalidValue;
    }
#undef SEM_FS
    return hipGetLastError();
}

hipError_t mid_schwarz(const Mesh &m, double h1, double h2, const HsmgBufs &b, int sym, hipStream_t s)
{
    const Hsmg &h = *m.hsmg;
    switch (h.lat_m.NP) {
    case 2: launch_schwarz<2, 2>(m, h.lat_m, b.rm, h.d_fdm_m, h1, h2, b.rows_m, h.d_Jmc, h.lat_c, b.rows_c, sym, s); break;
    case 3: launch_schwarz<3, 2>(m, h.lat_m, b.rm, h.d_fdm_m, h1, h2, b.rows_m, h.d_Jmc, h.lat_c, b.rows_c, sym, s); break;
    case 4: launch_schwarz<4, 2>(m, h.lat_m, b.rm, h.d_fdm_m, h1, h2, b.rows_m, h.d_Jmc, h.lat_c, b.rows_c, sym, s); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t prolong_fine(const Mesh &m, const HsmgBufs &b, hipStream_t s)
{
    const Hsmg &h = *m.hsmg;
#define SEM_PF(NP, NPM)                                                                                             \
    case NP:                                                                                                        \
        hipLaunchKernelGGL((mg::prolong_owned_kernel<NP, NPM>), dim3((unsigned)m.E), dim3(NP * NP * NP), 0, s, b.zm, \
                           h.lat_m, h.d_Jfm, m.lat, b.zp);                                                          \
        break;
    switch (m.NP) {
        SEM_PF(3, 2)
        SEM_PF(4, 3)
        SEM_PF(5, 4)
        SEM_PF(6, 4)
        SEM_PF(7, 4)
    case 8:
        hipLaunchKernelGGL(mg::prolong_pencil_kernel, dim3((unsigned)m.E), dim3(64), 0, s, b.zm, h.lat_m, h.d_Jfm, m.lat,
                           b.zp);
        break;
        SEM_PF(9, 4)
        SEM_PF(10, 4)
    default:
        return hipErrorInvalidValue;
    }
#undef SEM_PF
    return hipGetLastError();
}

hipError_t coarse_solve(const Mesh &m, double h1, double h2, const HsmgBufs &b, hipStream_t s)
{
    const Hsmg &h = *m.hsmg;
    const int nx = h.cn[0], ny = h.cn[1], nz = h.cn[2];
    if (nx * ny <= mg::kCoarsePlane && nz <= kBS) {
        const int ncol = kBS / nz;
        const unsigned ncb = (unsigned)(((int64_t)nx * ny + ncol - 1) / ncol);
        hipLaunchKernelGGL(mg::coarse_plane_kernel, dim3((unsigned)nz), dim3(mg::kPlaneThreads), 0, s, b.rc, h.d_cS[0],
                           h.d_cS[1], nx, ny, 1);
        hipLaunchKernelGGL(mg::coarse_column_kernel, dim3(ncb), dim3(kBS), 0, s, b.rc, h.d_cS[2], nx, ny, nz,
                           h.d_clam[0], h.d_clam[1], h.d_clam[2], h1, h2);
        hipLaunchKernelGGL(mg::coarse_plane_kernel, dim3((unsigned)nz), dim3(mg::kPlaneThreads), 0, s, b.rc, h.d_cS[0],
                           h.d_cS[1], nx, ny, 0);
        return hipGetLastError();
    }
    const int nb = cg_blocks(h.ng_c);
    double *in = b.rc, *out = b.tc;
    const int axes[6] = {0, 1, 2, 2, 1, 0};
    for (int q = 0; q < 6; ++q) {
        const int ax = axes[q];
        hipLaunchKernelGGL(mg::coarse_axis_kernel, dim3(nb), dim3(kBS), 0, s, in, out, h.d_cS[ax], ax, q < 3 ? 1 : 0,
                           nx, ny, nz, h.d_clam[0], h.d_clam[1], h.d_clam[2], h1, h2, q == 2 ? 1 : 0);
        std::swap(in, out);
    }
    // six passes: the result is back in b.rc
    return hipGetLastError();
}

hipError_t restrict_fine(const Mesh &m, const double *r, const HsmgBufs &b, hipStream_t s)
{
    const Hsmg &h = *m.hsmg;
#define SEM_RF(NP, NPM)                                                                                              \
    case NP:                                                                                                         \
        hipLaunchKernelGGL((mg::restrict_kernel<NP, NPM>), dim3((unsigned)m.E), dim3(NP * NP * NP), 0, s, r, m.lat, \
                           h.d_Jfm, h.lat_m, b.rows_m);                                                              \
        break;
    switch (m.NP) {
        SEM_RF(3, 2)
        SEM_RF(4, 3)
        SEM_RF(5, 4)
        SEM_RF(6, 4)
        SEM_RF(7, 4)
        SEM_RF(8, 4)
        SEM_RF(9, 4)
        SEM_RF(10, 4)
    default:
        return hipErrorInvalidValue;
    }
#undef SEM_RF
    return hipGetLastError();
}

// mid and coarse levels from the restricted residual in b.rows_m: b.zp =
// P_01 [Sw_1 r_1 + P_12 C^-1 R_21 r_1]
hipError_t coarser_levels(const Mesh &m, double h1, double h2, const HsmgBufs &b, int weight, hipStream_t s)
{
    const Hsmg &h = *m.hsmg;
    const int sym = weight == kWeightSym ? 1 : 0;
    hipError_t e;
    launch_assemble(h.lat_m, b.rows_m, kWeightNone, b.rm, nullptr, h.lat_c, nullptr, s);
    if ((e = mid_schwarz(m, h1, h2, b, sym, s)) != hipSuccess) return e;
    launch_assemble(h.lat_c, b.rows_c, kWeightNone, b.rc, nullptr, h.lat_c, nullptr, s);
    if ((e = coarse_solve(m, h1, h2, b, s)) != hipSuccess) return e;
    launch_assemble(h.lat_m, b.rows_m, weight, b.zm, b.rc, h.lat_c, h.d_Jmc, s);
    return prolong_fine(m, b, s);
}

}  // namespace

hipError_t hsmg_coarse_part(const Mesh &m, double h1, double h2, const double *r, const HsmgBufs &b, int weight,
                            hipStream_t s)
{
    hipError_t e = restrict_fine(m, r, b, s);
    if (e != hipSuccess) return e;
    return coarser_levels(m, h1, h2, b, weight, s);
}

hipError_t hsmg_coarse_part_fork(const Mesh &m, double h1, double h2, const double *r, const HsmgBufs &b, int weight,
                                 hipStream_t s)
{
    const Hsmg &h = *m.hsmg;
    hipError_t e;
    if ((e = hipEventRecord(h.fork, s)) != hipSuccess) return e;
    if ((e = hipStreamWaitEvent(h.side, h.fork, 0)) != hipSuccess) return e;
    if ((e = hsmg_coarse_part(m, h1, h2, r, b, weight, h.side)) != hipSuccess) return e;
    return hipEventRecord(h.join, h.side);
}

hipError_t hsmg_coarse_part_join(const Mesh &m, hipStream_t s)
{
    return hipStreamWaitEvent(s, m.hsmg->join, 0);
}

hipError_t hsmg_apply(const Mesh &m, double h1, double h2, const double *r, double *z, const HsmgBufs &b, int levels,
                      int weight, hipStream_t s, const FineHook *fine, double *part_rz)
{
    const Hsmg &h = *m.hsmg;
    const int sym = weight == kWeightSym ? 1 : 0;
    hipError_t e;
    if (fine) {
        // learned multigrid: the coarser levels (side stream) beside the
        // network, then z = M_learned(r) + zp
        if ((e = hsmg_coarse_part_fork(m, h1, h2, r, b, weight, s)) != hipSuccess) return e;
        e = fine->fp32 ? nn_infer32(*fine->sm, m, r, fine->dinv, fine->c_local, s)
                       : nn_infer<double>(*fine->sm, m, r, fine->dinv, fine->c_local, s, nullptr);
        if (e != hipSuccess) return e;
        if ((e = hsmg_coarse_part_join(m, s)) != hipSuccess) return e;
        return nn_assemble_z<double>(m, r, fine->dinv, fine->c_local, z, s, nullptr, b.zp);
    }
    if (levels == 1) {
        if ((e = fine_schwarz(m, r, h1, h2, b, false, sym, s)) != hipSuccess) return e;
        launch_assemble_fine(m.lat, b.rows_f, weight, nullptr, z, s, r, part_rz);
        return hipGetLastError();
    }
    if ((e = fine_schwarz(m, r, h1, h2, b, true, sym, s)) != hipSuccess) return e;
    launch_assemble(h.lat_m, b.rows_m, kWeightNone, b.rm, nullptr, h.lat_c, nullptr, s);
    if ((e = mid_schwarz(m, h1, h2, b, sym, s)) != hipSuccess) return e;
    launch_assemble(h.lat_c, b.rows_c, kWeightNone, b.rc, nullptr, h.lat_c, nullptr, s);
    if ((e = coarse_solve(m, h1, h2, b, s)) != hipSuccess) return e;
    launch_assemble(h.lat_m, b.rows_m, weight, b.zm, b.rc, h.lat_c, h.d_Jmc, s);
    if ((e = prolong_fine(m, b, s)) != hipSuccess) return e;
    launch_assemble_fine(m.lat, b.rows_f, weight, b.zp, z, s, r, part_rz);
    return hipGetLastError();
}

}  // namespace sem

// ---------------------------------------------------------------- solvers

namespace sem {
namespace {

sem_status read_st(CgState &h, const CgState *d, hipStream_t s)
{
    SEM_HIP_TRY(hipMemcpyAsync(&h, d, sizeof(CgState), hipMemcpyDeviceToHost, s));
    SEM_HIP_TRY(hipStreamSynchronize(s));
    return SEM_OK;
}

// sums of nv quantities from block partials part[q * nb + b] into host out
// sums of nv quantities from block partials into device h (skipped when *skip)
hipError_t reduce_to_dev(const double *part, int nb, int nv, double *stage, double *h, const int *skip, hipStream_t s)
{
    hipError_t e = cg_reduce(part, nb, nv, stage, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(mg::sums_finalize, dim3(1), dim3(kBS), 0, s, stage, nv, h, skip);
    return hipGetLastError();
}

sem_status reduce_to_host(const double *part, int nb, int nv, double *stage, double *hdev, double *out, hipStream_t s)
{
    SEM_HIP_TRY(cg_reduce(part, nb, nv, stage, s));
    hipLaunchKernelGGL(mg::sums_finalize, dim3(1), dim3(kBS), 0, s, stage, nv, hdev, nullptr);
    SEM_HIP_TRY(hipGetLastError());
    SEM_HIP_TRY(hipMemcpyAsync(out, hdev, sizeof(double) * nv, hipMemcpyDeviceToHost, s));
    SEM_HIP_TRY(hipStreamSynchronize(s));
    return SEM_OK;
}

#define SEM_TRY(x)                   \
    do {                             \
        sem_status _s = (x);         \
        if (_s != SEM_OK) return _s; \
    } while (0)

}  // namespace

size_t gmres_bufs_bytes(const Mesh &m, int mres)
{
    auto a = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t ng = (size_t)m.ng;
    const size_t nb = (size_t)std::max<int64_t>(node_grid(m.lat), cg_blocks(m.ng));
    return a((size_t)(mres + 1) * ng * 8) + a((size_t)mres * ng * 8) + a(nb * mg::kMaxDots * 8) +
           a((size_t)mg::kMaxDots * kStage * 8) + 3 * a(mg::kMaxDots * 8) + a(sizeof(GmresDev)) + hsmg_bufs_bytes(m);
}

GmresBufs gmres_bufs_carve(const Mesh &m, int mres, char *base)
{
    auto a = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t ng = (size_t)m.ng;
    const size_t nb = (size_t)std::max<int64_t>(node_grid(m.lat), cg_blocks(m.ng));
    GmresBufs g{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char *p = base + off;
        off += a(bytes);
        return p;
    };
    g.V = (double *)take((size_t)(mres + 1) * ng * 8);
    g.Z = (double *)take((size_t)mres * ng * 8);
    g.part = (double *)take(nb * mg::kMaxDots * 8);
    g.stage = (double *)take((size_t)mg::kMaxDots * kStage * 8);
    g.hdev = (double *)take(mg::kMaxDots * 8);
    g.h2dev = (double *)take(mg::kMaxDots * 8);
    g.ydev = (double *)take(mg::kMaxDots * 8);
    g.gd = (GmresDev *)take(sizeof(GmresDev));
    g.hb = hsmg_bufs_carve(m, base + off);
    return g;
}

sem_status solve_gmres_hsmg(const Mesh &m, const sem_solve_opts &o, const CgVecs<double> &v, const double *b,
                            CgState *st, const GmresBufs &gb, hipStream_t s, sem_solve_report *rep, CgState &h,
                            const FineHook *fine)
{
    const int mres = o.restart > 0 ? std::min(o.restart, kGmresMaxRestart) : kGmresMaxRestart;
    const int64_t ng = m.ng;
    const int nbf = cg_blocks(ng);
    double hv[mg::kMaxDots];
    std::vector<double> y(mres);
    h = CgState{};
    h.max_it = o.max_iter;
    // x = 0, r = b, |b|
    SEM_HIP_TRY(hipMemsetAsync(v.x, 0, sizeof(double) * ng, s));
    hipLaunchKernelGGL(mg::scale_kernel, dim3(nbf), dim3(kBS), 0, s, b, v.r, ng, 1.0);
    hipLaunchKernelGGL(mg::dots_kernel, dim3(nbf), dim3(kBS), 0, s, v.r, gb.V, ng, -1, gb.part);
    SEM_HIP_TRY(hipGetLastError());
    SEM_TRY(reduce_to_host(gb.part, nbf, 1, gb.stage, gb.hdev, hv, s));
    h.bb = hv[0];
    h.tol2 = o.rel_tol * o.rel_tol * h.bb;
    h.rr = h.true_rr = h.bb;
    int hist_written = 0;
    if (o.history && o.history_len > 0) o.history[hist_written++] = 1.0;
    if (h.bb == 0.0) {
        h.done = 1;
        rep->iterations = 0;
        rep->history_written = hist_written;
        return SEM_OK;
    }
    const double bn = std::sqrt(h.bb), tol_abs = o.rel_tol * bn;
    double beta = bn;
    int it = 0, restarts = 0;
    const Hsmg &hs = *m.hsmg;
    GmresDev gh;   // host copy of the cycle's device state
    for (;;) {
        hipLaunchKernelGGL(mg::scale_kernel, dim3(nbf), dim3(kBS), 0, s, v.r, gb.V, ng, 1.0 / beta);
        hipLaunchKernelGGL(mg::gmres_start_kernel, dim3(1), dim3(64), 0, s, gb.gd, beta, tol_abs, it, o.max_iter);
        SEM_HIP_TRY(hipGetLastError());
        // The Hessenberg column, the second-pass decision, the rotations and
        // the stop test run on the device; kernels of a stopped cycle return
        // at once.  The host reads step j's stop flag (copied to pinned
        // memory) after queueing step j + 1, so the stream never drains
        // inside a cycle; a cycle that stopped at step j has at most step
        // j + 1 queued after it, whose state-changing kernels skip.
        for (int j = 0; j < mres; ++j) {
            double *Vj = gb.V + (size_t)j * ng, *Vn = gb.V + (size_t)(j + 1) * ng, *Zj = gb.Z + (size_t)j * ng;
            SEM_HIP_TRY(hsmg_apply(m, o.h1, o.h2, Vj, Zj, gb.hb, 3, kWeightAvg, s, fine));
            SEM_HIP_TRY(launch_ax_f64_gather(m, o.h1, o.h2, Zj, v.w, nullptr, s));
            // Vn = mask(Q^T w), then (V_i, Vn) and (Vn, Vn) in a grid-stride pass
            launch_assemble_fine(m.lat, v.w, kWeightNone, nullptr, Vn, s, nullptr, nullptr);
            hipLaunchKernelGGL(mg::dots_kernel, dim3(nbf), dim3(kBS), 0, s, Vn, gb.V, ng, j, gb.part);
            SEM_HIP_TRY(hipGetLastError());
            SEM_HIP_TRY(reduce_to_dev(gb.part, nbf, j + 2, gb.stage, gb.hdev, nullptr, s));
            hipLaunchKernelGGL(mg::gmres_column_kernel, dim3(1), dim3(64), 0, s, gb.gd, gb.hdev, j);
            // second pass: the first update and its inner products share one read of V
            hipLaunchKernelGGL(mg::orth_dots_kernel, dim3(nbf), dim3(kBS), 0, s, Vn, gb.V, ng, j, gb.hdev, gb.part,
                               &gb.gd->skip_re);
            SEM_HIP_TRY(hipGetLastError());
            SEM_HIP_TRY(reduce_to_dev(gb.part, nbf, j + 2, gb.stage, gb.h2dev, &gb.gd->skip_re, s));
            hipLaunchKernelGGL(mg::gmres_givens_kernel, dim3(1), dim3(64), 0, s, gb.gd, gb.h2dev, j);
            hipLaunchKernelGGL(mg::orth_kernel, dim3(nbf), dim3(kBS), 0, s, Vn, gb.V, ng, j, gb.gd->coef,
                               &gb.gd->inv_bj, &gb.gd->stop);
            SEM_HIP_TRY(hipGetLastError());
            SEM_HIP_TRY(hipMemcpyAsync(hs.h_flag + (j & 1), &gb.gd->stop, sizeof(int), hipMemcpyDeviceToHost, s));
            SEM_HIP_TRY(hipEventRecord(hs.ev[j & 1], s));
            if (j > 0) {
                SEM_HIP_TRY(hipEventSynchronize(hs.ev[(j - 1) & 1]));
                if (hs.h_flag[(j - 1) & 1] != 0) break;
            }
        }
        SEM_HIP_TRY(hipMemcpyAsync(&gh, gb.gd, sizeof(GmresDev), hipMemcpyDeviceToHost, s));
        SEM_HIP_TRY(hipStreamSynchronize(s));
        const int k = gh.k;
        for (int j = 0; j < k; ++j)
            if (o.history && hist_written < o.history_len) o.history[hist_written++] = gh.res[j] / bn;
        it = gh.it;
        if (gh.stop == 2) {
            h.done = 2;
            rep->iterations = it;
            rep->history_written = hist_written;
            return SEM_OK;
        }
        auto Hs = [&](int r, int c) -> double { return gh.H[r * kGmresMaxRestart + c]; };
        // x += Z y, y from the triangular system H y = g
        for (int i = k - 1; i >= 0; --i) {
            double acc = gh.g[i];
            for (int c = i + 1; c < k; ++c) acc -= Hs(i, c) * y[c];
            y[i] = acc / Hs(i, i);
        }
        SEM_HIP_TRY(hipMemcpyAsync(gb.ydev, y.data(), sizeof(double) * k, hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(mg::combine_kernel, dim3(nbf), dim3(kBS), 0, s, v.x, gb.Z, ng, k, gb.ydev);
        // true residual r = b - S x
        SEM_HIP_TRY(launch_ax_f64_gather(m, o.h1, o.h2, v.x, v.w, nullptr, s));
        SEM_HIP_TRY(cg_resid<double>(m, v, b, v.r, st, s));
        CgState t;
        SEM_TRY(read_st(t, st, s));
        h.true_rr = h.rr = t.true_rr;
        if (!std::isfinite(h.true_rr)) {
            h.done = 2;
            break;
        }
        if (h.true_rr <= h.tol2) {
            h.done = 1;
            break;
        }
        if (it >= o.max_iter) {
            h.done = 3;
            break;
        }
        ++restarts;
        beta = std::sqrt(h.true_rr);
    }
    h.it = it;
    rep->iterations = it;
    rep->restarts = restarts;
    rep->outer_iterations = restarts + 1;
    rep->history_written = hist_written;
    return SEM_OK;
}

namespace {

// The next search direction of preconditioned CG after r changed: z = M r
// with the (r, z) partials from the preconditioner's last kernel, beta, and
// p = z (first) or z + beta p.
sem_status pc_direction(const Mesh &m, const sem_solve_opts &o, const CgVecs<double> &v, double *z, CgState *st,
                        const HsmgBufs &hb, int levels, int first, hipStream_t s)
{
    const int weight = levels == 1 ? kWeightNone : kWeightSym;
    const int64_t ng = m.ng;
    const int nbf = cg_blocks(ng);
    const int nbu = (int)((node_grid(m.lat) + mg::kRowsPerBlock - 1) / mg::kRowsPerBlock);
    SEM_HIP_TRY(hsmg_apply(m, o.h1, o.h2, v.r, z, hb, levels, weight, s, nullptr, v.part_b));
    const double *in;
    int64_t n = nbu;
    SEM_HIP_TRY(finalize_input(v.part_b, n, 1, v.stage, s, &in));
    hipLaunchKernelGGL(mg::bj_rz_finalize, dim3(1), dim3(kWide), 0, s, st, in, (int)n, first);
    if (first)
        hipLaunchKernelGGL(mg::scale_kernel, dim3(nbf), dim3(kBS), 0, s, z, v.p, ng, 1.0);
    else
        hipLaunchKernelGGL(mg::bj_p_kernel, dim3(nbf), dim3(kBS), 0, s, st, v.p, z, ng);
    SEM_HIP_TRY(hipGetLastError());
    return SEM_OK;
}

// The rest of an iteration once w = A_L p is in v.w and the (p, w) partials
// in v.part_e: alpha, x += alpha p and r -= alpha Q^T w (fused assembly),
// the convergence test, and the next direction.
sem_status pc_after_ax(const Mesh &m, const sem_solve_opts &o, const CgVecs<double> &v, double *z, CgState *st,
                       const HsmgBufs &hb, int levels, double *hist, hipStream_t s)
{
    const int nbu = (int)((node_grid(m.lat) + mg::kRowsPerBlock - 1) / mg::kRowsPerBlock);
    SEM_HIP_TRY(cg_alpha(m, v.part_e, v.stage, st, s));
    if (m.NP == 8)
        hipLaunchKernelGGL(mg::bj_update_kernel<8>, dim3(nbu), dim3(kBS), 0, s, st, v.w, v.x, v.r, v.p, v.dinv, m.lat,
                           v.part_b);
    else
        hipLaunchKernelGGL(mg::bj_update_kernel<0>, dim3(nbu), dim3(kBS), 0, s, st, v.w, v.x, v.r, v.p, v.dinv, m.lat,
                           v.part_b);
    const double *in;
    int64_t n = nbu;
    SEM_HIP_TRY(finalize_input(v.part_b, n, 1, v.stage, s, &in));
    hipLaunchKernelGGL(mg::bj_check_finalize, dim3(1), dim3(kWide), 0, s, st, in, (int)n, hist);
    return pc_direction(m, o, v, z, st, hb, levels, 0, s);
}

// x = 0, r = b, the first direction
sem_status pc_start(const Mesh &m, const sem_solve_opts &o, const CgVecs<double> &v, const double *b, double *z,
                    CgState *st, const HsmgBufs &hb, int levels, double *hist, int hist_len, hipStream_t s)
{
    const int nbf = cg_blocks(m.ng);
    CgState init{};
    init.max_it = o.max_iter;
    init.hist_len = hist_len;
    SEM_HIP_TRY(hipMemcpyAsync(st, &init, sizeof(CgState), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(mg::bj_init_kernel, dim3(nbf), dim3(kBS), 0, s, b, v.dinv, v.x, v.r, m.ng, v.part_b);
    hipLaunchKernelGGL(mg::bj_start_finalize, dim3(1), dim3(kBS), 0, s, st, v.part_b, nbf, o.rel_tol);
    if (hist && hist_len > 0) {
        const double one = 1.0;
        SEM_HIP_TRY(hipMemcpyAsync(hist, &one, sizeof(double), hipMemcpyHostToDevice, s));
        SEM_HIP_TRY(hipStreamSynchronize(s));
    }
    return pc_direction(m, o, v, z, st, hb, levels, 1, s);
}

// Iterate one field until its recursive residual converges, then let the
// FP64 true residual decide (up to three restarts from x with the true
// residual when the recursive one drifted).  A field whose device state is
// already done goes straight to that check.
sem_status pc_run(const Mesh &m, const sem_solve_opts &o, const CgVecs<double> &v, const double *b, double *z,
                  CgState *st, const HsmgBufs &hb, int levels, double *hist, int check_every, hipStream_t s,
                  sem_solve_report *rep, CgState &h)
{
    int restarts = 0;
    PollPlan plan;
    for (;;) {
        for (;;) {
            SEM_TRY(read_st(h, st, s));
            if (h.done) break;
            const int nq = plan.next(h, check_every);
            for (int q = 0; q < nq; ++q) {
                SEM_HIP_TRY(launch_ax_f64_gather(m, o.h1, o.h2, v.p, v.w, v.part_e, s, &st->done));
                SEM_TRY(pc_after_ax(m, o, v, z, st, hb, levels, hist, s));
            }
        }
        if (h.done != 1 || h.bb == 0.0) break;
        SEM_HIP_TRY(launch_ax_f64_gather(m, o.h1, o.h2, v.x, v.w, nullptr, s));
        SEM_HIP_TRY(cg_resid<double>(m, v, b, v.r, st, s));
        SEM_TRY(read_st(h, st, s));
        if (h.true_rr <= h.tol2 || restarts == 3 || h.it >= h.max_it) break;
        ++restarts;   // the recursive residual drifted: restart from x with the true residual
        CgState patch = h;
        patch.done = 0;
        patch.rr = h.true_rr;
        SEM_HIP_TRY(hipMemcpyAsync(st, &patch, sizeof(CgState), hipMemcpyHostToDevice, s));
        SEM_TRY(pc_direction(m, o, v, z, st, hb, levels, 1, s));
    }
    if (h.done != 1 && h.bb > 0.0) {
        SEM_HIP_TRY(launch_ax_f64_gather(m, o.h1, o.h2, v.x, v.w, nullptr, s));
        SEM_HIP_TRY(cg_resid<double>(m, v, b, v.r, st, s));
        SEM_TRY(read_st(h, st, s));
    }
    rep->iterations = h.it;
    rep->restarts = restarts;
    return SEM_OK;
}

}  // namespace

sem_status solve_pcg_precond(const Mesh &m, const sem_solve_opts &o, const CgVecs<double> &v, const double *b,
                             double *z, CgState *st, const HsmgBufs &hb, int levels, double *hist, int hist_len,
                             int check_every, hipStream_t s, sem_solve_report *rep, CgState &h)
{
    SEM_TRY(pc_start(m, o, v, b, z, st, hb, levels, hist, hist_len, s));
    return pc_run(m, o, v, b, z, st, hb, levels, hist, check_every, s, rep, h);
}

sem_status solve_pcg_precond_batched(const Mesh &m, const sem_solve_opts &o, int nrhs, const CgVecs<double> *v,
                                     const double *b, double *z, CgState *st, const HsmgBufs &hb, int levels,
                                     int check_every, hipStream_t s, sem_solve_report *reps, CgState *h)
{
    const int64_t ng = m.ng;
    for (int c = 0; c < nrhs; ++c)
        SEM_TRY(pc_start(m, o, v[c], b + c * ng, z + c * ng, st + c, hb, levels, nullptr, 0, s));
    for (;;) {
        bool all = true;
        for (int c = 0; c < nrhs; ++c) {
            SEM_TRY(read_st(h[c], st + c, s));
            all = all && h[c].done != 0;
        }
        if (all) break;
        for (int q = 0; q < check_every; ++q) {
            // one operator launch for every field (the geometric factors are
            // streamed once); fields already done skip inside it
            SEM_HIP_TRY(launch_ax_f64_gather_batched(m, nrhs, o.h1, o.h2, v[0].p, ng, v[0].w, v[0].part_e, &st->done,
                                                     (int)(sizeof(CgState) / sizeof(int32_t)), s));
            for (int c = 0; c < nrhs; ++c)
                if (!h[c].done) SEM_TRY(pc_after_ax(m, o, v[c], z + c * ng, st + c, hb, levels, nullptr, s));
        }
    }
    for (int c = 0; c < nrhs; ++c)
        SEM_TRY(pc_run(m, o, v[c], b + c * ng, z + c * ng, st + c, hb, levels, nullptr, check_every, s, reps + c, h[c]));
    return SEM_OK;
}

}  // namespace sem

// ---------------------------------------------------------------- C ABI

using namespace sem;

extern "C" {

sem_status sem_precond_workspace_bytes(const sem_mesh *mesh, size_t *bytes)
{
    if (!mesh || !bytes) return fail(SEM_ERR_INVALID_ARG, "null mesh or bytes");
    const Mesh &m = mesh->m;
    if (!m.hsmg) return fail(SEM_ERR_INVALID_ARG, "the mesh was created without SEM_PREP_HSMG");
    const size_t v = ((size_t)m.ng * 8 + 255) & ~(size_t)255;
    *bytes = hsmg_bufs_bytes(m) + 2 * v;
    return SEM_OK;
}

sem_status sem_precond_apply(const sem_mesh *mesh, int kind, double h1, double h2, const double *r_local,
                             double *z_local, void *workspace, size_t ws_bytes, void *stream)
{
    if (!mesh || !r_local || !z_local || !workspace) return fail(SEM_ERR_INVALID_ARG, "null argument");
    const Mesh &m = mesh->m;
    if (!m.hsmg) return fail(SEM_ERR_INVALID_ARG, "the mesh was created without SEM_PREP_HSMG");
    if (!(h1 > 0.0) || !(h2 >= 0.0) || !std::isfinite(h1) || !std::isfinite(h2))
        return fail(SEM_ERR_INVALID_ARG, "the preconditioners need h1 > 0 and h2 >= 0");
    int levels = 3, weight = kWeightAvg;
    switch (kind) {
    case SEM_PRECOND_HSMG: break;
    case SEM_PRECOND_SCHWARZ: levels = 1; break;
    case SEM_PRECOND_BLOCK_JACOBI: levels = 1; weight = kWeightNone; break;
    case SEM_PRECOND_HSMG_SYM: weight = kWeightSym; break;
    default: return fail(SEM_ERR_INVALID_ARG, "unknown preconditioner kind");
    }
    size_t need = 0;
    sem_status st = sem_precond_workspace_bytes(mesh, &need);
    if (st != SEM_OK) return st;
    if (ws_bytes < need) return fail(SEM_ERR_INVALID_ARG, "workspace too small: need " + std::to_string(need) + " bytes");
    hipStream_t s = (hipStream_t)stream;
    const size_t v = ((size_t)m.ng * 8 + 255) & ~(size_t)255;
    char *base = (char *)workspace;
    double *rg = (double *)base, *zg = (double *)(base + v);
    HsmgBufs hb = hsmg_bufs_carve(m, base + 2 * v);
    SEM_HIP_TRY(cg_gather<double>(m, r_local, rg, s));
    SEM_HIP_TRY(hsmg_apply(m, h1, h2, rg, zg, hb, levels, weight, s));
    SEM_HIP_TRY(cg_scatter<double>(m, zg, z_local, s));
    return SEM_OK;
}

}  // extern "C"
