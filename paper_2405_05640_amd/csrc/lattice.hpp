// lattice.hpp -- closed-form structure of a box of hexahedral spectral
// elements (device and host).
//
// Global node (gi, gj, gk), gi in [0, nx): the lexicographic numbering
// glo = gi + nx (gj + ny gk) with gi = ex N + i (mod nx in a periodic
// direction).  A node with gi a multiple of N lies on an element face and has
// one local copy on each side (two in total, or one on a non-periodic domain
// boundary).  Its copies across the three directions form a tensor product
// of up to 2 x 2 x 2 (element, local index) pairs.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace sem {

struct Lattice {
    int nelx, nely, nelz, N, NP;
    int64_t nx, ny, nz;   // global nodes per direction
    int64_t P;            // (N+1)^3
    uint8_t per[3];
    uint8_t dir;          // Dirichlet bits x-, x+, y-, y+, z-, z+
    // Per-axis copy tables (device), one int2 per global index g of the axis:
    //   .x = e0 | e1 << 16           element coordinates of the copies
    //   .y = l0 | l1 << 8 | cnt << 16 | masked << 24   local coordinates, count
    // so kernels enumerate copies with table reads instead of divisions.
    const int2 *tab[3];
    int unsorted;         // 1 if some axis is periodic with a single element
};

// Decode one axis entry.
__host__ __device__ inline int axis_count(int2 a) { return (a.y >> 16) & 0xff; }
__host__ __device__ inline int axis_elem(int2 a, int c) { return c ? (a.x >> 16) & 0xffff : a.x & 0xffff; }
__host__ __device__ inline int axis_loc(int2 a, int c) { return c ? (a.y >> 8) & 0xff : a.y & 0xff; }
__host__ __device__ inline bool axis_masked(int2 a) { return ((a.y >> 24) & 1) != 0; }

// Coordinates of element e = ex + nelx (ey + nely ez), 32-bit arithmetic
// (E < 2^31).
__device__ __forceinline__ void elem_coords(const Lattice &L, int64_t e, int &ex, int &ey, int &ez)
{
    const int ei = (int)e, t = ei / L.nelx;
    ex = ei - t * L.nelx;
    ez = t / L.nely;
    ey = t - ez * L.nely;
}

// Row layout of the solvers' unassembled operator output: the local points
// of all elements form one (nelx NP) x (nely NP) x (nelz NP) lattice, x
// fastest, so that the copies along one global lattice row -- including the
// two copies of every x-face node -- are contiguous.  (The C ABI's local
// fields use [E][k][j][i].)
__host__ __device__ inline int64_t rows_index(const Lattice &L, int64_t ex, int64_t ey, int64_t ez, int i, int j, int k)
{
    return ((ez * L.NP + k) * ((int64_t)L.nely * L.NP) + ey * L.NP + j) * ((int64_t)L.nelx * L.NP) + ex * L.NP + i;
}
// the same in 32-bit arithmetic (every local index is below 2^31)
__device__ __forceinline__ int rows_index32(const Lattice &L, int ex, int ey, int ez, int i, int j, int k)
{
    return ((ez * L.NP + k) * (L.nely * L.NP) + ey * L.NP + j) * (L.nelx * L.NP) + ex * L.NP + i;
}
// global index of local point (i, j, k) of element (ex, ey, ez), 32-bit
// (n_global <= n_local < 2^31); the periodic wrap is one compare per axis
__device__ __forceinline__ int gather_index32(const Lattice &L, int ex, int ey, int ez, int i, int j, int k)
{
    const int nx = (int)L.nx, ny = (int)L.ny, nz = (int)L.nz;
    int gi = ex * L.N + i, gj = ey * L.N + j, gk = ez * L.N + k;
    if (gi >= nx) gi -= nx;
    if (gj >= ny) gj -= ny;
    if (gk >= nz) gk -= nz;
    return gi + nx * (gj + ny * gk);
}

// All local indices (ascending) of global node (gi, gj, gk) of a local
// [E][k][j][i] field, from the axis tables, 32-bit arithmetic (n_local <
// 2^31).  Returns the copy count.
__device__ inline int node_locals(const Lattice &L, int gi, int gj, int gk, int loc[8], bool &masked)
{
    const int2 ax = L.tab[0][gi], ay = L.tab[1][gj], az = L.tab[2][gk];
    masked = axis_masked(ax) || axis_masked(ay) || axis_masked(az);
    const int cx = axis_count(ax), cy = axis_count(ay), cz = axis_count(az);
    const int P = (int)L.P, NP = L.NP;
    int n = 0;
    for (int c = 0; c < cz; ++c)
        for (int b = 0; b < cy; ++b)
            for (int a = 0; a < cx; ++a) {
                const int e = axis_elem(ax, a) + L.nelx * (axis_elem(ay, b) + L.nely * axis_elem(az, c));
                loc[n++] = e * P + axis_loc(ax, a) + NP * (axis_loc(ay, b) + NP * axis_loc(az, c));
            }
    if (L.unsorted) {
        for (int q = 1; q < n; ++q) {
            const int v = loc[q];
            int r = q - 1;
            while (r >= 0 && loc[r] > v) {
                loc[r + 1] = loc[r];
                --r;
            }
            loc[r + 1] = v;
        }
    }
    return n;
}

// Logical workgroup id with the XCD layout of the chip in mind.  Workgroups
// are handed to the 8 XCDs round-robin (workgroup b runs on XCD b mod 8) and
// every XCD has its own L2, so consecutive ids -- neighbouring elements or
// lattice rows, which share cache lines -- would land in 8 different L2s.
// The remap gives XCD x one contiguous range of logical ids (a bijection of
// 0 .. gridDim.x - 1, also when gridDim.x is not a multiple of 8).
constexpr int kNumXcd = 8;
__device__ __forceinline__ int64_t xcd_block()
{
    const int64_t b = blockIdx.x, n = gridDim.x;
    const int64_t q = n / kNumXcd, r = n % kNumXcd;
    const int64_t x = b % kNumXcd, i = b / kNumXcd;
    return x < r ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

// Copies of global index g along one axis, 32-bit arithmetic: returns the
// count (1 or 2) and X[c] = element * (N+1) + local coordinate, ascending
// (X[1] = X[0] for a single copy).  No table is read, so the addresses of a
// node's copies do not wait on a load.
__device__ __forceinline__ int axis_copies(int g, int nel, int N, bool per, int X[2])
{
    const int NP = N + 1;
    const int m = g / N, r = g - m * N;
    if (r != 0) {
        X[0] = X[1] = m * NP + r;
        return 1;
    }
    if (per) {
        if (m == 0) {
            X[0] = 0;
            X[1] = (nel - 1) * NP + N;
        } else {
            X[0] = (m - 1) * NP + N;
            X[1] = m * NP;
        }
        return 2;
    }
    if (m == 0) {
        X[0] = X[1] = 0;
        return 1;
    }
    if (m == nel) {
        X[0] = X[1] = (nel - 1) * NP + N;
        return 1;
    }
    X[0] = (m - 1) * NP + N;
    X[1] = m * NP;
    return 2;
}

// axis_copies with the order fixed at compile time when NPC = N + 1 > 0
// (the divisions by N become multiply-shifts); NPC = 0 takes N at run time.
template <int NPC>
__device__ __forceinline__ int axis_copies_t(int g, int nel, int Nrt, bool per, int X[2])
{
    if constexpr (NPC > 0) {
        constexpr int N = NPC - 1;
        const int m = g / N, r = g - m * N;
        if (r != 0) {
            X[0] = X[1] = m * NPC + r;
            return 1;
        }
        if (per) {
            X[0] = m == 0 ? 0 : (m - 1) * NPC + N;
            X[1] = m == 0 ? (nel - 1) * NPC + N : m * NPC;
            return 2;
        }
        if (m == 0 || m == nel) {
            X[0] = X[1] = m == 0 ? 0 : (nel - 1) * NPC + N;
            return 1;
        }
        X[0] = (m - 1) * NPC + N;
        X[1] = m * NPC;
        return 2;
    } else {
        return axis_copies(g, nel, Nrt, per, X);
    }
}

// Q^T w at node (gi, gj, gk) for w in the row layout, every copy computed per
// thread and every load issued before the first add (missing copies load
// nothing and add zero); summed in ascending local index.
template <int NPC, typename T>
__device__ __forceinline__ T node_assemble_rows(const Lattice &L, const T *__restrict__ w, int gi, int gj, int gk)
{
    const int NP = NPC > 0 ? NPC : L.NP;
    int X[2], Y[2], Z[2];
    const int cx = axis_copies_t<NPC>(gi, L.nelx, L.N, L.per[0] != 0, X);
    const int cy = axis_copies_t<NPC>(gj, L.nely, L.N, L.per[1] != 0, Y);
    const int cz = axis_copies_t<NPC>(gk, L.nelz, L.N, L.per[2] != 0, Z);
    const int nxl = L.nelx * NP, nyl = L.nely * NP;
    T v[8];
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                const bool ok = c < cz && b < cy && a < cx;
                v[4 * c + 2 * b + a] = ok ? w[(Z[c] * nyl + Y[b]) * nxl + X[a]] : T(0);
            }
    T s = v[0];
#pragma unroll
    for (int q = 1; q < 8; ++q) s += v[q];
    return s;
}

// Dirichlet flag of global index g along axis d
__device__ __forceinline__ bool axis_dirichlet(const Lattice &L, int d, int g, int nel)
{
    if (L.per[d]) return false;
    return (g == 0 && ((L.dir >> (2 * d)) & 1)) || (g == nel * L.N && ((L.dir >> (2 * d + 1)) & 1));
}

// Loop over the global nodes of lattice row blockIdx.x = gj + ny gk (one
// workgroup per row, threads over gi): no index is divided per node and every
// row is independent work for the scheduler.  Launch with ny * nz blocks.
// Binds gi, gj, gk (int) and g (int64 lexicographic id); `continue` skips a node.
#define SEM_FOR_EACH_NODE(L, gi, gj, gk, g)                                                            \
    for (int gj = (int)(blockIdx.x % (L).ny), gk = (int)(blockIdx.x / (L).ny), gi = (int)threadIdx.x; \
         gi < (L).nx; gi += (int)blockDim.x)                                                           \
        if (const int64_t g = gi + (L).nx * (int64_t)blockIdx.x; true)

// Copies of a global index g along one direction, ascending in (element, local).
// Returns the count (1 or 2); ec = element coordinate, lc = local coordinate.
__host__ __device__ inline int lattice_copies(int64_t g, int nel, int N, bool per, int ec[2], int lc[2])
{
    const int64_t m = g / N;
    const int r = (int)(g - m * N);
    if (r != 0) {
        ec[0] = (int)m;
        lc[0] = r;
        return 1;
    }
    if (per) {
        if (m == 0) {
            ec[0] = 0; lc[0] = 0;
            ec[1] = nel - 1; lc[1] = N;   // equals (0, N) when nel == 1
            return 2;
        }
        ec[0] = (int)m - 1; lc[0] = N;
        ec[1] = (int)m; lc[1] = 0;
        return 2;
    }
    if (m == 0) { ec[0] = 0; lc[0] = 0; return 1; }
    if (m == nel) { ec[0] = nel - 1; lc[0] = N; return 1; }
    ec[0] = (int)m - 1; lc[0] = N;
    ec[1] = (int)m; lc[1] = 0;
    return 2;
}

__host__ __device__ inline bool lattice_masked(const Lattice &L, int64_t gi, int64_t gj, int64_t gk)
{
    const int64_t g[3] = {gi, gj, gk};
    const int nel[3] = {L.nelx, L.nely, L.nelz};
    for (int d = 0; d < 3; ++d) {
        if (L.per[d]) continue;
        if (g[d] == 0 && ((L.dir >> (2 * d)) & 1)) return true;
        if (g[d] == (int64_t)nel[d] * L.N && ((L.dir >> (2 * d + 1)) & 1)) return true;
    }
    return false;
}

// All local indices of global node (gi, gj, gk), sorted ascending.  Returns
// the number of copies (1..8).
__host__ __device__ inline int lattice_locals(const Lattice &L, int64_t gi, int64_t gj, int64_t gk,
                                              int64_t loc[8])
{
    int ex[2], ix[2], ey[2], iy[2], ez[2], iz[2];
    const int cx = lattice_copies(gi, L.nelx, L.N, L.per[0], ex, ix);
    const int cy = lattice_copies(gj, L.nely, L.N, L.per[1], ey, iy);
    const int cz = lattice_copies(gk, L.nelz, L.N, L.per[2], ez, iz);
    int n = 0;
    for (int c = 0; c < cz; ++c)
        for (int b = 0; b < cy; ++b)
            for (int a = 0; a < cx; ++a) {
                const int64_t e = ex[a] + (int64_t)L.nelx * (ey[b] + (int64_t)L.nely * ez[c]);
                loc[n++] = e * L.P + ix[a] + L.NP * (iy[b] + (int64_t)L.NP * iz[c]);
            }
    // insertion sort (the enumeration is already ascending except in
    // periodic directions with a single element)
    for (int q = 1; q < n; ++q) {
        const int64_t v = loc[q];
        int r = q - 1;
        while (r >= 0 && loc[r] > v) {
            loc[r + 1] = loc[r];
            --r;
        }
        loc[r + 1] = v;
    }
    return n;
}

// Global id of local node (e, i, j, k).
__host__ __device__ inline int64_t lattice_glo(const Lattice &L, int64_t e, int i, int j, int k)
{
    const int64_t ex = e % L.nelx, ey = (e / L.nelx) % L.nely, ez = e / ((int64_t)L.nelx * L.nely);
    int64_t gi = ex * L.N + i, gj = ey * L.N + j, gk = ez * L.N + k;
    if (gi >= L.nx) gi -= L.nx;
    if (gj >= L.ny) gj -= L.ny;
    if (gk >= L.nz) gk -= L.nz;
    return gi + L.nx * (gj + L.ny * gk);
}

}  // namespace sem
