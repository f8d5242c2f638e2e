// Device-side lattice helpers for the gfx950 kernels.
//
// Population index a = ix + 3 iy (+ 9 iz), with velocity component
// c = index digit - 1, so every velocity component, weight and opposite
// direction is a compile-time function of a once the direction loops are
// unrolled.  Weights are the tensor products of the 1-D weights (1/6, 2/3,
// 1/6), written as exact ratios 4^(zero components) / 6^D.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mplb {

enum { BC_PER = 0, BC_WALL = 1, BC_SYM = 2 };

template <int D>
struct Lat {
    static constexpr int Q = D == 2 ? 9 : 27;
};

__host__ __device__ constexpr int cx_of(int a) { return a % 3 - 1; }
__host__ __device__ constexpr int cy_of(int a) { return (a / 3) % 3 - 1; }
template <int D>
__host__ __device__ constexpr int cz_of(int a) { return D == 3 ? a / 9 - 1 : 0; }

template <int D, typename T>
__host__ __device__ constexpr T weight(int a)
{
    return T(1 << (2 * ((cx_of(a) == 0) + (cy_of(a) == 0) + (D == 3 ? (cz_of<D>(a) == 0) : 0)))) /
           T(D == 3 ? 216 : 36);
}

template <int D>
__host__ __device__ constexpr int opposite(int a) { return Lat<D>::Q - 1 - a; }

// Lattice geometry as the kernels see it.  np is the stride between the
// planes of two consecutive directions in a population array.
struct Geom {
    int nx, ny, nz;
    int bcx, bcy, bcz;
    long long np;
};

__device__ __forceinline__ int cell_of(const Geom &g, int x, int y, int z)
{
    return (z * g.ny + y) * g.nx + x;
}

// Neighbour coordinate for the phi stencil: periodic wrap, otherwise the
// ghost layer mirrors the first fluid layer (walls and symmetry planes).
__device__ __forceinline__ int stencil_coord(int s, int n, int bc)
{
    if (s < 0) return bc == BC_PER ? s + n : 0;
    if (s >= n) return bc == BC_PER ? s - n : n - 1;
    return s;
}

// Where the pre-collision value f_a(x) sits in a post-collision buffer under
// pull streaming: the value left the source cell x - c_a in direction a; a
// source beyond a wall means the bounced-back f*_{opp(a)}(x); a source beyond
// a symmetry plane is the same-side cell with that velocity component
// reversed.  Returns the direction plane in *dir and the cell in *cell.
template <int D>
__device__ __forceinline__ void pull_src(const Geom &g, int x, int y, int z, int a, int *dir,
                                         int *cell)
{
    const int cx = cx_of(a), cy = cy_of(a), cz = cz_of<D>(a);
    int sx = x - cx, sy = y - cy, sz = z - cz;
    int b = a;
    bool bb = false;
    if (cx != 0 && (unsigned)sx >= (unsigned)g.nx) {
        if (g.bcx == BC_PER) sx += sx < 0 ? g.nx : -g.nx;
        else if (g.bcx == BC_WALL) bb = true;
        else { sx = x; b -= 2 * cx; }
    }
    if (cy != 0 && (unsigned)sy >= (unsigned)g.ny) {
        if (g.bcy == BC_PER) sy += sy < 0 ? g.ny : -g.ny;
        else if (g.bcy == BC_WALL) bb = true;
        else { sy = y; b -= 6 * cy; }
    }
    if (D == 3 && cz != 0 && (unsigned)sz >= (unsigned)g.nz) {
        if (g.bcz == BC_PER) sz += sz < 0 ? g.nz : -g.nz;
        else if (g.bcz == BC_WALL) bb = true;
        else { sz = z; b -= 18 * cz; }
    }
    if (bb) {
        *dir = opposite<D>(a);
        *cell = cell_of(g, x, y, z);
    } else {
        *dir = b;
        *cell = cell_of(g, sx, sy, sz);
    }
}

// The cell a thread works on.
struct Loc {
    const Geom *g;
    int x, y, z, me;
};

}  // namespace mplb
