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
// reversed.  Returns the direction plane in *dir and the cell in *cell, and
// in *bounced (if given) whether the value bounced back from a wall.
template <int D>
__device__ __forceinline__ void pull_src(const Geom &g, int x, int y, int z, int a, int *dir,
                                         int *cell, bool *bounced = nullptr)
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
    if (bounced) *bounced = bb;
}

// Neighbourhood of the cell a thread works on, general form: every lane
// applies the boundary rules to its own coordinates, for any block shape.
// row = (z ny + y) nx is the offset of the cell's x-row, me = row + x.
struct NbLane {
    const Geom *g;
    int x, y, z, row, me;
};

// Row form, for blocks a multiple of 64 cells wide in x on lattices periodic
// in x whose population arrays have fewer than 2^31 elements: the lanes of a
// wavefront then share y and z, so every decision along y and z (periodic
// wrap, bounce-back, mirroring) is wavefront-uniform.  It is taken once per
// wavefront into small tables: ry[k] = y'(y + k) nx and rz[k] = z'(z + k) nx ny
// for k = -1, 0, 1, with y', z' the wrapped coordinate on periodic axes and
// the cell's own one where the neighbour lies beyond a wall or symmetry plane
// (which is also the mirrored ghost of the phi stencil); bit k + 1 of bb and
// sym (y) and bit k + 4 (z) flag links through a wall or a symmetry plane.
// Lanes differ only in x, through xm = x - 1 and xp = x + 1 (wrapped).
struct NbRow {
    const Geom *g;
    int x, y, z, row, me;
    int xm, xp;
    int np;
    int ry[3], rz[3];
    unsigned bb, sym;
};

__device__ __forceinline__ NbLane make_nb(const Geom &g, int x, int y, int z, NbLane *)
{
    const int row = (z * g.ny + y) * g.nx;
    return NbLane{&g, x, y, z, row, row + x};
}

// y and z must be the same in every active lane of the wavefront.
__device__ __forceinline__ NbRow make_nb(const Geom &g, int x, int y, int z, NbRow *)
{
    NbRow n;
    n.g = &g;
    n.x = x;
    n.y = y;
    n.z = z;
    n.row = (z * g.ny + y) * g.nx;
    n.me = n.row + x;
    n.xm = x == 0 ? g.nx - 1 : x - 1;
    n.xp = x == g.nx - 1 ? 0 : x + 1;
    n.np = int(g.np);
    n.bb = 0;
    n.sym = 0;
    const int nxny = g.nx * g.ny;
#pragma unroll
    for (int k = -1; k <= 1; ++k) {
        const int yy = y + k, zz = z + k;
        const bool oy = (unsigned)yy >= (unsigned)g.ny, oz = (unsigned)zz >= (unsigned)g.nz;
        n.ry[k + 1] = (!oy ? yy : g.bcy == BC_PER ? yy - k * g.ny : y) * g.nx;
        n.rz[k + 1] = (!oz ? zz : g.bcz == BC_PER ? zz - k * g.nz : z) * nxny;
        n.bb |= ((oy && g.bcy == BC_WALL) ? 1u << (k + 1) : 0u) |
                ((oz && g.bcz == BC_WALL) ? 1u << (k + 4) : 0u);
        n.sym |= ((oy && g.bcy == BC_SYM) ? 1u << (k + 1) : 0u) |
                 ((oz && g.bcz == BC_SYM) ? 1u << (k + 4) : 0u);
    }
    return n;
}

}  // namespace mplb
