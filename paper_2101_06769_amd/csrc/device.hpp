// Device code (gfx950) shared by the kernels of one time step of the multiphase lattice Boltzmann
// method of arXiv 2101.06769: conservative Allen-Cahn phase-field populations
// (Sec. 2.2) coupled to pressure-based flow populations under the cumulant
// collision operator (Sec. 2.3).
//
// A step is two launches over the lattice:
//   k_phi      phi(x) = sum_a g_a(x), the g_a pulled from the post-collision
//              buffer of the previous step (Sec. 2.2, zeroth moment);
//   k_collide  per cell: isotropic gradient and Laplacian of phi (Sec. 2.2),
//              closure (density, chemical potential, forces, normal), flow
//              collision, phase-field collision, post-collision values
//              stored at the cell (pull streaming: the next step gathers);
// or, where the lattice allows it, k_phi_merge (phi from partial sums) and
// k_collide_nphi (the same update, which also sums the next phi from the
// values it stores; see "next order parameter" below).  The batched forms
// (kb_step, kb_collide_nphi) run the same per-cell bodies over a tile list of
// many independent domains.
//
// Flow collision.  All cumulant rates other than the viscous ones are unity
// (Sec. 2.3), so every post-collision cumulant above second order is zero and
// the post-collision set is determined by the conserved moments and the six
// (three in 2-D) relaxed second-order central moments.  The kernel therefore
// streams the Q pulled populations once, accumulating ten raw moments, adds
// the moments of the source Xi in closed form, relaxes in moment space, and
// rebuilds the populations from the central moments of the relaxed set
// (higher orders are products of second-order ones: the Gaussian moment
// closure implied by zero higher cumulants) with three 3-point sweeps.  The
// unit-mass set h = f^p - w (P - 1) is the one transformed; w (P - 1) passes
// through the collision unchanged.
//
// The work is memory-bound (about 440 B/cell/step in FP32 for D3Q27 at a few
// kflop), so the kernels are written for coalesced structure-of-arrays access:
// one thread per cell, x fastest across a 64-wide wavefront, each direction a
// separate plane.
#pragma once

#include <hip/hip_fp16.h>

#include <type_traits>

#include "internal.h"

namespace mplb {

// ------------------------------------------------------------------ storage
template <typename Raw>
struct Plain {
    using raw = Raw;
    static constexpr bool shifted = false;
};
struct Half16 {
    using raw = __half;
    static constexpr bool shifted = true;
};

template <class SF, class SG, typename TT>
struct Pol {
    using F = SF;
    using G = SG;
    using T = TT;
};
using P64 = Pol<Plain<double>, Plain<double>, double>;
using P32 = Pol<Plain<float>, Plain<float>, float>;
using P16 = Pol<Half16, Plain<float>, float>;
using P16A = Pol<Half16, Half16, float>;

// Element x of the row starting at base + off, in device memory (HBM).  The
// row offset is kept apart from the 32-bit lane offset so that, when it is
// wavefront-uniform, the address is a scalar base plus a per-lane byte
// offset.  The result is a global-address-space pointer: a base read from a
// table (the batched kernels) is otherwise a generic pointer, accessed with
// flat instructions that also count against the LDS wait counter.
// FP16 values (a class type, which cannot be copied through such a pointer)
// are accessed as their 16-bit patterns.
template <typename R>
using gptr = __attribute__((address_space(1))) R *;
template <typename R>
struct gelem {
    using type = R;
};
template <>
struct gelem<__half> {
    using type = unsigned short;
};
template <>
struct gelem<const __half> {
    using type = const unsigned short;
};

template <typename R>
__device__ __forceinline__ gptr<typename gelem<R>::type> lane_ptr(R *base, long long off, int x)
{
    using E = typename gelem<R>::type;
    using B = typename std::conditional<std::is_const<R>::value, const char, char>::type;
    const gptr<B> row = (gptr<B>)((gptr<E>)base + off);
    return (gptr<E>)(row + (unsigned)x * (unsigned)sizeof(R));
}

// Element i of an array in device memory, read as a global access (see lane_ptr).
template <typename R>
__device__ __forceinline__ R gld(const R *base, long long i)
{
    return ((gptr<const R>)base)[i];
}
__device__ __forceinline__ __half gld(const __half *base, long long i)
{
    return __ushort_as_half(((gptr<const unsigned short>)base)[i]);
}

// Where the pre-collision value of direction a comes from under pull
// streaming: the post-collision value in plane dir at cell rs + xs (row form:
// rs the wavefront-uniform row offset, xs the lane's column; per-lane form:
// rs the cell, xs 0), and whether it bounced back from a wall (then the cell
// is the reader itself).
struct PullLoc {
    int dir, rs, xs;
    bool bb;
};

// General form: the boundary rules of pull_src on each lane's coordinates.
template <int D>
__device__ __forceinline__ PullLoc pull_loc(const NbLane &n, int a)
{
    PullLoc l;
    pull_src<D>(*n.g, n.x, n.y, n.z, a, &l.dir, &l.rs, &l.bb);
    l.xs = 0;
    return l;
}

// Row form: the y and z rules are wavefront-uniform choices of plane and row
// read off the wavefront's tables; x wraps per lane.  Offsets are 32-bit
// element indices (the arrays hold fewer than 2^31 elements); the uniform
// part (plane and row) and the lane part (x) of an address stay apart, so the
// load is a scalar base plus a 32-bit lane offset (three distinct ones: x,
// x - 1, x + 1) with no per-load vector address arithmetic.
template <int D>
__device__ __forceinline__ PullLoc pull_loc(const NbRow &n, int a)
{
    const int cx = cx_of(a), cy = cy_of(a), cz = cz_of<D>(a);
    const int ky = 1 - cy, kz = 1 - cz;  // table index of y - cy, z - cz
    const unsigned by = cy ? 1u << ky : 0u, bz = cz ? 1u << (3 + kz) : 0u;
    PullLoc l;
    l.bb = (n.bb & (by | bz)) != 0;
    const int b = a - ((n.sym & by) ? 6 * cy : 0) - ((n.sym & bz) ? 18 * cz : 0);
    l.dir = l.bb ? opposite<D>(a) : b;
    l.rs = l.bb ? n.row : n.ry[ky] + n.rz[kz];
    l.xs = (l.bb || cx == 0) ? n.x : cx > 0 ? n.xm : n.xp;
    return l;
}

// Element (plane offset + location) of a device array, global access.  NT:
// a non-temporal load (the value is read once, by this cell).
template <bool NT = false, typename R>
__device__ __forceinline__ R load_loc(const NbLane &, const R *base, long long plane,
                                      const PullLoc &l)
{
    if constexpr (NT)
        return __builtin_nontemporal_load(&((gptr<const R>)base)[plane + l.rs]);
    else
        return gld(base, plane + l.rs);
}
template <bool NT = false, typename R>
__device__ __forceinline__ R load_loc(const NbRow &, const R *base, long long plane,
                                      const PullLoc &l)
{
    if constexpr (NT)
        return __builtin_nontemporal_load(lane_ptr(base, plane + l.rs, l.xs));
    else
        return *lane_ptr(base, plane + l.rs, l.xs);
}
// An FP16 code, as a float.  NT: non-temporal load, taken where both sets are
// FP16 (FP16S_ALL update 521 -> 501 us on 128 x 128 x 512; with the flow set
// alone in FP16, or in FP32 and FP64, non-temporal pulls measured slower:
// FP16S 586 -> 613, FP32 683 -> 702 us).
template <bool NT = false, class NB>
__device__ __forceinline__ float load_code(const NB &n, const void *base, long long plane,
                                           const PullLoc &l)
{
    const unsigned short c = load_loc<NT>(n, static_cast<const unsigned short *>(base), plane, l);
    return __half2float(__ushort_as_half(c));
}

// Pre-collision population a of a set in plain storage at the cell.
template <int D, class S, typename T, class NB>
__device__ __forceinline__ T pull(const NB &n, const void *base, long long np, int a)
{
    static_assert(!S::shifted, "FP16 sets decode with their references (pull_f16 / pull_g16)");
    const PullLoc l = pull_loc<D>(n, a);
    return T(load_loc(n, static_cast<const typename S::raw *>(base), (long long)l.dir * np, l));
}

// Whether the value the cell stores in direction a is read back by the cell
// itself (its neighbour x + c_a lies beyond a wall: bounce-back) rather than
// by that neighbour (periodic image, or the mirrored cell beyond a symmetry
// plane, which is the stencil's ghost).
template <int D>
__device__ __forceinline__ bool wall_out(const NbRow &n, int a)
{
    const int cy = cy_of(a), cz = cz_of<D>(a);
    const unsigned by = cy ? 1u << (1 + cy) : 0u, bz = cz ? 1u << (4 + cz) : 0u;
    return (n.bb & (by | bz)) != 0;
}
template <int D>
__device__ __forceinline__ bool wall_out(const NbLane &n, int a)
{
    const Geom &g = *n.g;
    auto out = [](int s, int m, int bc) { return bc == BC_WALL && (unsigned)s >= (unsigned)m; };
    return (cx_of(a) && out(n.x + cx_of(a), g.nx, g.bcx)) ||
           (cy_of(a) && out(n.y + cy_of(a), g.ny, g.bcy)) ||
           (D == 3 && cz_of<D>(a) && out(n.z + cz_of<D>(a), g.nz, g.bcz));
}

// phi at the stencil neighbour (x + cx, y + cy, z + cz): periodic wrap, or the
// mirrored first fluid layer beyond walls and symmetry planes.
template <typename T>
__device__ __forceinline__ T phi_at(const NbLane &n, const T *phi, int cx, int cy, int cz)
{
    const Geom &g = *n.g;
    const int xx = cx ? stencil_coord(n.x + cx, g.nx, g.bcx) : n.x;
    const int yy = cy ? stencil_coord(n.y + cy, g.ny, g.bcy) : n.y;
    const int zz = cz ? stencil_coord(n.z + cz, g.nz, g.bcz) : n.z;
    return gld(phi, cell_of(g, xx, yy, zz));
}

template <typename T>
__device__ __forceinline__ T phi_at(const NbRow &n, const T *phi, int cx, int cy, int cz)
{
    const int xx = cx == 0 ? n.x : cx > 0 ? n.xp : n.xm;
    return *lane_ptr(phi, (long long)(n.ry[1 + cy] + n.rz[1 + cz]), xx);
}

// Parameters in the arithmetic type.
template <typename T>
struct Phys {
    T rho_l, drho, nu_l, dnu, rnu_l, drnu, beta, kappa, gx, gy, gz, inv_tpb, src_pre, four_W;
    T scl_l, dscl;
    int visc_interp, collision, cac_edf;
};

template <typename T>
__host__ __device__ static Phys<T> to_phys(const PhysD &d)
{
    Phys<T> p;
    p.rho_l = T(d.rho_l);
    p.drho = T(d.drho);
    p.nu_l = T(d.nu_l);
    p.dnu = T(d.dnu);
    p.rnu_l = T(d.rnu_l);
    p.drnu = T(d.drnu);
    p.beta = T(d.beta);
    p.kappa = T(d.kappa);
    p.gx = T(d.gx);
    p.gy = T(d.gy);
    p.gz = T(d.gz);
    p.inv_tpb = T(d.inv_tpb);
    p.src_pre = T(d.src_pre);
    p.four_W = T(d.four_W);
    p.scl_l = T(d.scl_l);
    p.dscl = T(d.dscl);
    p.visc_interp = d.visc_interp;
    p.collision = d.collision;
    p.cac_edf = d.cac_edf;
    return p;
}

// ------------------------------------------------------------- FP16 storage
// The FP16 formats store, per direction and cell, a half-precision code q of
// the deviation of a post-collision value from a reference that both the
// cell writing it and the cell pulling it a step later hold without a
// per-population gather:
//  * flow set f': the writer's reference, v = w (P + s q), with P the fp16
//    rounding of the writer's pressure p* and s = rho(F) cs^2, F the fp16
//    rounding of its order parameter.  The reader pulls direction a from the
//    neighbour x - c_a, and the order-parameter record it loads from that
//    neighbour for the stencil carries the neighbour's (P, F).
//  * phase-field set g (FP16S_ALL): the reader's reference, v = w (F + q),
//    F the fp16 rounding of the reader's order parameter at the writer's
//    level, which the writer has from its own stencil.
// The deviations are O(u) in either phase, so half precision keeps about 11
// bits of them where the raw values at density ratio 1000 would lose ~6 bits
// to the pressure.  The rest direction of each FP16 set is not streamed: it
// is stored in FP32 as the remainder of the set's zeroth moment over the
// values the readers will decode, so pressure and phase mass stay exact to
// FP32 round-off.  The update writes each cell's reference (packed: low half
// P, high half F) to a reference array; the next step's order-parameter stage
// copies it into the cell's 8-byte record (phi, reference), which is what
// the stencil loads.
struct Ref16 {
    float P, F;
};
__device__ __forceinline__ Ref16 unpack_ref(unsigned r)
{
    Ref16 o;
    o.P = __half2float(__ushort_as_half((unsigned short)(r & 0xffffu)));
    o.F = __half2float(__ushort_as_half((unsigned short)(r >> 16)));
    return o;
}
__device__ __forceinline__ unsigned pack_ref(float P, float F)
{
    return unsigned(__half_as_ushort(__float2half(P))) |
           (unsigned(__half_as_ushort(__float2half(F))) << 16);
}
// Scale of the flow codes written by a cell whose reference has order
// parameter F: rho(F) cs^2, with cs^2 folded into the two coefficients.
__device__ __forceinline__ float flow_scale16(const Phys<float> &ph, float F)
{
    return __builtin_fmaf(ph.dscl, F, ph.scl_l);
}
__device__ __forceinline__ float dec_f16(float w, const Ref16 &r, float s, float q)
{
    return w * (r.P + s * q);
}
// w (F + q) as w q + w F: a reader decodes all its values against one F, so
// w F is formed once per weight and each value takes one mixed-precision
// multiply-add of its FP16 code.
__device__ __forceinline__ float dec_g16(float w, float F, float q) { return __builtin_fmaf(w, q, w * F); }
// Order-parameter record of the FP16 formats: phi (low word), reference.
__device__ __forceinline__ float rec_phi(unsigned long long v) { return __uint_as_float(unsigned(v)); }
__device__ __forceinline__ unsigned rec_ref(unsigned long long v) { return unsigned(v >> 32); }
__device__ __forceinline__ unsigned long long make_rec(float phi, unsigned ref)
{
    return (unsigned long long)__float_as_uint(phi) | ((unsigned long long)ref << 32);
}
// Element of a per-cell array at the thread's own cell.
template <typename R>
__device__ __forceinline__ R own_at(const NbLane &n, const R *base)
{
    return gld(base, n.me);
}
template <typename R>
__device__ __forceinline__ R own_at(const NbRow &n, const R *base)
{
    return *lane_ptr(base, n.row, n.x);
}
__device__ __forceinline__ unsigned short half_bits(float v) { return __half_as_ushort(__float2half(v)); }
__device__ __forceinline__ float half_val(unsigned short b) { return __half2float(__ushort_as_half(b)); }

// Stores the FP16 code of direction plane `plane` at the cell (row + x) of a
// population array, non-temporally: the next update reads it a launch later,
// and cached, the written lines were written back to HBM during the next
// order-parameter merge (FP16S_ALL merge 72.2 -> 57.9 us, step 0.604 -> 0.582
// ms on 128 x 128 x 512).  BUF (row form): through a buffer resource with
// the row as scalar offset and the column as per-lane offset, which leaves
// the 64-bit address arithmetic of the store to the scalar unit; taken where
// instruction issue bounds the update (both sets in FP16: 0.582 -> 0.577 ms;
// the FP16 flow set alone measured 0.642 against 0.645 ms without it).
template <bool BUF, class NB>
__device__ __forceinline__ void store_code(const NB &, void *base, long long plane, int row, int x,
                                           unsigned short bits)
{
    if constexpr (BUF && std::is_same<NB, NbRow>::value) {
        // raw buffer (stride 0) without a range limit; word 3 as gfx9 takes it for
        // untyped accesses; cache policy 2: non-temporal
        const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(
            static_cast<unsigned short *>(base) + plane, 0, -1, 0x00020000);
        __builtin_amdgcn_raw_buffer_store_b16(bits, r, unsigned(x) * 2u, unsigned(row) * 2u, 2);
    } else {
        __builtin_nontemporal_store(bits, lane_ptr(static_cast<unsigned short *>(base), plane + row, x));
    }
}

// ------------------------------------------------------------- cell state
template <typename T>
struct Cell {
    T phi, gx, gy, gz, lap;
    T rho, irho, drx, dry, drz, mu, Fx, Fy, Fz, omega;
    T S0, Sx, Sy, Sz, Sxx, Syy, Szz, Sxy, Sxz, Syz;
    T ux, uy, uz, pstar, U;
    T Fown;  // FP16 formats: the cell's own reference order parameter (fp16)
};

// LDS slot of a moving D3Q27 direction (the rest direction, 13, has none);
// for D2Q9 (a < 9) the direction itself.
__host__ __device__ constexpr int nphi_slot(int a) { return a < 13 ? a : a - 1; }

// grad(phi) = (1/cs^2) sum_a w_a c_a phi(x + c_a);
// lap(phi) = (2/cs^2) sum_a w_a [phi(x + c_a) - phi(x)]   (Sec. 2.2)
// Summed over pairs of opposite directions, w (phi(x+c) - phi(x-c)) and
// w (phi(x+c) + phi(x-c) - 2 phi(x)), so that uniform and mirror-symmetric
// fields give exactly zero gradient components.
template <int D, typename T, class NB>
__device__ __forceinline__ void stencil(const NB &n, const T *__restrict__ phi, Cell<T> &c)
{
    constexpr int Q = Lat<D>::Q;
    const T p0 = phi_at(n, phi, 0, 0, 0);
    T gx = 0, gy = 0, gz = 0, lap = 0;
#pragma unroll
    for (int a = Q / 2 + 1; a < Q; ++a) {
        const int cx = cx_of(a), cy = cy_of(a), cz = cz_of<D>(a);
        const T pp = phi_at(n, phi, cx, cy, cz);
        const T pm = phi_at(n, phi, -cx, -cy, -cz);
        const T w = weight<D, T>(a);
        const T d = w * (pp - pm);
        if (cx) gx += T(cx) * d;
        if (cy) gy += T(cy) * d;
        if (cz) gz += T(cz) * d;
        lap += w * ((pp - p0) + (pm - p0));
    }
    c.phi = p0;
    c.gx = T(3) * gx;
    c.gy = T(3) * gy;
    c.gz = T(3) * gz;
    c.lap = T(6) * lap;
}

// Density and its gradient, chemical potential, forces, relaxation rate
// (Sec. 2.1, 2.3).
template <int D, typename T>
__device__ __forceinline__ void closure(const Phys<T> &ph, Cell<T> &c)
{
    c.rho = ph.rho_l + ph.drho * c.phi;
    c.irho = T(1) / c.rho;
    c.drx = ph.drho * c.gx;
    c.dry = ph.drho * c.gy;
    c.drz = ph.drho * c.gz;
    c.mu = T(2) * ph.beta * c.phi * (c.phi - T(1)) * (T(2) * c.phi - T(1)) - ph.kappa * c.lap;
    c.Fx = c.mu * c.gx + c.rho * ph.gx;
    c.Fy = c.mu * c.gy + c.rho * ph.gy;
    c.Fz = D == 3 ? c.mu * c.gz + c.rho * ph.gz : T(0);
    const T nu = ph.visc_interp ? (ph.rnu_l + ph.drnu * c.phi) * c.irho : ph.nu_l + ph.dnu * c.phi;
    c.omega = T(1) / (T(3) * nu + T(0.5));
}

// Raw moments of the pulled flow populations (orders 0..2), accumulated over
// pairs of opposite directions (f_a + f_opp for even moments, f_a - f_opp for
// odd ones) so that the pressure part w p cancels exactly in the odd moments
// and the velocity part cancels before it reaches the even ones.  STASH: the
// pulled values are also kept for a collision that needs them one by one,
// the moving ones in stash[nphi_slot(a) * sstride], the rest value in
// *stash_rest.
template <int D, class P, bool STASH, class NB>
__device__ __forceinline__ void flow_moments(const NB &nb, long long np, const Ptrs &p,
                                             Cell<typename P::T> &c, typename P::T *stash,
                                             int sstride, typename P::T *stash_rest)
{
    using T = typename P::T;
    constexpr int Q = Lat<D>::Q;
    T S0 = pull<D, typename P::F, T>(nb, p.Fin, np, Q / 2);
    if constexpr (STASH) *stash_rest = S0;
    T Sx = 0, Sy = 0, Sz = 0, Sxx = 0, Syy = 0, Szz = 0, Sxy = 0, Sxz = 0, Syz = 0;
#pragma unroll
    for (int a = Q / 2 + 1; a < Q; ++a) {
        const int b = opposite<D>(a);
        const int cx = cx_of(a), cy = cy_of(a), cz = cz_of<D>(a);
        const T va = pull<D, typename P::F, T>(nb, p.Fin, np, a);
        const T vb = pull<D, typename P::F, T>(nb, p.Fin, np, b);
        if constexpr (STASH) {
            stash[nphi_slot(a) * sstride] = va;
            stash[nphi_slot(b) * sstride] = vb;
        }
        const T sp = va + vb, dm = va - vb;
        S0 += sp;
        if (cx) { Sx += T(cx) * dm; Sxx += sp; }
        if (cy) { Sy += T(cy) * dm; Syy += sp; }
        if (cz) { Sz += T(cz) * dm; Szz += sp; }
        if (cx && cy) Sxy += T(cx * cy) * sp;
        if (cx && cz) Sxz += T(cx * cz) * sp;
        if (cy && cz) Syz += T(cy * cz) * sp;
    }
    c.S0 = S0; c.Sx = Sx; c.Sy = Sy; c.Sz = Sz;
    c.Sxx = Sxx; c.Syy = Syy; c.Szz = Szz; c.Sxy = Sxy; c.Sxz = Sxz; c.Syz = Syz;
}

// Velocity: first moment of f^p = f'/(rho cs^2) + Xi/(2 rho cs^2), using
// sum_a c_a Xi_a = cs^2 F.  Pressure p* = sum f' + sum Xi / 2 with
// sum_a Xi_a = cs^2 u . grad(rho).
template <int D, typename T>
__device__ __forceinline__ void velocity(Cell<T> &c)
{
    const T h = T(0.5) * c.irho;
    c.ux = T(3) * c.Sx * c.irho + h * c.Fx;
    c.uy = T(3) * c.Sy * c.irho + h * c.Fy;
    c.uz = D == 3 ? T(3) * c.Sz * c.irho + h * c.Fz : T(0);
    c.U = c.ux * c.drx + c.uy * c.dry + c.uz * c.drz;
    c.pstar = c.S0 + T(0.5) * (T(1) / T(3)) * c.U;
}

// FP16 formats: the stencil and the raw flow moments in one pass over pairs
// of opposite directions.  The stencil neighbour x - c_a is the cell the
// pulled f'_a comes from (x + c_a that of f'_opp(a)), so the record loaded
// for the stencil also carries the reference that decodes the pulled value;
// a value that bounced back from a wall was written by the cell itself.
// gref (FP16 phase-field storage): per pair k of directions (a, opp(a)), the
// fp16 order parameters of the neighbours x + c_a (low half) and x - c_a
// (high half), the references of the cells that read the phase-field values
// this cell stores in directions a and opp(a).
// Phase-field collision of the plain formats: load every pulled value before
// the first store (true) or pair by pair (false).  The FP16 formats always
// preload (measured: the FP16S update 742 -> 642 us on 128 x 128 x 512); the
// FP32 update is faster without (697 against 715 us: the registers it
// would hold cost occupancy).
constexpr bool CAC_PRELOAD = false;

// Two schedules of the same pass.  paired: each pair's loads beside its
// arithmetic, the compiler free to overlap them (FP16S_ALL).  hoisted: every
// load of the pass (26 records, 26 codes) issued first, then a scheduling
// fence (FP16S): there, left to itself, the compiler trades the loads in
// flight for occupancy and waits on each pair in turn (update 600 -> 709 us
// on 128 x 128 x 512), while with both sets in FP16 the fence or the hoisted
// form costs it scalar-register spills.
template <int D, class P, class NB>
__device__ __forceinline__ void eval_cell16_paired(const NB &nb, long long np, const Phys<float> &ph,
                                            const Ptrs &p, Cell<float> &c, unsigned *gref)
{
    constexpr int Q = Lat<D>::Q;
    const unsigned long long *rec = static_cast<const unsigned long long *>(p.phi);
    const unsigned long long r0 = phi_at(nb, rec, 0, 0, 0);
    const float p0 = rec_phi(r0);
    const unsigned own_bits = rec_ref(r0);
    c.Fown = unpack_ref(own_bits).F;
    float gx = 0, gy = 0, gz = 0, lap = 0;
    float S0 = own_at(nb, p.frest_in);
    float Sx = 0, Sy = 0, Sz = 0, Sxx = 0, Syy = 0, Szz = 0, Sxy = 0, Sxz = 0, Syz = 0;
#pragma unroll
    for (int a = Q / 2 + 1; a < Q; ++a) {
        const int b = opposite<D>(a);
        const int cx = cx_of(a), cy = cy_of(a), cz = cz_of<D>(a);
        const unsigned long long rp = phi_at(nb, rec, cx, cy, cz);     // x + c_a
        const unsigned long long rm = phi_at(nb, rec, -cx, -cy, -cz);  // x - c_a
        const float pp = rec_phi(rp), pm = rec_phi(rm);
        const float w = weight<D, float>(a);
        const float d = w * (pp - pm);
        if (cx) gx += float(cx) * d;
        if (cy) gy += float(cy) * d;
        if (cz) gz += float(cz) * d;
        lap += w * ((pp - p0) + (pm - p0));
        if (gref) gref[a - (Q / 2 + 1)] = unsigned(half_bits(pp)) | (unsigned(half_bits(pm)) << 16);
        const PullLoc la = pull_loc<D>(nb, a), lb = pull_loc<D>(nb, b);
        const float qa = load_code<true>(nb, p.Fin, (long long)la.dir * np, la);
        const float qb = load_code<true>(nb, p.Fin, (long long)lb.dir * np, lb);
        // the reference words selected as integers: no branch on the
        // (wavefront-uniform in the row form) bounce-back flags
        const Ref16 ra = unpack_ref(la.bb ? own_bits : rec_ref(rm));
        const Ref16 rb = unpack_ref(lb.bb ? own_bits : rec_ref(rp));
        const float va = dec_f16(w, ra, flow_scale16(ph, ra.F), qa);
        const float vb = dec_f16(w, rb, flow_scale16(ph, rb.F), qb);
        const float sp = va + vb, dm = va - vb;
        S0 += sp;
        if (cx) { Sx += float(cx) * dm; Sxx += sp; }
        if (cy) { Sy += float(cy) * dm; Syy += sp; }
        if (cz) { Sz += float(cz) * dm; Szz += sp; }
        if (cx && cy) Sxy += float(cx * cy) * sp;
        if (cx && cz) Sxz += float(cx * cz) * sp;
        if (cy && cz) Syz += float(cy * cz) * sp;
    }
    c.phi = p0;
    c.gx = 3.0f * gx;
    c.gy = 3.0f * gy;
    c.gz = 3.0f * gz;
    c.lap = 6.0f * lap;
    c.S0 = S0; c.Sx = Sx; c.Sy = Sy; c.Sz = Sz;
    c.Sxx = Sxx; c.Syy = Syy; c.Szz = Szz; c.Sxy = Sxy; c.Sxz = Sxz; c.Syz = Syz;
    closure<D, float>(ph, c);
    velocity<D, float>(c);

}

template <int D, class P, bool STASH, class NB>
__device__ __forceinline__ void eval_cell16_hoisted(const NB &nb, long long np, const Phys<float> &ph,
                                            const Ptrs &p, Cell<float> &c, unsigned *gref,
                                            float *stash, int sstride, float *stash_rest)
{
    constexpr int Q = Lat<D>::Q, H = Q / 2;
    const unsigned long long *rec = static_cast<const unsigned long long *>(p.phi);
    const unsigned long long r0 = phi_at(nb, rec, 0, 0, 0);
    const float frest = own_at(nb, p.frest_in);
    if constexpr (STASH) *stash_rest = frest;
    unsigned long long rp[H], rm[H];
    unsigned short qa_bits[H], qb_bits[H];
    auto load_pair = [&](int a) {
        const int k = a - (H + 1), b = opposite<D>(a);
        const int cx = cx_of(a), cy = cy_of(a), cz = cz_of<D>(a);
        rp[k] = phi_at(nb, rec, cx, cy, cz);     // x + c_a
        rm[k] = phi_at(nb, rec, -cx, -cy, -cz);  // x - c_a
        const PullLoc la = pull_loc<D>(nb, a), lb = pull_loc<D>(nb, b);
        qa_bits[k] = load_loc(nb, static_cast<const unsigned short *>(p.Fin), (long long)la.dir * np, la);
        qb_bits[k] = load_loc(nb, static_cast<const unsigned short *>(p.Fin), (long long)lb.dir * np, lb);
    };
#pragma unroll
    for (int a = H + 1; a < Q; ++a) load_pair(a);
    __builtin_amdgcn_sched_barrier(0);
    const float p0 = rec_phi(r0);
    const unsigned own_bits = rec_ref(r0);
    c.Fown = unpack_ref(own_bits).F;
    float gx = 0, gy = 0, gz = 0, lap = 0;
    float S0 = frest;
    float Sx = 0, Sy = 0, Sz = 0, Sxx = 0, Syy = 0, Szz = 0, Sxy = 0, Sxz = 0, Syz = 0;
#pragma unroll
    for (int a = H + 1; a < Q; ++a) {
        const int k = a - (H + 1), b = opposite<D>(a);
        const int cx = cx_of(a), cy = cy_of(a), cz = cz_of<D>(a);
        const float pp = rec_phi(rp[k]), pm = rec_phi(rm[k]);
        const float w = weight<D, float>(a);
        const float d = w * (pp - pm);
        if (cx) gx += float(cx) * d;
        if (cy) gy += float(cy) * d;
        if (cz) gz += float(cz) * d;
        lap += w * ((pp - p0) + (pm - p0));
        if (gref) gref[k] = unsigned(half_bits(pp)) | (unsigned(half_bits(pm)) << 16);
        const PullLoc la = pull_loc<D>(nb, a), lb = pull_loc<D>(nb, b);
        const float qa = half_val(qa_bits[k]), qb = half_val(qb_bits[k]);
        // the reference words selected as integers: no branch on the
        // (wavefront-uniform in the row form) bounce-back flags
        const Ref16 ra = unpack_ref(la.bb ? own_bits : rec_ref(rm[k]));
        const Ref16 rb = unpack_ref(lb.bb ? own_bits : rec_ref(rp[k]));
        const float va = dec_f16(w, ra, flow_scale16(ph, ra.F), qa);
        const float vb = dec_f16(w, rb, flow_scale16(ph, rb.F), qb);
        if constexpr (STASH) {
            stash[nphi_slot(a) * sstride] = va;
            stash[nphi_slot(b) * sstride] = vb;
        }
        const float sp = va + vb, dm = va - vb;
        S0 += sp;
        if (cx) { Sx += float(cx) * dm; Sxx += sp; }
        if (cy) { Sy += float(cy) * dm; Syy += sp; }
        if (cz) { Sz += float(cz) * dm; Szz += sp; }
        if (cx && cy) Sxy += float(cx * cy) * sp;
        if (cx && cz) Sxz += float(cx * cz) * sp;
        if (cy && cz) Syz += float(cy * cz) * sp;
    }
    c.phi = p0;
    c.gx = 3.0f * gx;
    c.gy = 3.0f * gy;
    c.gz = 3.0f * gz;
    c.lap = 6.0f * lap;
    c.S0 = S0; c.Sx = Sx; c.Sy = Sy; c.Sz = Sz;
    c.Sxx = Sxx; c.Syy = Syy; c.Szz = Szz; c.Sxy = Sxy; c.Sxz = Sxz; c.Syz = Syz;
    closure<D, float>(ph, c);
    velocity<D, float>(c);
}

// STASH (not where both sets are FP16): the pulled flow values, decoded, are
// also kept as flow_moments describes.
template <int D, class P, bool STASH = false, class NB>
__device__ __forceinline__ void eval_cell(const NB &nb, long long np,
                                          const Phys<typename P::T> &ph, const Ptrs &p,
                                          Cell<typename P::T> &c, unsigned *gref = nullptr,
                                          typename P::T *stash = nullptr, int sstride = 0,
                                          typename P::T *stash_rest = nullptr)
{
    using T = typename P::T;
    if constexpr (P::F::shifted) {
        static_assert(!(STASH && P::G::shifted), "no stash where both sets are FP16");
        if constexpr (P::G::shifted)
            eval_cell16_paired<D, P>(nb, np, ph, p, c, gref);
        else
            eval_cell16_hoisted<D, P, STASH>(nb, np, ph, p, c, gref, stash, sstride, stash_rest);
    } else {
        stencil<D, T>(nb, static_cast<const T *>(p.phi), c);
        closure<D, T>(ph, c);
        flow_moments<D, P, STASH>(nb, np, p, c, stash, sstride, stash_rest);
        velocity<D, T>(c);
    }
}

// One 3-point sweep: central moments (k0, k1, k2) about u of a set on the
// velocities {-1, 0, +1} -> the three values.
// Written as its even and odd parts in u, E = (k0 u^2 + k2)/2 + k1 u and
// O = (k0 u + k1)/2: vm = E - O, v0 = k0 - 2E, vp = E + O.
template <typename T>
__device__ __forceinline__ void sweep3(T k0, T k1, T k2, T u, T &vm, T &v0, T &vp)
{
    const T E = k0 * (T(0.5) * (u * u)) + (k1 * u + T(0.5) * k2);
    const T O = k0 * (T(0.5) * u) + T(0.5) * k1;
    vm = E - O;
    v0 = k0 - T(2) * E;
    vp = E + O;
}

// Post-collision unit-mass set from velocity and relaxed second-order central
// moments (diagonal ones given as deviations dxx = Kxx - cs^2, ...): all
// cumulants above second order are zero, so the central moments are Gaussian
// (Isserlis) products of the second-order ones.  Returned as the
// deviation h*_a - w_a, computed without cancellation: the sweeps act on the
// central-moment deviations from the rest state (second moments cs^2), and the
// rest state's own image, prod_i (r + d(u_i)) - prod_i r with the D1Q3 weights
// r = (1/6, 2/3, 1/6) and d(u) = ((u^2 - u)/2, -u^2, (u^2 + u)/2), is added in
// expanded form.
template <int D, typename T>
__device__ __forceinline__ void rebuild(T ux, T uy, T uz, T dxx, T dyy, T dzz, T Kxy, T Kxz, T Kyz,
                                        T *hdev)
{
    constexpr T cs2 = T(1) / T(3);
    const T r[3] = {T(1) / T(6), T(2) / T(3), T(1) / T(6)};
    const T dx[3] = {T(0.5) * (ux * ux - ux), -ux * ux, T(0.5) * (ux * ux + ux)};
    const T dy[3] = {T(0.5) * (uy * uy - uy), -uy * uy, T(0.5) * (uy * uy + uy)};
    const T Kxx = cs2 + dxx, Kyy = cs2 + dyy;
    if constexpr (D == 3) {
        const T dz[3] = {T(0.5) * (uz * uz - uz), -uz * uz, T(0.5) * (uz * uz + uz)};
        const T Kzz = cs2 + dzz;
        // m[a + 3b + 9c] = deviation of the central moment x^a y^b z^c
        T m[27];
#pragma unroll
        for (int i = 0; i < 27; ++i) m[i] = T(0);
        m[2] = dxx;
        m[6] = dyy;
        m[18] = dzz;
        m[4] = Kxy;
        m[10] = Kxz;
        m[12] = Kyz;
        m[8] = dxx * Kyy + cs2 * dyy + T(2) * Kxy * Kxy;
        m[20] = dxx * Kzz + cs2 * dzz + T(2) * Kxz * Kxz;
        m[24] = dyy * Kzz + cs2 * dzz + T(2) * Kyz * Kyz;
        m[14] = Kxx * Kyz + T(2) * Kxy * Kxz;
        m[16] = Kyy * Kxz + T(2) * Kxy * Kyz;
        m[22] = Kzz * Kxy + T(2) * Kxz * Kyz;
        m[26] = dxx * Kyy * Kzz + cs2 * (dyy * Kzz + cs2 * dzz) +
                T(2) * (Kxx * Kyz * Kyz + Kyy * Kxz * Kxz + Kzz * Kxy * Kxy) +
                T(8) * Kxy * Kxz * Kyz;
        // z digit: exponent -> velocity.  Before it, every line (m[i],
        // m[i + 9], m[i + 18]) holds either its z-exponent-1 entry alone (odd
        // x+y exponent) or its z-exponent-0 and -2 ones (even), the entries
        // of odd total order being zero: each line is swept without its
        // products of zero.
        {
            const T uu = uz * uz, a1m = T(2) * uz - T(1), a1p = T(2) * uz + T(1);
            const T am = uu - uz, a0 = T(1) - uu, ap = uu + uz;
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                if (i == 0) {  // the rest-state deviation m[0] is zero too
                    const T k2 = m[18];
                    m[0] = T(0.5) * k2;
                    m[9] = -k2;
                    m[18] = T(0.5) * k2;
                } else if (i & 1) {
                    const T k1 = m[i + 9];
                    m[i] = T(0.5) * (k1 * a1m);
                    m[i + 9] = -(T(2) * uz * k1);
                    m[i + 18] = T(0.5) * (k1 * a1p);
                } else {
                    const T k0 = m[i], k2 = m[i + 18];
                    m[i] = T(0.5) * (k0 * am + k2);
                    m[i + 9] = k0 * a0 - k2;
                    m[i + 18] = T(0.5) * (k0 * ap + k2);
                }
            }
        }
        // y digit
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const int i = a + 9 * c;
                sweep3(m[i], m[i + 3], m[i + 6], uy, m[i], m[i + 3], m[i + 6]);
            }
        // x digit
#pragma unroll
        for (int j = 0; j < 9; ++j) {
            const int i = 3 * j;
            sweep3(m[i], m[i + 1], m[i + 2], ux, hdev[i], hdev[i + 1], hdev[i + 2]);
        }
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                const T t1 = (r[j] + dy[j]) * (r[k] + dz[k]);
                const T t2 = dy[j] * (r[k] + dz[k]) + r[j] * dz[k];
#pragma unroll
                for (int i = 0; i < 3; ++i) hdev[i + 3 * j + 9 * k] += dx[i] * t1 + r[i] * t2;
            }
    } else {
        T m[9];
        m[0] = T(0);
        m[1] = T(0);
        m[2] = dxx;
        m[3] = T(0);
        m[4] = Kxy;
        m[5] = T(0);
        m[6] = dyy;
        m[7] = T(0);
        m[8] = dxx * Kyy + cs2 * dyy + T(2) * Kxy * Kxy;
#pragma unroll
        for (int a = 0; a < 3; ++a) sweep3(m[a], m[a + 3], m[a + 6], uy, m[a], m[a + 3], m[a + 6]);
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const int i = 3 * j;
            sweep3(m[i], m[i + 1], m[i + 2], ux, hdev[i], hdev[i + 1], hdev[i + 2]);
        }
#pragma unroll
        for (int j = 0; j < 3; ++j)
#pragma unroll
            for (int i = 0; i < 3; ++i) hdev[i + 3 * j] += dx[i] * (r[j] + dy[j]) + r[i] * dy[j];
        (void)uz; (void)dzz; (void)Kxz; (void)Kyz; (void)Kxx;
    }
}

// c_a . v with the zero components of c_a dropped at compile time (a is a
// constant once the direction loops are unrolled; 0 * v cannot be folded
// away under IEEE rules, so the products are never formed).
template <int D, typename T>
__device__ __forceinline__ T cdot(int a, T vx, T vy, T vz)
{
    const int cx = cx_of(a), cy = cy_of(a), cz = cz_of<D>(a);
    T s = T(0);
    bool any = false;
    if (cx) { s = cx > 0 ? vx : -vx; any = true; }
    if (cy) { const T t = cy > 0 ? vy : -vy; s = any ? s + t : t; any = true; }
    if (cz) { const T t = cz > 0 ? vz : -vz; s = any ? s + t : t; any = true; }
    return s;
}

// Second-order equilibrium weights of a direction a and its opposite,
// Gamma = w (1 - 3/2 u^2 + 9/2 (c.u)^2) +- 3 w c.u (Appendix A), from
// base = 1 - 3/2 u^2 and cu = c_a . u.
template <typename T>
__device__ __forceinline__ void gamma_pair(T w, T base, T cu, T &ga, T &gb)
{
    const T e = w * (base + T(4.5) * cu * cu);
    const T o = T(3) * w * cu;
    ga = e + o;
    gb = e - o;
}

// Source term of the flow populations (Sec. 2.3, dilatation term dropped):
// Xi_a = cs^2 (Gamma_a - w_a)(c_a - u).grad(rho) + Gamma_a (c_a - u).F,
// Gamma_a = f_eq_a / rho (second-order Hermite equilibrium, Appendix A).
template <int D, typename T>
__device__ __forceinline__ T source_xi(const Cell<T> &c, int a, T usq, T V, T &gam)
{
    const T w = weight<D, T>(a);
    const T cu = cdot<D>(a, c.ux, c.uy, c.uz);
    gam = w * (T(1) + T(3) * cu + T(4.5) * cu * cu - T(1.5) * usq);
    const T cg = cdot<D>(a, c.drx, c.dry, c.drz) - c.U;
    const T cf = cdot<D>(a, c.Fx, c.Fy, c.Fz) - V;
    return (T(1) / T(3)) * (gam - w) * cg + gam * cf;
}

// ------------------------------------------------------------------ kernels

// Occupancy target of the cell update: four wavefronts per SIMD for the
// D3Q27 kernels with FP32 arithmetic and plain FP32 flow storage (at most 128
// VGPRs: measured faster than five, which spills, and than no cap); the
// compiler's choice otherwise (the FP16 formats gather a shift and a scale
// with every population and spill under the cap).
// Wavefronts per SIMD the FP16 formats' 3-D update is compiled for (1: the
// compiler's choice).
constexpr int FP16_WAVES = 1;

template <int D, class P, int COLL>
constexpr int collide_waves()
{
    return (D == 3 && sizeof(typename P::T) == 4) ? (P::F::shifted ? FP16_WAVES : 4) : 1;
}

// phi(x) = sum_a g_a(x) over the pulled phase-field populations (Sec. 2.2).
// FP16 formats store the record (phi, the cell's reference from the
// reference array); FP16 phase-field values decode with the cell's own
// reference, the fp16 order parameter of its previous level (rest direction
// in FP32).
template <class P, class NB>
__device__ __forceinline__ void store_phi(const NB &nb, const Ptrs &p, typename P::T v)
{
    using T = typename P::T;
    // non-temporal: read a launch later
    if constexpr (P::F::shifted)
        __builtin_nontemporal_store(make_rec(v, own_at(nb, static_cast<const unsigned *>(p.ref))),
                                    lane_ptr(static_cast<unsigned long long *>(p.phi), nb.row, nb.x));
    else
        __builtin_nontemporal_store(v, lane_ptr(static_cast<T *>(p.phi), nb.row, nb.x));
}

template <int D, class P, class NB>
__device__ __forceinline__ typename P::T phi_body(const NB &nb, long long np, const Ptrs &p)
{
    using T = typename P::T;
    constexpr int Q = Lat<D>::Q;
    T s = 0;
    if constexpr (P::G::shifted) {
        // the moving values in the order the writer sums its own (a and its
        // opposite, a = Q/2 + 1 ..), then the rest value, the remainder of
        // the writer's phi over that sum: where a cell receives the values it
        // sent (a uniform region) the sum reproduces its phi exactly, so the
        // rounding of the sums leaves the phase mass without bias
        const float F = unpack_ref(own_at(nb, static_cast<const unsigned *>(p.ref))).F;
        T m = 0;
#pragma unroll
        for (int a = Q / 2 + 1; a < Q; ++a) {
            const int b = opposite<D>(a);
            const PullLoc la = pull_loc<D>(nb, a), lb = pull_loc<D>(nb, b);
            m += dec_g16(weight<D, float>(a), F, load_code<true>(nb, p.Gin, (long long)la.dir * np, la));
            m += dec_g16(weight<D, float>(b), F, load_code<true>(nb, p.Gin, (long long)lb.dir * np, lb));
        }
        s = own_at(nb, p.grest_in) + m;
    } else {
#pragma unroll
        for (int a = 0; a < Q; ++a) s += pull<D, typename P::G, T>(nb, p.Gin, np, a);
    }
    store_phi<P>(nb, p, s);
    return s;
}

// x per lane; y and z wavefront-uniform when NB is NbRow.
template <int D, class P, class NB>
__device__ __forceinline__ typename P::T phi_cell(const Geom &g, const Ptrs &p, int x, int y, int z)
{
    const NB nb = make_nb(g, x, y, z, (NB *)nullptr);
    return phi_body<D, P>(nb, g.np, p);
}


// The update of one cell: stencil, closure, flow collision, phase-field
// collision; post-collision values stored at the cell.  COLL bit 0: flow
// collision (0 cumulant, 1 single relaxation time); bit 1: first-order
// phase-field equilibrium with the correction term.  KEEP: the stored
// phase-field values are also written to keep[nphi_slot(a) * kstride] (LDS),
// the rest direction's to *keep_rest, for the
// partial sums of the next order parameter.

// Single relaxation time in the 3-D update without partial sums keeps its
// pulled flow values in dynamic LDS, 26 per thread (the launch provides these
// bytes; a block has at most 256 threads); no LDS otherwise.
template <int D, class P, int COLL>
constexpr bool srt_lds_stash()
{
    return (COLL & 1) && D == 3 && !P::G::shifted;
}
template <int D, class P, int COLL>
constexpr size_t srt_lds_bytes(unsigned threads)
{
    return srt_lds_stash<D, P, COLL>() ? size_t(26) * threads * sizeof(typename P::T) : 0;
}

template <int D, class P, int COLL, class NB, bool KEEP = false>
__device__ __forceinline__ void collide_body(const NB &nb, const Geom &g,
                                             const Phys<typename P::T> &ph, const Ptrs &p,
                                             typename P::T *keep = nullptr, int kstride = 0,
                                             typename P::T *keep_rest = nullptr)
{
    using T = typename P::T;
    constexpr int Q = Lat<D>::Q;
    constexpr T cs2 = T(1) / T(3);
    const int row = nb.row, xl = nb.x;

    Cell<T> c;
    // FP16 phase-field storage: fp16 order parameters of the cells that read
    // the phase-field values stored here (see eval_cell16_paired)
    unsigned gref[P::G::shifted ? Q / 2 : 1];
    // single relaxation time needs the pulled flow values one by one: the
    // moment pass keeps them instead of the collision pulling them from
    // memory again.  In 3-D with partial sums: in the LDS slots of the stored
    // phase-field values, free until the flow collision (the flow set collides
    // first); in 3-D without: in the launch's dynamic LDS; in 2-D (eight
    // values): in registers
    constexpr bool STASH_LDS = KEEP && (COLL & 1) && D == 3 && !P::G::shifted;
    constexpr bool STASH_DYN = !KEEP && srt_lds_stash<D, P, COLL>();
    constexpr bool STASH_REG = !KEEP && (COLL & 1) && D == 2 && !P::G::shifted;
    constexpr bool STASH = STASH_LDS || STASH_DYN || STASH_REG;
    T fkeep[STASH_REG ? Q : 1];
    T fkeep_rest = 0;
    T *stash = STASH_LDS ? keep : fkeep;
    T *const stash_rest = STASH_LDS ? keep_rest : &fkeep_rest;
    int sstride = STASH_LDS ? kstride : 1;
    if constexpr (STASH_DYN) {
        // slot s of thread t at [s * threads + t]: each thread its own slots,
        // consecutive threads in consecutive words
        extern __shared__ double srt_lds[];
        const int threads = int(blockDim.x * blockDim.y * blockDim.z);
        const int tid = int(threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z));
        stash = reinterpret_cast<T *>(srt_lds) + tid;
        sstride = threads;
    }
    eval_cell<D, P, STASH>(nb, g.np, ph, p, c, P::G::shifted ? gref : nullptr, stash, sstride,
                           stash_rest);
    // Scheduling fences between the phases of the cell update keep the
    // compiler from hoisting every load of the kernel to its start, which
    // would hold them all in registers at once (spills, lower occupancy).
    __builtin_amdgcn_sched_barrier(0);
    const T usq = c.ux * c.ux + c.uy * c.uy + c.uz * c.uz;
    const T V = c.ux * c.Fx + c.uy * c.Fy + c.uz * c.Fz;
    const T rcs2 = c.rho * cs2;

    // --- flow set (Sec. 2.3)
    auto flow = [&]() {
        // FP16 flow storage: this cell's reference for the values it stores
        // (see "FP16 storage"); the decoded values are summed for the rest
        // direction's remainder
        unsigned rw = 0;
        Ref16 W{0.0f, 0.0f};
        float sw = 1.0f, isw = 1.0f;
        if constexpr (P::F::shifted) {
            rw = pack_ref(c.pstar, c.phi);
            W = unpack_ref(rw);
            sw = flow_scale16(ph, W.F);
            isw = 1.0f / sw;
        }
        T fsum = 0;
        auto emit = [&](int a, T dev) {
            if constexpr (P::F::shifted) {
                const float w = weight<D, float>(a);
                const __half h = __float2half((dev * (1.0f / w) + (c.pstar - W.P)) * isw);
                fsum += dec_f16(w, W, sw, __half2float(h));
                store_code<P::G::shifted>(nb, p.Fout, (long long)a * g.np, row, xl, __half_as_ushort(h));
            } else {
                const T v = dev + weight<D, T>(a) * c.pstar;
                fsum += v;
                __builtin_nontemporal_store(typename P::F::raw(v),
                    lane_ptr(static_cast<typename P::F::raw *>(p.Fout), (long long)a * g.np + row, xl));
            }
        };
        // the rest direction: the remainder of sum f'* = sum f' + sum Xi, so the
        // zeroth moment does not drift with the rounding of the stored values
        auto emit_rest = [&](T v0) {
            if constexpr (P::F::shifted)
                __builtin_nontemporal_store(float(v0), lane_ptr(p.frest_out, row, xl));
            else
                __builtin_nontemporal_store(typename P::F::raw(v0),
                    lane_ptr(static_cast<typename P::F::raw *>(p.Fout), (long long)(Q / 2) * g.np + row, xl));
        };
        if constexpr ((COLL & 1) == 0) {
            // second moments of Xi in closed form (4th-order isotropy of the lattice)
            auto xim = [&](T ui, T uj, T gi, T gj, T Fi, T Fj, bool diag) {
                return cs2 * (cs2 * ((diag ? c.U : T(0)) + ui * gj + uj * gi) - ui * uj * c.U) +
                       cs2 * (ui * Fj + uj * Fi) - ui * uj * V;
            };
            const T Mxx = c.Sxx + T(0.5) * xim(c.ux, c.ux, c.drx, c.drx, c.Fx, c.Fx, true);
            const T Myy = c.Syy + T(0.5) * xim(c.uy, c.uy, c.dry, c.dry, c.Fy, c.Fy, true);
            const T Mxy = c.Sxy + T(0.5) * xim(c.ux, c.uy, c.drx, c.dry, c.Fx, c.Fy, false);
            // second-order central moments of the unit-mass set, diagonal ones as
            // deviations from cs^2 (they are cs^2 + O(u^2) and relax by a small
            // amount, so carrying cs^2 along would cost digits in FP32)
            const T pc = cs2 * c.pstar;
            const T Pxx = T(3) * (Mxx - pc) * c.irho - c.ux * c.ux;
            const T Pyy = T(3) * (Myy - pc) * c.irho - c.uy * c.uy;
            const T Pxy = T(3) * Mxy * c.irho - c.ux * c.uy;
            const T om1 = T(1) - c.omega;
            T hd[Q];  // h* - w
            if constexpr (D == 3) {
                const T Mzz = c.Szz + T(0.5) * xim(c.uz, c.uz, c.drz, c.drz, c.Fz, c.Fz, true);
                const T Mxz = c.Sxz + T(0.5) * xim(c.ux, c.uz, c.drx, c.drz, c.Fx, c.Fz, false);
                const T Myz = c.Syz + T(0.5) * xim(c.uy, c.uz, c.dry, c.drz, c.Fy, c.Fz, false);
                const T Pzz = T(3) * (Mzz - pc) * c.irho - c.uz * c.uz;
                const T Pxz = T(3) * Mxz * c.irho - c.ux * c.uz;
                const T Pyz = T(3) * Myz * c.irho - c.uy * c.uz;
                // deviatoric parts relax with omega, the trace goes to 3 cs^2
                const T A = om1 * (Pxx - Pyy), B = om1 * (Pxx - Pzz);
                rebuild<D, T>(c.ux, c.uy, c.uz, (A + B) / T(3), (B - T(2) * A) / T(3),
                              (A - T(2) * B) / T(3), om1 * Pxy, om1 * Pxz, om1 * Pyz, hd);
            } else {
                const T A = om1 * (Pxx - Pyy);
                rebuild<D, T>(c.ux, c.uy, T(0), T(0.5) * A, T(-0.5) * A, T(0), om1 * Pxy, T(0), T(0),
                              hd);
            }
            // f'* = rho cs^2 (h* - w) + w p* + Xi/2, a direction and its opposite
            // together (c.u, c.grad(rho), c.F change sign)
            const T base = T(1) - T(1.5) * usq;
#pragma unroll
            for (int a = Q / 2 + 1; a < Q; ++a) {
                const int b = opposite<D>(a);
                const T w = weight<D, T>(a);
                const T cu = cdot<D>(a, c.ux, c.uy, c.uz);
                const T cg = cdot<D>(a, c.drx, c.dry, c.drz);
                const T cf = cdot<D>(a, c.Fx, c.Fy, c.Fz);
                T ga, gb;
                gamma_pair(w, base, cu, ga, gb);
                // Xi = cs^2 (Gamma - w)(c.grad(rho) - U) + Gamma (c.F - V)
                const T xa = cs2 * (ga - w) * (cg - c.U) + ga * (cf - V);
                const T xb = -(cs2 * (gb - w) * (cg + c.U) + gb * (cf + V));
                emit(a, rcs2 * hd[a] + T(0.5) * xa);
                emit(b, rcs2 * hd[b] + T(0.5) * xb);
            }
            emit_rest((c.S0 + cs2 * c.U) - fsum);
        } else {
            // single relaxation time: f'* = f' - omega (f' - f'_eq) + (1 - omega/2) Xi
#pragma unroll
            for (int a = 0; a < Q; ++a) {
                const int cx = cx_of(a), cy = cy_of(a), cz = cz_of<D>(a);
                T v;
                if constexpr (STASH) {
                    v = a == Q / 2 ? *stash_rest : stash[nphi_slot(a) * sstride];
                } else if constexpr (P::F::shifted) {
                    // decode with the writer's reference, from its record
                    const unsigned long long *rec = static_cast<const unsigned long long *>(p.phi);
                    if (a == Q / 2) {
                        v = own_at(nb, p.frest_in);
                    } else {
                        const PullLoc l = pull_loc<D>(nb, a);
                        const Ref16 R = unpack_ref(rec_ref(l.bb ? own_at(nb, rec) : load_loc(nb, rec, 0, l)));
                        v = dec_f16(weight<D, float>(a), R, flow_scale16(ph, R.F),
                                    load_code(nb, p.Fin, (long long)l.dir * g.np, l));
                    }
                } else {
                    v = pull<D, typename P::F, T>(nb, p.Fin, g.np, a);
                }
                const T w = weight<D, T>(a);
                const T cu = T(cx) * c.ux + T(cy) * c.uy + T(cz) * c.uz;
                T gam;
                const T xi = source_xi<D, T>(c, a, usq, V, gam);
                const T feq_dev = w * rcs2 * (T(3) * cu + T(4.5) * cu * cu - T(1.5) * usq);
                const T vdev = v - w * c.pstar;
                const T dev = vdev - c.omega * (vdev - feq_dev) + (T(1) - T(0.5) * c.omega) * xi;
                if (a == Q / 2)
                    emit_rest(dev + w * c.pstar);
                else
                    emit(a, dev);
            }
        }
        // non-temporal, as the codes: the order-parameter stage reads it a launch later
        if constexpr (P::F::shifted) __builtin_nontemporal_store(rw, lane_ptr(p.ref, row, xl));
    };

    // --- phase field (Sec. 2.2)
    // conservative Allen-Cahn: g* = g + (g_eq - g)/taubar + S_bar; the rest
    // direction is the remainder of sum g* = phi.
    auto phase = [&]() {
        const T nrm = sqrt(c.gx * c.gx + c.gy * c.gy + c.gz * c.gz + T(1e-24));
        const T nx = c.gx / nrm, ny = c.gy / nrm, nz = c.gz / nrm;
        const T src = ph.src_pre * ph.four_W * c.phi * (T(1) - c.phi);
        // g_eq = phi Gamma: a direction and its opposite together.  With the
        // first-order equilibrium (Sec. 2.2) g_eq = w phi (1 + c.u / cs^2) and the
        // correction (1 - 1/(2 taubar)) (w / cs^2) c.d(phi u)/dt is added, the time
        // derivative the backward difference of the cell's (phi u) over one step.
        const T gbase = T(1) - T(1.5) * usq;
        T gsum = 0;
        // FP16 phase-field storage: the reader's reference F, fp16 of its phi
        const unsigned short Fself_bits = P::G::shifted ? half_bits(float(c.phi)) : 0;
        auto gemit = [&](int a, T gout, float F) {
            if constexpr (P::G::shifted) {
                const float w = weight<D, float>(a);
                const __half h = __float2half(gout * (1.0f / w) - F);
                const float dec = dec_g16(w, F, __half2float(h));
                gsum += dec;
                store_code<P::G::shifted>(nb, p.Gout, (long long)a * g.np, row, xl, __half_as_ushort(h));
                if constexpr (KEEP) keep[nphi_slot(a) * kstride] = dec;
            } else {
                gsum += gout;
                __builtin_nontemporal_store(typename P::G::raw(gout),
                    lane_ptr(static_cast<typename P::G::raw *>(p.Gout), (long long)a * g.np + row, xl));
                if constexpr (KEEP) keep[nphi_slot(a) * kstride] = gout;
            }
        };
        auto cac = [&](auto first_order) {
            constexpr bool E1 = decltype(first_order)::value;
            T dx = 0, dy = 0, dz = 0;
            if constexpr (E1) {
                T *out = static_cast<T *>(p.phiu_out);
                const T *in = static_cast<const T *>(p.phiu_in);
                const T qx = c.phi * c.ux, qy = c.phi * c.uy, qz = c.phi * c.uz;
                if (p.have_prev) {
                    dx = qx - *lane_ptr(in, row, xl);
                    dy = qy - *lane_ptr(in, g.np + row, xl);
                    dz = qz - *lane_ptr(in, 2 * g.np + row, xl);
                }
                // non-temporal: read by the next update
                __builtin_nontemporal_store(qx, lane_ptr(out, row, xl));
                __builtin_nontemporal_store(qy, lane_ptr(out, g.np + row, xl));
                __builtin_nontemporal_store(qz, lane_ptr(out, 2 * g.np + row, xl));
            }
            // the pulled values: all loads issued before the first store (the
            // compiler cannot prove the stored set apart from the pulled one,
            // and would otherwise wait on each pair before storing it)
            constexpr bool preload = P::F::shifted || P::G::shifted || CAC_PRELOAD;
            T pre[preload ? Q : 1];
            if constexpr (preload) {
#pragma unroll
                for (int a = 0; a < Q; ++a) {
                    if (a == Q / 2) continue;
                    if constexpr (P::G::shifted) {
                        const PullLoc l = pull_loc<D>(nb, a);
                        pre[a] = dec_g16(weight<D, float>(a), c.Fown,
                                         load_code<true>(nb, p.Gin, (long long)l.dir * g.np, l));
                    } else {
                        pre[a] = pull<D, typename P::G, T>(nb, p.Gin, g.np, a);
                    }
                }
            }
#pragma unroll
            for (int a = Q / 2 + 1; a < Q; ++a) {
                const int b = opposite<D>(a);
                const T w = weight<D, T>(a);
                T va, vb;
                float Fa = 0.0f, Fb = 0.0f;
                if constexpr (preload) {
                    va = pre[a];
                    vb = pre[b];
                } else {
                    va = pull<D, typename P::G, T>(nb, p.Gin, g.np, a);
                    vb = pull<D, typename P::G, T>(nb, p.Gin, g.np, b);
                }
                if constexpr (P::G::shifted) {
                    const unsigned r = gref[a - (Q / 2 + 1)];
                    Fa = half_val(wall_out<D>(nb, a) ? Fself_bits : (unsigned short)(r & 0xffffu));
                    Fb = half_val(wall_out<D>(nb, b) ? Fself_bits : (unsigned short)(r >> 16));
                }
                const T cu = cdot<D>(a, c.ux, c.uy, c.uz);
                T ga, gb;
                T s = w * cdot<D>(a, nx, ny, nz) * src;
                if constexpr (E1) {
                    const T o = T(3) * w * cu;
                    ga = w + o;
                    gb = w - o;
                    s += ph.src_pre * T(3) * w * cdot<D>(a, dx, dy, dz);
                } else {
                    gamma_pair(w, gbase, cu, ga, gb);
                }
                gemit(a, va + (c.phi * ga - va) * ph.inv_tpb + s, Fa);
                gemit(b, vb + (c.phi * gb - vb) * ph.inv_tpb - s, Fb);
            }
            const T g0 = c.phi - gsum;
            if constexpr (P::G::shifted)
                __builtin_nontemporal_store(float(g0), lane_ptr(p.grest_out, row, xl));
            else
                __builtin_nontemporal_store(typename P::G::raw(g0),
                    lane_ptr(static_cast<typename P::G::raw *>(p.Gout), (long long)(Q / 2) * g.np + row, xl));
            if constexpr (KEEP) *keep_rest = g0;
        };
        cac(std::integral_constant<bool, (COLL & 2) != 0>{});
    };

    // FP16 phase-field storage updates the phase field first, while the
    // readers' references from the stencil are still live; otherwise the flow
    // set first
    if constexpr (P::G::shifted) {
        phase();
        __builtin_amdgcn_sched_barrier(0);
        flow();
    } else {
        flow();
        __builtin_amdgcn_sched_barrier(0);
        phase();
    }
}

template <int D, class P, int COLL, class NB>
__device__ __forceinline__ void collide_cell(const Geom &g, const Phys<typename P::T> &ph,
                                             const Ptrs &p, int x, int y, int z)
{
    const NB nb = make_nb(g, x, y, z, (NB *)nullptr);
    collide_body<D, P, COLL>(nb, g, ph, p);
}

template <bool ROW>
using NbOf = typename std::conditional<ROW, NbRow, NbLane>::type;

// Thread -> cell for a block starting at (x0, y0, z0).  ROW: the block is a
// multiple of 64 wide in x, so each wavefront lies in one x-row and y, z are
// taken from its first lane as wavefront-uniform values.
template <bool ROW>
__device__ __forceinline__ void thread_cell(int x0, int y0, int z0, int &x, int &y, int &z)
{
    x = x0 + int(threadIdx.x);
    y = y0 + int(threadIdx.y);
    z = z0 + int(threadIdx.z);
    if constexpr (ROW) {
        y = __builtin_amdgcn_readfirstlane(y);
        z = __builtin_amdgcn_readfirstlane(z);
    }
}


// ------------------------------------------------------- next order parameter
// phi^{n+1}(x) is the zeroth moment of the populations pulled at x (Sec. 2.2),
// sum_a g*_a(x - c_a) under periodic wrap, with bounced-back values where the
// source lies beyond a wall.  Instead of a separate pass that re-reads all Q
// post-collision values of every cell, the update kernel sums them where they
// are produced.  A block updates whole x-rows (block.x = nx, x periodic) of
// by = block.y rows of one plane z (by from nphi_rows), keeps its 26 moving
// post-collision g* in LDS ([row][slot][x], 53 KB for 512 FP32 or 256 FP64
// threads: three tiles per CU) and the rest value in a register, and after a
// barrier sums for every destination cell the values it received from this
// tile, split by the source plane:
//   part[oz][d]     (oz = -1, 0, 1; d in the tile's rows of plane z + oz): the
//                   values that left this tile's plane z towards d, plus, for
//                   oz = 0, the cell's own values that bounced back from a wall
//                   in y or z;
//   edge[0][oz][t]  the values from the last row of tile t - 1 to the first
//                   row of tile t; edge[1][oz][t] from the first row of tile
//                   t + 1 to the last row of tile t ([2][3][ny / by][nz][nx];
//                   tiles wrap in periodic y, end at walls).
// k_phi_merge adds the pieces of each cell in a fixed order.  Lattices: 3-D,
// x periodic with nx a multiple of 64 up to 256 (512 with 512-thread tiles),
// y and z periodic or walls; any storage format (an FP16 phase-field set
// keeps the values its readers will decode).

// Threads of a tile (its rows: as many as fit, dividing ny): 512 for FP32
// (four wavefronts per SIMD, three tiles per CU); 256 for FP64, whose LDS
// tile would otherwise pass 64 KiB; 256 for the FP16 formats, whose update
// holds more registers, except on 512-cell rows, which take one row per
// 512-thread tile.
constexpr int NPHI_THREADS = 512;
constexpr int FP16_NPHI_THREADS = 256;
inline int nphi_threads(int storage, int nx)
{
    if (storage == ST_FP32) return NPHI_THREADS;
    if (storage == ST_FP64) return 256;
    return nx > FP16_NPHI_THREADS ? NPHI_THREADS : FP16_NPHI_THREADS;
}
__device__ __forceinline__ long long nphi_edge_at(const Geom &g, int ntiles, int kind, int oz, int t,
                                                  int z, int x)
{
    return ((((long long)kind * 3 + oz + 1) * ntiles + t) * g.nz + z) * g.nx + x;
}

// The sums of the phi-summing update after its barrier, for the thread's cell
// as destination (row ty of tile t, planes z - 1 .. z + 1) and, in the first
// and last tile rows, for the neighbouring tiles' edge rows.  BX: the row
// length nx, or 0 for a run-time one (bx_rt).
template <class P, int BX, int B>
__device__ __forceinline__ void nphi_gather(const Geom &g, const NextPhi &q,
                                            const typename P::T *lds, typename P::T rest, int x,
                                            int xm, int xp, int t, int ty, int y, int z, int bx_rt)
{
    using T = typename P::T;
    const int bx = BX ? BX : bx_rt, RS = 26 * bx;
    const int by = q.by;
    // value a of tile row r, source column x - ox: col[ox + 1][(r - ty + B) RS + slot(a) bx]
    const T *col[3] = {lds + (ty - B) * RS + xp, lds + (ty - B) * RS + x, lds + (ty - B) * RS + xm};
    auto V = [&](int a, int r, int c) {
        return a == 13 ? rest : col[c][(r - ty + B) * RS + nphi_slot(a) * bx];
    };
    T *part = static_cast<T *>(q.part);
    T *edge = static_cast<T *>(q.edge);
    const int ntiles = g.ny / by;
    const bool wy = g.bcy == BC_WALL, wz = g.bcz == BC_WALL;
    const bool ylo = wy && y == 0, yhi = wy && y == g.ny - 1;
    const bool zlo = wz && z == 0, zhi = wz && z == g.nz - 1;
#pragma unroll
    for (int oz = -1; oz <= 1; ++oz) {
        int zd = z + oz;
        if (zd < 0 || zd >= g.nz) {
            if (wz) continue;  // those values bounced back (oz = 0 below)
            zd += zd < 0 ? g.nz : -g.nz;
        }
        T s = 0;
#pragma unroll
        for (int oy = -1; oy <= 1; ++oy) {
            const int r = ty - oy;
            if (r >= 0 && r < by) {
#pragma unroll
                for (int ox = -1; ox <= 1; ++ox)
                    s += V((ox + 1) + 3 * (oy + 1) + 9 * (oz + 1), r, ox + 1);
            }
        }
        if (oz == 0 && (ylo || yhi || zlo || zhi)) {
#pragma unroll
            for (int b = 0; b < 27; ++b) {
                const int by_ = cy_of(b), bz = cz_of<3>(b);
                if ((ylo && by_ == -1) || (yhi && by_ == 1) || (zlo && bz == -1) || (zhi && bz == 1))
                    s += V(b, ty, 1);
            }
        }
        // non-temporal, as the populations: the merge reads them a launch later
        __builtin_nontemporal_store(s, lane_ptr(part, (long long)(oz + 1) * g.np + (zd * g.ny + y) * g.nx, x));
        if (ty == 0 && (!wy || t > 0)) {
            T e = 0;
#pragma unroll
            for (int ox = -1; ox <= 1; ++ox) e += V((ox + 1) + 9 * (oz + 1), 0, ox + 1);
            __builtin_nontemporal_store(
                e, lane_ptr(edge, nphi_edge_at(g, ntiles, 1, oz, t > 0 ? t - 1 : ntiles - 1, zd, 0), x));
        }
        if (ty == by - 1 && (!wy || t < ntiles - 1)) {
            T e = 0;
#pragma unroll
            for (int ox = -1; ox <= 1; ++ox) e += V((ox + 1) + 6 + 9 * (oz + 1), by - 1, ox + 1);
            __builtin_nontemporal_store(
                e, lane_ptr(edge, nphi_edge_at(g, ntiles, 0, oz, t < ntiles - 1 ? t + 1 : 0, zd, 0), x));
        }
    }
}


// One tile of the phi-summing update: rows t by .. t by + by - 1 of plane z,
// thread (x, ty).  Every thread of the block calls it (it holds a barrier);
// threads with active false (rows beyond the tile in a larger block) only
// take part in the barrier.  BX as for nphi_gather.
template <class P, int COLL, int BX>
__device__ __forceinline__ void nphi_tile(const Geom &g, const Phys<typename P::T> &ph,
                                          const Ptrs &p, const NextPhi &q, typename P::T *lds,
                                          int bx_rt, int t, int ty, int x, int z, bool active)
{
    using T = typename P::T;
    const int bx = BX ? BX : bx_rt, RS = 26 * bx;
    const int y = __builtin_amdgcn_readfirstlane(t * q.by + ty);
    using NB = NbRow;
    NB nb;
    T rest = 0;
    if (active) {
        nb = make_nb(g, x, y, z, (NB *)nullptr);
        collide_body<3, P, COLL, NB, true>(nb, g, ph, p, lds + ty * RS + x, bx, &rest);
    }
    __syncthreads();
    if (!active) return;
    // rows ty - 1 .. ty + 1 are read from a base at row ty - B (B = 1, or 0 in
    // the first tile row, which reads no row above): every LDS offset is a
    // non-negative constant when BX is
    if (ty == 0)
        nphi_gather<P, BX, 0>(g, q, lds, rest, x, nb.xm, nb.xp, t, ty, y, z, bx_rt);
    else
        nphi_gather<P, BX, 1>(g, q, lds, rest, x, nb.xm, nb.xp, t, ty, y, z, bx_rt);
}

// The pieces of one cell's phi in a fixed order: for source planes z + 1, z,
// z - 1 (oz = -1, 0, 1) the tile's own sum, then the sums from the tiles
// below and above where the cell lies on a tile's first or last row.
template <typename T>
__device__ __forceinline__ T nphi_merge_sum(const Geom &g, const T (&v)[3][3], int z, bool first,
                                            bool last)
{
    const bool wz = g.bcz == BC_WALL;
    T s = 0;
#pragma unroll
    for (int oz = 0; oz < 3; ++oz) {
        const int zs = z - (oz - 1);
        if (wz && (zs < 0 || zs >= g.nz)) continue;
        s += v[oz][0];
        if (first) s += v[oz][1];
        if (last) s += v[oz][2];
    }
    return s;
}

// Block (64, 4): each wavefront is 64 cells of one row, so y, z and every
// index but x are wavefront-uniform; each thread merges merge_planes<P>()
// planes, all loads issued before the sums: four in FP32, two in FP64 and in
// the FP16 formats, whose merge also copies the 4-byte references into the
// 8-byte records (measured per format: FP32 37.1 us with four against 39.9
// with two and 40.7 with eight planes; FP16S_ALL 72.3 us with two against
// 74.8 and 86.1; FP64 88.6 us with two against 90.0 with four).
template <class P>
constexpr int merge_planes()
{
    return (P::F::shifted || sizeof(typename P::T) == 8) ? 2 : 4;
}

// phi of cell (x, y, z) from its pieces, loaded one by one (batched form).
template <class P>
__device__ __forceinline__ typename P::T nphi_merge_cell(const Geom &g, const Ptrs &p,
                                                         const NextPhi &q, int x, int y, int z)
{
    using T = typename P::T;
    const int by = q.by, ntiles = g.ny / by;
    const int t = y / by, r = y - t * by;
    const bool wy = g.bcy == BC_WALL, wz = g.bcz == BC_WALL;
    const bool first = r == 0 && (!wy || t > 0), last = r == by - 1 && (!wy || t < ntiles - 1);
    const T *part = static_cast<const T *>(q.part);
    const T *edge = static_cast<const T *>(q.edge);
    const long long row = (long long)(z * g.ny + y) * g.nx;
    T v[3][3];
#pragma unroll
    for (int oz = -1; oz <= 1; ++oz) {
        const int zs = z - oz;
        const bool ok = !(wz && (zs < 0 || zs >= g.nz));
        v[oz + 1][0] = ok ? *lane_ptr(part, (oz + 1) * g.np + row, x) : T(0);
        v[oz + 1][1] = ok && first ? *lane_ptr(edge, nphi_edge_at(g, ntiles, 0, oz, t, z, 0), x) : T(0);
        v[oz + 1][2] = ok && last ? *lane_ptr(edge, nphi_edge_at(g, ntiles, 1, oz, t, z, 0), x) : T(0);
    }
    const T s = nphi_merge_sum(g, v, z, first, last);
    if constexpr (P::F::shifted)
        __builtin_nontemporal_store(make_rec(s, *lane_ptr(static_cast<const unsigned *>(p.ref), row, x)),
                                    lane_ptr(static_cast<unsigned long long *>(p.phi), row, x));
    else
        __builtin_nontemporal_store(s, lane_ptr(static_cast<T *>(p.phi), row, x));
    return s;
}

// ------------------------------------------------------------------ batches
// Many independent domains advance in the same launches.  Blocks stride over
// a tile list (one block per tile when the launch has a block per tile); each
// tile names its domain, whose geometry, parameters, buffers and active step
// window are read from the domain table.  The per-cell arithmetic is the
// single-domain path's (phi_cell, collide_cell, nphi_merge_sum, nphi_tile),
// so a domain's result does not depend on the batch it is in.

__device__ __forceinline__ Ptrs batch_ptrs(const BatchDom &d, int in, bool have_prev)
{
    Ptrs p;
    p.phiu_in = d.phiu[in];
    p.phiu_out = d.phiu[1 - in];
    p.have_prev = have_prev ? 1 : 0;
    p.Fin = d.F[in];
    p.Gin = d.G[in];
    p.Fout = d.F[1 - in];
    p.Gout = d.G[1 - in];
    p.phi = d.phi;
    p.ref = d.ref;
    p.frest_in = d.frest[in];
    p.grest_in = d.grest[in];
    p.frest_out = d.frest[1 - in];
    p.grest_out = d.grest[1 - in];
    return p;
}

// --------------------------------------------------------------- launchers

inline dim3 grid_for(const Ctx &c)
{
    return dim3((c.g.nx + c.block.x - 1) / c.block.x, (c.g.ny + c.block.y - 1) / c.block.y,
                (c.g.nz + c.block.z - 1) / c.block.z);
}

// Calls fn.template operator()<D, P>() for the context's dimension and storage.
template <class Fn>
inline hipError_t dispatch(const Ctx &c, Fn &&fn)
{
    if (c.dim == 2) {
        switch (c.storage) {
        case ST_FP64: return fn.template operator()<2, P64>();
        case ST_FP32: return fn.template operator()<2, P32>();
        case ST_FP16S: return fn.template operator()<2, P16>();
        case ST_FP16S_ALL: return fn.template operator()<2, P16A>();
        }
    } else if (c.dim == 3) {
        switch (c.storage) {
        case ST_FP64: return fn.template operator()<3, P64>();
        case ST_FP32: return fn.template operator()<3, P32>();
        case ST_FP16S: return fn.template operator()<3, P16>();
        case ST_FP16S_ALL: return fn.template operator()<3, P16A>();
        }
    }
    return hipErrorInvalidValue;
}

inline bool row_form(const Ctx &c) { return row_form_ok(c.dim, c.g, c.block); }

// Compile-time operator selection: bit 0 of COLL the flow collision, bit 1
// the first-order phase-field equilibrium.
inline int coll_code(const PhysD &ph) { return (ph.collision ? 1 : 0) | (ph.cac_edf ? 2 : 0); }

template <class Fn>
inline hipError_t with_coll(int code, Fn &&fn)
{
    switch (code) {
    case 0: return fn(std::integral_constant<int, 0>{});
    case 1: return fn(std::integral_constant<int, 1>{});
    case 2: return fn(std::integral_constant<int, 2>{});
    case 3: return fn(std::integral_constant<int, 3>{});
    }
    return hipErrorInvalidValue;
}

}  // namespace mplb
