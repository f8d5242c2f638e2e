// HIP kernels (gfx950) for one time step of the multiphase lattice Boltzmann
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

// Value of direction plane `dir` at `cell`.  Shifted FP16 values decode as
// w (shift + scale q) with the shift/scale of the cell that stored them
// (scale 1 when sc is null).
template <int D, class S, typename T>
__device__ __forceinline__ T load_pop(const void *base, long long np, int dir, int cell, int a,
                                      const float *sh, const float *sc)
{
    if constexpr (S::shifted) {
        const float q = __half2float(gld(static_cast<const __half *>(base), (long long)dir * np + cell));
        const float w = weight<D, float>(a);
        return T(w * (gld(sh, cell) + (sc ? gld(sc, cell) : 1.0f) * q));
    } else {
        return T(gld(static_cast<const typename S::raw *>(base), (long long)dir * np + cell));
    }
}

// Store dev + w shift (plain) or dev / (w scale) (shifted) as direction a
// of the cell (row + x).
template <int D, class S, typename T>
__device__ __forceinline__ void store_dev(void *base, long long np, int a, int row, int x, T dev,
                                          T shift, T scale)
{
    if constexpr (S::shifted) {
        const float w = weight<D, float>(a);
        *lane_ptr(static_cast<__half *>(base), (long long)a * np + row, x) =
            __half_as_ushort(__float2half(float(dev) / (w * float(scale))));
    } else {
        __builtin_nontemporal_store(typename S::raw(dev + weight<D, T>(a) * shift),
                                    lane_ptr(static_cast<typename S::raw *>(base),
                                             (long long)a * np + row, x));
    }
}

// Value of direction a held in plane `dir` at cell (row + x); see load_pop.
template <int D, class S, typename T>
__device__ __forceinline__ T load_at(const void *base, long long plane, int row, int x, int a,
                                     const float *sh, const float *sc)
{
    if constexpr (S::shifted) {
        const float q =
            __half2float(__ushort_as_half(*lane_ptr(static_cast<const __half *>(base), plane + row, x)));
        const float w = weight<D, float>(a);
        const float s = *lane_ptr(sh, row, x);
        const float r = sc ? *lane_ptr(sc, row, x) : 1.0f;
        return T(w * (s + r * q));
    } else {
        return T(*lane_ptr(static_cast<const typename S::raw *>(base), plane + row, x));
    }
}

// Pre-collision population a at the cell (pull streaming with the boundary
// rules of pull_src), general form.
template <int D, class S, typename T>
__device__ __forceinline__ T pull(const NbLane &n, const void *base, long long np, int a,
                                  const float *sh, const float *sc)
{
    int dir, cell;
    pull_src<D>(*n.g, n.x, n.y, n.z, a, &dir, &cell);
    return load_pop<D, S, T>(base, np, dir, cell, a, sh, sc);
}

// Row form: the y and z rules are wavefront-uniform choices of plane and row
// read off the wavefront's tables; x wraps per lane.  Offsets are 32-bit
// element indices (the arrays hold fewer than 2^31 elements); the uniform
// part (plane and row) and the lane part (x) of an address stay apart, so the
// load is a scalar base plus a 32-bit lane offset (three distinct ones: x,
// x - 1, x + 1) with no per-load vector address arithmetic.
// Source of the pulled value of direction a: plane dir, row offset rs (both
// wavefront-uniform), column xs.
template <int D>
__device__ __forceinline__ void row_src(const NbRow &n, int a, int &dir, int &rs, int &xs)
{
    const int cx = cx_of(a), cy = cy_of(a), cz = cz_of<D>(a);
    const int ky = 1 - cy, kz = 1 - cz;  // table index of y - cy, z - cz
    const unsigned by = cy ? 1u << ky : 0u, bz = cz ? 1u << (3 + kz) : 0u;
    const bool bb = (n.bb & (by | bz)) != 0;
    const int b = a - ((n.sym & by) ? 6 * cy : 0) - ((n.sym & bz) ? 18 * cz : 0);
    dir = bb ? opposite<D>(a) : b;
    rs = bb ? n.row : n.ry[ky] + n.rz[kz];
    xs = (bb || cx == 0) ? n.x : cx > 0 ? n.xm : n.xp;
}

template <int D, class S, typename T>
__device__ __forceinline__ T pull(const NbRow &n, const void *base, long long, int a,
                                  const float *sh, const float *sc)
{
    int dir, rs, xs;
    row_src<D>(n, a, dir, rs, xs);
    const long long off = dir * n.np + rs;
    if constexpr (S::shifted) {
        const float q = __half2float(__ushort_as_half(*lane_ptr(static_cast<const __half *>(base), off, xs)));
        const float w = weight<D, float>(a);
        const float s0 = *lane_ptr(sh, (long long)rs, xs);
        return T(w * (s0 + (sc ? *lane_ptr(sc, (long long)rs, xs) : 1.0f) * q));
    } else {
        return T(*lane_ptr(static_cast<const typename S::raw *>(base), off, xs));
    }
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
    p.visc_interp = d.visc_interp;
    p.collision = d.collision;
    p.cac_edf = d.cac_edf;
    return p;
}

// ------------------------------------------------------------- cell state
template <typename T>
struct Cell {
    T phi, gx, gy, gz, lap;
    T rho, irho, drx, dry, drz, mu, Fx, Fy, Fz, omega;
    T S0, Sx, Sy, Sz, Sxx, Syy, Szz, Sxy, Sxz, Syz;
    T ux, uy, uz, pstar, U;
};

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
// and the velocity part cancels before it reaches the even ones.
template <int D, class P, class NB>
__device__ __forceinline__ void flow_moments(const NB &nb, long long np, const Ptrs &p,
                                             Cell<typename P::T> &c)
{
    using T = typename P::T;
    constexpr int Q = Lat<D>::Q;
    T S0 = pull<D, typename P::F, T>(nb, p.Fin, np, Q / 2, p.fp_in, p.fr_in);
    T Sx = 0, Sy = 0, Sz = 0, Sxx = 0, Syy = 0, Szz = 0, Sxy = 0, Sxz = 0, Syz = 0;
#pragma unroll
    for (int a = Q / 2 + 1; a < Q; ++a) {
        const int b = opposite<D>(a);
        const int cx = cx_of(a), cy = cy_of(a), cz = cz_of<D>(a);
        const T va = pull<D, typename P::F, T>(nb, p.Fin, np, a, p.fp_in, p.fr_in);
        const T vb = pull<D, typename P::F, T>(nb, p.Fin, np, b, p.fp_in, p.fr_in);
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

template <int D, class P, class NB>
__device__ __forceinline__ void eval_cell(const NB &nb, long long np,
                                          const Phys<typename P::T> &ph, const Ptrs &p,
                                          Cell<typename P::T> &c)
{
    using T = typename P::T;
    stencil<D, T>(nb, static_cast<const T *>(p.phi), c);
    closure<D, T>(ph, c);
    flow_moments<D, P>(nb, np, p, c);
    velocity<D, T>(c);
}

// One 3-point sweep: central moments (k0, k1, k2) about u of a set on the
// velocities {-1, 0, +1} -> the three values.
template <typename T>
__device__ __forceinline__ void sweep3(T k0, T k1, T k2, T u, T &vm, T &v0, T &vp)
{
    const T uu = u * u;
    vm = T(0.5) * (k0 * (uu - u) + k1 * (T(2) * u - T(1)) + k2);
    v0 = k0 * (T(1) - uu) - T(2) * u * k1 - k2;
    vp = T(0.5) * (k0 * (uu + u) + k1 * (T(2) * u + T(1)) + k2);
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
        // z digit: exponent -> velocity
#pragma unroll
        for (int i = 0; i < 9; ++i) sweep3(m[i], m[i + 9], m[i + 18], uz, m[i], m[i + 9], m[i + 18]);
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
template <int D, class P, int COLL>
constexpr int collide_waves()
{
    return (D == 3 && sizeof(typename P::T) == 4 && !P::F::shifted) ? 4 : 1;
}

// phi(x) = sum_a g_a(x) over the pulled phase-field populations (Sec. 2.2).
template <int D, class P, class NB>
__device__ __forceinline__ typename P::T phi_body(const NB &nb, long long np, const Ptrs &p)
{
    using T = typename P::T;
    constexpr int Q = Lat<D>::Q;
    T s = 0;
#pragma unroll
    for (int a = 0; a < Q; ++a) s += pull<D, typename P::G, T>(nb, p.Gin, np, a, p.gp_in, nullptr);
    __builtin_nontemporal_store(s, lane_ptr(static_cast<T *>(p.phi), nb.row, nb.x));  // read a launch later
    return s;
}

// x per lane; y and z wavefront-uniform when NB is NbRow.
template <int D, class P, class NB>
__device__ __forceinline__ typename P::T phi_cell(const Geom &g, const Ptrs &p, int x, int y, int z)
{
    const NB nb = make_nb(g, x, y, z, (NB *)nullptr);
    return phi_body<D, P>(nb, g.np, p);
}

template <int D, class P, bool ROW>
__global__ void __launch_bounds__(256) k_phi(Geom g, Ptrs p);

// The update of one cell: stencil, closure, flow collision, phase-field
// collision; post-collision values stored at the cell.  COLL bit 0: flow
// collision (0 cumulant, 1 single relaxation time); bit 1: first-order
// phase-field equilibrium with the correction term.  KEEP: the stored
// phase-field values are also written to keep[nphi_slot(a) * kstride] (LDS),
// the rest direction's to *keep_rest, for the
// partial sums of the next order parameter.
// LDS slot of a moving D3Q27 direction (the rest direction, 13, has none).
__host__ __device__ constexpr int nphi_slot(int a) { return a < 13 ? a : a - 1; }

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
    eval_cell<D, P>(nb, g.np, ph, p, c);
    // Scheduling fences between the phases of the cell update keep the
    // compiler from hoisting every load of the kernel to its start, which
    // would hold them all in registers at once (spills, lower occupancy).
    __builtin_amdgcn_sched_barrier(0);
    const T usq = c.ux * c.ux + c.uy * c.uy + c.uz * c.uz;
    const T V = c.ux * c.Fx + c.uy * c.Fy + c.uz * c.Fz;
    const T rcs2 = c.rho * cs2;

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
        // together (c.u, c.grad(rho), c.F change sign).  Plain formats take
        // the rest direction as the remainder of sum f'* = sum f' + sum Xi, so
        // the zeroth moment does not drift with the rounding of the weights.
        const T base = T(1) - T(1.5) * usq;
        T fsum = 0;
        auto emit = [&](int a, T dev) {
            if constexpr (P::F::shifted) {
                store_dev<D, typename P::F, T>(p.Fout, g.np, a, row, xl, dev, c.pstar, rcs2);
            } else {
                const T v = dev + weight<D, T>(a) * c.pstar;
                fsum += v;
                __builtin_nontemporal_store(typename P::F::raw(v),
                    lane_ptr(static_cast<typename P::F::raw *>(p.Fout), (long long)a * g.np + row, xl));
            }
        };
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
        if constexpr (P::F::shifted) {
            constexpr int a0 = Q / 2;
            const T w0 = weight<D, T>(a0);
            const T g0 = w0 * base;
            emit(a0, rcs2 * hd[a0] + T(0.5) * (-(cs2 * (g0 - w0) * c.U + g0 * V)));
        } else {
            __builtin_nontemporal_store(typename P::F::raw((c.S0 + cs2 * c.U) - fsum),
                lane_ptr(static_cast<typename P::F::raw *>(p.Fout), (long long)(Q / 2) * g.np + row, xl));
        }
    } else {
        // single relaxation time: f'* = f' - omega (f' - f'_eq) + (1 - omega/2) Xi
#pragma unroll
        for (int a = 0; a < Q; ++a) {
            const int cx = cx_of(a), cy = cy_of(a), cz = cz_of<D>(a);
            const T v = pull<D, typename P::F, T>(nb, p.Fin, g.np, a, p.fp_in, p.fr_in);
            const T w = weight<D, T>(a);
            const T cu = T(cx) * c.ux + T(cy) * c.uy + T(cz) * c.uz;
            T gam;
            const T xi = source_xi<D, T>(c, a, usq, V, gam);
            const T feq_dev = w * rcs2 * (T(3) * cu + T(4.5) * cu * cu - T(1.5) * usq);
            const T vdev = v - w * c.pstar;
            const T dev = vdev - c.omega * (vdev - feq_dev) + (T(1) - T(0.5) * c.omega) * xi;
            store_dev<D, typename P::F, T>(p.Fout, g.np, a, row, xl, dev, c.pstar, rcs2);
        }
    }
    if constexpr (P::F::shifted) {
        *lane_ptr(p.fp_out, row, xl) = float(c.pstar);
        *lane_ptr(p.fr_out, row, xl) = float(rcs2);
    }

    __builtin_amdgcn_sched_barrier(0);
    // conservative Allen-Cahn: g* = g + (g_eq - g)/taubar + S_bar (Sec. 2.2).
    // Plain formats take the rest direction as the remainder of sum g* = phi.
    const T nrm = sqrt(c.gx * c.gx + c.gy * c.gy + c.gz * c.gz + T(1e-24));
    const T nx = c.gx / nrm, ny = c.gy / nrm, nz = c.gz / nrm;
    const T src = ph.src_pre * ph.four_W * c.phi * (T(1) - c.phi);
    // g_eq = phi Gamma: a direction and its opposite together.  With the
    // first-order equilibrium (Sec. 2.2) g_eq = w phi (1 + c.u / cs^2) and the
    // correction (1 - 1/(2 taubar)) (w / cs^2) c.d(phi u)/dt is added, the time
    // derivative the backward difference of the cell's (phi u) over one step.
    const T gbase = T(1) - T(1.5) * usq;
    T gsum = 0;
    auto gemit = [&](int a, T gout) {
        if constexpr (P::G::shifted) {
            store_dev<D, typename P::G, T>(p.Gout, g.np, a, row, xl, gout - weight<D, T>(a) * c.phi,
                                           c.phi, T(1));
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
            *lane_ptr(out, row, xl) = qx;
            *lane_ptr(out, g.np + row, xl) = qy;
            *lane_ptr(out, 2 * g.np + row, xl) = qz;
        }
#pragma unroll
        for (int a = Q / 2 + 1; a < Q; ++a) {
            const int b = opposite<D>(a);
            const T w = weight<D, T>(a);
            const T va = pull<D, typename P::G, T>(nb, p.Gin, g.np, a, p.gp_in, nullptr);
            const T vb = pull<D, typename P::G, T>(nb, p.Gin, g.np, b, p.gp_in, nullptr);
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
            gemit(a, va + (c.phi * ga - va) * ph.inv_tpb + s);
            gemit(b, vb + (c.phi * gb - vb) * ph.inv_tpb - s);
        }
        if constexpr (P::G::shifted) {
            constexpr int a0 = Q / 2;
            const T v0 = pull<D, typename P::G, T>(nb, p.Gin, g.np, a0, p.gp_in, nullptr);
            const T g0 = E1 ? weight<D, T>(a0) : weight<D, T>(a0) * gbase;
            gemit(a0, v0 + (c.phi * g0 - v0) * ph.inv_tpb);
        } else {
            const T g0 = c.phi - gsum;
            __builtin_nontemporal_store(typename P::G::raw(g0),
                lane_ptr(static_cast<typename P::G::raw *>(p.Gout), (long long)(Q / 2) * g.np + row, xl));
            if constexpr (KEEP) *keep_rest = g0;
        }
    };
    cac(std::integral_constant<bool, (COLL & 2) != 0>{});
    if constexpr (P::G::shifted) *lane_ptr(p.gp_out, row, xl) = float(c.phi);
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

template <int D, class P, bool ROW>
__global__ void __launch_bounds__(256) k_phi(Geom g, Ptrs p)
{
    int x, y, z;
    thread_cell<ROW>(blockIdx.x * blockDim.x, blockIdx.y * blockDim.y, blockIdx.z * blockDim.z, x,
                     y, z);
    if (x >= g.nx || y >= g.ny || z >= g.nz) return;
    phi_cell<D, P, NbOf<ROW>>(g, p, x, y, z);
}

template <int D, class P, int COLL, bool ROW>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(collide_waves<D, P, COLL>())))
k_collide(Geom g, Phys<typename P::T> ph, Ptrs p)
{
    int x, y, z;
    thread_cell<ROW>(blockIdx.x * blockDim.x, blockIdx.y * blockDim.y, blockIdx.z * blockDim.z, x,
                     y, z);
    if (x >= g.nx || y >= g.ny || z >= g.nz) return;
    collide_cell<D, P, COLL, NbOf<ROW>>(g, ph, p, x, y, z);
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
// x periodic with nx a multiple of 64 up to 256, y and z periodic or walls;
// phase-field populations in plain storage.

// Rows per tile: as many as the thread budget allows, dividing ny.  512
// threads for FP32 (four wavefronts per SIMD, two tiles per CU); 256 for
// FP64, whose LDS tile would otherwise pass 64 KiB, and for FP16S, whose
// update holds too many registers for two 512-thread tiles per CU.
constexpr int NPHI_THREADS = 512;
static int nphi_threads(int storage) { return storage == ST_FP32 ? NPHI_THREADS : 256; }
// Row lengths with a kernel (a multiple of 64 up to 256; 512, one row per
// tile, where a tile has 512 threads).
bool nphi_width_ok(int nx, int storage)
{
    return (nx % 64 == 0 && nx <= 256) || (nx == 512 && nphi_threads(storage) >= 512);
}
int nphi_rows(int nx, int ny, int storage)
{
    const int cap = nphi_threads(storage) / nx;
    for (int by = cap; by > 1; --by)
        if (ny % by == 0) return by;
    return 1;
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

// BX = nx, a compile-time row length so that every LDS offset is an immediate.
template <class P, int COLL, int BX>
__global__ void __launch_bounds__(NPHI_THREADS) __attribute__((amdgpu_waves_per_eu(collide_waves<3, P, COLL>())))
k_collide_nphi(Geom g, Phys<typename P::T> ph, Ptrs p, NextPhi q)
{
    using T = typename P::T;
    extern __shared__ double nphi_lds[];
    nphi_tile<P, COLL, BX>(g, ph, p, q, reinterpret_cast<T *>(nphi_lds), BX, int(blockIdx.y),
                           __builtin_amdgcn_readfirstlane(int(threadIdx.y)), int(threadIdx.x),
                           __builtin_amdgcn_readfirstlane(int(blockIdx.z)), true);
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
// index but x are wavefront-uniform; each thread merges MERGE_Z planes, all
// loads issued before the sums.
constexpr int MERGE_Z = 4;

template <typename T>
__global__ void __launch_bounds__(256) k_phi_merge(Geom g, Ptrs p, NextPhi q)
{
    const int x = blockIdx.x * 64 + threadIdx.x;
    const int y = __builtin_amdgcn_readfirstlane(int(blockIdx.y * 4 + threadIdx.y));
    const int z0 = int(blockIdx.z) * MERGE_Z;
    if (y >= g.ny) return;
    const int by = q.by, ntiles = g.ny / by;
    const int t = y / by, r = y - t * by;
    const bool wy = g.bcy == BC_WALL, wz = g.bcz == BC_WALL;
    const bool first = r == 0 && (!wy || t > 0), last = r == by - 1 && (!wy || t < ntiles - 1);
    const T *__restrict__ part = static_cast<const T *>(q.part);
    const T *__restrict__ edge = static_cast<const T *>(q.edge);
    T v[MERGE_Z][3][3];
#pragma unroll
    for (int k = 0; k < MERGE_Z; ++k) {
        const int z = z0 + k;
#pragma unroll
        for (int oz = -1; oz <= 1; ++oz) {
            const int zs = z - oz;
            const bool ok = z < g.nz && !(wz && (zs < 0 || zs >= g.nz));
            const long long row = (long long)(z * g.ny + y) * g.nx;
            v[k][oz + 1][0] = ok ? *lane_ptr(part, (oz + 1) * g.np + row, x) : T(0);
            v[k][oz + 1][1] = ok && first ? *lane_ptr(edge, nphi_edge_at(g, ntiles, 0, oz, t, z, 0), x) : T(0);
            v[k][oz + 1][2] = ok && last ? *lane_ptr(edge, nphi_edge_at(g, ntiles, 1, oz, t, z, 0), x) : T(0);
        }
    }
#pragma unroll
    for (int k = 0; k < MERGE_Z; ++k) {
        const int z = z0 + k;
        if (z >= g.nz) break;
        // non-temporal, as the partial sums: the next update reads phi a launch later
        __builtin_nontemporal_store(nphi_merge_sum(g, v[k], z, first, last),
                                    lane_ptr(static_cast<T *>(p.phi), (long long)(z * g.ny + y) * g.nx, x));
    }
}

// phi of cell (x, y, z) from its pieces, loaded one by one (batched form).
template <typename T>
__device__ __forceinline__ T nphi_merge_cell(const Geom &g, const Ptrs &p, const NextPhi &q,
                                                int x, int y, int z)
{
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
    __builtin_nontemporal_store(s, lane_ptr(static_cast<T *>(p.phi), row, x));
    return s;
}

// Equilibrium initial state, computed in FP64 for every storage format and
// scattered to the slots the first step pulls from.
template <int D, class P>
__global__ void __launch_bounds__(256) k_init(Geom g, PhysD ph, Ptrs p, const double *dphi,
                                              const double *du, const double *dp)
{
    constexpr int Q = Lat<D>::Q;
    constexpr double cs2 = 1.0 / 3.0;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z = blockIdx.z * blockDim.z + threadIdx.z;
    if (x >= g.nx || y >= g.ny || z >= g.nz) return;
    const int me = cell_of(g, x, y, z);
    const long long N = (long long)g.nx * g.ny * g.nz;
    Cell<double> c;
    stencil<D, double>(make_nb(g, x, y, z, (NbLane *)nullptr), dphi, c);
    closure<D, double>(to_phys<double>(ph), c);
    const double ux = du[me], uy = du[N + me], uz = D == 3 ? du[2 * N + me] : 0.0;
    const double h = 0.5 * c.irho;
    // population velocity and pressure such that the scheme reports u and p
    const double vx = ux - h * c.Fx, vy = uy - h * c.Fy, vz = uz - h * c.Fz;
    const double U = ux * c.drx + uy * c.dry + uz * c.drz;
    const double ppop = dp[me] - 0.5 * cs2 * U;
    const double usq = ux * ux + uy * uy + uz * uz, vsq = vx * vx + vy * vy + vz * vz;
    const double rcs2 = c.rho * cs2;
#pragma unroll
    for (int a = 0; a < Q; ++a) {
        const int cx = cx_of(a), cy = cy_of(a), cz = cz_of<D>(a);
        const double w = weight<D, double>(a);
        const double cv = cx * vx + cy * vy + cz * vz;
        const double cu = cx * ux + cy * uy + cz * uz;
        const double fdev = w * rcs2 * (3.0 * cv + 4.5 * cv * cv - 1.5 * vsq);
        const double gval = w * c.phi * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * usq);
        int dir, cell;
        pull_src<D>(g, x, y, z, a, &dir, &cell);
        // the slot's own cell supplies the shift/scale of shifted formats
        if constexpr (P::F::shifted) {
            const float w32 = weight<D, float>(a);
            const double f = w * ppop + fdev;
            static_cast<__half *>(p.Fout)[(long long)dir * g.np + cell] =
                __float2half(float((f - w * p.fp_out[cell]) / (w32 * p.fr_out[cell])));
        } else {
            static_cast<typename P::F::raw *>(p.Fout)[(long long)dir * g.np + cell] =
                typename P::F::raw(w * ppop + fdev);
        }
        if constexpr (P::G::shifted) {
            const float w32 = weight<D, float>(a);
            static_cast<__half *>(p.Gout)[(long long)dir * g.np + cell] =
                __float2half(float((gval - w * p.gp_out[cell]) / w32));
        } else {
            static_cast<typename P::G::raw *>(p.Gout)[(long long)dir * g.np + cell] =
                typename P::G::raw(gval);
        }
    }
}

// Shift/scale of shifted formats from FP64 phi and pressure fields.
template <int D>
__global__ void __launch_bounds__(256) k_set_refs(Geom g, PhysD ph, Ptrs p, const double *dphi,
                                                  const double *dp)
{
    const long long N = (long long)g.nx * g.ny * g.nz;
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    if (p.fp_out) {
        p.fp_out[i] = float(dp[i]);
        p.fr_out[i] = float((ph.rho_l + ph.drho * dphi[i]) / 3.0);
    }
    if (p.gp_out) p.gp_out[i] = float(dphi[i]);
}

template <int D, class P>
__global__ void __launch_bounds__(256) k_get_pop(Geom g, Ptrs p, int which, int a0, int a1,
                                                 double *dst)
{
    using T = typename P::T;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z = blockIdx.z * blockDim.z + threadIdx.z;
    if (x >= g.nx || y >= g.ny || z >= g.nz) return;
    const int me = cell_of(g, x, y, z);
    const long long N = (long long)g.nx * g.ny * g.nz;
#pragma unroll
    for (int a = 0; a < Lat<D>::Q; ++a) {
        if (a < a0 || a >= a1) continue;
        int dir, cell;
        pull_src<D>(g, x, y, z, a, &dir, &cell);
        const T v = which == 0
                        ? load_pop<D, typename P::F, T>(p.Fin, g.np, dir, cell, a, p.fp_in, p.fr_in)
                        : load_pop<D, typename P::G, T>(p.Gin, g.np, dir, cell, a, p.gp_in, nullptr);
        dst[(long long)(a - a0) * N + me] = double(v);
    }
}

template <int D, class P>
__global__ void __launch_bounds__(256) k_set_pop(Geom g, Ptrs p, int which, int a0, int a1,
                                                 const double *src)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z = blockIdx.z * blockDim.z + threadIdx.z;
    if (x >= g.nx || y >= g.ny || z >= g.nz) return;
    const int me = cell_of(g, x, y, z);
    const long long N = (long long)g.nx * g.ny * g.nz;
#pragma unroll
    for (int a = 0; a < Lat<D>::Q; ++a) {
        if (a < a0 || a >= a1) continue;
        int dir, cell;
        pull_src<D>(g, x, y, z, a, &dir, &cell);
        const double v = src[(long long)(a - a0) * N + me];
        const double w = weight<D, double>(a);
        const float w32 = weight<D, float>(a);
        if (which == 0) {
            if constexpr (P::F::shifted)
                static_cast<__half *>(p.Fout)[(long long)dir * g.np + cell] =
                    __float2half(float((v - w * p.fp_out[cell]) / (w32 * p.fr_out[cell])));
            else
                static_cast<typename P::F::raw *>(p.Fout)[(long long)dir * g.np + cell] =
                    typename P::F::raw(v);
        } else {
            if constexpr (P::G::shifted)
                static_cast<__half *>(p.Gout)[(long long)dir * g.np + cell] =
                    __float2half(float((v - w * p.gp_out[cell]) / w32));
            else
                static_cast<typename P::G::raw *>(p.Gout)[(long long)dir * g.np + cell] =
                    typename P::G::raw(v);
        }
    }
}

template <int D, class P>
__global__ void __launch_bounds__(256) k_field(Geom g, Phys<typename P::T> ph, Ptrs p, int field,
                                               double *dst)
{
    using T = typename P::T;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z = blockIdx.z * blockDim.z + threadIdx.z;
    if (x >= g.nx || y >= g.ny || z >= g.nz) return;
    Cell<T> c;
    const NbLane nb = make_nb(g, x, y, z, (NbLane *)nullptr);
    eval_cell<D, P>(nb, g.np, ph, p, c);
    T v = field == 0 ? c.phi : field == 1 ? c.rho : field == 2 ? c.ux : field == 3 ? c.uy
        : field == 4 ? c.uz : c.pstar;
    dst[cell_of(g, x, y, z)] = double(v);
}

constexpr int RED_BLOCKS = 1024;
constexpr int RED_THREADS = 256;

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}
__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_down(v, off, 64));
    return v;
}

// Per-block partial sums in a fixed order: grid-stride over cells, wavefront
// shuffles, then the four wavefronts of the block in order.
template <int D, class P>
__global__ void __launch_bounds__(RED_THREADS) k_reduce_partial(Geom g, Phys<typename P::T> ph,
                                                               Ptrs p, double *partials)
{
    using T = typename P::T;
    const long long N = (long long)g.nx * g.ny * g.nz;
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (long long i = (long long)blockIdx.x * RED_THREADS + threadIdx.x; i < N;
         i += (long long)gridDim.x * RED_THREADS) {
        const int x = int(i % g.nx), y = int((i / g.nx) % g.ny), z = int(i / ((long long)g.nx * g.ny));
        Cell<T> c;
        const NbLane nb = make_nb(g, x, y, z, (NbLane *)nullptr);
        eval_cell<D, P>(nb, g.np, ph, p, c);
        const double rho = double(c.rho);
        const double ux = double(c.ux), uy = double(c.uy), uz = double(c.uz);
        const double um = sqrt(ux * ux + uy * uy + uz * uz);
        const double ph0 = double(c.phi);
        acc[0] += ph0;
        acc[1] += rho * ux;
        acc[2] += rho * uy;
        acc[3] += rho * uz;
        acc[4] = fmax(acc[4], um);
        if (!isfinite(ph0) || !isfinite(rho * ux) || !isfinite(rho * uy) || !isfinite(rho * uz) ||
            !isfinite(um))
            acc[5] += 1.0;
    }
    __shared__ double red[RED_THREADS / 64][6];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const double v = k == 4 ? wave_max(acc[k]) : wave_sum(acc[k]);
        if (lane == 0) red[wv][k] = v;
    }
    __syncthreads();
    if (threadIdx.x < 6) {
        const int k = threadIdx.x;
        double v = red[0][k];
        for (int w = 1; w < RED_THREADS / 64; ++w) v = k == 4 ? fmax(v, red[w][k]) : v + red[w][k];
        partials[blockIdx.x * 8 + k] = v;
    }
}

__global__ void __launch_bounds__(RED_THREADS) k_reduce_final(const double *partials, int nblocks,
                                                             double *out)
{
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < nblocks; b += RED_THREADS)
#pragma unroll
        for (int k = 0; k < 6; ++k)
            acc[k] = k == 4 ? fmax(acc[k], partials[b * 8 + k]) : acc[k] + partials[b * 8 + k];
    __shared__ double red[RED_THREADS / 64][6];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const double v = k == 4 ? wave_max(acc[k]) : wave_sum(acc[k]);
        if (lane == 0) red[wv][k] = v;
    }
    __syncthreads();
    if (threadIdx.x < 6) {
        const int k = threadIdx.x;
        double v = red[0][k];
        for (int w = 1; w < RED_THREADS / 64; ++w) v = k == 4 ? fmax(v, red[w][k]) : v + red[w][k];
        out[k] = v;
    }
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
    p.fp_in = d.fp[in];
    p.fr_in = d.fr[in];
    p.gp_in = d.gp[in];
    p.fp_out = d.fp[1 - in];
    p.fr_out = d.fr[1 - in];
    p.gp_out = d.gp[1 - in];
    return p;
}

template <int D, class P, int COLL, bool PHI, bool ROW>
__global__ void __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(PHI ? 1 : collide_waves<D, P, COLL>()))) kb_step(const BatchDom *__restrict__ doms,
                                               const BatchTile *__restrict__ tiles,
                                               const int *ntiles, const long long *tbase,
                                               int step_off, int *status)
{
    using T = typename P::T;
    const long long t = *tbase + step_off;
    // the phi stage covers every domain, the update those without nphi_by;
    // the phi stage also flags a domain whose order parameter is not finite
    // (status[dom] != 0): a non-finite population of either set reaches phi
    // within a step
    const int nt = PHI ? ntiles[1] : ntiles[0];
    for (int ti = blockIdx.x; ti < nt; ti += gridDim.x) {
        const BatchTile tl = tiles[ti];
        // the domain's record by value: read once, not re-read after every
        // population store the compiler cannot prove to be elsewhere
        const Geom g = doms[tl.dom].g;
        const long long first = doms[tl.dom].first, last = doms[tl.dom].last;
        if (t < first || t >= last) continue;
        const Ptrs p = batch_ptrs(doms[tl.dom], int((t - first) & 1), t >= doms[tl.dom].hist_from);
        // the tile is tl.w cells wide in x and (block threads) / tl.w rows
        // high, one plane deep; the width is the domain's own (a multiple of
        // 64 in the row form, so that each wavefront lies in one x-row)
        const int tid = int(threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z));
        const int x = tl.x0 + tid % tl.w;
        int y = tl.y0 + tid / tl.w;
        const int z = tl.z0;
        if constexpr (ROW) y = __builtin_amdgcn_readfirstlane(y);
        if (x >= g.nx || y >= g.ny || z >= tl.z1) continue;
        const int nby = doms[tl.dom].nphi_by;
        if constexpr (PHI) {
            const T ph = (D == 3 && nby && t >= doms[tl.dom].nphi_from)
                             ? nphi_merge_cell<T>(g, p, NextPhi{doms[tl.dom].npart,
                                                                doms[tl.dom].nedge, nby}, x, y, z)
                             : phi_cell<D, P, NbOf<ROW>>(g, p, x, y, z);
            if (!__builtin_isfinite(ph)) atomicOr(status + tl.dom, 1);
        } else {
            const Phys<T> ph = to_phys<T>(doms[tl.dom].ph);
            collide_cell<D, P, COLL, NbOf<ROW>>(g, ph, p, x, y, z);
        }
    }
}

// Batched phi-summing update for domains with rows of BX cells (64, 128,
// 192, 256 or 512): blocks stride over the ntiles[3 + 2k] tiles from index
// ntiles[2 + 2k], k = nphi_group(BX) (domain, rows y0 .. y0 + nphi_by - 1 of
// plane z0), each an nphi_tile of its domain.  (A loop over several planes
// per tile keeps the tile's pointers and parameters live across the update
// and spills: measured slower even for one plane.)  FP32: at most 80 VGPRs (six
// wavefronts per SIMD), so that three tiles fit a CU as in the
// single-domain kernel.
template <class P, int COLL>
constexpr int kb_nphi_waves()
{
    return collide_waves<3, P, COLL>() == 4 ? 6 : collide_waves<3, P, COLL>();
}

template <class P, int COLL, int BX>
__global__ void __launch_bounds__(NPHI_THREADS) __attribute__((amdgpu_waves_per_eu(kb_nphi_waves<P, COLL>())))
kb_collide_nphi(const BatchDom *__restrict__ doms, const BatchTile *__restrict__ tiles,
                const int *ntiles, const long long *tbase, int step_off)
{
    using T = typename P::T;
    extern __shared__ double nphi_lds[];
    constexpr int k = nphi_group(BX);
    const long long t = *tbase + step_off;
    const int n0 = ntiles[2 + 2 * k], nt = ntiles[3 + 2 * k];
    for (int ti = blockIdx.x; ti < nt; ti += gridDim.x) {
        const BatchTile tl = tiles[n0 + ti];
        const Geom g = doms[tl.dom].g;  // by value, see kb_step
        const long long first = doms[tl.dom].first, last = doms[tl.dom].last;
        if (t < first || t >= last) continue;  // the whole block
        const Ptrs p = batch_ptrs(doms[tl.dom], int((t - first) & 1), t >= doms[tl.dom].hist_from);
        const Phys<T> ph = to_phys<T>(doms[tl.dom].ph);
        const NextPhi q{doms[tl.dom].npart, doms[tl.dom].nedge, doms[tl.dom].nphi_by};
        const int tid = int(threadIdx.x);
        const int ty = __builtin_amdgcn_readfirstlane(tid / BX);
        nphi_tile<P, COLL, BX>(g, ph, p, q, reinterpret_cast<T *>(nphi_lds), BX, tl.y0 / q.by, ty,
                               tid - ty * BX, tl.z0, ty < q.by);
        __syncthreads();  // the next tile of this block reuses the LDS
    }
}

__global__ void k_set_i64(long long *ptr, long long v) { *ptr = v; }

__global__ void __launch_bounds__(256) k_fill_i32(int *ptr, int n, int v)
{
    const int i = int(blockIdx.x * blockDim.x + threadIdx.x);
    if (i < n) ptr[i] = v;
}

// --------------------------------------------------------------- launchers

static dim3 grid_for(const Ctx &c)
{
    return dim3((c.g.nx + c.block.x - 1) / c.block.x, (c.g.ny + c.block.y - 1) / c.block.y,
                (c.g.nz + c.block.z - 1) / c.block.z);
}

// Calls fn.template operator()<D, P>() for the context's dimension and storage.
template <class Fn>
static hipError_t dispatch(const Ctx &c, Fn &&fn)
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

// Row-form addressing: every wavefront inside one x-row of the block, x
// periodic, population arrays of fewer than 2^31 elements.
bool row_form_ok(int dim, const Geom &g, dim3 block)
{
    const long long Q = dim == 2 ? 9 : 27;
    return block.x % 64 == 0 && g.bcx == BC_PER && Q * g.np < (1ll << 31);
}

static bool row_form(const Ctx &c) { return row_form_ok(c.dim, c.g, c.block); }

hipError_t launch_phi(const Ctx &c)
{
    return dispatch(c, [&]<int D, class P>() {
        if (row_form(c))
            hipLaunchKernelGGL((k_phi<D, P, true>), grid_for(c), c.block, 0, c.stream, c.g, c.p);
        else
            hipLaunchKernelGGL((k_phi<D, P, false>), grid_for(c), c.block, 0, c.stream, c.g, c.p);
        return hipGetLastError();
    });
}

// Compile-time operator selection: bit 0 of COLL the flow collision, bit 1
// the first-order phase-field equilibrium.
static int coll_code(const PhysD &ph) { return (ph.collision ? 1 : 0) | (ph.cac_edf ? 2 : 0); }

template <class Fn>
static hipError_t with_coll(int code, Fn &&fn)
{
    switch (code) {
    case 0: return fn(std::integral_constant<int, 0>{});
    case 1: return fn(std::integral_constant<int, 1>{});
    case 2: return fn(std::integral_constant<int, 2>{});
    case 3: return fn(std::integral_constant<int, 3>{});
    }
    return hipErrorInvalidValue;
}

hipError_t launch_collide(const Ctx &c)
{
    return dispatch(c, [&]<int D, class P>() {
        using T = typename P::T;
        const bool row = row_form(c);
        return with_coll(coll_code(c.ph), [&](auto cc) {
            constexpr int COLL = decltype(cc)::value;
            if (row)
                hipLaunchKernelGGL((k_collide<D, P, COLL, true>), grid_for(c), c.block, 0, c.stream,
                                   c.g, to_phys<T>(c.ph), c.p);
            else
                hipLaunchKernelGGL((k_collide<D, P, COLL, false>), grid_for(c), c.block, 0,
                                   c.stream, c.g, to_phys<T>(c.ph), c.p);
            return hipGetLastError();
        });
    });
}

bool nphi_ok(const Ctx &c)
{
    const Geom &g = c.g;
    return c.dim == 3 && (c.storage == ST_FP64 || c.storage == ST_FP32 || c.storage == ST_FP16S) &&
           g.bcx == BC_PER && (g.bcy == BC_PER || g.bcy == BC_WALL) &&
           (g.bcz == BC_PER || g.bcz == BC_WALL) && nphi_width_ok(g.nx, c.storage) &&
           27 * g.np < (1ll << 31);
}

static bool nphi_tile_ok(const Ctx &c, const NextPhi &q)
{
    return nphi_ok(c) && q.by == nphi_rows(c.g.nx, c.g.ny, c.storage);
}

hipError_t launch_collide_nphi(const Ctx &c, const NextPhi &q)
{
    if (!nphi_tile_ok(c, q)) return hipErrorInvalidValue;
    return dispatch(c, [&]<int D, class P>() {
        using T = typename P::T;
        if constexpr (D != 3 || P::G::shifted) {
            return hipErrorInvalidValue;
        } else {
            const dim3 block(c.g.nx, q.by, 1);
            const dim3 grid(1, c.g.ny / q.by, c.g.nz);
            const size_t lds = size_t(26) * block.x * block.y * sizeof(T);
            return with_coll(coll_code(c.ph), [&](auto cc) {
                constexpr int COLL = decltype(cc)::value;
                auto go = [&](auto kernel) {
                    hipLaunchKernelGGL(kernel, grid, block, lds, c.stream, c.g, to_phys<T>(c.ph),
                                       c.p, q);
                    return hipGetLastError();
                };
                switch (c.g.nx) {
                case 64: return go(k_collide_nphi<P, COLL, 64>);
                case 128: return go(k_collide_nphi<P, COLL, 128>);
                case 192: return go(k_collide_nphi<P, COLL, 192>);
                case 256: return go(k_collide_nphi<P, COLL, 256>);
                case 512:
                    // one row per tile: 512 threads, FP32 only
                    if constexpr (std::is_same<P, P32>::value) return go(k_collide_nphi<P, COLL, 512>);
                    break;
                }
                return hipErrorInvalidValue;
            });
        }
    });
}

hipError_t launch_phi_merge(const Ctx &c, const NextPhi &q)
{
    if (!nphi_tile_ok(c, q)) return hipErrorInvalidValue;
    const dim3 grid(c.g.nx / 64, (c.g.ny + 3) / 4, (c.g.nz + MERGE_Z - 1) / MERGE_Z);
    return dispatch(c, [&]<int D, class P>() {
        hipLaunchKernelGGL((k_phi_merge<typename P::T>), grid, dim3(64, 4, 1), 0, c.stream, c.g,
                           c.p, q);
        return hipGetLastError();
    });
}

hipError_t launch_init(const Ctx &c, const double *phi, const double *u, const double *pr)
{
    return dispatch(c, [&]<int D, class P>() {
        hipLaunchKernelGGL((k_init<D, P>), grid_for(c), c.block, 0, c.stream, c.g, c.ph, c.p, phi,
                           u, pr);
        return hipGetLastError();
    });
}

hipError_t launch_set_refs(const Ctx &c, const double *phi, const double *pr)
{
    const long long N = (long long)c.g.nx * c.g.ny * c.g.nz;
    const dim3 grid((unsigned)((N + 255) / 256));
    if (c.dim == 2)
        hipLaunchKernelGGL(k_set_refs<2>, grid, dim3(256), 0, c.stream, c.g, c.ph, c.p, phi, pr);
    else
        hipLaunchKernelGGL(k_set_refs<3>, grid, dim3(256), 0, c.stream, c.g, c.ph, c.p, phi, pr);
    return hipGetLastError();
}

hipError_t launch_get_pop(const Ctx &c, int which, int a0, int a1, double *dst)
{
    return dispatch(c, [&]<int D, class P>() {
        hipLaunchKernelGGL((k_get_pop<D, P>), grid_for(c), c.block, 0, c.stream, c.g, c.p, which,
                           a0, a1, dst);
        return hipGetLastError();
    });
}

hipError_t launch_set_pop(const Ctx &c, int which, int a0, int a1, const double *src)
{
    return dispatch(c, [&]<int D, class P>() {
        hipLaunchKernelGGL((k_set_pop<D, P>), grid_for(c), c.block, 0, c.stream, c.g, c.p, which,
                           a0, a1, src);
        return hipGetLastError();
    });
}

hipError_t launch_field(const Ctx &c, int field, double *dst)
{
    return dispatch(c, [&]<int D, class P>() {
        hipLaunchKernelGGL((k_field<D, P>), grid_for(c), c.block, 0, c.stream, c.g,
                           to_phys<typename P::T>(c.ph), c.p, field, dst);
        return hipGetLastError();
    });
}

int nphi_block_threads(int storage) { return nphi_threads(storage); }

hipError_t launch_batch_step(int dim, int storage, int collision, bool row,
                             const BatchDom *doms, const BatchTile *tiles, const int *ntiles,
                             const long long *tbase, int step_off, dim3 block, const int *grid,
                             int *status, hipStream_t stream)
{
    Ctx c{};
    c.dim = dim;
    c.storage = storage;

    auto go = [&](auto k, dim3 blk, int nblk) {
        hipLaunchKernelGGL(k, dim3(nblk), blk, 0, stream, doms, tiles, ntiles, tbase, step_off,
                           status);
        return hipGetLastError();
    };
    // the phi-summing domains' update (plain phase-field storage only), one
    // launch per row length present (grid[2 + k] blocks for NPHI_WIDTHS[k])
    auto go_nphi = [&]<class P>(auto cc) -> hipError_t {
        constexpr int COLL = decltype(cc)::value;
        if constexpr (P::G::shifted) {
            return hipErrorInvalidValue;
        } else {
            const int threads = nphi_threads(storage);
            const size_t lds = size_t(26) * threads * sizeof(typename P::T);
            auto one = [&](auto kernel, int nblk) {
                if (nblk == 0) return hipSuccess;
                hipLaunchKernelGGL(kernel, dim3(nblk), dim3(threads), lds, stream, doms, tiles,
                                   ntiles, tbase, step_off);
                return hipGetLastError();
            };
            hipError_t e = one(kb_collide_nphi<P, COLL, 64>, grid[2]);
            if (e == hipSuccess) e = one(kb_collide_nphi<P, COLL, 128>, grid[3]);
            if (e == hipSuccess) e = one(kb_collide_nphi<P, COLL, 192>, grid[4]);
            if (e == hipSuccess) e = one(kb_collide_nphi<P, COLL, 256>, grid[5]);
            if constexpr (std::is_same<P, P32>::value) {
                if (e == hipSuccess) e = one(kb_collide_nphi<P, COLL, 512>, grid[6]);
            } else {
                if (grid[6]) e = hipErrorInvalidValue;
            }
            return e;
        }
    };
    // collision: the operator code (bit 0 flow collision, bit 1 first-order
    // phase-field equilibrium), shared by every domain of the batch
    return dispatch(c, [&]<int D, class P>() {
        hipError_t e = row ? go(kb_step<D, P, 0, true, true>, block, grid[0])
                           : go(kb_step<D, P, 0, true, false>, block, grid[0]);
        if (e != hipSuccess) return e;
        return with_coll(collision, [&](auto cc) {
            constexpr int COLL = decltype(cc)::value;
            hipError_t e2 = row ? go(kb_step<D, P, COLL, false, true>, block, grid[1])
                                : go(kb_step<D, P, COLL, false, false>, block, grid[1]);
            const bool nphi = grid[2] || grid[3] || grid[4] || grid[5] || grid[6];
            if constexpr (D == 3) {
                if (e2 == hipSuccess && nphi) e2 = go_nphi.template operator()<P>(cc);
            } else {
                if (nphi) e2 = hipErrorInvalidValue;
            }
            return e2;
        });
    });
}

hipError_t launch_set_i64(long long *ptr, long long v, hipStream_t stream)
{
    hipLaunchKernelGGL(k_set_i64, dim3(1), dim3(1), 0, stream, ptr, v);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int *ptr, int n, int v, hipStream_t stream)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_i32, dim3((n + 255) / 256), dim3(256), 0, stream, ptr, n, v);
    return hipGetLastError();
}

int reduce_blocks(const Ctx &c)
{
    const long long N = (long long)c.g.nx * c.g.ny * c.g.nz;
    const long long need = (N + RED_THREADS - 1) / RED_THREADS;
    return int(need < RED_BLOCKS ? need : RED_BLOCKS);
}

hipError_t launch_reduce(const Ctx &c, double *partials, double *out)
{
    const int nb = reduce_blocks(c);
    hipError_t e = dispatch(c, [&]<int D, class P>() {
        hipLaunchKernelGGL((k_reduce_partial<D, P>), dim3(nb), dim3(RED_THREADS), 0, c.stream, c.g,
                           to_phys<typename P::T>(c.ph), c.p, partials);
        return hipGetLastError();
    });
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(RED_THREADS), 0, c.stream, partials, nb, out);
    return hipGetLastError();
}

}  // namespace mplb
