// Host exchange (initial state, populations in and out, fields) and the
// deterministic FP64 reductions.
#include <map>
#include <mutex>

#include "device.hpp"

namespace mplb {

// A pre-collision value v of direction a of set `which` (0 f', 1 g) that
// cell `me` pulls from slot (dir, cell), in the set's storage format: plain
// as is; FP16 as a code against the references of "FP16 storage" (flow: the
// writing cell's, phase field: the reader's, both from the reference array),
// the rest direction in FP32.
template <int D, class P>
__device__ __forceinline__ void put_value(const Geom &g, const Ptrs &p, const Phys<float> &pf,
                                          int which, int a, int dir, int cell, int me, double v)
{
    constexpr int Q = Lat<D>::Q;
    const long long e = (long long)dir * g.np + cell;
    const double w = weight<D, double>(a);
    if (which == 0) {
        if constexpr (P::F::shifted) {
            if (a == Q / 2) {
                p.frest_out[me] = float(v);
            } else {
                const Ref16 R = unpack_ref(p.ref[cell]);
                static_cast<unsigned short *>(p.Fout)[e] =
                    half_bits(float((v / w - double(R.P)) / double(flow_scale16(pf, R.F))));
            }
        } else {
            static_cast<typename P::F::raw *>(p.Fout)[e] = typename P::F::raw(v);
        }
    } else {
        if constexpr (P::G::shifted) {
            if (a == Q / 2) {
                p.grest_out[me] = float(v);
            } else {
                const float F = unpack_ref(p.ref[me]).F;
                static_cast<unsigned short *>(p.Gout)[e] = half_bits(float(v / w - double(F)));
            }
        } else {
            static_cast<typename P::G::raw *>(p.Gout)[e] = typename P::G::raw(v);
        }
    }
}

// The inverse of put_value (from the Fin / Gin buffers).
template <int D, class P>
__device__ __forceinline__ double get_value(const Geom &g, const Ptrs &p, const Phys<float> &pf,
                                            int which, int a, int dir, int cell, int me)
{
    constexpr int Q = Lat<D>::Q;
    const long long e = (long long)dir * g.np + cell;
    if (which == 0) {
        if constexpr (P::F::shifted) {
            if (a == Q / 2) return p.frest_in[me];
            const Ref16 R = unpack_ref(p.ref[cell]);
            return dec_f16(weight<D, float>(a), R, flow_scale16(pf, R.F),
                           half_val(static_cast<const unsigned short *>(p.Fin)[e]));
        } else {
            return double(static_cast<const typename P::F::raw *>(p.Fin)[e]);
        }
    } else {
        if constexpr (P::G::shifted) {
            if (a == Q / 2) return p.grest_in[me];
            return dec_g16(weight<D, float>(a), unpack_ref(p.ref[me]).F,
                           half_val(static_cast<const unsigned short *>(p.Gin)[e]));
        } else {
            return double(static_cast<const typename P::G::raw *>(p.Gin)[e]);
        }
    }
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
    const Phys<float> pf = to_phys<float>(ph);
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
        put_value<D, P>(g, p, pf, 0, a, dir, cell, me, w * ppop + fdev);
        put_value<D, P>(g, p, pf, 1, a, dir, cell, me, gval);
    }
}

// References of the FP16 formats for an initial state: the prescribed
// pressure and order parameter of each cell, rounded to FP16.
template <int D>
__global__ void __launch_bounds__(256) k_set_refs(Geom g, PhysD ph, Ptrs p, const double *dphi,
                                                  const double *dp)
{
    const long long N = (long long)g.nx * g.ny * g.nz;
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    p.ref[i] = pack_ref(float(dp[i]), float(dphi[i]));
}

template <int D, class P>
__global__ void __launch_bounds__(256) k_get_pop(Geom g, PhysD ph, Ptrs p, int which, int a0,
                                                 int a1, double *dst)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z = blockIdx.z * blockDim.z + threadIdx.z;
    if (x >= g.nx || y >= g.ny || z >= g.nz) return;
    const int me = cell_of(g, x, y, z);
    const long long N = (long long)g.nx * g.ny * g.nz;
    const Phys<float> pf = to_phys<float>(ph);
#pragma unroll
    for (int a = 0; a < Lat<D>::Q; ++a) {
        if (a < a0 || a >= a1) continue;
        int dir, cell;
        pull_src<D>(g, x, y, z, a, &dir, &cell);
        dst[(long long)(a - a0) * N + me] = get_value<D, P>(g, p, pf, which, a, dir, cell, me);
    }
}

template <int D, class P>
__global__ void __launch_bounds__(256) k_set_pop(Geom g, PhysD ph, Ptrs p, int which, int a0,
                                                 int a1, const double *src)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z = blockIdx.z * blockDim.z + threadIdx.z;
    if (x >= g.nx || y >= g.ny || z >= g.nz) return;
    const int me = cell_of(g, x, y, z);
    const long long N = (long long)g.nx * g.ny * g.nz;
    const Phys<float> pf = to_phys<float>(ph);
#pragma unroll
    for (int a = 0; a < Lat<D>::Q; ++a) {
        if (a < a0 || a >= a1) continue;
        int dir, cell;
        pull_src<D>(g, x, y, z, a, &dir, &cell);
        put_value<D, P>(g, p, pf, which, a, dir, cell, me, src[(long long)(a - a0) * N + me]);
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
        hipLaunchKernelGGL((k_get_pop<D, P>), grid_for(c), c.block, 0, c.stream, c.g, c.ph, c.p,
                           which, a0, a1, dst);
        return hipGetLastError();
    });
}

hipError_t launch_set_pop(const Ctx &c, int which, int a0, int a1, const double *src)
{
    return dispatch(c, [&]<int D, class P>() {
        hipLaunchKernelGGL((k_set_pop<D, P>), grid_for(c), c.block, 0, c.stream, c.g, c.ph, c.p,
                           which, a0, a1, src);
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


// ---------------------------------------------------- static scratch
// The reduction's partial sums and result in a file-scope device array, for
// callers that cannot allocate device memory (see mplb_reduce_noalloc): room
// for RED_BLOCKS blocks of 8 partials and the 8 results.  Each device holds
// its own copy at its own address, looked up once per device; calls that
// overlap on one device share it and race.
constexpr int SCRATCH_DOUBLES = RED_BLOCKS * 8 + 8;
static __device__ __align__(256) double scratch[SCRATCH_DOUBLES];

namespace {
std::mutex scratch_mu;
std::map<int, double *> scratch_ptr;  // device -> address of `scratch` there
}  // namespace

static hipError_t scratch_base(double **base)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lock(scratch_mu);
    auto it = scratch_ptr.find(dev);
    if (it != scratch_ptr.end()) {
        *base = it->second;
        return hipSuccess;
    }
    void *ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    scratch_ptr[dev] = static_cast<double *>(ptr);
    *base = static_cast<double *>(ptr);
    return hipSuccess;
}

int reduce_scratch_max_blocks() { return RED_BLOCKS; }

hipError_t launch_reduce_static(const Ctx &c, double **result)
{
    if (reduce_blocks(c) > RED_BLOCKS) return hipErrorInvalidValue;
    double *base = nullptr;
    const hipError_t e = scratch_base(&base);
    if (e != hipSuccess) return e;
    *result = base + RED_BLOCKS * 8;
    return launch_reduce(c, base, *result);
}

}  // namespace mplb
