// The update that sums the next order parameter and the merge of its
// partial sums (see device.hpp, "next order parameter").
#include "device.hpp"

namespace mplb {

// Row lengths with a kernel (a multiple of 64 up to 256; 512, one row per
// tile, where a tile has 512 threads).
bool nphi_width_ok(int nx, int storage)
{
    return (nx % 64 == 0 && nx <= 256) || (nx == 512 && nphi_threads(storage, nx) >= 512);
}
int nphi_rows(int nx, int ny, int storage)
{
    const int cap = nphi_threads(storage, nx) / nx;
    for (int by = cap; by > 1; --by)
        if (ny % by == 0) return by;
    return 1;
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

template <class P>
__global__ void __launch_bounds__(256) k_phi_merge(Geom g, Ptrs p, NextPhi q)
{
    using T = typename P::T;
    constexpr int MERGE_Z = merge_planes<P>();
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
            // every partial sum and edge value is read once: non-temporal
            v[k][oz + 1][0] = ok ? __builtin_nontemporal_load(lane_ptr(part, (oz + 1) * g.np + row, x)) : T(0);
            v[k][oz + 1][1] = ok && first ? __builtin_nontemporal_load(lane_ptr(edge, nphi_edge_at(g, ntiles, 0, oz, t, z, 0), x)) : T(0);
            v[k][oz + 1][2] = ok && last ? __builtin_nontemporal_load(lane_ptr(edge, nphi_edge_at(g, ntiles, 1, oz, t, z, 0), x)) : T(0);
        }
    }
#pragma unroll
    for (int k = 0; k < MERGE_Z; ++k) {
        const int z = z0 + k;
        if (z >= g.nz) break;
        // non-temporal, as the partial sums: the next update reads phi a launch
        // later (FP16 formats: the record of phi and the cell's reference)
        const long long row = (long long)(z * g.ny + y) * g.nx;
        const T s = nphi_merge_sum(g, v[k], z, first, last);
        if constexpr (P::F::shifted)
            __builtin_nontemporal_store(make_rec(s, *lane_ptr(static_cast<const unsigned *>(p.ref), row, x)),
                                        lane_ptr(static_cast<unsigned long long *>(p.phi), row, x));
        else
            __builtin_nontemporal_store(s, lane_ptr(static_cast<T *>(p.phi), row, x));
    }
}

bool nphi_ok(const Ctx &c)
{
    const Geom &g = c.g;
    return c.dim == 3 && g.bcx == BC_PER && (g.bcy == BC_PER || g.bcy == BC_WALL) &&
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
        if constexpr (D != 3) {
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
                    // one row per tile: 512 threads, FP32 arithmetic only
                    if constexpr (sizeof(T) == 4) return go(k_collide_nphi<P, COLL, 512>);
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
    return dispatch(c, [&]<int D, class P>() {
        constexpr int MERGE_Z = merge_planes<P>();
        const dim3 grid(c.g.nx / 64, (c.g.ny + 3) / 4, (c.g.nz + MERGE_Z - 1) / MERGE_Z);
        hipLaunchKernelGGL((k_phi_merge<P>), grid, dim3(64, 4, 1), 0, c.stream, c.g,
                           c.p, q);
        return hipGetLastError();
    });
}

int nphi_block_threads(int storage, int nx) { return nphi_threads(storage, nx); }


}  // namespace mplb
