// The step kernels of one domain: the order-parameter pass and the cell
// update (see device.hpp).
#include "device.hpp"

namespace mplb {

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

// Row-form addressing: every wavefront inside one x-row of the block, x
// periodic, population arrays of fewer than 2^31 elements.
bool row_form_ok(int dim, const Geom &g, dim3 block)
{
    const long long Q = dim == 2 ? 9 : 27;
    return block.x % 64 == 0 && g.bcx == BC_PER && Q * g.np < (1ll << 31);
}

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

hipError_t launch_collide(const Ctx &c)
{
    return dispatch(c, [&]<int D, class P>() {
        using T = typename P::T;
        const bool row = row_form(c);
        return with_coll(coll_code(c.ph), [&](auto cc) {
            constexpr int COLL = decltype(cc)::value;
            // dynamic LDS: single relaxation time's flow values (3-D)
            const size_t lds = srt_lds_bytes<D, P, COLL>(c.block.x * c.block.y * c.block.z);
            if (row)
                hipLaunchKernelGGL((k_collide<D, P, COLL, true>), grid_for(c), c.block, lds,
                                   c.stream, c.g, to_phys<T>(c.ph), c.p);
            else
                hipLaunchKernelGGL((k_collide<D, P, COLL, false>), grid_for(c), c.block, lds,
                                   c.stream, c.g, to_phys<T>(c.ph), c.p);
            return hipGetLastError();
        });
    });
}


}  // namespace mplb
