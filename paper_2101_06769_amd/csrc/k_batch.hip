// Batched kernels: many independent domains in the same launches (see
// device.hpp, "batches").
#include "device.hpp"

namespace mplb {

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
                             ? nphi_merge_cell<P>(g, p, NextPhi{doms[tl.dom].npart,
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

hipError_t launch_batch_step(int dim, int storage, int collision, bool row,
                             const BatchDom *doms, const BatchTile *tiles, const int *ntiles,
                             const long long *tbase, int step_off, dim3 block, const int *grid,
                             int *status, hipStream_t stream)
{
    Ctx c{};
    c.dim = dim;
    c.storage = storage;

    auto go = [&](auto k, dim3 blk, int nblk, size_t lds = 0) {
        hipLaunchKernelGGL(k, dim3(nblk), blk, lds, stream, doms, tiles, ntiles, tbase, step_off,
                           status);
        return hipGetLastError();
    };
    // the phi-summing domains' update, one launch per row length present
    // (grid[2 + k] blocks for NPHI_WIDTHS[k])
    auto go_nphi = [&]<class P>(auto cc) -> hipError_t {
        constexpr int COLL = decltype(cc)::value;
        {
            // a group's tiles have the threads its row length takes alone
            auto one = [&](auto kernel, int nx, int nblk) {
                if (nblk == 0) return hipSuccess;
                const int threads = nphi_threads(storage, nx);
                const size_t lds = size_t(26) * threads * sizeof(typename P::T);
                hipLaunchKernelGGL(kernel, dim3(nblk), dim3(threads), lds, stream, doms, tiles,
                                   ntiles, tbase, step_off);
                return hipGetLastError();
            };
            hipError_t e = one(kb_collide_nphi<P, COLL, 64>, 64, grid[2]);
            if (e == hipSuccess) e = one(kb_collide_nphi<P, COLL, 128>, 128, grid[3]);
            if (e == hipSuccess) e = one(kb_collide_nphi<P, COLL, 192>, 192, grid[4]);
            if (e == hipSuccess) e = one(kb_collide_nphi<P, COLL, 256>, 256, grid[5]);
            if constexpr (sizeof(typename P::T) == 4) {
                if (e == hipSuccess) e = one(kb_collide_nphi<P, COLL, 512>, 512, grid[6]);
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
            // dynamic LDS: single relaxation time's flow values (3-D)
            const size_t lds = srt_lds_bytes<D, P, COLL>(block.x * block.y * block.z);
            hipError_t e2 = row ? go(kb_step<D, P, COLL, false, true>, block, grid[1], lds)
                                : go(kb_step<D, P, COLL, false, false>, block, grid[1], lds);
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

// flag |= 1 if the order parameter of the context's current level holds a
// non-finite value anywhere (grid-stride over the cells).
template <class P>
__global__ void __launch_bounds__(256) k_flag_nonfinite(const void *phi, long long n, int *flag)
{
    using T = typename P::T;
    bool bad = false;
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256) {
        T v;
        if constexpr (P::F::shifted)
            v = rec_phi(gld(static_cast<const unsigned long long *>(phi), i));
        else
            v = gld(static_cast<const T *>(phi), i);
        bad = bad || !__builtin_isfinite(v);
    }
    if (bad) atomicOr(flag, 1);
}

hipError_t launch_flag_nonfinite(const Ctx &c, int *flag)
{
    const long long n = (long long)c.g.nx * c.g.ny * c.g.nz;
    const long long need = (n + 255) / 256;
    const int blocks = int(need < 1024 ? need : 1024);
    return dispatch(c, [&]<int D, class P>() {
        hipLaunchKernelGGL((k_flag_nonfinite<P>), dim3(blocks), dim3(256), 0, c.stream, c.p.phi, n,
                           flag);
        return hipGetLastError();
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


}  // namespace mplb
