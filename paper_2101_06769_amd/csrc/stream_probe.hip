// Streaming ceiling of the update's access pattern, with no arithmetic to
// speak of: 54 planes of FP32 in and 54 out per cell (the 27 f' and 27 g
// populations of a D3Q27 step, structure-of-arrays with plane stride N), on
// the 128 x 128 x 512 benchmark grid.  Two shapes, each with 1, 2 or 4
// consecutive cells per thread (4, 8 or 16 bytes per lane and access):
//   all  - every plane loaded, then every plane stored (the update's shape:
//          all loads in flight before the first store);
//   copy - plane after plane, each load followed by its store.
// Stores are non-temporal, as the update's.  Prints one line per variant:
// average launch time over 20 launches and the rate at 2 x 54 x 4 B per
// cell.  Standalone: it shares nothing with the solver library.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>

#define PROBE_CHECK(x)                                                                         \
    do {                                                                                       \
        hipError_t e_ = (x);                                                                   \
        if (e_ != hipSuccess) {                                                                \
            std::fprintf(stderr, "stream_probe: %s failed: %s\n", #x, hipGetErrorString(e_)); \
            std::exit(1);                                                                      \
        }                                                                                      \
    } while (0)

namespace {

constexpr int PLANES = 54;
constexpr long long CELLS = 128LL * 128 * 512;

typedef float f2 __attribute__((ext_vector_type(2)));
typedef float f4 __attribute__((ext_vector_type(4)));
template <int W> struct Lane;
template <> struct Lane<1> { using V = float; static __device__ float sum(float v) { return v; } };
template <> struct Lane<2> { using V = f2; static __device__ float sum(f2 v) { return v.x + v.y; } };
template <> struct Lane<4> {
    using V = f4;
    static __device__ float sum(f4 v) { return (v.x + v.y) + (v.z + v.w); }
};

// Thread t owns cells t*W .. t*W + W - 1; the grid covers n / W threads
// (n a multiple of W * block), so no thread indexes past plane end.
template <int W, int NB>
__global__ void __launch_bounds__(NB) k_all(const float *__restrict__ in, float *__restrict__ out, long long n)
{
    using V = typename Lane<W>::V;
    const long long t = (long long)blockIdx.x * NB + threadIdx.x;
    const long long nv = n / W;
    if (t >= nv) return;
    const V *vin = reinterpret_cast<const V *>(in);
    V *vout = reinterpret_cast<V *>(out);
    V v[PLANES];
#pragma unroll
    for (int a = 0; a < PLANES; ++a) v[a] = vin[a * nv + t];
    // a dependency of every store on every load, so the loads cannot be
    // interleaved with the stores; the added term is below FP32 resolution
    float s = 0;
#pragma unroll
    for (int a = 0; a < PLANES; ++a) s += Lane<W>::sum(v[a]);
#pragma unroll
    for (int a = 0; a < PLANES; ++a) __builtin_nontemporal_store(v[a] + s * 1e-30f, &vout[a * nv + t]);
}

template <int W>
__global__ void __launch_bounds__(256) k_copy(const float *__restrict__ in, float *__restrict__ out, long long n)
{
    using V = typename Lane<W>::V;
    const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
    const long long nv = n / W;
    if (t >= nv) return;
    const V *vin = reinterpret_cast<const V *>(in);
    V *vout = reinterpret_cast<V *>(out);
#pragma unroll 6
    for (int a = 0; a < PLANES; ++a) __builtin_nontemporal_store(vin[a * nv + t], &vout[a * nv + t]);
}

template <class L>
double average_ms(L launch)
{
    hipEvent_t e0, e1;
    PROBE_CHECK(hipEventCreate(&e0));
    PROBE_CHECK(hipEventCreate(&e1));
    launch();
    launch();
    PROBE_CHECK(hipGetLastError());
    PROBE_CHECK(hipDeviceSynchronize());
    constexpr int reps = 20;
    PROBE_CHECK(hipEventRecord(e0));
    for (int r = 0; r < reps; ++r) launch();
    PROBE_CHECK(hipEventRecord(e1));
    PROBE_CHECK(hipEventSynchronize(e1));
    PROBE_CHECK(hipGetLastError());
    float ms = 0;
    PROBE_CHECK(hipEventElapsedTime(&ms, e0, e1));
    PROBE_CHECK(hipEventDestroy(e0));
    PROBE_CHECK(hipEventDestroy(e1));
    return double(ms) / reps;
}

} // namespace

int main()
{
    static_assert(CELLS % (4 * 512) == 0, "every variant's grid must tile the planes exactly");
    const size_t bytes = size_t(PLANES) * CELLS * sizeof(float);
    float *in = nullptr, *out = nullptr;
    PROBE_CHECK(hipMalloc(&in, bytes));
    PROBE_CHECK(hipMalloc(&out, bytes));
    PROBE_CHECK(hipMemset(in, 0, bytes));
    PROBE_CHECK(hipMemset(out, 0, bytes));
    const double moved = 2.0 * double(bytes);
    std::printf("stream_probe: %d FP32 planes in and out, %lld cells, %.3f GB per launch\n", PLANES, CELLS,
                moved * 1e-9);
    auto report = [&](const char *name, double ms) {
        std::printf("%-24s %9.1f us %8.1f GB/s\n", name, ms * 1e3, moved / (ms * 1e-3) * 1e-9);
        std::fflush(stdout);
    };
    const long long n = CELLS;
    report("all W=1 block 256", average_ms([&] {
               hipLaunchKernelGGL((k_all<1, 256>), dim3(unsigned(n / 256)), dim3(256), 0, 0, in, out, n);
           }));
    report("all W=1 block 512", average_ms([&] {
               hipLaunchKernelGGL((k_all<1, 512>), dim3(unsigned(n / 512)), dim3(512), 0, 0, in, out, n);
           }));
    report("all W=2 block 256", average_ms([&] {
               hipLaunchKernelGGL((k_all<2, 256>), dim3(unsigned(n / 512)), dim3(256), 0, 0, in, out, n);
           }));
    report("all W=4 block 256", average_ms([&] {
               hipLaunchKernelGGL((k_all<4, 256>), dim3(unsigned(n / 1024)), dim3(256), 0, 0, in, out, n);
           }));
    report("copy W=1", average_ms([&] {
               hipLaunchKernelGGL((k_copy<1>), dim3(unsigned(n / 256)), dim3(256), 0, 0, in, out, n);
           }));
    report("copy W=2", average_ms([&] {
               hipLaunchKernelGGL((k_copy<2>), dim3(unsigned(n / 512)), dim3(256), 0, 0, in, out, n);
           }));
    report("copy W=4", average_ms([&] {
               hipLaunchKernelGGL((k_copy<4>), dim3(unsigned(n / 1024)), dim3(256), 0, 0, in, out, n);
           }));
    PROBE_CHECK(hipFree(in));
    PROBE_CHECK(hipFree(out));
    return 0;
}
