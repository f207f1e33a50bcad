// Achievable-rate probes of one MI355X: the denominators against which the
// library's kernels are judged beside the published peaks.  Each probe is a
// plain kernel timed with HIP events on its own stream; the host entry point
// runs it `reps` times after one warm-up launch and returns the best rate.
//
//   hbm_read     every thread streams float4 loads over a buffer far larger than
//                the caches (default 4 GiB) and folds them into one value;
//   hbm_copy     the same buffer copied into a second one (read + write bytes);
//   cache_read   a footprint small enough to stay in the L2 of each XCD (2 MiB)
//                or in the Infinity Cache (64, 192 MiB) read again and again by
//                every workgroup from rotating offsets;
//   lds_read     ds_read_b128 loops over a 64 KiB LDS array;
//   fma_f32      independent chains of FP32 fused multiply-adds (the build has
//                packed FP32 disabled, so one FMA per lane per instruction);
//   fma_f64      the same in FP64.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "dic_roofs.h"

namespace {

__global__ __launch_bounds__(256) void k_read(const float4 *src, int64_t n, float *sink)
{
    float acc = 0.0f;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) {
        const float4 v = src[i];
        acc += (v.x + v.y) + (v.z + v.w);
    }
    if (acc == 1234.5f) sink[blockIdx.x] = acc;   // never true for the zero-filled buffer
}

__global__ __launch_bounds__(256) void k_copy(const float4 *src, float4 *dst, int64_t n)
{
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

// workgroup b reads `chunk` float4 of the n-float4 footprint from offset
// b * chunk (mod n), `reps` times: every part of the footprint is read by many
// workgroups, so after the first touch the reads hit the cache that holds it
__global__ __launch_bounds__(256) void k_reread(const float4 *src, int64_t n, int64_t chunk, int reps, float *sink)
{
    float acc = 0.0f;
    const int64_t off = (static_cast<int64_t>(blockIdx.x) * chunk) % n;
    for (int r = 0; r < reps; ++r)
        for (int64_t i = threadIdx.x; i < chunk; i += blockDim.x) {
            int64_t j = off + i;
            j = j >= n ? j - n : j;
            const float4 v = src[j];
            acc += (v.x + v.y) + (v.z + v.w);
        }
    if (acc == 1234.5f) sink[blockIdx.x] = acc;
}

__global__ __launch_bounds__(256) void k_lds(int iters, float *sink)
{
    __shared__ float4 a[4096];   // 64 KiB
    for (int i = threadIdx.x; i < 4096; i += blockDim.x) a[i] = make_float4(i, 0, 0, 0);
    __syncthreads();
    float4 acc = make_float4(0, 0, 0, 0);
    int idx = threadIdx.x;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const float4 v = a[(idx + k * 256) & 4095];
            acc.x += v.x;
            acc.y += v.y;
            acc.z += v.z;
            acc.w += v.w;
        }
        idx = (idx + 1) & 4095;
    }
    if (acc.x + acc.y + acc.z + acc.w == 1234.5f) sink[blockIdx.x] = acc.x;
}

template <typename T> __global__ __launch_bounds__(256) void k_fma(int iters, T a, T b, T *sink)
{
    T x[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) x[k] = static_cast<T>(threadIdx.x + k);
    for (int it = 0; it < iters; ++it)
#pragma unroll
        for (int k = 0; k < 8; ++k) x[k] = x[k] * a + b;
    T s = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) s += x[k];
    if (s == static_cast<T>(1234.5)) sink[blockIdx.x] = s;
}

} // namespace

namespace {

constexpr int kBlocks = 2048;   // 8 workgroups of 256 threads per compute unit
constexpr int kThreads = 256;

// best time of `reps` launches after one warm-up, in ms; < 0 on a HIP error
template <typename F> double best_ms(F launch, int reps, hipStream_t s)
{
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess) return -1.0;
    if (hipEventCreate(&b) != hipSuccess) {
        (void)hipEventDestroy(a);
        return -1.0;
    }
    double best = -1.0;
    launch();
    for (int r = 0; r < reps; ++r) {
        (void)hipEventRecord(a, s);
        launch();
        (void)hipEventRecord(b, s);
        if (hipEventSynchronize(b) != hipSuccess) {
            best = -1.0;
            break;
        }
        float ms = 0.0f;
        (void)hipEventElapsedTime(&ms, a, b);
        if (best < 0.0 || ms < best) best = ms;
    }
    if (hipGetLastError() != hipSuccess) best = -1.0;
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return best;
}

struct Buffers {
    void *a = nullptr, *b = nullptr;
    float *sink = nullptr;
    hipStream_t s = nullptr;
    bool ok = true;
    Buffers(size_t na, size_t nb)
    {
        ok = hipStreamCreate(&s) == hipSuccess && hipMalloc(&sink, sizeof(float) * kBlocks) == hipSuccess &&
             (na == 0 || (hipMalloc(&a, na) == hipSuccess && hipMemsetAsync(a, 0, na, s) == hipSuccess)) &&
             (nb == 0 || hipMalloc(&b, nb) == hipSuccess) && hipStreamSynchronize(s) == hipSuccess;
    }
    ~Buffers()
    {
        if (a) (void)hipFree(a);
        if (b) (void)hipFree(b);
        if (sink) (void)hipFree(sink);
        if (s) (void)hipStreamDestroy(s);
    }
};

} // namespace

extern "C" {

double dic_roof_hbm_read(int64_t bytes, int reps)
{
    if (bytes < (1 << 20) || reps < 1) return -1.0;
    Buffers B(static_cast<size_t>(bytes), 0);
    if (!B.ok) return -1.0;
    const int64_t n = bytes / 16;
    const double ms = best_ms([&] { k_read<<<kBlocks, kThreads, 0, B.s>>>(static_cast<const float4 *>(B.a), n, B.sink); },
                              reps, B.s);
    return ms > 0.0 ? n * 16.0 / (ms * 1e-3) / 1e9 : -1.0;
}

double dic_roof_hbm_copy(int64_t bytes, int reps)
{
    if (bytes < (1 << 20) || reps < 1) return -1.0;
    Buffers B(static_cast<size_t>(bytes), static_cast<size_t>(bytes));
    if (!B.ok) return -1.0;
    const int64_t n = bytes / 16;
    const double ms = best_ms(
        [&] { k_copy<<<kBlocks, kThreads, 0, B.s>>>(static_cast<const float4 *>(B.a), static_cast<float4 *>(B.b), n); },
        reps, B.s);
    return ms > 0.0 ? 2.0 * n * 16.0 / (ms * 1e-3) / 1e9 : -1.0;
}

double dic_roof_cache_read(int64_t footprint_bytes, int64_t chunk_bytes, int inner, int reps)
{
    if (footprint_bytes < 4096 || chunk_bytes < 4096 || chunk_bytes > footprint_bytes || inner < 1 || reps < 1)
        return -1.0;
    Buffers B(static_cast<size_t>(footprint_bytes), 0);
    if (!B.ok) return -1.0;
    const int64_t n = footprint_bytes / 16, chunk = chunk_bytes / 16;
    const double ms = best_ms(
        [&] { k_reread<<<kBlocks, kThreads, 0, B.s>>>(static_cast<const float4 *>(B.a), n, chunk, inner, B.sink); },
        reps, B.s);
    return ms > 0.0 ? static_cast<double>(kBlocks) * chunk * 16.0 * inner / (ms * 1e-3) / 1e9 : -1.0;
}

double dic_roof_lds_read(int iters, int reps)
{
    if (iters < 1 || reps < 1) return -1.0;
    Buffers B(0, 0);
    if (!B.ok) return -1.0;
    const double ms = best_ms([&] { k_lds<<<kBlocks, kThreads, 0, B.s>>>(iters, B.sink); }, reps, B.s);
    return ms > 0.0 ? static_cast<double>(kBlocks) * kThreads * iters * 16.0 * 16.0 / (ms * 1e-3) / 1e9 : -1.0;
}

double dic_roof_fma(int fp64, int iters, int reps)
{
    if (iters < 1 || reps < 1) return -1.0;
    Buffers B(0, fp64 ? sizeof(double) * kBlocks : 0);
    if (!B.ok) return -1.0;
    double ms;
    if (fp64)
        ms = best_ms([&] { k_fma<double><<<kBlocks, kThreads, 0, B.s>>>(iters, 0.999, 1e-3, static_cast<double *>(B.b)); },
                     reps, B.s);
    else
        ms = best_ms([&] { k_fma<float><<<kBlocks, kThreads, 0, B.s>>>(iters, 0.999f, 1e-3f, B.sink); }, reps, B.s);
    return ms > 0.0 ? static_cast<double>(kBlocks) * kThreads * iters * 8.0 * 2.0 / (ms * 1e-3) / 1e12 : -1.0;
}

} // extern "C"
