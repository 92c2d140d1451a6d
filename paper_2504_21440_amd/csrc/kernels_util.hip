// kernels_util.hip -- measurement utility: the device's achievable HBM bandwidth, from a streaming
// copy kernel and a streaming read kernel timed with HIP events (the reference points beside the
// published peak for the bandwidth-bound SpMV kernels, whose traffic is nearly all reads).
#include <hip/hip_runtime.h>

#include <string>

#include "qt_host.h"

namespace qt {

typedef float cpy4 __attribute__((ext_vector_type(4)));

// b = a over n16 16-byte items, grid-stride with four items in flight per lane, non-temporal on both
// sides (the data is touched once).
__global__ __launch_bounds__(256) void k_stream_copy(const cpy4 *__restrict__ a, cpy4 *__restrict__ b, int64_t n16)
{
    const int64_t st = (int64_t)gridDim.x * 256;
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    for (; i + 3 * st < n16; i += 4 * st) {
        cpy4 v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = __builtin_nontemporal_load(a + i + u * st);
#pragma unroll
        for (int u = 0; u < 4; ++u) __builtin_nontemporal_store(v[u], b + i + u * st);
    }
    for (; i < n16; i += st) __builtin_nontemporal_store(__builtin_nontemporal_load(a + i), b + i);
}

// Sum of a over n16 16-byte items, the same access pattern without the stores.  The sums are
// written only in the impossible case that one equals `never`, which keeps the loads alive at no
// cost in traffic.
__global__ __launch_bounds__(256) void k_stream_read(const cpy4 *__restrict__ a, int64_t n16, float never,
                                                     float *__restrict__ out)
{
    const int64_t st = (int64_t)gridDim.x * 256;
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    cpy4 acc = {0.f, 0.f, 0.f, 0.f};
    for (; i + 3 * st < n16; i += 4 * st) {
        cpy4 v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = __builtin_nontemporal_load(a + i + u * st);
#pragma unroll
        for (int u = 0; u < 4; ++u) acc += v[u];
    }
    for (; i < n16; i += st) acc += __builtin_nontemporal_load(a + i);
    const float t = acc.x + acc.y + acc.z + acc.w;
    if (t == never) out[blockIdx.x] = t;
}

// Launches per compute unit of the two kernels (the fastest of 4 to 64 on MI355X over 2 GiB).
constexpr int COPY_WG_PER_CU = 64, READ_WG_PER_CU = 32;

// Times `reps` launches of the copy (read = false) or read kernel over n16 items on the context's
// stream; returns the bytes moved per second in GB/s through *gbs.
static qt_status stream_measure(qt_ctx *ctx, int64_t bytes, int32_t reps, bool read, double *gbs, const char *who)
{
    QT_HIP(hipSetDevice(ctx->device));
    const int64_t n16 = bytes / 16;
    void *a = nullptr, *b = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int cus = 256;
    hipError_t e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device);
    const unsigned grid = (unsigned)((read ? READ_WG_PER_CU : COPY_WG_PER_CU) * cus);
    if (!e) e = hipMalloc(&a, (size_t)n16 * 16);
    if (!e) e = hipMalloc(&b, read ? (size_t)grid * 4 : (size_t)n16 * 16);
    if (!e) e = hipMemsetAsync(a, 0, (size_t)n16 * 16, ctx->stream);
    if (!e) e = hipEventCreate(&e0);
    if (!e) e = hipEventCreate(&e1);
    float ms = 0.f;
    auto launch = [&] {
        if (read)
            hipLaunchKernelGGL(k_stream_read, dim3(grid), dim3(256), 0, ctx->stream, (const cpy4 *)a, n16, -1.0f,
                               (float *)b);
        else
            hipLaunchKernelGGL(k_stream_copy, dim3(grid), dim3(256), 0, ctx->stream, (const cpy4 *)a, (cpy4 *)b, n16);
    };
    if (!e) {
        launch();
        e = hipEventRecord(e0, ctx->stream);
    }
    for (int r = 0; r < reps && !e; ++r) {
        launch();
        e = hipGetLastError();
    }
    if (!e) e = hipEventRecord(e1, ctx->stream);
    if (!e) e = hipEventSynchronize(e1);
    if (!e) e = hipEventElapsedTime(&ms, e0, e1);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (a) (void)hipFree(a);
    if (b) (void)hipFree(b);
    if (e) return set_error(QT_EDEVICE, std::string(who) + ": " + hipGetErrorString(e));
    *gbs = (read ? 1.0 : 2.0) * (double)n16 * 16.0 * reps / (ms * 1e-3) / 1e9;
    return QT_OK;
}

}  // namespace qt

using namespace qt;

extern "C" qt_status qt_measure_copy_bandwidth(qt_ctx *ctx, int64_t bytes, int32_t reps, double *gbs)
{
    if (!ctx || !gbs || bytes < 16 || reps < 1) return set_error(QT_EINVAL, "qt_measure_copy_bandwidth: bad arguments");
    return stream_measure(ctx, bytes, reps, false, gbs, "qt_measure_copy_bandwidth");
}

extern "C" qt_status qt_measure_read_bandwidth(qt_ctx *ctx, int64_t bytes, int32_t reps, double *gbs)
{
    if (!ctx || !gbs || bytes < 16 || reps < 1) return set_error(QT_EINVAL, "qt_measure_read_bandwidth: bad arguments");
    return stream_measure(ctx, bytes, reps, true, gbs, "qt_measure_read_bandwidth");
}
