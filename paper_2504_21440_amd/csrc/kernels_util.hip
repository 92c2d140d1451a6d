// kernels_util.hip -- measurement utility: the device's achievable HBM bandwidth, from a streaming
// copy kernel timed with HIP events (the reference point beside the published peak for the
// bandwidth-bound SpMV kernels).
#include <hip/hip_runtime.h>

#include <string>

#include "qt_host.h"

namespace qt {

typedef float cpy4 __attribute__((ext_vector_type(4)));

// b = a over n16 16-byte items, grid-stride, non-temporal on both sides (the data is touched once).
__global__ __launch_bounds__(256) void k_stream_copy(const cpy4 *__restrict__ a, cpy4 *__restrict__ b, int64_t n16)
{
    const int64_t st = (int64_t)gridDim.x * 256;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n16; i += st)
        __builtin_nontemporal_store(__builtin_nontemporal_load(a + i), b + i);
}

}  // namespace qt

using namespace qt;

extern "C" qt_status qt_measure_copy_bandwidth(qt_ctx *ctx, int64_t bytes, int32_t reps, double *gbs)
{
    if (!ctx || !gbs || bytes < 16 || reps < 1) return set_error(QT_EINVAL, "qt_measure_copy_bandwidth: bad arguments");
    QT_HIP(hipSetDevice(ctx->device));
    const int64_t n16 = bytes / 16;
    void *a = nullptr, *b = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipMalloc(&a, (size_t)n16 * 16);
    if (!e) e = hipMalloc(&b, (size_t)n16 * 16);
    if (!e) e = hipMemsetAsync(a, 0, (size_t)n16 * 16, ctx->stream);
    if (!e) e = hipEventCreate(&e0);
    if (!e) e = hipEventCreate(&e1);
    int cus = 256;
    if (!e) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device);
    const unsigned grid = (unsigned)(16 * cus);  // 16 workgroups per compute unit, grid-stride
    float ms = 0.f;
    if (!e) {
        hipLaunchKernelGGL(k_stream_copy, dim3(grid), dim3(256), 0, ctx->stream, (const cpy4 *)a, (cpy4 *)b, n16);
        e = hipEventRecord(e0, ctx->stream);
    }
    for (int r = 0; r < reps && !e; ++r) {
        hipLaunchKernelGGL(k_stream_copy, dim3(grid), dim3(256), 0, ctx->stream, (const cpy4 *)a, (cpy4 *)b, n16);
        e = hipGetLastError();
    }
    if (!e) e = hipEventRecord(e1, ctx->stream);
    if (!e) e = hipEventSynchronize(e1);
    if (!e) e = hipEventElapsedTime(&ms, e0, e1);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (a) (void)hipFree(a);
    if (b) (void)hipFree(b);
    if (e) return set_error(QT_EDEVICE, std::string("qt_measure_copy_bandwidth: ") + hipGetErrorString(e));
    *gbs = 2.0 * (double)n16 * 16.0 * reps / (ms * 1e-3) / 1e9;
    return QT_OK;
}
