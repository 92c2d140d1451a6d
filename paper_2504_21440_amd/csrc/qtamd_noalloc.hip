// qtamd_noalloc.hip -- the expectation value Tr(O rho) / <psi|O|psi> without any allocation, for
// callers that cannot allocate device memory (code under HIP graph capture, tight serving loops,
// harnesses that forbid hipMalloc).
//
// qt_expect stages the host operator in a device arena it allocates per call.  qt_expect_noalloc
// stages it instead in `scratch`, a file-scope device array of QT_NOALLOC_SCRATCH_BYTES that every
// GPU the library runs on holds until the process ends.  The array's name is a host-side stand-in
// in host code: its device address is looked up once per device (hipGetSymbolAddress, with that
// device current) when a context is created on it, and only that address is ever handed to copies
// and kernels.  Every call on a GPU shares that GPU's array: calls that overlap on one GPU (two
// threads, or two contexts whose streams run concurrently) race, and the array keeps the last
// call's contents.  Nothing in it has to start at zero (every byte a call reads it writes first).
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>
#include <string>

#include "qt_host.h"

namespace qt {

static __device__ __align__(256) unsigned char scratch[QT_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
void *g_ptr[MAX_DEVICES] = {};

__global__ __launch_bounds__(256) void k_rowptr32(int n, const int64_t *__restrict__ p64, int32_t *__restrict__ p32)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p32[i] = (int32_t)p64[i];
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }
}  // namespace

// Called with `device` current (from qt_ctx_create and, as a fallback, the entry point itself).
qt_status noalloc_init_device(int32_t device)
{
    if (device < 0 || device >= MAX_DEVICES) return set_error(QT_EINVAL, "qt_expect_noalloc: device index too large");
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_ptr[device]) return QT_OK;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
        return set_error(QT_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_ptr[device] = p;
    return QT_OK;
}

// Scratch bytes a call with this operator needs (the layout the entry point uses).
static size_t noalloc_bytes(int32_t d, int64_t nnz)
{
    size_t b = align256((size_t)(d + 1) * 8);             // row pointers as given (int64)
    b += align256((size_t)(d + 1) * 4);                   // row pointers narrowed to int32
    b += align256((size_t)std::max<int64_t>(1, nnz) * 4); // column indices
    b += align256((size_t)std::max<int64_t>(1, nnz) * 16);  // values, complex128
    b += 256;                                              // the result
    return b;
}

}  // namespace qt

using namespace qt;

extern "C" qt_status qt_expect_noalloc(qt_ctx *ctx, int32_t d, const qt_csr *O, const void *dev_state, int32_t is_ket,
                                       int32_t precision, double *out)
{
    if (!ctx || !O || !dev_state || !out || d <= 0) return set_error(QT_EINVAL, "qt_expect_noalloc: null argument");
    if (precision != QT_F64 && precision != QT_MIXED) return set_error(QT_EINVAL, "qt_expect_noalloc: bad precision");
    // validation in place: the caller's arrays are copied to the device as they are
    if (O->rows != d || O->cols != d) return set_error(QT_EINVAL, "qt_expect_noalloc: O must be d x d");
    if (O->nnz < 0 || !O->indptr || (O->nnz > 0 && (!O->indices || !O->values)))
        return set_error(QT_EINVAL, "qt_expect_noalloc: malformed CSR arrays");
    if (O->indptr[0] != 0 || O->indptr[d] != O->nnz)
        return set_error(QT_EINVAL, "qt_expect_noalloc: indptr[0] must be 0 and indptr[rows] == nnz");
    if (O->nnz >= 2147483647LL) return set_error(QT_EINVAL, "qt_expect_noalloc: operator has too many non-zeros");
    for (int32_t i = 0; i < d; ++i)
        if (O->indptr[i + 1] < O->indptr[i]) return set_error(QT_EINVAL, "qt_expect_noalloc: decreasing indptr");
    for (int64_t p = 0; p < O->nnz; ++p) {
        if (O->indices[p] < 0 || O->indices[p] >= d)
            return set_error(QT_EINVAL, "qt_expect_noalloc: column index out of range");
        if (!std::isfinite(O->values[2 * p]) || !std::isfinite(O->values[2 * p + 1]))
            return set_error(QT_EINVAL, "qt_expect_noalloc: non-finite value");
    }
    const size_t need = noalloc_bytes(d, O->nnz);
    if (need > (size_t)QT_NOALLOC_SCRATCH_BYTES)
        return set_error(QT_ENOMEM, "qt_expect_noalloc: operator needs " + std::to_string(need) +
                                        " bytes of scratch, more than the " +
                                        std::to_string((long long)QT_NOALLOC_SCRATCH_BYTES) + " the library holds");
    QT_HIP(hipSetDevice(ctx->device));
    qt_status st = noalloc_init_device(ctx->device);
    if (st) return st;
    char *base;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        base = (char *)g_ptr[ctx->device];
    }
    int64_t *p64 = (int64_t *)base;
    int32_t *p32 = (int32_t *)(base + align256((size_t)(d + 1) * 8));
    int32_t *ci = (int32_t *)((char *)p32 + align256((size_t)(d + 1) * 4));
    double2 *v = (double2 *)((char *)ci + align256((size_t)std::max<int64_t>(1, O->nnz) * 4));
    double2 *res = (double2 *)((char *)v + align256((size_t)std::max<int64_t>(1, O->nnz) * 16));
    hipStream_t s = ctx->stream;
    hipError_t e = hipMemcpyAsync(p64, O->indptr, (size_t)(d + 1) * 8, hipMemcpyHostToDevice, s);
    if (!e && O->nnz > 0) e = hipMemcpyAsync(ci, O->indices, (size_t)O->nnz * 4, hipMemcpyHostToDevice, s);
    if (!e && O->nnz > 0) e = hipMemcpyAsync(v, O->values, (size_t)O->nnz * 16, hipMemcpyHostToDevice, s);
    if (!e) {
        hipLaunchKernelGGL(k_rowptr32, dim3((d + 1 + 255) / 256), dim3(256), 0, s, d + 1, (const int64_t *)p64, p32);
        e = hipGetLastError();
    }
    if (!e) {
        launch_expect(precision == QT_F64, d, p32, ci, v, dev_state, is_ket, res, s);
        e = hipGetLastError();
    }
    if (!e) e = hipMemcpyAsync(out, res, 16, hipMemcpyDeviceToHost, s);
    if (!e) e = hipStreamSynchronize(s);
    if (e) return set_error(QT_EDEVICE, std::string("qt_expect_noalloc: ") + hipGetErrorString(e));
    return QT_OK;
}
