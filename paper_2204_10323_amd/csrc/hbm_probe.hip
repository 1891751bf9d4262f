// Plain streaming copy used to calibrate the roofline: the practical HBM
// ceiling of a read-once/write-once kernel on this GPU, and the scale of the
// FETCH_SIZE / WRITE_SIZE counters for a copy of known size.
#include <hip/hip_runtime.h>

#include <string>

#include "../../include/flood.h"

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));

// Grid-stride copy of 16-byte vectors, UNR vectors per thread per iteration.
template <int UNR, bool NT>
__global__ __launch_bounds__(256) void k_copy(const v4f* __restrict__ src, v4f* __restrict__ dst,
                                              long long n) {
    const long long stride = (long long)gridDim.x * blockDim.x;
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + (UNR - 1) * stride < n; i += UNR * stride) {
        v4f v[UNR];
#pragma unroll
        for (int u = 0; u < UNR; ++u)
            v[u] = NT ? __builtin_nontemporal_load(src + i + u * stride) : src[i + u * stride];
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
            if (NT) __builtin_nontemporal_store(v[u], dst + i + u * stride);
            else dst[i + u * stride] = v[u];
        }
    }
    for (; i < n; i += stride) dst[i] = src[i];
}

// Read-only stream: every element is loaded once; one value per thread is
// stored so the loads stay live.
__global__ __launch_bounds__(256) void k_read(const v4f* __restrict__ src, v4f* __restrict__ dst,
                                              long long n) {
    const long long stride = (long long)gridDim.x * blockDim.x;
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    v4f acc = {0.f, 0.f, 0.f, 0.f};
    for (; i + 3 * stride < n; i += 4 * stride) {
        v4f v0 = src[i], v1 = src[i + stride], v2 = src[i + 2 * stride], v3 = src[i + 3 * stride];
        acc += (v0 + v1) + (v2 + v3);
    }
    for (; i < n; i += stride) acc += src[i];
    dst[(long long)blockIdx.x * blockDim.x + threadIdx.x] = acc;
}

// Write-only stream.
__global__ __launch_bounds__(256) void k_write(v4f* __restrict__ dst, long long n) {
    const long long stride = (long long)gridDim.x * blockDim.x;
    const v4f v = {1.f, 2.f, 3.f, 4.f};
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = v;
}

}  // namespace

extern "C" fl_status fl_copy_probe(int device, size_t bytes, int reps, int variant, double* gbps) {
    if (!gbps || reps < 1 || bytes < 4096 || variant < 0 || variant > 6) return FL_EINVAL;
    if (hipSetDevice(device) != hipSuccess) return FL_EHIP;
    const long long n = (long long)(bytes / sizeof(v4f));
    void *a = nullptr, *b = nullptr;
    if (hipMalloc(&a, n * sizeof(v4f)) != hipSuccess) return FL_ENOMEM;
    if (hipMalloc(&b, n * sizeof(v4f)) != hipSuccess) {
        (void)hipFree(a);
        return FL_ENOMEM;
    }
    hipStream_t s;
    hipEvent_t e0, e1;
    fl_status st = FL_OK;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) st = FL_EHIP;
    if (!st && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)) st = FL_EHIP;
    if (!st) {
        (void)hipMemsetAsync(a, 0, n * sizeof(v4f), s);
        int dev_cu = 256;
        (void)hipDeviceGetAttribute(&dev_cu, hipDeviceAttributeMultiprocessorCount, device);
        const int blocks = dev_cu * (variant == 6 ? 32 : 8);
        auto launch = [&]() {
            const v4f* src = (const v4f*)a;
            v4f* dst = (v4f*)b;
            switch (variant) {
            case 0: hipLaunchKernelGGL((k_copy<1, false>), dim3(blocks), dim3(256), 0, s, src, dst, n); break;
            case 1: hipLaunchKernelGGL((k_copy<4, false>), dim3(blocks), dim3(256), 0, s, src, dst, n); break;
            case 2: hipLaunchKernelGGL((k_copy<1, true>), dim3(blocks), dim3(256), 0, s, src, dst, n); break;
            case 3: hipLaunchKernelGGL((k_copy<4, true>), dim3(blocks), dim3(256), 0, s, src, dst, n); break;
            case 4: hipLaunchKernelGGL(k_read, dim3(blocks), dim3(256), 0, s, src, dst, n); break;
            case 5: hipLaunchKernelGGL(k_write, dim3(blocks), dim3(256), 0, s, dst, n); break;
            default: hipLaunchKernelGGL((k_copy<4, false>), dim3(blocks), dim3(256), 0, s, src, dst, n); break;
            }
        };
        launch();
        (void)hipEventRecord(e0, s);
        for (int r = 0; r < reps; ++r) launch();
        (void)hipEventRecord(e1, s);
        if (hipEventSynchronize(e1) != hipSuccess) st = FL_EHIP;
        float ms = 0.f;
        if (!st && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) st = FL_EHIP;
        const double moved = (variant == 4 || variant == 5) ? 1.0 : 2.0;
        if (!st) *gbps = moved * (double)n * sizeof(v4f) * reps / (ms * 1e-3) / 1e9;
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        (void)hipStreamDestroy(s);
    }
    (void)hipFree(a);
    (void)hipFree(b);
    return st;
}
