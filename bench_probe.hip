// Bandwidth probes of the benchmark (not part of libflood): plain streams that
// calibrate the roofline -- the practical HBM ceiling of a read-once /
// write-once kernel on this GPU, the HIP runtime's own device-to-device copy
// as an independent reference, and the scale of the FETCH_SIZE / WRITE_SIZE
// counters for a copy of known size.  Built into bench_probe.so, loaded only
// by bench.py.
#include <hip/hip_runtime.h>

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

enum { P_OK = 0, P_EINVAL = 1, P_ENOMEM = 2, P_EHIP = 3 };

// Achieved bandwidth (bytes read + bytes written per second, GB/s) of
// `reps` repetitions of a stream over `bytes` bytes on `device`, timed with HIP
// events on the probe's own stream after one untimed repetition.
// variant: 0 copy, 1 copy unrolled x4, 2 non-temporal copy, 3 non-temporal
// copy unrolled x4, 4 read-only stream, 5 write-only stream, 6 copy unrolled
// x4 with 4x more workgroups, 7 hipMemcpyAsync device to device (the
// runtime's own copy).  Allocates and frees its two buffers.  Returns 0, or
// 1 bad argument (bytes < 4096, reps < 1, unknown variant), 2 no memory,
// 3 a HIP error.
extern "C" int probe_stream(int device, size_t bytes, int reps, int variant, double* gbps) {
    if (!gbps || reps < 1 || bytes < 4096 || variant < 0 || variant > 7) return P_EINVAL;
    if (hipSetDevice(device) != hipSuccess) return P_EHIP;
    const long long n = (long long)(bytes / sizeof(v4f));
    void *a = nullptr, *b = nullptr;
    if (hipMalloc(&a, n * sizeof(v4f)) != hipSuccess) return P_ENOMEM;
    if (hipMalloc(&b, n * sizeof(v4f)) != hipSuccess) {
        (void)hipFree(a);
        return P_ENOMEM;
    }
    hipStream_t s;
    hipEvent_t e0, e1;
    int st = P_OK;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) st = P_EHIP;
    if (!st && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)) st = P_EHIP;
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
            case 7: (void)hipMemcpyAsync(dst, src, n * sizeof(v4f), hipMemcpyDeviceToDevice, s); break;
            default: hipLaunchKernelGGL((k_copy<4, false>), dim3(blocks), dim3(256), 0, s, src, dst, n); break;
            }
        };
        launch();
        (void)hipEventRecord(e0, s);
        for (int r = 0; r < reps; ++r) launch();
        (void)hipEventRecord(e1, s);
        if (hipEventSynchronize(e1) != hipSuccess) st = P_EHIP;
        float ms = 0.f;
        if (!st && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) st = P_EHIP;
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
