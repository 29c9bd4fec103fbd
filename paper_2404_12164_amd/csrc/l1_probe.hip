// Measurement aid, not part of the transport path: the rate at which a CU's
// vector L1 cache processes cache-line lookups when every lane of a
// wavefront load touches a different 128-B line, the access pattern of the
// step kernel's corner gather.  The loads stay within a 16 KB array, so they
// hit in L1 and only the lookup rate limits them.
//
//   int l1_probe_lines_per_ns(double *lines_per_cu_ns, int *n_cu)
//     Runs the probe three times on the current device's default stream and
//     returns, in *lines_per_cu_ns, the best rate in lines per CU per
//     nanosecond and, in *n_cu, the device's compute-unit count.  Allocates
//     and frees its own 16 KB and output buffers.  Returns 0, or the HIP
//     error code of the first call that failed.
#include <hip/hip_runtime.h>

namespace {

constexpr int kLines = 128;                 // 16 KB of 128-B lines
constexpr int kBlocks = 2048, kThreads = 256, kIters = 4096;

__global__ __launch_bounds__(256) void k_divergent_lines(const float4 *__restrict__ a, float *__restrict__ out) {
    const int lane = threadIdx.x & 63;
    float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
    for (int it = 0; it < kIters; ++it) {
        // each lane a different line, rotating so the pattern is not static
        const float4 v = a[((lane + it) & (kLines - 1)) * 8];
        acc.x += v.x;
        acc.y += v.y;
        acc.z += v.z;
        acc.w += v.w;
    }
    out[blockIdx.x * blockDim.x + threadIdx.x] = acc.x + acc.y + acc.z + acc.w;
}

}  // namespace

extern "C" int l1_probe_lines_per_ns(double *lines_per_cu_ns, int *n_cu) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return (int)e;
    hipDeviceProp_t prop;
    if ((e = hipGetDeviceProperties(&prop, dev)) != hipSuccess) return (int)e;
    float4 *a = nullptr;
    float *out = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    double best = 0.0;
    if ((e = hipMalloc(&a, kLines * 8 * sizeof(float4))) != hipSuccess) goto done;
    if ((e = hipMalloc(&out, (size_t)kBlocks * kThreads * sizeof(float))) != hipSuccess) goto done;
    if ((e = hipMemset(a, 0, kLines * 8 * sizeof(float4))) != hipSuccess) goto done;
    if ((e = hipEventCreate(&e0)) != hipSuccess) goto done;
    if ((e = hipEventCreate(&e1)) != hipSuccess) goto done;
    for (int rep = 0; rep < 3; ++rep) {
        if ((e = hipEventRecord(e0, nullptr)) != hipSuccess) goto done;
        k_divergent_lines<<<kBlocks, kThreads, 0, nullptr>>>(a, out);
        if ((e = hipEventRecord(e1, nullptr)) != hipSuccess) goto done;
        if ((e = hipEventSynchronize(e1)) != hipSuccess) goto done;
        if ((e = hipGetLastError()) != hipSuccess) goto done;
        float ms = 0.f;
        if ((e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) goto done;
        const double lines = (double)kBlocks * kThreads * kIters;   // one line per lane-load
        const double rate = lines / prop.multiProcessorCount / (ms * 1e6);
        if (rate > best) best = rate;
    }
done:
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (a) (void)hipFree(a);
    if (out) (void)hipFree(out);
    *lines_per_cu_ns = best;
    *n_cu = prop.multiProcessorCount;
    return (int)e;
}
