// Measurement aid, not part of the transport path: how fast a CU's vector L1
// cache serves the step kernel's corner gather when every access hits in it.
// The step kernel reads, per particle-step, 8 pairs of neighbouring 10-float
// records (2 snapshots x 4 corner rows, 80 contiguous bytes at a 40-byte
// stride each), one pair per lane, different for each lane of a wavefront.
// The probe repeats exactly that access pattern over a 10 KB table that stays
// resident in L1, so only the L1's handling of divergent accesses limits it.
// A second probe loads one 16-byte vector per lane from 64 distinct 128-byte
// lines (the L1's rate of line lookups); a third reads the same record pairs
// from a copy of the table in LDS (what staging records in LDS could serve).
//
//   int l1_probe_rates(double *pairs_per_cu_ns, double *lines_per_cu_ns,
//                      double *lds_pairs_per_cu_ns, int *n_cu)
//     Runs each probe three times on the current device's default stream and
//     returns the best rates per compute unit and nanosecond, and the
//     device's compute-unit count.  Allocates and frees its own buffers.
//     Returns 0, or the HIP error code of the first call that failed.
#include <hip/hip_runtime.h>

namespace {

constexpr int kRecords = 256;               // 10-float records: 10 KB
constexpr int kRecFloats = 10;
constexpr int kLines = 128;                 // 16 KB of 128-B lines for the line probe
constexpr int kBlocks = 2048, kThreads = 256;
constexpr int kPairIters = 1024, kLineIters = 4096;

__global__ __launch_bounds__(256) void k_pair_gather(const float *__restrict__ rec, float *__restrict__ out) {
    const int lane = threadIdx.x & 63;
    float acc = 0.f;
    for (int it = 0; it < kPairIters; ++it) {
        // distinct records for the 64 lanes (5 lane mod 256 is one-to-one),
        // rotating with the iteration; records r and r + 1 are read
        const int r = (lane * 5 + it * 3) & (kRecords - 1);
        const float *p = rec + (size_t)r * kRecFloats;
#pragma unroll
        for (int q = 0; q < 2 * kRecFloats; ++q) acc += p[q];
    }
    out[blockIdx.x * blockDim.x + threadIdx.x] = acc;
}

__global__ __launch_bounds__(256) void k_pair_gather_lds(const float *__restrict__ rec, float *__restrict__ out) {
    constexpr int kTab = (kRecords + 1) * kRecFloats;   // record 255 reads its neighbour 256
    __shared__ float tab[kTab];
    for (int k = threadIdx.x; k < kTab; k += blockDim.x) tab[k] = rec[k];
    __syncthreads();
    const int lane = threadIdx.x & 63;
    float acc = 0.f;
    for (int it = 0; it < kPairIters; ++it) {
        const int r = (lane * 5 + it * 3) & (kRecords - 1);
        const float *p = tab + r * kRecFloats;
#pragma unroll
        for (int q = 0; q < 2 * kRecFloats; ++q) acc += p[q];
    }
    out[blockIdx.x * blockDim.x + threadIdx.x] = acc;
}

__global__ __launch_bounds__(256) void k_divergent_lines(const float4 *__restrict__ a, float *__restrict__ out) {
    const int lane = threadIdx.x & 63;
    float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
    for (int it = 0; it < kLineIters; ++it) {
        const float4 v = a[((lane + it) & (kLines - 1)) * 8];
        acc.x += v.x;
        acc.y += v.y;
        acc.z += v.z;
        acc.w += v.w;
    }
    out[blockIdx.x * blockDim.x + threadIdx.x] = acc.x + acc.y + acc.z + acc.w;
}

}  // namespace

extern "C" int l1_probe_rates(double *pairs_per_cu_ns, double *lines_per_cu_ns, double *lds_pairs_per_cu_ns,
                              int *n_cu) {
    *pairs_per_cu_ns = 0.0;
    *lines_per_cu_ns = 0.0;
    *lds_pairs_per_cu_ns = 0.0;
    *n_cu = 0;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return (int)e;
    hipDeviceProp_t prop;
    if ((e = hipGetDeviceProperties(&prop, dev)) != hipSuccess) return (int)e;
    const double ncu = prop.multiProcessorCount;
    const size_t table_bytes = (size_t)kLines * 128;                     // covers both probes' tables
    static_assert((kRecords + 1) * kRecFloats * 4 <= kLines * 128, "record table fits the buffer");
    void *buf = nullptr;
    float *out = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if ((e = hipMalloc(&buf, table_bytes)) != hipSuccess) goto done;
    if ((e = hipMalloc(&out, (size_t)kBlocks * kThreads * sizeof(float))) != hipSuccess) goto done;
    if ((e = hipMemset(buf, 0, table_bytes)) != hipSuccess) goto done;
    if ((e = hipEventCreate(&e0)) != hipSuccess) goto done;
    if ((e = hipEventCreate(&e1)) != hipSuccess) goto done;
    for (int probe = 0; probe < 3; ++probe) {
        for (int rep = 0; rep < 3; ++rep) {
            if ((e = hipEventRecord(e0, nullptr)) != hipSuccess) goto done;
            if (probe == 0) k_pair_gather<<<kBlocks, kThreads, 0, nullptr>>>((const float *)buf, out);
            else if (probe == 1) k_divergent_lines<<<kBlocks, kThreads, 0, nullptr>>>((const float4 *)buf, out);
            else k_pair_gather_lds<<<kBlocks, kThreads, 0, nullptr>>>((const float *)buf, out);
            if ((e = hipGetLastError()) != hipSuccess) goto done;
            if ((e = hipEventRecord(e1, nullptr)) != hipSuccess) goto done;
            if ((e = hipEventSynchronize(e1)) != hipSuccess) goto done;
            float ms = 0.f;
            if ((e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) goto done;
            const double n = (double)kBlocks * kThreads * (probe == 1 ? kLineIters : kPairIters);
            const double rate = n / ncu / (ms * 1e6);
            double *dst = probe == 0 ? pairs_per_cu_ns : (probe == 1 ? lines_per_cu_ns : lds_pairs_per_cu_ns);
            if (rate > *dst) *dst = rate;
        }
    }
    *n_cu = prop.multiProcessorCount;
done:
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (buf) (void)hipFree(buf);
    if (out) (void)hipFree(out);
    return (int)e;
}
