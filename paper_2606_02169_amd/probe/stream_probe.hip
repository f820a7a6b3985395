// Stream ceilings of the GPU, measured with plain kernels: the rates that bound the gather kernels of the
// library (its matvecs move their bytes between the L2 and the memory fabric).  A standalone program, not
// part of libmrmf.so; bench.py (--workload stream) runs it and reports its lines.
//
//  read     : every element of a footprint of F bytes read once per pass, passes repeated to about 8 GB,
//             with the default cache policy and with non-temporal loads.  Footprints from 2 MB (inside the
//             L2 of one XCD) through 64-256 MB (inside the 256 MB Infinity Cache) to 1-4 GB (HBM).
//  copy     : y = x over 64 MB .. 2 GB (read + write bytes counted).
//  gather8  : y_i = x_i + sum of 8 rows x_{i +- R / 2^k} (k = 0..3), 1 GB footprint, for window spans R
//             from 16 KB to 512 MB: the access pattern of a matvec's channels, one row per thread.
//
// Output: one JSON object per line on stdout.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <vector>

#define CHECK(call)                                                                                 \
    do {                                                                                            \
        const hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess) {                                                                     \
            std::fprintf(stderr, "stream_probe: %s at line %d\n", hipGetErrorString(e_), __LINE__); \
            std::exit(1);                                                                           \
        }                                                                                           \
    } while (0)

namespace {

constexpr int kThreads = 256;

// the sums are kept alive by a store that never happens for the zero-filled inputs used here
template <bool NT>
__global__ __launch_bounds__(kThreads) void k_read(const double2* __restrict__ x, size_t n, int passes,
                                                   double* __restrict__ sink) {
    double acc = 0.0;
    const size_t stride = size_t(gridDim.x) * kThreads;
    for (int r = 0; r < passes; ++r)
        for (size_t i = size_t(blockIdx.x) * kThreads + threadIdx.x; i < n; i += stride) {
            if constexpr (NT) {
                const double* p = reinterpret_cast<const double*>(x + i);
                acc += __builtin_nontemporal_load(p) + __builtin_nontemporal_load(p + 1);
            } else {
                const double2 v = x[i];
                acc += v.x + v.y;
            }
        }
    if (acc == 1.0e300) sink[0] = acc;
}

__global__ __launch_bounds__(kThreads) void k_copy(const double2* __restrict__ x, double2* __restrict__ y,
                                                   size_t n) {
    const size_t stride = size_t(gridDim.x) * kThreads;
    for (size_t i = size_t(blockIdx.x) * kThreads + threadIdx.x; i < n; i += stride) y[i] = x[i];
}

// n is a power of two, so (i + off) & (n - 1) stays inside the footprint for any offset
__global__ __launch_bounds__(kThreads) void k_gather8(const double2* __restrict__ x, double2* __restrict__ y,
                                                      size_t n, const long long* __restrict__ off) {
    const size_t stride = size_t(gridDim.x) * kThreads, mask = n - 1;
    for (size_t i = size_t(blockIdx.x) * kThreads + threadIdx.x; i < n; i += stride) {
        double2 a = x[i];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const double2 v = x[(i + size_t(off[k])) & mask];
            a.x += v.x;
            a.y += v.y;
        }
        y[i] = a;
    }
}

float time_ms(hipEvent_t a, hipEvent_t b) {
    CHECK(hipEventSynchronize(b));
    float ms = 0.f;
    CHECK(hipEventElapsedTime(&ms, a, b));
    return ms;
}

}  // namespace

int main() {
    const size_t max_bytes = size_t(4) << 30;
    double2 *x = nullptr, *y = nullptr;
    double* sink = nullptr;
    long long* d_off = nullptr;
    CHECK(hipMalloc(&x, max_bytes));
    CHECK(hipMalloc(&y, max_bytes));
    CHECK(hipMalloc(&sink, 64));
    CHECK(hipMalloc(&d_off, 8 * sizeof(long long)));
    CHECK(hipMemset(x, 0, max_bytes));
    CHECK(hipMemset(y, 0, max_bytes));
    hipEvent_t a, b;
    CHECK(hipEventCreate(&a));
    CHECK(hipEventCreate(&b));
    int cus = 0;
    CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, 0));
    const int grid = cus * 8;
    std::printf("{\"kind\": \"device\", \"compute_units\": %d, \"grid\": %d, \"threads\": %d}\n", cus, grid, kThreads);
    std::fflush(stdout);

    const size_t foot[] = {size_t(2) << 20,   size_t(16) << 20,  size_t(64) << 20, size_t(128) << 20,
                           size_t(256) << 20, size_t(384) << 20, size_t(1) << 30,  size_t(4) << 30};
    for (int nt = 0; nt < 2; ++nt)
        for (const size_t f : foot) {
            const size_t n = f / sizeof(double2);
            const int passes = static_cast<int>(std::max<size_t>(1, (size_t(8) << 30) / f));
            auto kern = nt ? k_read<true> : k_read<false>;
            hipLaunchKernelGGL(kern, dim3(grid), dim3(kThreads), 0, 0, x, n, 1, sink);  // warm-up pass
            CHECK(hipEventRecord(a));
            hipLaunchKernelGGL(kern, dim3(grid), dim3(kThreads), 0, 0, x, n, passes, sink);
            CHECK(hipEventRecord(b));
            const float ms = time_ms(a, b);
            std::printf("{\"kind\": \"read\", \"policy\": \"%s\", \"footprint_MB\": %.0f, \"passes\": %d, "
                        "\"GBps\": %.1f}\n",
                        nt ? "nontemporal" : "default", f / 1048576.0, passes, double(f) * passes / ms / 1e6);
            std::fflush(stdout);
        }
    for (const size_t f : {size_t(64) << 20, size_t(256) << 20, size_t(1) << 30, size_t(2) << 30}) {
        const size_t n = f / sizeof(double2);
        hipLaunchKernelGGL(k_copy, dim3(grid), dim3(kThreads), 0, 0, x, y, n);
        CHECK(hipEventRecord(a));
        for (int r = 0; r < 10; ++r) hipLaunchKernelGGL(k_copy, dim3(grid), dim3(kThreads), 0, 0, x, y, n);
        CHECK(hipEventRecord(b));
        const float ms = time_ms(a, b);
        std::printf("{\"kind\": \"copy\", \"footprint_MB\": %.0f, \"GBps_read_plus_write\": %.1f}\n", f / 1048576.0,
                    2.0 * double(f) * 10 / ms / 1e6);
        std::fflush(stdout);
    }
    const size_t n = size_t(1) << 26;  // 1 GB of c128 rows
    for (const long long R : {1LL << 10, 1LL << 14, 1LL << 18, 1LL << 20, 1LL << 22, 1LL << 24, 1LL << 25}) {
        std::vector<long long> off(8);
        for (int k = 0; k < 8; ++k) off[k] = (k % 2 ? 1 : -1) * (R >> (k / 2));
        CHECK(hipMemcpy(d_off, off.data(), 8 * sizeof(long long), hipMemcpyHostToDevice));
        hipLaunchKernelGGL(k_gather8, dim3(grid), dim3(kThreads), 0, 0, x, y, n, d_off);
        CHECK(hipEventRecord(a));
        for (int r = 0; r < 5; ++r) hipLaunchKernelGGL(k_gather8, dim3(grid), dim3(kThreads), 0, 0, x, y, n, d_off);
        CHECK(hipEventRecord(b));
        const double ms = time_ms(a, b) / 5;
        std::printf("{\"kind\": \"gather8\", \"span_rows\": %lld, \"span_MB\": %.2f, \"ms\": %.3f, "
                    "\"algorithmic_GBps\": %.1f, \"row_requests_GBps\": %.1f}\n",
                    R, R * 16.0 / 1048576, ms, 2.0 * n * 16 / ms / 1e6, 10.0 * n * 16 / ms / 1e6);
        std::fflush(stdout);
    }
    CHECK(hipFree(d_off));
    CHECK(hipFree(sink));
    CHECK(hipFree(y));
    CHECK(hipFree(x));
    return 0;
}
