// psl_bench_atomics: measured roofs for the dose tally -- 64-bit atomic adds
// scattered over many addresses (the tally's access pattern) and atomic adds
// that all hit one address (the pattern this library avoids).
#include "common.hpp"

namespace psl {
namespace {

__global__ void __launch_bounds__(256)
k_atomic_scatter(unsigned long long *a, int64_t n, int iters) {
    const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int i = 0; i < iters; ++i) {
        uint64_t h = t * 0x9E3779B97F4A7C15ull + (uint64_t)i * 0xBF58476D1CE4E5B9ull;
        h ^= h >> 31;
        atomicAdd(&a[h % (uint64_t)n], 1ull);
    }
}

__global__ void __launch_bounds__(256)
k_atomic_same(uint32_t *c, int iters) {
    if (__lane_id() == 0)
        for (int i = 0; i < iters; ++i) atomicAdd(c, 1u);
}

}  // namespace
}  // namespace psl

using namespace psl;

extern "C" size_t psl_bench_atomics_workspace_bytes(int64_t n_addresses) {
    return n_addresses > 0 ? (size_t)n_addresses * 8 + 256 : 0;
}

extern "C" psl_status psl_bench_atomics(int64_t n_addresses, double *rates,
                                        void *d_ws, size_t ws_bytes,
                                        void *stream) {
    PSL_REQUIRE(rates && d_ws, "NULL argument");
    PSL_REQUIRE(n_addresses >= 1024, "n_addresses < 1024");
    if (ws_bytes < psl_bench_atomics_workspace_bytes(n_addresses)) {
        set_error("workspace too small");
        return PSL_ENOSPC;
    }
    if (psl_status s = check_device()) return s;
    hipStream_t st = (hipStream_t)stream;
    auto *a = static_cast<unsigned long long *>(d_ws);
    auto *c = reinterpret_cast<uint32_t *>(static_cast<char *>(d_ws) +
                                           n_addresses * 8);
    hipEvent_t e0, e1;
    PSL_HIP(hipEventCreate(&e0));
    PSL_HIP(hipEventCreate(&e1));
    const int blocks = device_cu_count() * 32;
    const int iters = 16;
    float ms = 0.0f;
    // scattered u64 atomics
    hipLaunchKernelGGL(k_atomic_scatter, dim3(blocks), dim3(256), 0, st, a,
                       n_addresses, 2);
    PSL_HIP(hipEventRecord(e0, st));
    hipLaunchKernelGGL(k_atomic_scatter, dim3(blocks), dim3(256), 0, st, a,
                       n_addresses, iters);
    PSL_HIP(hipEventRecord(e1, st));
    PSL_HIP(hipEventSynchronize(e1));
    PSL_HIP(hipEventElapsedTime(&ms, e0, e1));
    rates[0] = (double)blocks * 256 * iters / (ms * 1e-3);
    // one address, one atomic per wave per iteration
    const int blocks1 = device_cu_count() * 2;
    PSL_HIP(hipEventRecord(e0, st));
    hipLaunchKernelGGL(k_atomic_same, dim3(blocks1), dim3(256), 0, st, c,
                       64);
    PSL_HIP(hipEventRecord(e1, st));
    PSL_HIP(hipEventSynchronize(e1));
    PSL_HIP(hipEventElapsedTime(&ms, e0, e1));
    rates[1] = (double)blocks1 * 4 * 64 / (ms * 1e-3);
    PSL_HIP(hipEventDestroy(e0));
    PSL_HIP(hipEventDestroy(e1));
    PSL_LAUNCHED();
    return PSL_OK;
}
