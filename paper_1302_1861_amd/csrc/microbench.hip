// psl_bench_atomics: measured roofs for the dose tally -- 64-bit atomic adds
// scattered over many addresses and atomic adds that all hit one address
// (the pattern this library avoids); psl_bench_atomics_replay: the tally's
// own recorded deposit addresses replayed at several occupancies.
#include "common.hpp"

namespace psl {
namespace {

// Uniformly scattered addresses: a 32-bit multiplicative hash of (thread,
// iteration) masked to the largest power of two <= the address count.
__global__ void __launch_bounds__(256)
k_atomic_scatter(unsigned long long *a, uint32_t mask, int iters) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    for (int i = 0; i < iters; ++i) {
        uint32_t h = t * 0x9E3779B9u ^ (uint32_t)i * 0x85EBCA6Bu;
        h ^= h >> 15;
        atomicAdd(&a[h & mask], 1ull);
    }
}

// Replay of a recorded deposit-address trace: entry j goes to thread
// j mod (grid size), so the lanes of a wave issue consecutive entries
// together, as the waves that recorded them did.
__global__ void __launch_bounds__(256)
k_atomic_replay(unsigned long long *a, uint32_t n_addr,
                const uint32_t *__restrict__ trace, int64_t n, int reps) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int r = 0; r < reps; ++r)
        for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
             j < n; j += stride) {
            const uint32_t v = trace[j];
            if (v < n_addr) atomicAdd(&a[v], 1ull);
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
    uint32_t mask = 1;
    while ((int64_t)mask * 2 <= n_addresses && mask < (1u << 31)) mask *= 2;
    mask -= 1;
    hipLaunchKernelGGL(k_atomic_scatter, dim3(blocks), dim3(256), 0, st, a,
                       mask, 2);
    PSL_HIP(hipEventRecord(e0, st));
    hipLaunchKernelGGL(k_atomic_scatter, dim3(blocks), dim3(256), 0, st, a,
                       mask, iters);
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

extern "C" psl_status psl_bench_atomics_replay(
    const uint32_t *d_trace, int64_t n_trace, int64_t n_addresses,
    const int32_t *blocks_per_cu, int32_t n_shapes, int32_t reps,
    double *rates, void *d_ws, size_t ws_bytes, void *stream) {
    PSL_REQUIRE(d_trace && blocks_per_cu && rates && d_ws, "NULL argument");
    PSL_REQUIRE(n_trace >= 1 && n_addresses >= 1 &&
                    n_addresses < ((int64_t)1 << 32),
                "empty trace, or address count outside 1..2^32-1");
    PSL_REQUIRE(n_shapes >= 1 && n_shapes <= 64 && reps >= 1 && reps <= 1000,
                "n_shapes outside 1..64 or reps outside 1..1000");
    for (int i = 0; i < n_shapes; ++i)
        PSL_REQUIRE(blocks_per_cu[i] >= 1 && blocks_per_cu[i] <= 64,
                    "blocks_per_cu[%d] outside 1..64", i);
    if (ws_bytes < psl_bench_atomics_workspace_bytes(n_addresses)) {
        set_error("workspace too small");
        return PSL_ENOSPC;
    }
    if (psl_status s = check_device()) return s;
    hipStream_t st = (hipStream_t)stream;
    auto *a = static_cast<unsigned long long *>(d_ws);
    hipEvent_t e0, e1;
    PSL_HIP(hipEventCreate(&e0));
    PSL_HIP(hipEventCreate(&e1));
    const int cu = device_cu_count();
    for (int i = 0; i < n_shapes; ++i) {
        const int blocks = cu * blocks_per_cu[i];
        float ms = 0.0f;
        hipLaunchKernelGGL(k_atomic_replay, dim3(blocks), dim3(256), 0, st, a,
                           (uint32_t)n_addresses, d_trace, n_trace, 1);
        PSL_HIP(hipEventRecord(e0, st));
        hipLaunchKernelGGL(k_atomic_replay, dim3(blocks), dim3(256), 0, st, a,
                           (uint32_t)n_addresses, d_trace, n_trace, reps);
        PSL_HIP(hipEventRecord(e1, st));
        PSL_HIP(hipEventSynchronize(e1));
        PSL_HIP(hipEventElapsedTime(&ms, e0, e1));
        rates[i] = (double)n_trace * reps / (ms * 1e-3);
    }
    PSL_HIP(hipEventDestroy(e0));
    PSL_HIP(hipEventDestroy(e1));
    PSL_LAUNCHED();
    return PSL_OK;
}
