// Block-wide and device-wide exclusive prefix sums (64-wide waves).
#pragma once

#include "common.hpp"

namespace psl {

// Exclusive scan of one value per thread over a block of BLOCK threads.
// s_wave: LDS scratch of BLOCK/64 entries.  Returns the exclusive prefix;
// *total receives the block sum.  Contains __syncthreads: call from all
// threads of the block.
template <int BLOCK>
__device__ __forceinline__ uint64_t block_exclusive_scan(uint64_t v,
                                                         uint64_t *total,
                                                         uint64_t *s_wave) {
    constexpr int NW = BLOCK / 64;
    const int lane = __lane_id();
    const int wid = threadIdx.x >> 6;
    uint64_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint64_t y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    if (lane == 63) s_wave[wid] = x;
    __syncthreads();
    if (wid == 0) {
        uint64_t w = lane < NW ? s_wave[lane] : 0;
#pragma unroll
        for (int o = 1; o < NW; o <<= 1) {
            uint64_t y = __shfl_up(w, o);
            if (lane >= o) w += y;
        }
        if (lane < NW) s_wave[lane] = w;
    }
    __syncthreads();
    uint64_t off = wid ? s_wave[wid - 1] : 0;
    *total = s_wave[NW - 1];
    __syncthreads();
    return off + x - v;
}

constexpr int kScanBlock = 1024;
constexpr int kScanItems = 4;
constexpr int kScanChunk = kScanBlock * kScanItems;

// Pass 1: per-chunk sums.
template <class Tin>
__global__ void __launch_bounds__(kScanBlock)
k_scan_reduce(const Tin *__restrict__ in, int64_t n,
              uint64_t *__restrict__ chunk_sums) {
    __shared__ uint64_t s_wave[kScanBlock / 64];
    int64_t base = (int64_t)blockIdx.x * kScanChunk +
                   (int64_t)threadIdx.x * kScanItems;
    uint64_t s = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i)
        if (base + i < n) s += (uint64_t)in[base + i];
    uint64_t tot;
    block_exclusive_scan<kScanBlock>(s, &tot, s_wave);
    if (threadIdx.x == 0) chunk_sums[blockIdx.x] = tot;
}

// Pass 2: exclusive scan of the chunk sums in one block (any length).
static __global__ void __launch_bounds__(kScanBlock)
k_scan_chunks(uint64_t *__restrict__ sums, int64_t n_chunks,
              uint64_t *__restrict__ grand_total) {
    __shared__ uint64_t s_wave[kScanBlock / 64];
    uint64_t carry = 0;
    for (int64_t b = 0; b < n_chunks; b += kScanBlock) {
        int64_t i = b + threadIdx.x;
        uint64_t v = i < n_chunks ? sums[i] : 0;
        uint64_t tot;
        uint64_t ex = block_exclusive_scan<kScanBlock>(v, &tot, s_wave);
        if (i < n_chunks) sums[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0 && grand_total) *grand_total = carry;
}

// Pass 3: exclusive scan inside each chunk plus the chunk offset.
template <class Tin, class Tout>
__global__ void __launch_bounds__(kScanBlock)
k_scan_apply(const Tin *in, int64_t n,
             const uint64_t *__restrict__ chunk_off, Tout *out) {
    __shared__ uint64_t s_wave[kScanBlock / 64];
    int64_t base = (int64_t)blockIdx.x * kScanChunk +
                   (int64_t)threadIdx.x * kScanItems;
    uint64_t v[kScanItems];
    uint64_t s = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        v[i] = base + i < n ? (uint64_t)in[base + i] : 0;
        s += v[i];
    }
    uint64_t tot;
    uint64_t ex = block_exclusive_scan<kScanBlock>(s, &tot, s_wave) +
                  chunk_off[blockIdx.x];
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        if (base + i < n) out[base + i] = (Tout)ex;
        ex += v[i];
    }
}

inline int64_t scan_chunks(int64_t n) {
    return (n + kScanChunk - 1) / kScanChunk;
}

// Exclusive scan of n values (out may alias in).  chunk_scratch holds
// scan_chunks(n) uint64 values; total (device, optional) gets the sum.
template <class Tin, class Tout>
inline psl_status exclusive_scan(const Tin *in, Tout *out, int64_t n,
                                 uint64_t *chunk_scratch, uint64_t *total,
                                 hipStream_t st) {
    int64_t nc = scan_chunks(n);
    if (nc == 0) nc = 1;
    hipLaunchKernelGGL((k_scan_reduce<Tin>), dim3((unsigned)nc),
                       dim3(kScanBlock), 0, st, in, n, chunk_scratch);
    hipLaunchKernelGGL(k_scan_chunks, dim3(1), dim3(kScanBlock), 0, st,
                       chunk_scratch, nc, total);
    hipLaunchKernelGGL((k_scan_apply<Tin, Tout>), dim3((unsigned)nc),
                       dim3(kScanBlock), 0, st, in, n, chunk_scratch, out);
    PSL_LAUNCHED();
    return PSL_OK;
}

}  // namespace psl
