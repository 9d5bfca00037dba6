// Slot compaction into typed, energy-bucketed queues (see compact.hpp).
#include "compact.hpp"
#include "scan.hpp"

namespace psl {
namespace {

__device__ __forceinline__ int64_t slot_count(int64_t n_host,
                                              const uint32_t *n_dev,
                                              int64_t mult, int64_t add) {
    if (!n_dev) return n_host;
    int64_t n = (int64_t)n_dev[0] * mult + add;
    return n < n_host ? n : n_host;
}

__global__ void __launch_bounds__(kCompactBlock)
k_compact_count(const uint8_t *__restrict__ code, int64_t n_host,
                const uint32_t *n_dev, int64_t mult, int64_t add, int nq,
                uint32_t *__restrict__ tile_counts, int64_t n_tiles) {
    __shared__ uint32_t cnt[kMaxQ];
    if (threadIdx.x < kMaxQ) cnt[threadIdx.x] = 0;
    __syncthreads();
    const int64_t n = slot_count(n_host, n_dev, mult, add);
    const int64_t base = (int64_t)blockIdx.x * kCompactTile;
    if (base < n) {
        for (int r = 0; r < kCompactItems; ++r) {
            int64_t i = base + r * kCompactBlock + threadIdx.x;
            if (i < n) {
                uint32_t c = code[i];
                if (c < (uint32_t)nq) atomicAdd(&cnt[c], 1u);
            }
        }
    }
    __syncthreads();
    if (threadIdx.x < nq)
        tile_counts[(int64_t)threadIdx.x * n_tiles + blockIdx.x] =
            cnt[threadIdx.x];
}

constexpr int kOffBlock = 1024;

__global__ void __launch_bounds__(kOffBlock)
k_compact_offsets(uint32_t *__restrict__ tile_counts, int64_t n_tiles,
                  uint32_t *__restrict__ counts) {
    __shared__ uint64_t s_wave[kOffBlock / 64];
    const int q = blockIdx.x;
    uint64_t carry = counts[q];
    uint32_t *row = tile_counts + (int64_t)q * n_tiles;
    for (int64_t b = 0; b < n_tiles; b += kOffBlock) {
        int64_t i = b + threadIdx.x;
        uint64_t v = i < n_tiles ? row[i] : 0;
        uint64_t tot;
        uint64_t ex = block_exclusive_scan<kOffBlock>(v, &tot, s_wave);
        if (i < n_tiles) row[i] = (uint32_t)(carry + ex);
        carry += tot;
    }
    if (threadIdx.x == 0) counts[q] = (uint32_t)carry;
}

__global__ void __launch_bounds__(kCompactBlock)
k_compact_scatter(Slots s, int64_t n_host, const uint32_t *n_dev,
                  int64_t mult, int64_t add, QueueRegions q,
                  const uint32_t *__restrict__ tile_off, int64_t n_tiles) {
    constexpr int NW = kCompactBlock / 64;
    __shared__ uint32_t s_base[kMaxQ];
    __shared__ uint32_t s_w[NW][kMaxQ];
    const int tid = threadIdx.x, wid = tid >> 6;
    const int64_t n = slot_count(n_host, n_dev, mult, add);
    const int64_t base = (int64_t)blockIdx.x * kCompactTile;
    if (base >= n) return;   // uniform per block
    if (tid < q.nq) s_base[tid] = tile_off[(int64_t)tid * n_tiles + blockIdx.x];
    uint32_t lost = 0;
    for (int r = 0; r < kCompactItems; ++r) {
        if (tid < NW * kMaxQ) (&s_w[0][0])[tid] = 0;
        __syncthreads();
        const int64_t i = base + r * kCompactBlock + tid;
        const uint32_t c = i < n ? (uint32_t)s.code[i] : (uint32_t)kEmpty;
        const bool valid = c < (uint32_t)q.nq;
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 5; ++b) {
            uint64_t bb = __ballot((c >> b) & 1u);
            peers &= ((c >> b) & 1u) ? bb : ~bb;
        }
        const uint32_t rank = (uint32_t)__popcll(peers & lanemask_lt());
        if (valid && rank == 0) s_w[wid][c] = (uint32_t)__popcll(peers);
        __syncthreads();
        if (tid < q.nq) {
            uint32_t run = s_base[tid];
#pragma unroll
            for (int w = 0; w < NW; ++w) {
                uint32_t t = s_w[w][tid];
                s_w[w][tid] = run;
                run += t;
            }
            s_base[tid] = run;
        }
        __syncthreads();
        if (valid) {
            const uint32_t dst = s_w[wid][c] + rank;
            const psl_particles &P = c == 0 ? q.ph : q.el;
            const int64_t cap = c == 0 ? q.ph.capacity : q.cap_b;
            if ((int64_t)dst < cap) {
                const int64_t d = c == 0 ? (int64_t)dst
                                         : (int64_t)(c - 1) * q.cap_b + dst;
                P.E[d] = s.p.E[i];
                P.x[d] = s.p.x[i];
                P.y[d] = s.p.y[i];
                P.z[d] = s.p.z[i];
                P.u[d] = s.p.u[i];
                P.v[d] = s.p.v[i];
                P.w[d] = s.p.w[i];
                P.wt[d] = s.p.wt[i];
                P.uid[d] = s.p.uid[i];
                P.ctr[d] = s.p.ctr[i];
            } else {
                ++lost;
            }
        }
        __syncthreads();
    }
    if (lost) atomicAdd(&q.counts[PSL_QCOUNTS - 1], lost);
}

}  // namespace

psl_status compact_slots(const Slots &s, int64_t n_host, const uint32_t *n_dev,
                         int64_t mult, int64_t add, const QueueRegions &q,
                         uint32_t *tile_counts, hipStream_t st) {
    const int64_t n_tiles = compact_tiles(n_host);
    if (n_tiles == 0) return PSL_OK;
    hipLaunchKernelGGL(k_compact_count, dim3((unsigned)n_tiles),
                       dim3(kCompactBlock), 0, st, s.code, n_host, n_dev,
                       mult, add, q.nq, tile_counts, n_tiles);
    hipLaunchKernelGGL(k_compact_offsets, dim3((unsigned)q.nq),
                       dim3(kOffBlock), 0, st, tile_counts, n_tiles,
                       q.counts);
    hipLaunchKernelGGL(k_compact_scatter, dim3((unsigned)n_tiles),
                       dim3(kCompactBlock), 0, st, s, n_host, n_dev, mult,
                       add, q, tile_counts, n_tiles);
    PSL_LAUNCHED();
    return PSL_OK;
}

}  // namespace psl
