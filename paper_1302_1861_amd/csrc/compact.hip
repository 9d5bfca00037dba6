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

// one wave per 1024-slot tile
__global__ void __launch_bounds__(kCompactBlock)
k_compact_count(const uint8_t *__restrict__ code, int64_t n_host,
                const uint32_t *n_dev, int64_t mult, int64_t add, int nq,
                uint32_t *__restrict__ tile_counts, int64_t n_tiles) {
    const int lane = __lane_id();
    const int64_t tile = (int64_t)blockIdx.x * (kCompactBlock / 64) +
                         (threadIdx.x >> 6);
    if (tile >= n_tiles) return;
    const int64_t n = slot_count(n_host, n_dev, mult, add);
    const int64_t base = tile * kCompactTile;
    uint32_t mine = 0;   // lane c counts code c
    if (base < n) {
        for (int r = 0; r < kCompactRounds; ++r) {
            const int64_t i = base + r * 64 + lane;
            const uint32_t c = i < n ? (uint32_t)code[i] : (uint32_t)kEmpty;
            for (int q = 0; q < nq; ++q) {
                uint64_t m = __ballot(c == (uint32_t)q);
                if (lane == q) mine += (uint32_t)__popcll(m);
            }
        }
    }
    if (lane < nq) tile_counts[(int64_t)lane * n_tiles + tile] = mine;
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
    const int lane = __lane_id();
    const int64_t tile = (int64_t)blockIdx.x * (kCompactBlock / 64) +
                         (threadIdx.x >> 6);
    if (tile >= n_tiles) return;
    const int64_t n = slot_count(n_host, n_dev, mult, add);
    const int64_t base = tile * kCompactTile;
    if (base >= n) return;
    uint32_t run = lane < q.nq ? tile_off[(int64_t)lane * n_tiles + tile] : 0;
    uint32_t lost = 0;
    for (int r = 0; r < kCompactRounds; ++r) {
        const int64_t i = base + r * 64 + lane;
        const uint32_t c = i < n ? (uint32_t)s.code[i] : (uint32_t)kEmpty;
        uint64_t my = 0;
        uint32_t add_c = 0;
        for (int qq = 0; qq < q.nq; ++qq) {
            uint64_t m = __ballot(c == (uint32_t)qq);
            if (c == (uint32_t)qq) my = m;
            if (lane == qq) add_c = (uint32_t)__popcll(m);
        }
        const bool valid = c < (uint32_t)q.nq;
        const uint32_t cb = __shfl(run, valid ? (int)c : 0);
        run += add_c;
        if (valid) {
            const uint32_t dst = cb + (uint32_t)__popcll(my & lanemask_lt());
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
    }
    for (int o = 32; o > 0; o >>= 1) lost += __shfl_xor(lost, o);
    if (lane == 0 && lost) atomicAdd(&q.counts[PSL_QCOUNTS - 1], lost);
}

}  // namespace

psl_status compact_slots(const Slots &s, int64_t n_host, const uint32_t *n_dev,
                         int64_t mult, int64_t add, const QueueRegions &q,
                         uint32_t *tile_counts, hipStream_t st) {
    const int64_t n_tiles = compact_tiles(n_host);
    if (n_tiles == 0) return PSL_OK;
    const int64_t wpb = kCompactBlock / 64;
    const unsigned blocks = (unsigned)((n_tiles + wpb - 1) / wpb);
    hipLaunchKernelGGL(k_compact_count, dim3(blocks),
                       dim3(kCompactBlock), 0, st, s.code, n_host, n_dev,
                       mult, add, q.nq, tile_counts, n_tiles);
    hipLaunchKernelGGL(k_compact_offsets, dim3((unsigned)q.nq),
                       dim3(kOffBlock), 0, st, tile_counts, n_tiles,
                       q.counts);
    hipLaunchKernelGGL(k_compact_scatter, dim3(blocks),
                       dim3(kCompactBlock), 0, st, s, n_host, n_dev, mult,
                       add, q, tile_counts, n_tiles);
    PSL_LAUNCHED();
    return PSL_OK;
}

}  // namespace psl
