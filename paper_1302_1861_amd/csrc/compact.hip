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

// One wave per tile of kCompactRounds x 64 slots: all codes of the tile are
// loaded first (independent loads, one wait), every destination is then
// ranked with ballots, and the payload moves in groups of kMoveGroup rounds
// whose loads are issued together.
constexpr int kMoveGroup = 4;
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
    uint32_t code[kCompactRounds];
#pragma unroll
    for (int r = 0; r < kCompactRounds; ++r) {
        const int64_t i = base + r * 64 + lane;
        code[r] = i < n ? (uint32_t)s.code[i] : (uint32_t)kEmpty;
    }
    uint32_t run = lane < q.nq ? tile_off[(int64_t)lane * n_tiles + tile] : 0;
    int64_t dst[kCompactRounds];   // queue index, or -1 (empty or lost)
    uint32_t lost = 0;
#pragma unroll
    for (int r = 0; r < kCompactRounds; ++r) {
        const uint32_t c = code[r];
        uint64_t my = 0;
        uint32_t add_c = 0;
        for (int qq = 0; qq < q.nq; ++qq) {
            const uint64_t m = __ballot(c == (uint32_t)qq);
            if (c == (uint32_t)qq) my = m;
            if (lane == qq) add_c = (uint32_t)__popcll(m);
        }
        const bool valid = c < (uint32_t)q.nq;
        const uint32_t cb = __shfl(run, valid ? (int)c : 0);
        run += add_c;
        dst[r] = -1;
        if (valid) {
            const uint32_t k = cb + (uint32_t)__popcll(my & lanemask_lt());
            const int64_t cap = c == 0 ? q.ph.capacity : q.cap_b;
            if ((int64_t)k < cap)
                dst[r] = c == 0 ? (int64_t)k : (int64_t)(c - 1) * q.cap_b + k;
            else
                ++lost;
        }
    }
#pragma unroll
    for (int g = 0; g < kCompactRounds; g += kMoveGroup) {
        // masked loads of the group (only lanes with a destination touch
        // memory), then the stores
        float E[kMoveGroup], x[kMoveGroup], y[kMoveGroup], z[kMoveGroup];
        float u[kMoveGroup], v[kMoveGroup], w[kMoveGroup], wt[kMoveGroup];
        uint64_t uid[kMoveGroup];
        uint32_t ctr[kMoveGroup];
#pragma unroll
        for (int j = 0; j < kMoveGroup; ++j) {
            const int64_t i = base + (g + j) * 64 + lane;
            if (dst[g + j] >= 0) {
                E[j] = s.p.E[i]; x[j] = s.p.x[i]; y[j] = s.p.y[i];
                z[j] = s.p.z[i]; u[j] = s.p.u[i]; v[j] = s.p.v[i];
                w[j] = s.p.w[i]; wt[j] = s.p.wt[i]; uid[j] = s.p.uid[i];
                ctr[j] = s.p.ctr[i];
            }
        }
#pragma unroll
        for (int j = 0; j < kMoveGroup; ++j) {
            const int64_t d = dst[g + j];
            if (d >= 0) {
                const psl_particles &P = code[g + j] == 0 ? q.ph : q.el;
                P.E[d] = E[j]; P.x[d] = x[j]; P.y[d] = y[j]; P.z[d] = z[j];
                P.u[d] = u[j]; P.v[d] = v[j]; P.w[d] = w[j];
                P.wt[d] = wt[j]; P.uid[d] = uid[j]; P.ctr[d] = ctr[j];
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
