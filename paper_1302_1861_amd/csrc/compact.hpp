// Slot compaction: re-bucketing of particles into typed, energy-bucketed
// queues without contended atomics.
//
// Producers (the sampler, the photon kernel) write each particle they emit
// into a slot whose index they own (history h, or photon i's j-th
// secondary), with a one-byte queue code (0 photons, 1 + b electron bucket
// b, kEmpty nothing).  Three kernels then move the occupied slots into the
// queue regions:
//   k_compact_count    per 1024-slot wave tile, counts per queue code from
//                      ballots (no LDS, no barriers)
//   k_compact_offsets  per queue, exclusive scan of the tile counts on top of
//                      the queue's current count; the count is advanced
//   k_compact_scatter  stable scatter: one wave per tile takes 16 rounds of
//                      64 slots; a slot's rank among equal codes is a
//                      popcount of the ballot for its code, the base of
//                      code c is held by lane c and advanced each round
// Queue order is the slot order, so the result is deterministic.
#pragma once

#include "common.hpp"

namespace psl {

constexpr uint8_t kEmpty = 0xFF;
constexpr int kCompactBlock = 256;
constexpr int kCompactRounds = 16;
constexpr int kCompactTile = 64 * kCompactRounds;   // slots per wave
constexpr int kMaxQ = 1 + PSL_MAX_QBUCKETS;

struct Slots {
    psl_particles p;     // records, p.capacity slots
    uint8_t *code;       // queue code per slot
};

struct QueueRegions {
    psl_particles ph, el;
    int32_t nq;          // 1 + number of electron buckets
    int64_t cap_b;       // electron region size
    uint32_t *counts;    // queue counts (d_counts layout)
};

inline int64_t compact_tiles(int64_t n_max) {
    return (n_max + kCompactTile - 1) / kCompactTile;
}

// Enqueues the three kernels over slots [0, n) where n = n_host, or, if
// n_dev is given, n = min(n_host, n_dev[0] * mult + add).
// tile_counts: workspace of kMaxQ * compact_tiles(n_host) uint32.
// Codes >= nq (kEmpty) are skipped; nq <= kMaxQ.
psl_status compact_slots(const Slots &s, int64_t n_host,
                         const uint32_t *n_dev, int64_t mult, int64_t add,
                         const QueueRegions &q, uint32_t *tile_counts,
                         hipStream_t st);

}  // namespace psl
