// Internal helpers shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstddef>
#include <cstdint>
#include <cstdio>
#include <string>

#include "../../include/psl.h"

namespace psl {

// ---------------------------------------------------------------- errors --
void set_error(const char *fmt, ...);
psl_status check_device();          // PSL_EUNSUPPORTED unless gfx950
int device_cu_count();

// Brackets the launches in its scope with hipEvents when profiling is on.
class ProfScope {
  public:
    ProfScope(int group, hipStream_t st);
    ~ProfScope();
    ProfScope(const ProfScope &) = delete;
    ProfScope &operator=(const ProfScope &) = delete;

  private:
    int group_;
    hipStream_t st_;
    hipEvent_t a_{}, b_{};
    bool active_ = false;
};

#define PSL_REQUIRE(cond, ...)                                                \
    do {                                                                      \
        if (!(cond)) {                                                        \
            ::psl::set_error(__VA_ARGS__);                                    \
            return PSL_EINVAL;                                                \
        }                                                                     \
    } while (0)

#define PSL_HIP(call)                                                         \
    do {                                                                      \
        hipError_t e_ = (call);                                               \
        if (e_ != hipSuccess) {                                               \
            ::psl::set_error("%s failed: %s", #call, hipGetErrorString(e_));  \
            return PSL_EHIP;                                                  \
        }                                                                     \
    } while (0)

#define PSL_LAUNCHED()                                                        \
    do {                                                                      \
        hipError_t e_ = hipGetLastError();                                    \
        if (e_ != hipSuccess) {                                               \
            ::psl::set_error("kernel launch failed: %s",                      \
                             hipGetErrorString(e_));                          \
            return PSL_EHIP;                                                  \
        }                                                                     \
    } while (0)

// -------------------------------------------------------------- workspace --
// Carves 256-byte aligned regions out of a caller workspace.  With base ==
// nullptr it only measures.
struct Carver {
    char *base;
    size_t used = 0;
    explicit Carver(void *b) : base(static_cast<char *>(b)) {}
    template <class T> T *take(size_t count) {
        used = (used + 255) & ~size_t(255);
        T *p = base ? reinterpret_cast<T *>(base + used) : nullptr;
        used += count * sizeof(T);
        return p;
    }
};

// ------------------------------------------------------------ wave utils --
__device__ __forceinline__ uint64_t lanemask_lt() {
    uint32_t lane = __lane_id();
    return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// --------------------------------------------------------------- Philox --
// Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11).
struct u32x4 { uint32_t x, y, z, w; };

__host__ __device__ __forceinline__ u32x4 philox4x32_10(u32x4 c,
                                                        uint32_t k0,
                                                        uint32_t k1) {
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        // each 32 x 32 -> 64-bit product as one multiply-add instruction
        // (both halves) instead of separate high and low multiplies
        const uint64_t p0 = (uint64_t)M0 * c.x, p1 = (uint64_t)M1 * c.z;
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        c = u32x4{hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0};
        k0 += W0;
        k1 += W1;
    }
    return c;
}

// Uniform in (0, 1) from the top 24 bits.
__device__ __forceinline__ float u01(uint32_t x) {
    return ((float)(x >> 8) + 0.5f) * (1.0f / 16777216.0f);
}

// The random blocks of one particle: block n is Philox of the counter
// (uid_lo, uid_hi, c2, tag | n), n = n0, n0 + 1, ...  Each sampling step
// (a free flight, one rejection trial, one deflection) takes a whole block
// at a fixed point of the code, so the lanes of a wave run the generator
// together instead of whenever one lane's buffer runs dry.
struct Rng {
    uint32_t k0, k1, uid_lo, uid_hi, c2, tag, n;
    __device__ void init(uint64_t seed, uint64_t uid, uint32_t c2_,
                         uint32_t tag_, uint32_t n0) {
        k0 = (uint32_t)seed;
        k1 = (uint32_t)(seed >> 32);
        uid_lo = (uint32_t)uid;
        uid_hi = (uint32_t)(uid >> 32);
        c2 = c2_;
        tag = tag_;
        n = n0;
    }
    __device__ u32x4 draw() {
        const u32x4 r =
            philox4x32_10(u32x4{uid_lo, uid_hi, c2, tag | n}, k0, k1);
        ++n;
        return r;
    }
};

// splitmix64 finaliser (Steele, Lea & Flood, OOPSLA 2014).
__host__ __device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Physics table layout inside the PSL_TABLE_BYTES device block.
struct TableHeader {
    int32_t n_mu, n_rng, n_inv, pad;
    float mu_lnE0, mu_inv_dlnE;     // mu table on ln E
    float rng_lnT0, rng_inv_dlnT;   // residual range on ln T
    float inv_r0, inv_inv_dr;       // energy on residual range
    float t_cut, p_cut, r_max, e_max;
    float kn_lnE0, kn_inv_dlnE;     // Compton fraction table on ln E
};
constexpr int kTabMu = 2048;
constexpr int kTabRange = 2048;
constexpr int kTabInv = 4096;
constexpr int kKnE = 64;    // energies of the Compton fraction table
constexpr int kKnQ = 96;    // quantiles per energy
constexpr size_t kTabHeaderBytes = 256;
// floats after the header: mu[kTabMu], range[kTabRange], inv[kTabInv],
// kn[kKnE][kKnQ]

}  // namespace psl

namespace psl {

// --------------------------------------------------------- block stats ----
// psl_stats as words: counters first, then doubles.
constexpr int kStatWords = (int)(sizeof(psl_stats) / 8);
constexpr int kStatFirstDouble = (int)(offsetof(psl_stats, e_in) / 8);

// Per-thread statistics, reduced per block into a partial record (plain
// stores) and summed by k_stats_reduce: no contended atomics.
struct StatAcc {
    uint64_t w[kStatWords];
    __device__ void zero() {
#pragma unroll
        for (int i = 0; i < kStatWords; ++i) w[i] = 0;
    }
    __device__ void add(int word, uint64_t v) { w[word] += v; }
    __device__ void addf(int word, double v) {
        w[word] = __double_as_longlong(__longlong_as_double(w[word]) + v);
    }
};

#define PSL_STAT(field) ((int)(offsetof(psl_stats, field) / 8))

// Block reduction of StatAcc into part[blockIdx.x * kStatWords + i].  All
// threads of the block must call it; s_red: LDS of (blockDim/64) *
// kStatWords words.
__device__ __forceinline__ void block_stats_write(StatAcc &a, uint64_t *s_red,
                                                  uint64_t *part) {
    const int lane = __lane_id(), wid = threadIdx.x >> 6;
    const int nw = blockDim.x >> 6;
#pragma unroll
    for (int i = 0; i < kStatWords; ++i) {
        uint64_t v = a.w[i];
        if (i < kStatFirstDouble) {
            for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
        } else {
            double d = __longlong_as_double(v);
            for (int o = 32; o > 0; o >>= 1) d += __shfl_xor(d, o);
            v = __double_as_longlong(d);
        }
        if (lane == 0) s_red[wid * kStatWords + i] = v;
    }
    __syncthreads();
    if (threadIdx.x < kStatWords) {
        const int i = threadIdx.x;
        uint64_t v = 0;
        double d = 0.0;
        for (int w = 0; w < nw; ++w) {
            if (i < kStatFirstDouble) v += s_red[w * kStatWords + i];
            else d += __longlong_as_double(s_red[w * kStatWords + i]);
        }
        part[(int64_t)blockIdx.x * kStatWords + i] =
            i < kStatFirstDouble ? v : (uint64_t)__double_as_longlong(d);
    }
}

// Adds the per-block partial records part[n_blocks][kStatWords] to *out.
psl_status stats_reduce(const uint64_t *part, int n_blocks, psl_stats *out,
                        hipStream_t st);

// --------------------------------------------------- work distribution ----
// Work items are claimed from kParts counters on separate cache lines, each
// owning a contiguous partition of the items; a wave starts at its own
// partition and moves on when it is drained.
constexpr int kParts = 64;
constexpr int kPartStride = 32;   // uint32 per counter (128 bytes)

}  // namespace psl
