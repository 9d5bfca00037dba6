// Internal helpers shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <string>

#include "../../include/psl.h"

namespace psl {

// ---------------------------------------------------------------- errors --
void set_error(const char *fmt, ...);
psl_status check_device();          // PSL_EUNSUPPORTED unless gfx950
int device_cu_count();

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

// Wave-aggregated reservation of `want` (0 or 1) slots in one of several
// counters: lanes choosing the same counter share one atomic.  Returns the
// slot index for lanes with want != 0.  Must be reached by all lanes that
// may want a slot (divergent lanes simply do not take part).
__device__ __forceinline__ uint32_t wave_reserve(uint32_t *counters, int which,
                                                 bool want) {
    uint64_t pending = __ballot(want);
    uint32_t slot = 0;
    while (pending) {
        int leader = __ffsll((unsigned long long)pending) - 1;
        int w = __shfl(which, leader);
        uint64_t grp = __ballot(want && which == w) & pending;
        uint32_t base = 0;
        if ((int)__lane_id() == leader)
            base = atomicAdd(&counters[w], (uint32_t)__popcll(grp));
        base = __shfl(base, leader);
        if (want && which == w)
            slot = base + (uint32_t)__popcll(grp & lanemask_lt());
        pending &= ~grp;
    }
    return slot;
}

// Wave sum then one atomic (for statistics).
__device__ __forceinline__ void wave_add_u64(uint64_t *dst, uint64_t v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if (__lane_id() == 0 && v) atomicAdd((unsigned long long *)dst,
                                         (unsigned long long)v);
}
__device__ __forceinline__ void wave_add_f64(double *dst, double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if (__lane_id() == 0 && v != 0.0) unsafeAtomicAdd(dst, v);
}

// --------------------------------------------------------------- Philox --
// Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11).
struct u32x4 { uint32_t x, y, z, w; };

__device__ __forceinline__ u32x4 philox4x32_10(u32x4 c, uint32_t k0,
                                               uint32_t k1) {
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        uint32_t hi0 = __umulhi(M0, c.x), lo0 = M0 * c.x;
        uint32_t hi1 = __umulhi(M1, c.z), lo1 = M1 * c.z;
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

// A stream of uniforms for one particle: counter (uid_lo, uid_hi, c2,
// tag | n) for n = 0, 1, 2, ...
struct Rng {
    uint32_t k0, k1, uid_lo, uid_hi, c2, tag, n;
    float b0, b1, b2, b3;   // scalars, not an array: no private memory
    int left;
    __device__ void init(uint64_t seed, uint64_t uid, uint32_t c2_,
                         uint32_t tag_, uint32_t n0) {
        k0 = (uint32_t)seed;
        k1 = (uint32_t)(seed >> 32);
        uid_lo = (uint32_t)uid;
        uid_hi = (uint32_t)(uid >> 32);
        c2 = c2_;
        tag = tag_;
        n = n0;
        left = 0;
    }
    __device__ void refill() {
        u32x4 r = philox4x32_10(u32x4{uid_lo, uid_hi, c2, tag | n}, k0, k1);
        ++n;
        b0 = u01(r.x);
        b1 = u01(r.y);
        b2 = u01(r.z);
        b3 = u01(r.w);
        left = 4;
    }
    __device__ float next() {
        if (left == 0) refill();
        float v = left == 4 ? b0 : left == 3 ? b1 : left == 2 ? b2 : b3;
        --left;
        return v;
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
};
constexpr int kTabMu = 2048;
constexpr int kTabRange = 2048;
constexpr int kTabInv = 4096;
constexpr size_t kTabHeaderBytes = 256;
// floats after the header: mu[kTabMu], range[kTabRange], inv[kTabInv]

}  // namespace psl
