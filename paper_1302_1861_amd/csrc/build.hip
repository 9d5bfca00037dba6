// psl_build: PSL generation (Sec. 2.3.2) as a stable LSD radix sort by key
// that carries the particles with it.
//
//   k_keys            key per particle by comparison against the grid edges
//                     (staged in LDS); no atomics
//   radix passes      8-bit digits, 4096-item tiles: tile histograms
//                     (digit-major), device scan, stable scatter ranked with
//                     wave ballots; every pass moves the key and the seven
//                     float columns (E x y u v w wt), the first reading the
//                     input in file order, the last writing the output
//   k_offsets         PSL offsets from the boundaries of equal keys in the
//                     sorted keys (lower bound of every key), the particle
//                     type from the key, and the dropped count
// Each pass reads and writes whole columns in tile order, so the payload is
// never gathered at random positions.
#include "common.hpp"
#include "radix.hpp"
#include "scan.hpp"

namespace psl {
namespace {

constexpr int kRadixBlock = 256;
constexpr int kRadixItems = 32;
constexpr int kTile = kRadixBlock * kRadixItems;

// Largest k with v >= e[k], top edge closed; -1 outside [e[0], e[n]] or NaN.
__device__ __forceinline__ int bin_search(float v, const float *e, int n) {
    if (!(v >= e[0] && v <= e[n])) return -1;
    int lo = 0, hi = n;
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (v >= e[mid]) lo = mid; else hi = mid;
    }
    return lo;
}

__global__ void __launch_bounds__(256)
k_keys(psl_phsp in, psl_grid g, uint32_t n_keys, uint32_t *__restrict__ keys) {
    __shared__ float se[PSL_MAX_EBINS + 1], sx[PSL_MAX_POSBINS + 1],
        sy[PSL_MAX_POSBINS + 1];
    for (int i = threadIdx.x; i <= g.n_e; i += blockDim.x) se[i] = g.e_edges[i];
    for (int i = threadIdx.x; i <= g.n_x; i += blockDim.x) sx[i] = g.x_edges[i];
    for (int i = threadIdx.x; i <= g.n_y; i += blockDim.x) sy[i] = g.y_edges[i];
    __syncthreads();
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < in.n;
         i += stride) {
        uint32_t t = in.type[i];
        int e = bin_search(in.E[i], se, g.n_e);
        int ix = bin_search(in.x[i], sx, g.n_x);
        int iy = bin_search(in.y[i], sy, g.n_y);
        uint32_t key = n_keys;  // sentinel: dropped
        if (t <= 1 && e >= 0 && ix >= 0 && iy >= 0)
            key = ((t * g.n_e + e) * g.n_y + iy) * g.n_x + ix;
        keys[i] = key;
    }
}

__global__ void __launch_bounds__(kRadixBlock)
k_tile_hist(const uint32_t *__restrict__ keys, int64_t n, int shift,
            uint32_t *__restrict__ tile_hist, int64_t n_tiles) {
    __shared__ uint32_t s[256];
    s[threadIdx.x] = 0;
    __syncthreads();
    int64_t base = (int64_t)blockIdx.x * kTile;
#pragma unroll 4
    for (int r = 0; r < kRadixItems; ++r) {
        int64_t i = base + r * kRadixBlock + threadIdx.x;
        if (i < n) atomicAdd(&s[(keys[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    tile_hist[(int64_t)threadIdx.x * n_tiles + blockIdx.x] = s[threadIdx.x];
}

// What a k_radix_scatter pass moves besides the key: an index (the stable
// partition of the Method 1/2 source) or the seven float columns of the
// azimuthally turned copies (the first pass of an APR build; the other
// psl_build passes use k_radix_scatter_lds).
struct MoveIdx {
    const uint32_t *in;
    uint32_t *out;
    struct V { uint32_t id; };
    __device__ V load(int64_t i) const { return V{in[i]}; }
    __device__ void store(int64_t d, const V &v) const { out[d] = v.id; }
};

struct Cols7 { float *c[7]; };

// Azimuthal particle redistribution (Sec. 2.3.1): the turn of copy m, a
// point uniform in the unit disk by rejection from the counter-based
// stream splitmix64(splitmix64(seed ^ m) + t), whose doubled angle gives
// cos = (a^2 - b^2) / r^2, sin = 2ab / r^2 (IEEE arithmetic only, so the
// value does not depend on the machine); unturned after 64 failures.
__device__ __forceinline__ void apr_rotation(uint64_t seed, uint64_t m,
                                             double &c, double &s) {
#pragma clang fp contract(off)
    const uint64_t key = splitmix64(seed ^ m);
    for (uint64_t t = 0; t < 64; ++t) {
        const double a =
            (double)(splitmix64(key + 2 * t) >> 11) * 0x1.0p-53 * 2.0 - 1.0;
        const double b =
            (double)(splitmix64(key + 2 * t + 1) >> 11) * 0x1.0p-53 * 2.0 -
            1.0;
        const double r2 = a * a + b * b;
        if (r2 > 0.0 && r2 <= 1.0) {
            c = (a * a - b * b) / r2;
            s = 2.0 * a * b / r2;
            return;
        }
    }
    c = 1.0;
    s = 0.0;
}

// Copy m = i k + j of particle i, turned about the central axis.
struct AprIn {
    psl_phsp in;
    int64_t k;
    uint64_t seed;
    __device__ void particle(int64_t m, float &x, float &y, float &u,
                             float &v) const {
#pragma clang fp contract(off)
        const int64_t i = m / k;
        double c, s;
        apr_rotation(seed, (uint64_t)m, c, s);
        const double px = in.x[i], py = in.y[i], du = in.u[i], dv = in.v[i];
        x = (float)(c * px - s * py);
        y = (float)(s * px + c * py);
        u = (float)(c * du - s * dv);
        v = (float)(s * du + c * dv);
    }
};

__global__ void __launch_bounds__(256)
k_keys_apr(AprIn A, psl_grid g, uint32_t n_keys, int64_t n_items,
           uint32_t *__restrict__ keys) {
    __shared__ float se[PSL_MAX_EBINS + 1], sx[PSL_MAX_POSBINS + 1],
        sy[PSL_MAX_POSBINS + 1];
    for (int i = threadIdx.x; i <= g.n_e; i += blockDim.x) se[i] = g.e_edges[i];
    for (int i = threadIdx.x; i <= g.n_x; i += blockDim.x) sx[i] = g.x_edges[i];
    for (int i = threadIdx.x; i <= g.n_y; i += blockDim.x) sy[i] = g.y_edges[i];
    __syncthreads();
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
         m < n_items; m += stride) {
        const int64_t i = m / A.k;
        float x, y, u, v;
        A.particle(m, x, y, u, v);
        uint32_t t = A.in.type[i];
        int e = bin_search(A.in.E[i], se, g.n_e);
        int ix = bin_search(x, sx, g.n_x);
        int iy = bin_search(y, sy, g.n_y);
        uint32_t key = n_keys;
        if (t <= 1 && e >= 0 && ix >= 0 && iy >= 0)
            key = ((t * g.n_e + e) * g.n_y + iy) * g.n_x + ix;
        keys[m] = key;
    }
}

// The first pass of an APR build reads the turned copies.
struct MoveApr {
    AprIn a;
    Cols7 out;
    struct V { float c[7]; };
    __device__ V load(int64_t m) const {
        V v;
        const int64_t i = m / a.k;
        a.particle(m, v.c[1], v.c[2], v.c[3], v.c[4]);
        v.c[0] = a.in.E[i];
        v.c[5] = a.in.w[i];
        v.c[6] = (float)((double)a.in.wt[i] / (double)a.k);
        return v;
    }
    __device__ void store(int64_t d, const V &v) const {
#pragma unroll
        for (int k = 0; k < 7; ++k) out.c[k][d] = v.c[k];
    }
};

// Stable scatter of one tile.  Items are taken in rounds of 256 in index
// order; within a wave, lanes with equal digits are found with 8 ballots
// and ranked by lane; per-wave digit counts in LDS order the waves; a
// running per-digit base carries the rounds.  The payload of a round is
// loaded before its ranking so the loads overlap the ballots; items whose
// key is skip_key move their key only.
template <class M>
__global__ void __launch_bounds__(kRadixBlock)
k_radix_scatter(const uint32_t *__restrict__ keys_in, M mv, int64_t n,
                int shift, const uint32_t *__restrict__ tile_off,
                int64_t n_tiles, uint32_t *__restrict__ keys_out,
                uint32_t skip_key) {
    constexpr int NW = kRadixBlock / 64;
    __shared__ uint32_t s_base[256];
    __shared__ uint32_t s_w[NW][256];
    const int tid = threadIdx.x, wid = tid >> 6;
    s_base[tid] = tile_off[(int64_t)tid * n_tiles + blockIdx.x];
    const int64_t base = (int64_t)blockIdx.x * kTile;
    for (int r = 0; r < kRadixItems; ++r) {
#pragma unroll
        for (int w = 0; w < NW; ++w) s_w[w][tid] = 0;
        __syncthreads();
        int64_t i = base + r * kRadixBlock + tid;
        bool valid = i < n;
        uint32_t key = valid ? keys_in[i] : 0u;
        typename M::V val{};
        if (valid) val = mv.load(i);
        uint32_t d = (key >> shift) & 255u;
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            uint64_t bb = __ballot((d >> b) & 1u);
            peers &= ((d >> b) & 1u) ? bb : ~bb;
        }
        uint32_t rank = (uint32_t)__popcll(peers & lanemask_lt());
        if (valid && rank == 0) s_w[wid][d] = (uint32_t)__popcll(peers);
        __syncthreads();
        {
            uint32_t run = s_base[tid];
#pragma unroll
            for (int w = 0; w < NW; ++w) {
                uint32_t c = s_w[w][tid];
                s_w[w][tid] = run;
                run += c;
            }
            s_base[tid] = run;
        }
        __syncthreads();
        if (valid) {
            uint32_t dst = s_w[wid][d] + rank;
            keys_out[dst] = key;
            if (key != skip_key) mv.store(dst, val);
        }
        __syncthreads();
    }
}

// The same stable pass for the particle columns, with the tile put in
// order in LDS first: the ranking of k_radix_scatter, started from the
// tile's own digit offsets, gives every item its place in the tile sorted
// by digit; the keys and then each column go through LDS into that order
// and leave it by consecutive threads, so equal digits are written as
// contiguous runs (on average kTile / 256 items) instead of one item per
// round.  tile_off is the exclusive scan over (digit, tile) of the tile
// histograms: a tile's count of digit d is the next entry minus its own.
__global__ void __launch_bounds__(kRadixBlock)
k_radix_scatter_lds(const uint32_t *__restrict__ keys_in, Cols7 in,
                    Cols7 out, int64_t n, int shift,
                    const uint32_t *__restrict__ tile_off, int64_t n_tiles,
                    uint32_t *__restrict__ keys_out, uint32_t skip_key) {
    constexpr int NW = kRadixBlock / 64, R = kRadixItems;
    __shared__ uint32_t s_buf[kTile];      // keys, then one column at a time
    __shared__ uint32_t s_base[256];       // running local base per digit
    __shared__ uint32_t s_glob[256];       // global offset - local start
    __shared__ uint32_t s_w[NW][256];
    const int tid = threadIdx.x, wid = tid >> 6, lane = tid & 63;
    const int64_t base = (int64_t)blockIdx.x * kTile;
    const int m = (int)std::min<int64_t>(kTile, n - base);   // items here
    {
        const int64_t e = (int64_t)tid * n_tiles + blockIdx.x;
        const uint32_t g0 = tile_off[e];
        const uint32_t g1 =
            e + 1 < 256 * n_tiles ? tile_off[e + 1] : (uint32_t)n;
        // exclusive scan of the tile's digit counts: per wave, then waves
        uint32_t c = g1 - g0, incl = c;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t t = __shfl_up(incl, o);
            if (lane >= o) incl += t;
        }
        if (lane == 63) s_w[0][wid] = incl;
        __syncthreads();
        uint32_t before = 0;
        for (int w = 0; w < wid; ++w) before += s_w[0][w];
        const uint32_t lstart = before + incl - c;
        s_base[tid] = lstart;
        s_glob[tid] = g0 - lstart;
        __syncthreads();
    }
    uint32_t lp[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (r) __syncthreads();            // the last round's reads of s_w
#pragma unroll
        for (int w = 0; w < NW; ++w) s_w[w][tid] = 0;
        __syncthreads();
        const int li = r * kRadixBlock + tid;
        const bool valid = li < m;
        const uint32_t key = valid ? keys_in[base + li] : 0u;
        const uint32_t d = (key >> shift) & 255u;
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const uint64_t bb = __ballot((d >> b) & 1u);
            peers &= ((d >> b) & 1u) ? bb : ~bb;
        }
        const uint32_t rank = (uint32_t)__popcll(peers & lanemask_lt());
        if (valid && rank == 0) s_w[wid][d] = (uint32_t)__popcll(peers);
        __syncthreads();
        {
            uint32_t run = s_base[tid];
#pragma unroll
            for (int w = 0; w < NW; ++w) {
                const uint32_t c = s_w[w][tid];
                s_w[w][tid] = run;
                run += c;
            }
            s_base[tid] = run;
        }
        __syncthreads();
        lp[r] = valid ? s_w[wid][d] + rank : 0u;
        if (valid) s_buf[lp[r]] = key;
    }
    __syncthreads();
    // the keys in tile order: destinations, and which items carry payload
    uint32_t dst[R];
    uint32_t keep = 0;
#pragma unroll
    for (int j = 0; j < R; ++j) {
        const int p = j * kRadixBlock + tid;
        dst[j] = 0;
        if (p < m) {
            const uint32_t key = s_buf[p];
            dst[j] = s_glob[(key >> shift) & 255u] + (uint32_t)p;
            if (dst[j] < (uint64_t)n) {        // always, for consistent offsets
                keys_out[dst[j]] = key;
                if (key != skip_key) keep |= 1u << j;
            }
        }
    }
#pragma unroll 1
    for (int k = 0; k < 7; ++k) {
        const float *src = in.c[k];
        float v[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int li = r * kRadixBlock + tid;
            v[r] = li < m ? src[base + li] : 0.0f;
        }
        __syncthreads();                   // the last reads of s_buf
#pragma unroll
        for (int r = 0; r < R; ++r)
            if (r * kRadixBlock + tid < m) s_buf[lp[r]] = __float_as_uint(v[r]);
        __syncthreads();
        float *o = out.c[k];
#pragma unroll
        for (int j = 0; j < R; ++j)
            if ((keep >> j) & 1u)
                o[dst[j]] = __uint_as_float(s_buf[j * kRadixBlock + tid]);
    }
}

// Sorted keys -> PSL offsets (offsets[k] = items with key < k, for k = 0
// .. n_keys; the sentinel n_keys marks dropped particles and sorts last),
// the type column from the key, and the dropped count.
__global__ void __launch_bounds__(256)
k_offsets(const uint32_t *__restrict__ keys, int64_t n, uint32_t n_keys,
          uint32_t per_type, int64_t *__restrict__ off,
          uint8_t *__restrict__ type_out, int64_t *__restrict__ n_dropped) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j <= n;
         j += stride) {
        const int64_t kp = j == 0 ? -1 : (int64_t)keys[j - 1];
        const int64_t kc = j == n ? (int64_t)n_keys : (int64_t)keys[j];
        for (int64_t k = kp + 1; k <= kc; ++k) off[k] = j;
        if (j < n && kc < (int64_t)n_keys) type_out[j] = (uint8_t)(kc / per_type);
        if (kc == (int64_t)n_keys && kp < (int64_t)n_keys)
            *n_dropped = n - j;   // first dropped item (or the end)
    }
}

struct BuildWs {
    uint32_t *ka, *kb, *tile;
    Cols7 pa, pb;           // payload between passes (pb: three passes)
    uint64_t *chunks;
    size_t bytes;
};

int build_passes(int64_t n_keys) {
    int bits = 0;   // bits of keys 0 .. n_keys (the sentinel included)
    while ((1LL << bits) <= n_keys) ++bits;
    return std::max(1, (bits + 7) / 8);
}

BuildWs carve_build(void *base, int64_t n, int64_t n_keys) {
    Carver c(base);
    BuildWs w;
    const int64_t nn = n > 0 ? n : 1;
    const int64_t n_tiles = (nn + kTile - 1) / kTile;
    const int passes = build_passes(n_keys);
    w.ka = c.take<uint32_t>(nn);
    w.kb = c.take<uint32_t>(nn);
    w.tile = c.take<uint32_t>(256 * n_tiles);
    w.chunks = c.take<uint64_t>(scan_chunks(256 * n_tiles) + 1);
    for (int k = 0; k < 7; ++k) w.pa.c[k] = passes > 1 ? c.take<float>(nn)
                                                        : nullptr;
    for (int k = 0; k < 7; ++k) w.pb.c[k] = passes > 2 ? c.take<float>(nn)
                                                        : nullptr;
    w.bytes = c.used;
    return w;
}

psl_status validate_grid(const psl_grid *g) {
    PSL_REQUIRE(g, "grid is NULL");
    PSL_REQUIRE(g->n_e >= 1 && g->n_e <= PSL_MAX_EBINS,
                "n_e = %d outside 1..%d", g->n_e, PSL_MAX_EBINS);
    PSL_REQUIRE(g->n_x >= 1 && g->n_x <= PSL_MAX_POSBINS &&
                    g->n_y >= 1 && g->n_y <= PSL_MAX_POSBINS,
                "position bins %d x %d outside 1..%d", g->n_x, g->n_y,
                PSL_MAX_POSBINS);
    for (int i = 0; i < g->n_e; ++i)
        PSL_REQUIRE(g->e_edges[i] < g->e_edges[i + 1],
                    "energy edges not strictly increasing at %d", i);
    for (int i = 0; i < g->n_x; ++i)
        PSL_REQUIRE(g->x_edges[i] < g->x_edges[i + 1],
                    "x edges not strictly increasing at %d", i);
    for (int i = 0; i < g->n_y; ++i)
        PSL_REQUIRE(g->y_edges[i] < g->y_edges[i + 1],
                    "y edges not strictly increasing at %d", i);
    return PSL_OK;
}

}  // namespace

psl_status validate_grid_public(const psl_grid *g) { return validate_grid(g); }

namespace {
__global__ void k_digit_start(const uint32_t *__restrict__ tile_off,
                              int64_t n_tiles, uint32_t *__restrict__ out) {
    out[threadIdx.x] = tile_off[(int64_t)threadIdx.x * n_tiles];
}
}  // namespace

size_t radix_pass_ws_bytes(int64_t n) {
    const int64_t nn = n > 0 ? n : 1;
    const int64_t n_tiles = (nn + kTile - 1) / kTile;
    Carver c(nullptr);
    c.take<uint32_t>(256 * n_tiles);
    c.take<uint64_t>(scan_chunks(256 * n_tiles) + 1);
    return c.used;
}

psl_status radix_pass(const uint32_t *keys_in, const uint32_t *idx_in,
                      int64_t n, int shift, uint32_t *keys_out,
                      uint32_t *idx_out, uint32_t *digit_start, void *ws,
                      hipStream_t st) {
    const int64_t nn = n > 0 ? n : 1;
    const int64_t n_tiles = (nn + kTile - 1) / kTile;
    Carver c(ws);
    uint32_t *tile = c.take<uint32_t>(256 * n_tiles);
    uint64_t *chunks = c.take<uint64_t>(scan_chunks(256 * n_tiles) + 1);
    hipLaunchKernelGGL(k_tile_hist, dim3((unsigned)n_tiles),
                       dim3(kRadixBlock), 0, st, keys_in, n, shift, tile,
                       n_tiles);
    psl_status s = exclusive_scan<uint32_t, uint32_t>(tile, tile,
                                                      256 * n_tiles, chunks,
                                                      nullptr, st);
    if (s) return s;
    if (n > 0)
        hipLaunchKernelGGL(k_radix_scatter<MoveIdx>, dim3((unsigned)n_tiles),
                           dim3(kRadixBlock), 0, st, keys_in,
                           MoveIdx{idx_in, idx_out}, n, shift, tile, n_tiles,
                           keys_out, 0xFFFFFFFFu);
    if (digit_start)
        hipLaunchKernelGGL(k_digit_start, dim3(1), dim3(256), 0, st, tile,
                           n_tiles, digit_start);
    PSL_LAUNCHED();
    return PSL_OK;
}

}  // namespace psl

using namespace psl;

extern "C" size_t psl_build_workspace_bytes(int64_t n, const psl_grid *g) {
    if (!g || n < 0) return 0;
    int64_t n_keys = 2LL * g->n_e * g->n_x * g->n_y;
    return carve_build(nullptr, n, n_keys).bytes;
}

namespace {

psl_status build_impl(const psl_phsp *in, const psl_grid *g, bool apr_on,
                      int64_t copies, uint64_t seed, psl_phsp *out,
                      int64_t *d_offsets,
                      int64_t *d_n_dropped, void *d_ws, size_t ws_bytes,
                      void *stream) {
    PSL_REQUIRE(in && out && d_offsets && d_n_dropped, "NULL argument");
    psl_status s = validate_grid(g);
    if (s) return s;
    PSL_REQUIRE(copies >= 1 && copies <= 4096, "copies = %lld outside 1..4096",
                (long long)copies);
    PSL_REQUIRE(in->n >= 0 && in->n * copies < (int64_t)0x7fffffff,
                "n x copies = %lld outside 0 .. 2^31-2",
                (long long)(in->n * copies));
    const int64_t n = in->n * copies;
    PSL_REQUIRE(out->n >= n, "output capacity %lld < %lld",
                (long long)out->n, (long long)n);
    if (in->n > 0)
        PSL_REQUIRE(in->type && in->E && in->x && in->y && in->u && in->v &&
                        in->w && in->wt && out->type && out->E && out->x &&
                        out->y && out->u && out->v && out->w && out->wt,
                    "NULL phase-space array");
    const int64_t n_keys = 2LL * g->n_e * g->n_x * g->n_y;
    BuildWs need = carve_build(nullptr, n, n_keys);
    if (ws_bytes < need.bytes || !d_ws) {
        set_error("workspace %zu bytes < %zu required", ws_bytes, need.bytes);
        return PSL_ENOSPC;
    }
    if ((s = check_device())) return s;
    hipStream_t st = (hipStream_t)stream;
    BuildWs w = carve_build(d_ws, n, n_keys);
    const int cu = device_cu_count();
    ProfScope prof(PSL_PROF_BUILD, st);
    const int blocks = (int)std::max<int64_t>(
        1, std::min<int64_t>((n + 255) / 256, (int64_t)cu * 8));
    const uint32_t per_type = (uint32_t)(g->n_e * g->n_x * g->n_y);
    if (n > 0) {
        const AprIn apr{*in, copies, seed};
        if (apr_on)
            hipLaunchKernelGGL(k_keys_apr, dim3(blocks), dim3(256), 0, st,
                               apr, *g, (uint32_t)n_keys, n, w.ka);
        else
            hipLaunchKernelGGL(k_keys, dim3(blocks), dim3(256), 0, st, *in,
                               *g, (uint32_t)n_keys, w.ka);
        const int passes = build_passes(n_keys);
        const int64_t n_tiles = (n + kTile - 1) / kTile;
        const Cols7 src{{const_cast<float *>(in->E), const_cast<float *>(in->x),
                         const_cast<float *>(in->y), const_cast<float *>(in->u),
                         const_cast<float *>(in->v), const_cast<float *>(in->w),
                         const_cast<float *>(in->wt)}};
        const Cols7 dst{{out->E, out->x, out->y, out->u, out->v, out->w,
                         out->wt}};
        uint32_t *ki = w.ka, *ko = w.kb;
        Cols7 pi = src;
        for (int p = 0; p < passes; ++p) {
            const bool last = p == passes - 1;
            const Cols7 po = last ? dst : (p % 2 == 0 ? w.pa : w.pb);
            const uint32_t skip = last ? (uint32_t)n_keys : 0xFFFFFFFFu;
            hipLaunchKernelGGL(k_tile_hist, dim3((unsigned)n_tiles),
                               dim3(kRadixBlock), 0, st, ki, n, 8 * p, w.tile,
                               n_tiles);
            s = exclusive_scan<uint32_t, uint32_t>(w.tile, w.tile,
                                                   256 * n_tiles, w.chunks,
                                                   nullptr, st);
            if (s) return s;
            if (p == 0 && apr_on)
                hipLaunchKernelGGL(k_radix_scatter<MoveApr>,
                                   dim3((unsigned)n_tiles), dim3(kRadixBlock),
                                   0, st, ki, MoveApr{apr, po}, n, 8 * p,
                                   w.tile, n_tiles, ko, skip);
            else
                hipLaunchKernelGGL(k_radix_scatter_lds,
                                   dim3((unsigned)n_tiles), dim3(kRadixBlock),
                                   0, st, ki, pi, po, n, 8 * p, w.tile,
                                   n_tiles, ko, skip);
            std::swap(ki, ko);
            pi = po;
        }
        // ki holds the sorted keys
        hipLaunchKernelGGL(k_offsets, dim3(blocks), dim3(256), 0, st, ki, n,
                           (uint32_t)n_keys, per_type, d_offsets, out->type,
                           d_n_dropped);
    } else {
        hipLaunchKernelGGL(k_offsets, dim3(1), dim3(256), 0, st, w.ka, n,
                           (uint32_t)n_keys, per_type, d_offsets, out->type,
                           d_n_dropped);
    }
    PSL_LAUNCHED();
    return PSL_OK;
}

}  // namespace

extern "C" psl_status psl_build(const psl_phsp *in, const psl_grid *g,
                                psl_phsp *out, int64_t *d_offsets,
                                int64_t *d_n_dropped, void *d_ws,
                                size_t ws_bytes, void *stream) {
    return build_impl(in, g, false, 1, 0, out, d_offsets, d_n_dropped, d_ws,
                      ws_bytes, stream);
}

extern "C" size_t psl_build_apr_workspace_bytes(int64_t n, int64_t copies,
                                                const psl_grid *g) {
    if (!g || n < 0 || copies < 1) return 0;
    int64_t n_keys = 2LL * g->n_e * g->n_x * g->n_y;
    return carve_build(nullptr, n * copies, n_keys).bytes;
}

extern "C" psl_status psl_build_apr(const psl_phsp *in, const psl_grid *g,
                                    int64_t copies, uint64_t seed,
                                    psl_phsp *out, int64_t *d_offsets,
                                    int64_t *d_n_dropped, void *d_ws,
                                    size_t ws_bytes, void *stream) {
    return build_impl(in, g, true, copies, seed, out, d_offsets, d_n_dropped,
                      d_ws, ws_bytes, stream);
}
