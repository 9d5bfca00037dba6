// psl_build: PSL generation (Sec. 2.3.2) as a stable LSD radix sort of
// (key, index) pairs followed by one gather of the 29-byte payload.
//
//   k_keys        key per particle by comparison against the grid edges
//                 (staged in LDS), global histogram of keys
//   radix passes  8-bit digits, 4096-item tiles: tile histograms
//                 (digit-major), device scan, stable scatter ranked with
//                 wave ballots
//   offsets       exclusive scan of the key histogram (int64)
//   k_gather      payload copy in PSL order
#include "common.hpp"
#include "radix.hpp"
#include "scan.hpp"

namespace psl {
namespace {

constexpr int kRadixBlock = 256;
constexpr int kRadixItems = 16;
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
k_keys(psl_phsp in, psl_grid g, uint32_t n_keys, uint32_t *__restrict__ keys,
       uint32_t *__restrict__ idx, uint32_t *__restrict__ hist) {
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
        idx[i] = (uint32_t)i;
        atomicAdd(&hist[key], 1u);
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

// Stable scatter of one tile.  Items are taken in rounds of 256 in index
// order; within a wave, lanes with equal digits are found with 8 ballots
// and ranked by lane; per-wave digit counts in LDS order the waves; a
// running per-digit base carries the rounds.
__global__ void __launch_bounds__(kRadixBlock)
k_radix_scatter(const uint32_t *__restrict__ keys_in,
                const uint32_t *__restrict__ idx_in, int64_t n, int shift,
                const uint32_t *__restrict__ tile_off, int64_t n_tiles,
                uint32_t *__restrict__ keys_out,
                uint32_t *__restrict__ idx_out) {
    constexpr int NW = kRadixBlock / 64;
    __shared__ uint32_t s_base[256];
    __shared__ uint32_t s_w[NW][256];
    const int tid = threadIdx.x, lane = __lane_id(), wid = tid >> 6;
    s_base[tid] = tile_off[(int64_t)tid * n_tiles + blockIdx.x];
    const int64_t base = (int64_t)blockIdx.x * kTile;
    for (int r = 0; r < kRadixItems; ++r) {
#pragma unroll
        for (int w = 0; w < NW; ++w) s_w[w][tid] = 0;
        __syncthreads();
        int64_t i = base + r * kRadixBlock + tid;
        bool valid = i < n;
        uint32_t key = valid ? keys_in[i] : 0u;
        uint32_t id = valid ? idx_in[i] : 0u;
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
            idx_out[dst] = id;
        }
        __syncthreads();
        (void)lane;
    }
}

__global__ void __launch_bounds__(256)
k_gather(psl_phsp in, const uint32_t *__restrict__ idx,
         const int64_t *__restrict__ n_kept, psl_phsp out) {
    const int64_t m = *n_kept;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < m;
         j += stride) {
        uint32_t i = idx[j];
        out.type[j] = in.type[i];
        out.E[j] = in.E[i];
        out.x[j] = in.x[i];
        out.y[j] = in.y[i];
        out.u[j] = in.u[i];
        out.v[j] = in.v[i];
        out.w[j] = in.w[i];
        out.wt[j] = in.wt[i];
    }
}

__global__ void k_fill_u32(uint32_t *p, int64_t n, uint32_t v) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += stride)
        p[i] = v;
}

__global__ void k_dropped(const uint32_t *hist, uint32_t n_keys,
                          int64_t *n_dropped) {
    *n_dropped = hist[n_keys];
}

struct BuildWs {
    uint32_t *ka, *ia, *kb, *ib, *hist, *tile;
    uint64_t *chunks;
    size_t bytes;
};

BuildWs carve_build(void *base, int64_t n, int64_t n_keys) {
    Carver c(base);
    BuildWs w;
    int64_t nn = n > 0 ? n : 1;
    int64_t n_tiles = (nn + kTile - 1) / kTile;
    w.ka = c.take<uint32_t>(nn);
    w.ia = c.take<uint32_t>(nn);
    w.kb = c.take<uint32_t>(nn);
    w.ib = c.take<uint32_t>(nn);
    w.hist = c.take<uint32_t>(n_keys + 1);
    w.tile = c.take<uint32_t>(256 * n_tiles);
    int64_t big = std::max<int64_t>(256 * n_tiles, n_keys + 1);
    w.chunks = c.take<uint64_t>(scan_chunks(big) + 1);
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
        hipLaunchKernelGGL(k_radix_scatter, dim3((unsigned)n_tiles),
                           dim3(kRadixBlock), 0, st, keys_in, idx_in, n,
                           shift, tile, n_tiles, keys_out, idx_out);
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

extern "C" psl_status psl_build(const psl_phsp *in, const psl_grid *g,
                                psl_phsp *out, int64_t *d_offsets,
                                int64_t *d_n_dropped, void *d_ws,
                                size_t ws_bytes, void *stream) {
    PSL_REQUIRE(in && out && d_offsets && d_n_dropped, "NULL argument");
    psl_status s = validate_grid(g);
    if (s) return s;
    PSL_REQUIRE(in->n >= 0 && in->n < (int64_t)0x7fffffff,
                "n = %lld outside 0 .. 2^31-2", (long long)in->n);
    PSL_REQUIRE(out->n >= in->n, "output capacity %lld < n %lld",
                (long long)out->n, (long long)in->n);
    if (in->n > 0)
        PSL_REQUIRE(in->type && in->E && in->x && in->y && in->u && in->v &&
                        in->w && in->wt && out->type && out->E && out->x &&
                        out->y && out->u && out->v && out->w && out->wt,
                    "NULL phase-space array");
    const int64_t n = in->n;
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

    hipLaunchKernelGGL(k_fill_u32, dim3(64), dim3(256), 0, st, w.hist,
                       n_keys + 1, 0u);
    if (n > 0) {
        int blocks = (int)std::min<int64_t>((n + 255) / 256, cu * 8);
        hipLaunchKernelGGL(k_keys, dim3(blocks), dim3(256), 0, st, *in, *g,
                           (uint32_t)n_keys, w.ka, w.ia, w.hist);
        // passes over the bits needed for keys 0 .. n_keys (sentinel)
        int bits = 0;
        while ((1LL << bits) <= n_keys) ++bits;
        int passes = (bits + 7) / 8;
        int64_t n_tiles = (n + kTile - 1) / kTile;
        uint32_t *ki = w.ka, *ii = w.ia, *ko = w.kb, *io = w.ib;
        for (int p = 0; p < passes; ++p) {
            hipLaunchKernelGGL(k_tile_hist, dim3((unsigned)n_tiles),
                               dim3(kRadixBlock), 0, st, ki, n, 8 * p, w.tile,
                               n_tiles);
            s = exclusive_scan<uint32_t, uint32_t>(w.tile, w.tile,
                                                   256 * n_tiles, w.chunks,
                                                   nullptr, st);
            if (s) return s;
            hipLaunchKernelGGL(k_radix_scatter, dim3((unsigned)n_tiles),
                               dim3(kRadixBlock), 0, st, ki, ii, n, 8 * p,
                               w.tile, n_tiles, ko, io);
            std::swap(ki, ko);
            std::swap(ii, io);
        }
        s = exclusive_scan<uint32_t, int64_t>(w.hist, d_offsets, n_keys + 1,
                                              w.chunks, nullptr, st);
        if (s) return s;
        hipLaunchKernelGGL(k_gather, dim3(blocks), dim3(256), 0, st, *in, ii,
                           d_offsets + n_keys, *out);
    } else {
        s = exclusive_scan<uint32_t, int64_t>(w.hist, d_offsets, n_keys + 1,
                                              w.chunks, nullptr, st);
        if (s) return s;
    }
    hipLaunchKernelGGL(k_dropped, dim3(1), dim3(1), 0, st, w.hist,
                       (uint32_t)n_keys, d_n_dropped);
    PSL_LAUNCHED();
    return PSL_OK;
}
