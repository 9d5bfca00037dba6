// psl_stream_sample: Methods 1 and 2 (Sec. 2.1, 2.2), the sources the PSL
// method replaces: the unsorted phase space read in file order, the beam
// model (Method 2), and the on-the-fly bins by type and energy that are
// flushed to transport when they hold bin_capacity particles and at the end
// of the batch.
//
// The sequential process is reproduced exactly with data-parallel steps:
//   k_stream_classify   one thread per history: file position, beam model,
//                       bin code (255 when not accepted)
//   radix_pass          stable partition of the histories by bin code: the
//                       rank of a history in its bin is its arrival rank
//   k_stream_triggers   the history whose arrival completes a multiple of
//                       the capacity in its bin triggers a flush: flag it at
//                       its stream position; a scan of the flags numbers the
//                       full flushes in the order they happen
//   k_stream_full       full-flush descriptors and the (bin, k) -> flush
//                       table
//   k_stream_partial    end-of-batch flushes, in bin order after the full
//                       ones
//   scan                first element of each flush in the flushed sequence
//   k_stream_place      each accepted history recomputes its particle and
//                       writes it to its slot in the flushed sequence
//   compact_slots       photons to the photon queue, electrons to their
//                       energy buckets, both in flushed-sequence order
#include "compact.hpp"
#include "radix.hpp"
#include "sample.hpp"
#include "scan.hpp"

#include <cmath>

namespace psl {
namespace {

constexpr int kStreamBlock = 256;
constexpr uint32_t kRejected = 255u;
constexpr uint32_t kSourceElectronCtr = 0xFFFFFFFFu;

__global__ void k_stream_init(psl_stats *stats, uint32_t *counts,
                              int64_t *n_flushes) {
    const int t = threadIdx.x;
    if (t < (int)(sizeof(psl_stats) / 8))
        reinterpret_cast<uint64_t *>(stats)[t] = 0;
    if (t < PSL_QCOUNTS) counts[t] = 0;
    if (t == 0) *n_flushes = 0;
}

__global__ void k_fill32(uint32_t *p, int64_t n, uint32_t v) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += stride)
        p[i] = v;
}

__global__ void k_fill64(int64_t *p, int64_t n, int64_t v) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += stride)
        p[i] = v;
}

struct StreamArgs {
    psl_phsp ps;
    FieldDev F;
    Geo geo;
    uint64_t start;       // (s + b n_hist) mod n
    int64_t n_hist;
    double g;
    int n_e;
    int method;
};

// Energy bin: largest k with E >= e_k, clamped to 0 .. n_e-1.
__device__ __forceinline__ int energy_bin(float E, const float *e, int n_e) {
    int k = 0;
    for (int j = 1; j < n_e; ++j)
        if (E >= e[j]) k = j;
    return k;
}

__device__ __forceinline__ int64_t file_pos(const StreamArgs &A, int64_t r) {
    return (int64_t)((A.start + (uint64_t)r) % (uint64_t)A.ps.n);
}

__global__ void __launch_bounds__(kStreamBlock)
k_stream_classify(StreamArgs A, const float *__restrict__ e_edges,
                  uint32_t *__restrict__ keys, uint32_t *__restrict__ idx,
                  uint64_t *part) {
    __shared__ float s_e[PSL_MAX_EBINS + 1];
    __shared__ uint64_t s_red[(kStreamBlock / 64) * kStatWords];
    for (int i = threadIdx.x; i <= A.n_e; i += blockDim.x) s_e[i] = e_edges[i];
    __syncthreads();
    StatAcc st;
    st.zero();
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
         r < A.n_hist; r += stride) {
        const int64_t p = file_pos(A, r);
        const uint32_t type = A.ps.type[p];
        const float E = A.ps.E[p];
        uint32_t code = kRejected;
        st.add(PSL_STAT(histories), 1);
        if (type > 1u || E != E) {
            st.add(PSL_STAT(dropped), 1);
        } else {
            float o[7];
            const int status = beam_model(A.F, A.geo, A.ps.x[p], A.ps.y[p],
                                          A.ps.u[p], A.ps.v[p], A.ps.w[p],
                                          A.ps.wt[p], A.g, o);
            if (status == 1) {
                code = type * (uint32_t)A.n_e +
                       (uint32_t)energy_bin(E, s_e, A.n_e);
                st.add(type ? PSL_STAT(electrons) : PSL_STAT(photons), 1);
                st.addf(PSL_STAT(e_in), (double)E * (double)o[6]);
            } else if (status == 0) {
                st.add(PSL_STAT(jaw_rejected), 1);
            } else if (status == 2) {
                st.add(PSL_STAT(fluence_zero), 1);
            } else {
                st.add(PSL_STAT(missed), 1);
            }
        }
        keys[r] = code;
        idx[r] = (uint32_t)r;
    }
    block_stats_write(st, s_red, part);
}

// Sorted position j (digit order, arrival order within a digit) of an
// accepted history: rank within its bin b = j - start[b].
__global__ void __launch_bounds__(kStreamBlock)
k_stream_triggers(const uint32_t *__restrict__ keys,
                  const uint32_t *__restrict__ idx,
                  const uint32_t *__restrict__ start, int64_t cap,
                  uint32_t *__restrict__ flag) {
    const int64_t n_acc = start[kRejected];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
         j < n_acc; j += stride) {
        const int64_t rank = j - (int64_t)start[keys[j]];
        if ((rank + 1) % cap == 0) flag[idx[j]] = 1u;
    }
}

// Per bin: table base (flushes of earlier bins), full flushes, and the
// ordinal of the end-of-batch flush.  One block; bins <= 2 PSL_MAX_EBINS.
__global__ void __launch_bounds__(2 * PSL_MAX_EBINS)
k_stream_partial(const uint32_t *__restrict__ start, int n_bins,
                 int64_t cap, const uint64_t *__restrict__ n_full_p,
                 int64_t *__restrict__ tab_base,
                 int32_t *__restrict__ table, psl_flush *__restrict__ fl,
                 int64_t *__restrict__ count, int64_t *__restrict__ n_fl) {
    __shared__ int64_t s_tab[2 * PSL_MAX_EBINS];
    __shared__ int64_t s_part[2 * PSL_MAX_EBINS];
    const int b = threadIdx.x;
    int64_t c = 0;
    if (b < n_bins) c = (int64_t)start[b + 1] - (int64_t)start[b];
    const int64_t nf = (c + cap - 1) / cap;
    const int64_t rem = c % cap;
    s_tab[b] = b < n_bins ? nf : 0;
    s_part[b] = (b < n_bins && rem) ? 1 : 0;
    __syncthreads();
    if (b == 0) {
        int64_t t = 0, q = 0;
        for (int i = 0; i < n_bins; ++i) {
            const int64_t a = s_tab[i], pq = s_part[i];
            s_tab[i] = t;
            s_part[i] = q;
            t += a;
            q += pq;
        }
        *n_fl = (int64_t)*n_full_p + q;
    }
    __syncthreads();
    if (b < n_bins) {
        tab_base[b] = s_tab[b];
        if (rem) {
            const int64_t f = (int64_t)*n_full_p + s_part[b];
            fl[f].bin = b;
            fl[f].pad = 0;
            fl[f].count = rem;
            fl[f].trigger = -1;
            count[f] = rem;
            table[s_tab[b] + c / cap] = (int32_t)f;
        }
    }
}

__global__ void __launch_bounds__(kStreamBlock)
k_stream_full(const uint32_t *__restrict__ keys,
              const uint32_t *__restrict__ idx,
              const uint32_t *__restrict__ start, int64_t cap,
              const uint32_t *__restrict__ ordinal,
              const int64_t *__restrict__ tab_base,
              int32_t *__restrict__ table, psl_flush *__restrict__ fl,
              int64_t *__restrict__ count) {
    const int64_t n_acc = start[kRejected];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
         j < n_acc; j += stride) {
        const uint32_t b = keys[j];
        const int64_t rank = j - (int64_t)start[b];
        if ((rank + 1) % cap != 0) continue;
        const uint32_t r = idx[j];
        const int64_t f = ordinal[r];
        fl[f].bin = (int32_t)b;
        fl[f].pad = 0;
        fl[f].count = cap;
        fl[f].trigger = r;
        count[f] = cap;
        table[tab_base[b] + rank / cap] = (int32_t)f;
    }
}

__global__ void k_stream_first(const int64_t *__restrict__ first,
                               const int64_t *__restrict__ n_fl,
                               psl_flush *__restrict__ fl) {
    const int64_t n = *n_fl;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; f < n;
         f += stride)
        fl[f].first = first[f];
}

__global__ void __launch_bounds__(kStreamBlock)
k_stream_place(StreamArgs A, const uint32_t *__restrict__ keys,
               const uint32_t *__restrict__ idx,
               const uint32_t *__restrict__ start, int64_t cap,
               const int64_t *__restrict__ tab_base,
               const int32_t *__restrict__ table,
               const int64_t *__restrict__ first, uint64_t uid0,
               psl_queue qcfg, Slots slots) {
    __shared__ float s_edges[PSL_MAX_QBUCKETS + 1];
    if (threadIdx.x <= PSL_MAX_QBUCKETS)
        s_edges[threadIdx.x] = qcfg.e_bucket_edges[threadIdx.x];
    __syncthreads();
    const int64_t n_acc = start[kRejected];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
         j < n_acc; j += stride) {
        const uint32_t b = keys[j];
        const int64_t rank = j - (int64_t)start[b];
        const int64_t f = table[tab_base[b] + rank / cap];
        const int64_t seq = first[f] + rank % cap;
        const uint32_t r = idx[j];
        const int64_t p = file_pos(A, r);
        float o[7];
        (void)beam_model(A.F, A.geo, A.ps.x[p], A.ps.y[p], A.ps.u[p],
                         A.ps.v[p], A.ps.w[p], A.ps.wt[p], A.g, o);
        const float E = A.ps.E[p];
        int which = 0;
        if (b >= (uint32_t)A.n_e) {
            int q = 0;
            for (int k = 1; k < qcfg.n_ebuckets; ++k)
                if (E >= s_edges[k]) q = k;
            which = 1 + q;
        }
        slots.p.E[seq] = E;
        slots.p.x[seq] = o[0];
        slots.p.y[seq] = o[1];
        slots.p.z[seq] = o[2];
        slots.p.u[seq] = o[3];
        slots.p.v[seq] = o[4];
        slots.p.w[seq] = o[5];
        slots.p.wt[seq] = o[6];
        slots.p.uid[seq] = uid0 + r;
        slots.p.ctr[seq] = which ? kSourceElectronCtr : 0u;
        slots.code[seq] = (uint8_t)which;
    }
}

constexpr int kStreamMaxBlocks = 8192;

struct StreamWs {
    uint32_t *ka, *ia, *kb, *ib, *start, *flag;
    int64_t *tab_base, *count, *first;
    float *edges;
    int32_t *table;
    uint64_t *chunks, *n_full, *part;
    void *radix;
    Slots slots;
    uint32_t *tiles;
    size_t bytes;
};

int64_t stream_max_flushes(int64_t n_hist, int n_e, int64_t cap) {
    return n_hist / cap + 2LL * n_e + 1;
}

StreamWs carve_stream(void *base, int64_t n_hist, int n_e, int64_t cap) {
    Carver c(base);
    StreamWs w;
    const int64_t nn = std::max<int64_t>(n_hist, 1);
    const int64_t mf = stream_max_flushes(n_hist, n_e, cap);
    w.ka = c.take<uint32_t>(nn);
    w.ia = c.take<uint32_t>(nn);
    w.kb = c.take<uint32_t>(nn);
    w.ib = c.take<uint32_t>(nn);
    w.start = c.take<uint32_t>(256);
    w.flag = c.take<uint32_t>(nn);
    w.tab_base = c.take<int64_t>(2 * PSL_MAX_EBINS);
    w.table = c.take<int32_t>(mf);
    w.count = c.take<int64_t>(mf);
    w.first = c.take<int64_t>(mf);
    w.edges = c.take<float>(PSL_MAX_EBINS + 1);
    w.chunks = c.take<uint64_t>(scan_chunks(std::max<int64_t>(nn, mf)) + 1);
    w.n_full = c.take<uint64_t>(1);
    w.part = c.take<uint64_t>((int64_t)kStreamMaxBlocks * kStatWords);
    w.radix = c.take<char>(radix_pass_ws_bytes(nn));
    w.slots.p.capacity = nn;
    w.slots.p.E = c.take<float>(nn);
    w.slots.p.x = c.take<float>(nn);
    w.slots.p.y = c.take<float>(nn);
    w.slots.p.z = c.take<float>(nn);
    w.slots.p.u = c.take<float>(nn);
    w.slots.p.v = c.take<float>(nn);
    w.slots.p.w = c.take<float>(nn);
    w.slots.p.wt = c.take<float>(nn);
    w.slots.p.uid = c.take<uint64_t>(nn);
    w.slots.p.ctr = c.take<uint32_t>(nn);
    w.slots.code = c.take<uint8_t>(nn);
    w.tiles = c.take<uint32_t>((int64_t)kMaxQ * compact_tiles(nn));
    w.bytes = c.used;
    return w;
}

}  // namespace
}  // namespace psl

using namespace psl;

extern "C" size_t psl_stream_workspace_bytes(int64_t n_histories, int32_t n_e,
                                             int64_t bin_capacity) {
    if (n_histories < 0 || n_e < 1 || n_e > PSL_MAX_EBINS ||
        bin_capacity < 1)
        return 0;
    return carve_stream(nullptr, n_histories, n_e, bin_capacity).bytes;
}

extern "C" psl_status psl_stream_sample(const psl_phsp *phsp,
                                        const psl_field *field,
                                        const psl_stream_cfg *cfg,
                                        psl_queue *q, psl_flush *d_flushes,
                                        int64_t max_flushes,
                                        int64_t *d_n_flushes,
                                        psl_stats *d_stats, void *d_ws,
                                        size_t ws_bytes, void *stream) {
    PSL_REQUIRE(phsp && field && cfg && q && d_flushes && d_n_flushes &&
                    d_stats,
                "NULL argument");
    psl_status s = validate_queue(q);
    if (s) return s;
    PSL_REQUIRE(phsp->n >= 1 && phsp->n < ((int64_t)1 << 40),
                "phase space of %lld particles", (long long)phsp->n);
    PSL_REQUIRE(phsp->type && phsp->E && phsp->x && phsp->y && phsp->u &&
                    phsp->v && phsp->w && phsp->wt,
                "NULL phase-space array");
    PSL_REQUIRE(cfg->method == 1 || cfg->method == 2, "method = %d",
                cfg->method);
    PSL_REQUIRE(cfg->n_e >= 1 && cfg->n_e <= PSL_MAX_EBINS && cfg->e_edges,
                "n_e = %d outside 1..%d", cfg->n_e, PSL_MAX_EBINS);
    for (int i = 0; i < cfg->n_e; ++i)
        PSL_REQUIRE(cfg->e_edges[i] < cfg->e_edges[i + 1],
                    "energy edges not strictly increasing at %d", i);
    PSL_REQUIRE(cfg->batch >= 0, "batch < 0");
    PSL_REQUIRE(cfg->n_histories >= 0 &&
                    cfg->n_histories < (int64_t)0x7fffffff,
                "n_histories = %lld outside 0 .. 2^31-2",
                (long long)cfg->n_histories);
    PSL_REQUIRE(cfg->bin_capacity >= 1, "bin_capacity < 1");
    PSL_REQUIRE((unsigned __int128)cfg->batch * (uint64_t)cfg->n_histories <
                    ((unsigned __int128)1 << 62),
                "batch * n_histories overflows");
    PSL_REQUIRE(cfg->weight > 0 && std::isfinite(cfg->weight),
                "weight must be positive");
    PSL_REQUIRE(cfg->sad > 0, "sad must be positive");
    const bool jaws = cfg->method == 2 && field->jaws_on;
    PSL_REQUIRE(!jaws || (cfg->z_jaw_x < cfg->sad && cfg->z_jaw_y < cfg->sad &&
                          cfg->z_plane < cfg->z_jaw_x &&
                          cfg->z_plane < cfg->z_jaw_y),
                "a field with jaws needs z_plane < z_jaw < sad");
    PSL_REQUIRE(!jaws || (field->X1 <= field->X2 && field->Y1 <= field->Y2),
                "jaw X1 > X2 or Y1 > Y2");
    PSL_REQUIRE(cfg->method == 1 || !field->fluence ||
                    (field->nfx > 0 && field->nfy > 0 && field->f_pix > 0),
                "bad fluence map");
    for (int a = 0; a < 3; ++a)
        PSL_REQUIRE(cfg->box_lo[a] < cfg->box_hi[a], "empty phantom box");
    PSL_REQUIRE(q->ph.capacity >= cfg->n_histories,
                "photon queue capacity %lld < n_histories %lld",
                (long long)q->ph.capacity, (long long)cfg->n_histories);
    const int64_t n_hist = cfg->n_histories;
    const int64_t cap = cfg->bin_capacity;
    const int n_e = cfg->n_e;
    const int64_t mf = stream_max_flushes(n_hist, n_e, cap);
    PSL_REQUIRE(max_flushes >= mf - 1,
                "max_flushes %lld < %lld (n_histories / bin_capacity + "
                "2 n_e)", (long long)max_flushes, (long long)(mf - 1));
    StreamWs need = carve_stream(nullptr, n_hist, n_e, cap);
    if (!d_ws || ws_bytes < need.bytes) {
        set_error("workspace %zu bytes < %zu required", ws_bytes, need.bytes);
        return PSL_ENOSPC;
    }
    if ((s = check_device())) return s;
    hipStream_t st = (hipStream_t)stream;
    StreamWs w = carve_stream(d_ws, n_hist, n_e, cap);

    const FieldDev F = make_field_dev(
        *field, jaws, cfg->method == 2 && field->fluence != nullptr);
    Geo geo{cfg->sad, cfg->z_jaw_x, cfg->z_jaw_y, cfg->z_plane,
            {cfg->iso[0], cfg->iso[1], cfg->iso[2]},
            {cfg->box_lo[0], cfg->box_lo[1], cfg->box_lo[2]},
            {cfg->box_hi[0], cfg->box_hi[1], cfg->box_hi[2]}};
    const uint64_t n = (uint64_t)phsp->n;
    const uint64_t s0 = splitmix64(cfg->seed) % n;
    const uint64_t start = (uint64_t)(
        ((unsigned __int128)s0 +
         (unsigned __int128)cfg->batch * (uint64_t)n_hist) % n);
    StreamArgs A{*phsp, F, geo, start, n_hist, cfg->weight, n_e,
                 cfg->method};
    float *d_edges = w.edges;
    PSL_HIP(hipMemcpyAsync(d_edges, cfg->e_edges, sizeof(float) * (n_e + 1),
                           hipMemcpyHostToDevice, st));
    ProfScope prof(PSL_PROF_SAMPLE, st);
    hipLaunchKernelGGL(k_stream_init, dim3(1), dim3(64), 0, st, d_stats,
                       q->d_counts, d_n_flushes);
    const int cu = device_cu_count();
    const int blocks = (int)std::max<int64_t>(
        1, std::min<int64_t>((n_hist + kStreamBlock - 1) / kStreamBlock,
                             std::min<int64_t>((int64_t)cu * 16,
                                               kStreamMaxBlocks)));
    hipLaunchKernelGGL(k_stream_classify, dim3(blocks), dim3(kStreamBlock), 0,
                       st, A, d_edges, w.ka, w.ia, w.part);
    if ((s = stats_reduce(w.part, blocks, d_stats, st))) return s;
    if ((s = radix_pass(w.ka, w.ia, n_hist, 0, w.kb, w.ib, w.start, w.radix,
                        st)))
        return s;
    hipLaunchKernelGGL(k_fill32, dim3(std::min<int64_t>(
                                     (n_hist + 255) / 256 + 1, 4096)),
                       dim3(256), 0, st, w.flag, std::max<int64_t>(n_hist, 1),
                       0u);
    hipLaunchKernelGGL(k_fill64, dim3(std::min<int64_t>(mf / 256 + 1, 4096)),
                       dim3(256), 0, st, w.count, mf, (int64_t)0);
    hipLaunchKernelGGL(k_stream_triggers, dim3(blocks), dim3(kStreamBlock), 0,
                       st, w.kb, w.ib, w.start, cap, w.flag);
    if ((s = exclusive_scan<uint32_t, uint32_t>(w.flag, w.flag,
                                                std::max<int64_t>(n_hist, 1),
                                                w.chunks, w.n_full, st)))
        return s;
    hipLaunchKernelGGL(k_stream_partial, dim3(1), dim3(2 * PSL_MAX_EBINS), 0,
                       st, w.start, 2 * n_e, cap, w.n_full, w.tab_base,
                       w.table, d_flushes, w.count, d_n_flushes);
    hipLaunchKernelGGL(k_stream_full, dim3(blocks), dim3(kStreamBlock), 0, st,
                       w.kb, w.ib, w.start, cap, w.flag, w.tab_base, w.table,
                       d_flushes, w.count);
    if ((s = exclusive_scan<int64_t, int64_t>(w.count, w.first, mf, w.chunks,
                                              nullptr, st)))
        return s;
    hipLaunchKernelGGL(k_stream_first, dim3(std::min<int64_t>(mf / 256 + 1,
                                                             4096)),
                       dim3(256), 0, st, w.first, d_n_flushes, d_flushes);
    const uint64_t uid0 = (uint64_t)cfg->batch * (uint64_t)n_hist;
    hipLaunchKernelGGL(k_stream_place, dim3(blocks), dim3(kStreamBlock), 0, st,
                       A, w.kb, w.ib, w.start, cap, w.tab_base, w.table,
                       w.first, uid0, *q, w.slots);
    QueueRegions qr{q->ph, q->el, 1 + q->n_ebuckets,
                    q->el.capacity / q->n_ebuckets, q->d_counts};
    if ((s = compact_slots(w.slots, std::max<int64_t>(n_hist, 1),
                           w.start + kRejected, 1, 0, qr, w.tiles, st)))
        return s;
    PSL_LAUNCHED();
    return PSL_OK;
}
