// psl_sample: the PSL source of one batch (Sec. 2.2, 2.3.3, 2.4).
//
//   k_cull          ROI selection per (field, position bin)
//   k_field_pop     C_i: particles in the selected PSLs of field i (Eq. 1)
//   k_field_totals  N_i by prefix-floor over fields (Eq. 2 or MU)
//   k_key_alloc     N_ik by prefix-floor over keys, g_ik (Eq. 2-4)
//   k_cursor        particles already read from each PSL (cyclic cursor)
//   scan            history ranges of (field, PSL)
//   k_sample        one thread per history: read, jaw test, fluence, weight,
//                   gantry, projection, wave-aggregated push to the queues
//
// The per-history decisions (jaw acceptance, fluence pixel, hitting the
// phantom) are taken in double precision with floating-point contraction
// disabled, so they are reproducible operation by operation.
#include "sample.hpp"
#include "scan.hpp"

#include <cmath>
#include <memory>
#include <mutex>
#include <vector>

namespace psl {

psl_status validate_grid_public(const psl_grid *g);

namespace {

__global__ void k_sample_init(psl_stats *stats, uint32_t *counts) {
    int t = threadIdx.x;
    if (t < (int)(sizeof(psl_stats) / 8))
        reinterpret_cast<uint64_t *>(stats)[t] = 0;
    if (t < PSL_QCOUNTS) counts[t] = 0;
}

// ROI at the PSL plane from the field centre at SAD through the jaw edges
// (Sec. 2.3.3, Fig. 1); a bin is kept when it overlaps the ROI with
// positive area.
__device__ void roi(double lo_sad, double hi_sad, double z_jaw, double sad,
                    double z_psl, double *lo, double *hi) {
#pragma clang fp contract(off)
    double c = (lo_sad + hi_sad) * 0.5;
    double f = (sad - z_psl) / (sad - z_jaw);
    double a_lo = lo_sad * z_jaw / sad;
    double a_hi = hi_sad * z_jaw / sad;
    *lo = c + (a_lo - c) * f;
    *hi = c + (a_hi - c) * f;
}

__global__ void __launch_bounds__(256)
k_cull(const FieldDev *__restrict__ fields, int n_fields, Geo geo,
       psl_grid g, int cull, uint8_t *__restrict__ mask) {
#pragma clang fp contract(off)
    const int P = g.n_x * g.n_y;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)n_fields * P) return;
    int f = (int)(i / P), p = (int)(i % P);
    int ix = p % g.n_x, iy = p / g.n_x;
    const FieldDev F = fields[f];
    uint8_t keep = 1;
    if (cull && F.jaws_on) {
        double xlo, xhi, ylo, yhi;
        roi(F.X1, F.X2, geo.z_x, geo.sad, geo.z_psl, &xlo, &xhi);
        roi(F.Y1, F.Y2, geo.z_y, geo.sad, geo.z_psl, &ylo, &yhi);
        keep = ((double)g.x_edges[ix] < xhi) &&
               ((double)g.x_edges[ix + 1] > xlo) &&
               ((double)g.y_edges[iy] < yhi) &&
               ((double)g.y_edges[iy + 1] > ylo);
    }
    mask[i] = keep;
}

constexpr int kAllocBlock = 1024;

__global__ void __launch_bounds__(kAllocBlock)
k_field_pop(const int64_t *__restrict__ off, int64_t n_keys, int P,
            const uint8_t *__restrict__ mask, int64_t *__restrict__ C) {
    __shared__ uint64_t s_wave[kAllocBlock / 64];
    const int f = blockIdx.x;
    const uint8_t *m = mask + (int64_t)f * P;
    uint64_t s = 0;
    for (int64_t k = threadIdx.x; k < n_keys; k += kAllocBlock)
        if (m[k % P]) s += (uint64_t)(off[k + 1] - off[k]);
    uint64_t tot;
    block_exclusive_scan<kAllocBlock>(s, &tot, s_wave);
    if (threadIdx.x == 0) C[f] = (int64_t)tot;
}

// Field totals by prefix-floor (one thread; fields are few).
__global__ void k_field_totals(const FieldDev *__restrict__ fields,
                               int n_fields, const int64_t *__restrict__ C,
                               int mode, int64_t n_sim,
                               int64_t *__restrict__ NF,
                               double *__restrict__ mu_tot_out) {
#pragma clang fp contract(off)
    double mu_tot = 0.0;
    for (int f = 0; f < n_fields; ++f) mu_tot += fields[f].MU;
    *mu_tot_out = mu_tot;
    int64_t prev = 0;
    if (mode == PSL_ALLOC_COUNTS) {
        int64_t c_all = 0;
        for (int f = 0; f < n_fields; ++f) c_all += C[f];
        int64_t acc = 0;
        for (int f = 0; f < n_fields; ++f) {
            acc += C[f];
            int64_t F = (f == n_fields - 1 || c_all == 0)
                            ? (f == n_fields - 1 && c_all ? n_sim : 0)
                            : (int64_t)(((unsigned __int128)n_sim * acc) /
                                        (uint64_t)c_all);
            NF[f] = F - prev;
            prev = F;
        }
    } else {
        double m = 0.0;
        for (int f = 0; f < n_fields; ++f) {
            m += fields[f].MU;
            int64_t F = (f == n_fields - 1)
                            ? n_sim
                            : (int64_t)floor((double)n_sim * m / mu_tot);
            NF[f] = F - prev;
            prev = F;
        }
    }
}

// Selected population per (field, key): sel_ik * n_k.
__global__ void k_masked_counts(const int64_t *__restrict__ off,
                                int64_t n_keys, int P, int n_fields,
                                const uint8_t *__restrict__ mask,
                                int64_t *__restrict__ v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)n_fields * n_keys) return;
    const int64_t f = i / n_keys, k = i % n_keys;
    v[i] = mask[f * P + k % P] ? off[k + 1] - off[k] : 0;
}

// N_ik = floor(N_i S_k / C_i) - floor(N_i S_k-1 / C_i), S the running
// selected population of field i in key order (from a device-wide exclusive
// scan Pm of the masked counts v); g_ik = (MU_i / MU_tot) n_k / N_ik.
__global__ void k_key_alloc(const FieldDev *__restrict__ fields,
                            const int64_t *__restrict__ off, int64_t n_keys,
                            int n_fields, const int64_t *__restrict__ v,
                            const int64_t *__restrict__ Pm,
                            const int64_t *__restrict__ C,
                            const int64_t *__restrict__ NF,
                            const double *__restrict__ mu_tot,
                            int64_t *__restrict__ N, double *__restrict__ g) {
#pragma clang fp contract(off)
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)n_fields * n_keys) return;
    const int64_t f = i / n_keys, k = i % n_keys;
    const uint64_t Cf = (uint64_t)C[f];
    const uint64_t Ni = (uint64_t)NF[f];
    const uint64_t vi = (uint64_t)v[i];
    int64_t Nik = 0;
    if (vi > 0 && Cf > 0) {
        const uint64_t Sp = (uint64_t)(Pm[i] - Pm[f * n_keys]);
        const uint64_t Sk = Sp + vi;
        const uint64_t a = (uint64_t)(((unsigned __int128)Ni * Sk) / Cf);
        const uint64_t b = (uint64_t)(((unsigned __int128)Ni * Sp) / Cf);
        Nik = (int64_t)(a - b);
    }
    N[i] = Nik;
    const double nk = (double)(off[k + 1] - off[k]);
    g[i] = Nik > 0 ? (fields[f].MU / *mu_tot) * (nk / (double)Nik) : 0.0;
}

// Per PSL: particles read by earlier fields of a batch, and per batch.
__global__ void k_cursor(const int64_t *__restrict__ N, int n_fields,
                         int64_t n_keys, int64_t *__restrict__ before,
                         int64_t *__restrict__ T) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_keys) return;
    int64_t run = 0;
    for (int f = 0; f < n_fields; ++f) {
        before[(int64_t)f * n_keys + k] = run;
        run += N[(int64_t)f * n_keys + k];
    }
    T[k] = run;
}

constexpr uint32_t kSourceElectronCtr = 0xFFFFFFFFu;
constexpr int kSampleBlock = 256;

// The last index idx >= from with H[idx] <= h, given H[from] <= h < total
// (H non-decreasing with n entries; entry n, which is not stored, is the
// total): a galloping search, short when the answer is near `from`.
__device__ __forceinline__ int64_t range_at(const int64_t *__restrict__ H,
                                            int64_t n, int64_t total,
                                            int64_t from, int64_t h) {
    auto at = [&](int64_t i) { return i < n ? H[i] : total; };
    if (at(from + 1) > h) return from;
    int64_t a = from + 1, step = 1, b = a + 1;   // H[a] <= h
    while (b < n && H[b] <= h) {
        a = b;
        step *= 2;
        b = a + step;
    }
    if (b > n) b = n;                             // at(b) > h
    while (b - a > 1) {
        const int64_t mid = (a + b) >> 1;        // a < mid < b <= n
        if (H[mid] <= h) a = mid; else b = mid;
    }
    return a;
}

__global__ void __launch_bounds__(kSampleBlock)
k_sample(psl_phsp ps, const int64_t *__restrict__ off, int64_t n_keys,
         const FieldDev *__restrict__ fields, Geo geo,
         const int64_t *__restrict__ H, int64_t n_ranges,
         const uint64_t *__restrict__ h_total_p,
         const int64_t *__restrict__ before, const int64_t *__restrict__ T,
         const double *__restrict__ g, uint64_t seed,
         const int64_t *__restrict__ batch_p, Slots slots, int64_t n_slots,
         psl_queue qcfg, uint64_t *part) {
#pragma clang fp contract(off)
    const int64_t batch = *batch_p;
    __shared__ float s_edges[PSL_MAX_QBUCKETS + 1];
    __shared__ uint64_t s_red[(kSampleBlock / 64) * kStatWords];
    if (threadIdx.x <= PSL_MAX_QBUCKETS)
        s_edges[threadIdx.x] = qcfg.e_bucket_edges[threadIdx.x];
    __syncthreads();
    StatAcc st;
    st.zero();
    const int64_t h_total = (int64_t)*h_total_p;
    // Each wave takes a contiguous run of 64-history chunks.  The range of
    // a chunk's first and last history is found by a wave-uniform search
    // that starts from the previous chunk's range (ranges are sorted), so
    // lanes search on their own only where a chunk straddles ranges.
    const int lane = __lane_id();
    const int64_t n_waves = (int64_t)gridDim.x * (kSampleBlock / 64);
    // the wave index, and so the chunk bounds, the range search and all
    // that depends on a chunk's range alone, are wave-uniform (scalar
    // registers and scalar loads)
    const int64_t wave_g = (int64_t)blockIdx.x * (kSampleBlock / 64) +
                           __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t n_chunks = (n_slots + 63) / 64;
    const int64_t per_wave = (n_chunks + n_waves - 1) / n_waves;
    const int64_t ch_end = min(n_chunks, (wave_g + 1) * per_wave);
    int64_t lo = 0;   // wave-uniform, H[lo] <= first history of the chunk
    for (int64_t ch = wave_g * per_wave; ch < ch_end; ++ch) {
        const int64_t h0 = ch * 64 + lane;
        const int64_t hf = ch * 64;
        int64_t hi = lo;
        if (hf < h_total) {
            const int64_t hl = min(hf + 63, h_total - 1);
            lo = range_at(H, n_ranges, h_total, lo, hf);
            hi = range_at(H, n_ranges, h_total, lo, hl);
        }
        if (h0 >= n_slots) continue;
        // the lane's accepted particle, written below
        bool acc_ok = false;
        float rE = 0.0f, rwt = 0.0f;
        float ro[6] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
        uint64_t ruid = 0;
        uint8_t rcode = kEmpty;
        if (h0 < h_total) {
            st.add(PSL_STAT(histories), 1);
            // range containing h0 (last idx with H[idx] <= h0) and the
            // particle it reads: p = off[k] + (s_k + c + r) mod n_k with
            // r = h0 - H[idx], c = batch * T[k] + before[idx]
            int64_t idx, p;
            if (hi == lo) {
                // one range for the whole chunk: r advances by one per
                // lane from the chunk's first history, so the residue is
                // taken once and each lane adds its offset
                idx = lo;
                const int64_t k = lo % n_keys;
                const int64_t o0 = off[k];
                const uint64_t nk = (uint64_t)(off[k + 1] - o0);
                const uint64_t s0 = splitmix64(seed ^ (uint64_t)k) % nk +
                                    (uint64_t)batch * (uint64_t)T[k] +
                                    (uint64_t)before[lo] +
                                    (uint64_t)(hf - H[lo]);
                const uint64_t l = (uint64_t)lane;
                uint64_t j;
                if (s0 > ~0ull - 63) {            // the sum wraps 2^64
                    j = (s0 + l) % nk;
                } else if (nk >= 64) {
                    j = s0 % nk + l;
                    if (j >= nk) j -= nk;
                } else {
                    j = (uint32_t)(s0 % nk + l) % (uint32_t)nk;
                }
                p = o0 + (int64_t)j;
            } else {
                // H[a0] <= h0 < H[b0] (b0 <= n_ranges; only H[mid], mid <
                // b0, is read)
                int64_t a0 = lo, b0 = hi + 1;
                while (b0 - a0 > 1) {
                    const int64_t mid = (a0 + b0) >> 1;
                    if (H[mid] <= h0) a0 = mid; else b0 = mid;
                }
                idx = a0;
                const int64_t k = idx % n_keys;
                const int64_t r = h0 - H[idx];
                const uint64_t nk = (uint64_t)(off[k + 1] - off[k]);
                const uint64_t sk = splitmix64(seed ^ (uint64_t)k) % nk;
                const uint64_t c = (uint64_t)batch * (uint64_t)T[k] +
                                   (uint64_t)before[idx];
                p = off[k] + (int64_t)((sk + c + (uint64_t)r) % nk);
            }
            const int f = (int)(idx / n_keys);
            const uint8_t type = ps.type[p];
            const float px = ps.x[p], py = ps.y[p], pu = ps.u[p],
                        pv = ps.v[p], pw = ps.w[p], pwt = ps.wt[p];
            const double gi = g[idx];
            // the beam model with its field's constants in scalar
            // registers, once per distinct field among the lanes (one,
            // except where a chunk crosses into the next field)
            float o[7];
            int status = 0;
            for (uint64_t pend = __ballot(1); pend;) {
                const int fl = __builtin_amdgcn_readlane(
                    f, (int)__builtin_ctzll(pend));
                if (f == fl)
                    status = beam_model(fields[fl], geo, px, py, pu, pv, pw,
                                        pwt, gi, o);
                pend &= ~__ballot(f == fl);
            }
            if (status == 1) {
                const float oE = ps.E[p];
                const float owt = o[6];
                int which = 0;
                if (type != 0) {
                    int b = 0;
                    for (int j = 1; j < qcfg.n_ebuckets; ++j)
                        if (oE >= s_edges[j]) b = j;
                    which = 1 + b;
                }
                acc_ok = true;
                rE = oE;
                rwt = owt;
#pragma unroll
                for (int j = 0; j < 6; ++j) ro[j] = o[j];
                ruid = (uint64_t)batch * (uint64_t)h_total + (uint64_t)h0;
                rcode = (uint8_t)which;
                st.add(which ? PSL_STAT(electrons) : PSL_STAT(photons), 1);
                st.addf(PSL_STAT(e_in), (double)oE * owt);
            }
            if (status == 0) st.add(PSL_STAT(jaw_rejected), 1);
            if (status == 2) st.add(PSL_STAT(fluence_zero), 1);
            if (status == 3) st.add(PSL_STAT(missed), 1);
        }
        // the chunk's accepted particles packed into its first slots in
        // history order (the queues keep that order; each carries its
        // uid), the other slots of the chunk marked empty: the
        // compaction then reads whole lines of packed slots
        const uint64_t am = __ballot(acc_ok);
        if (acc_ok) {
            const int64_t d = hf + __popcll(am & lanemask_lt());
            slots.p.E[d] = rE;
            slots.p.x[d] = ro[0];
            slots.p.y[d] = ro[1];
            slots.p.z[d] = ro[2];
            slots.p.u[d] = ro[3];
            slots.p.v[d] = ro[4];
            slots.p.w[d] = ro[5];
            slots.p.wt[d] = rwt;
            slots.p.uid[d] = ruid;
            slots.p.ctr[d] = rcode != 0 ? kSourceElectronCtr : 0u;
            slots.code[d] = rcode;
        }
        if (lane >= __popcll(am)) slots.code[h0] = kEmpty;
    }
    block_stats_write(st, s_red, part);
}

constexpr int kSampleMaxBlocks = 16384;


psl_status validate_particles(const psl_particles &p, const char *name) {
    PSL_REQUIRE(p.capacity >= 0, "%s capacity < 0", name);
    if (p.capacity > 0)
        PSL_REQUIRE(p.E && p.x && p.y && p.z && p.u && p.v && p.w && p.wt &&
                        p.uid && p.ctr,
                    "NULL array in %s", name);
    return PSL_OK;
}

__global__ void k_set_i64(int64_t *p, int64_t v) { *p = v; }
__global__ void k_inc_i64(int64_t *p) { *p += 1; }
__global__ void k_add_i64(int64_t *p, int64_t v) { *p += v; }

}  // namespace

SampleWs carve_sample_impl(void *base, int64_t n_keys, int P, int F,
                           int64_t n_hist) {
    Carver c(base);
    SampleWs w;
    const int64_t ns = std::max<int64_t>(n_hist, 1);
    w.fields = c.take<FieldDev>(F);
    w.mask = c.take<uint8_t>((int64_t)F * P);
    w.C = c.take<int64_t>(F);
    w.NF = c.take<int64_t>(F);
    w.mu_tot = c.take<double>(1);
    w.N = c.take<int64_t>((int64_t)F * n_keys);
    w.g = c.take<double>((int64_t)F * n_keys);
    w.H = c.take<int64_t>((int64_t)F * n_keys + 1);
    w.before = c.take<int64_t>((int64_t)F * n_keys);
    w.T = c.take<int64_t>(n_keys);
    w.chunks = c.take<uint64_t>(scan_chunks((int64_t)F * n_keys + 1) + 1);
    w.h_total = c.take<uint64_t>(1);
    w.batch = c.take<int64_t>(1);
    w.part = c.take<uint64_t>((int64_t)kSampleMaxBlocks * kStatWords);
    w.slots.p.capacity = ns;
    w.slots.p.E = c.take<float>(ns);
    w.slots.p.x = c.take<float>(ns);
    w.slots.p.y = c.take<float>(ns);
    w.slots.p.z = c.take<float>(ns);
    w.slots.p.u = c.take<float>(ns);
    w.slots.p.v = c.take<float>(ns);
    w.slots.p.w = c.take<float>(ns);
    w.slots.p.wt = c.take<float>(ns);
    w.slots.p.uid = c.take<uint64_t>(ns);
    w.slots.p.ctr = c.take<uint32_t>(ns);
    w.slots.code = c.take<uint8_t>(ns);
    w.tiles = c.take<uint32_t>((int64_t)kMaxQ * compact_tiles(ns));
    w.bytes = c.used;
    return w;
}

psl_status set_i64(int64_t *p, int64_t v, hipStream_t st) {
    hipLaunchKernelGGL(k_set_i64, dim3(1), dim3(1), 0, st, p, v);
    PSL_LAUNCHED();
    return PSL_OK;
}

psl_status inc_i64(int64_t *p, hipStream_t st) {
    hipLaunchKernelGGL(k_inc_i64, dim3(1), dim3(1), 0, st, p);
    PSL_LAUNCHED();
    return PSL_OK;
}

psl_status add_i64(int64_t *p, int64_t v, hipStream_t st) {
    hipLaunchKernelGGL(k_add_i64, dim3(1), dim3(1), 0, st, p, v);
    PSL_LAUNCHED();
    return PSL_OK;
}


psl_status validate_queue(const psl_queue *q) {
    PSL_REQUIRE(q && q->d_counts, "queue or its counts are NULL");
    psl_status s;
    if ((s = validate_particles(q->ph, "photon queue"))) return s;
    if ((s = validate_particles(q->el, "electron queue"))) return s;
    PSL_REQUIRE(q->n_ebuckets >= 1 && q->n_ebuckets <= PSL_MAX_QBUCKETS,
                "n_ebuckets = %d outside 1..%d", q->n_ebuckets,
                PSL_MAX_QBUCKETS);
    for (int b = 0; b + 1 < q->n_ebuckets; ++b)
        PSL_REQUIRE(q->e_bucket_edges[b] < q->e_bucket_edges[b + 1],
                    "bucket edges not increasing at %d", b);
    PSL_REQUIRE(q->ph.capacity < (int64_t)0xFFFFFFFF &&
                    q->el.capacity / q->n_ebuckets < (int64_t)0xFFFFFFFF,
                "queue capacity must stay below 2^32 per region");
    return PSL_OK;
}

}  // namespace psl

using namespace psl;

extern "C" size_t psl_sample_workspace_bytes(const psl_grid *g,
                                             int32_t n_fields,
                                             int64_t n_histories) {
    if (!g || n_fields < 1 || n_histories < 0) return 0;
    int64_t n_keys = 2LL * g->n_e * g->n_x * g->n_y;
    return carve_sample_impl(nullptr, n_keys, g->n_x * g->n_y, n_fields,
                             n_histories).bytes;
}

namespace psl {

psl_status sample_setup(const psl_phsp *sorted, const int64_t *d_offsets,
                        const psl_grid *g, const psl_field *fields,
                        int32_t n_fields, const psl_sample_cfg *cfg,
                        const psl_queue *q, uint8_t *d_mask, int64_t *d_alloc,
                        psl_stats *d_stats, void *d_ws, size_t ws_bytes,
                        SampleCtx *ctx) {
    PSL_REQUIRE(sorted && d_offsets && fields && cfg && q && d_stats,
                "NULL argument");
    psl_status s = validate_grid_public(g);
    if (s) return s;
    if ((s = validate_queue(q))) return s;
    PSL_REQUIRE(n_fields >= 1 && n_fields <= 4096, "n_fields = %d",
                n_fields);
    PSL_REQUIRE(sorted->n >= 1, "empty phase space");
    PSL_REQUIRE(sorted->type && sorted->E && sorted->x && sorted->y &&
                    sorted->u && sorted->v && sorted->w && sorted->wt,
                "NULL phase-space array");
    PSL_REQUIRE(cfg->batch >= 0, "batch < 0");
    PSL_REQUIRE(cfg->n_histories >= 0 &&
                    cfg->n_histories < (int64_t)0x7fffffff,
                "n_histories = %lld outside 0 .. 2^31-2",
                (long long)cfg->n_histories);
    PSL_REQUIRE(cfg->alloc_mode == PSL_ALLOC_COUNTS ||
                    cfg->alloc_mode == PSL_ALLOC_MU,
                "alloc_mode = %d", cfg->alloc_mode);
    PSL_REQUIRE(cfg->sad > 0, "sad must be positive");
    bool any_jaws = false;
    for (int i = 0; i < n_fields; ++i) any_jaws |= fields[i].jaws_on != 0;
    PSL_REQUIRE(!any_jaws || (cfg->z_jaw_x < cfg->sad &&
                              cfg->z_jaw_y < cfg->sad &&
                              g->z_plane < cfg->z_jaw_x &&
                              g->z_plane < cfg->z_jaw_y),
                "fields with jaws need z_psl < z_jaw < sad");
    for (int a = 0; a < 3; ++a)
        PSL_REQUIRE(cfg->box_lo[a] < cfg->box_hi[a], "empty phantom box");
    PSL_REQUIRE(q->ph.capacity >= cfg->n_histories,
                "photon queue capacity %lld < n_histories %lld",
                (long long)q->ph.capacity, (long long)cfg->n_histories);
    // products N_i * S_k must stay in 64 bits
    PSL_REQUIRE((unsigned __int128)cfg->n_histories * (uint64_t)sorted->n <
                    ((unsigned __int128)1 << 63),
                "n_histories * n_particles overflows 64 bits");
    ctx->fd.resize(n_fields);
    for (int i = 0; i < n_fields; ++i) {
        const psl_field &f = fields[i];
        PSL_REQUIRE(f.MU > 0, "field %d: MU <= 0", i);
        PSL_REQUIRE(!f.jaws_on || (f.X1 <= f.X2 && f.Y1 <= f.Y2),
                    "field %d: jaw X1 > X2 or Y1 > Y2", i);
        PSL_REQUIRE(!f.fluence || (f.nfx > 0 && f.nfy > 0 && f.f_pix > 0),
                    "field %d: bad fluence map", i);
        ctx->fd[i] = make_field_dev(f, f.jaws_on != 0, f.fluence != nullptr);
    }
    ctx->n_keys = 2LL * g->n_e * g->n_x * g->n_y;
    ctx->P = g->n_x * g->n_y;
    SampleWs need = carve_sample_impl(nullptr, ctx->n_keys, ctx->P, n_fields,
                                      cfg->n_histories);
    if (!d_ws || ws_bytes < need.bytes) {
        set_error("workspace %zu bytes < %zu required", ws_bytes, need.bytes);
        return PSL_ENOSPC;
    }
    ctx->w = carve_sample_impl(d_ws, ctx->n_keys, ctx->P, n_fields,
                               cfg->n_histories);
    ctx->sorted = *sorted;
    ctx->offsets = d_offsets;
    ctx->g = *g;
    ctx->geo = Geo{cfg->sad, cfg->z_jaw_x, cfg->z_jaw_y, g->z_plane,
                   {cfg->iso[0], cfg->iso[1], cfg->iso[2]},
                   {cfg->box_lo[0], cfg->box_lo[1], cfg->box_lo[2]},
                   {cfg->box_hi[0], cfg->box_hi[1], cfg->box_hi[2]}};
    ctx->n_fields = n_fields;
    ctx->cull = cfg->cull;
    ctx->alloc_mode = cfg->alloc_mode;
    ctx->n_ranges = (int64_t)n_fields * ctx->n_keys;
    ctx->n_hist = cfg->n_histories;
    ctx->seed = cfg->seed;
    ctx->q = *q;
    ctx->stats = d_stats;
    ctx->mask = d_mask ? d_mask : ctx->w.mask;
    ctx->N = d_alloc ? d_alloc : ctx->w.N;
    return PSL_OK;
}

psl_status sample_alloc(const SampleCtx &c, hipStream_t st) {
    psl_status s;
    const SampleWs &w = c.w;
    PSL_HIP(hipMemcpyAsync(w.fields, c.fd.data(),
                           sizeof(FieldDev) * c.n_fields,
                           hipMemcpyHostToDevice, st));
    ProfScope prof(PSL_PROF_ALLOC, st);
    const int64_t nm = (int64_t)c.n_fields * c.P;
    hipLaunchKernelGGL(k_cull, dim3((unsigned)((nm + 255) / 256)), dim3(256),
                       0, st, w.fields, c.n_fields, c.geo, c.g, c.cull,
                       c.mask);
    hipLaunchKernelGGL(k_field_pop, dim3(c.n_fields), dim3(kAllocBlock), 0,
                       st, c.offsets, c.n_keys, c.P, c.mask, w.C);
    hipLaunchKernelGGL(k_field_totals, dim3(1), dim3(1), 0, st, w.fields,
                       c.n_fields, w.C, c.alloc_mode, c.n_hist, w.NF,
                       w.mu_tot);
    {
        // masked counts in H, their scan in `before` (both rewritten below)
        const int64_t nr = c.n_ranges;
        const unsigned nb = (unsigned)((nr + 255) / 256);
        hipLaunchKernelGGL(k_masked_counts, dim3(nb), dim3(256), 0, st,
                           c.offsets, c.n_keys, c.P, c.n_fields, c.mask, w.H);
        if ((s = exclusive_scan<int64_t, int64_t>(w.H, w.before, nr, w.chunks,
                                                  nullptr, st)))
            return s;
        hipLaunchKernelGGL(k_key_alloc, dim3(nb), dim3(256), 0, st, w.fields,
                           c.offsets, c.n_keys, c.n_fields, w.H, w.before,
                           w.C, w.NF, w.mu_tot, c.N, w.g);
    }
    hipLaunchKernelGGL(k_cursor, dim3((unsigned)((c.n_keys + 255) / 256)),
                       dim3(256), 0, st, c.N, c.n_fields, c.n_keys, w.before,
                       w.T);
    if ((s = exclusive_scan<int64_t, int64_t>(c.N, w.H, c.n_ranges, w.chunks,
                                              w.h_total, st)))
        return s;
    PSL_LAUNCHED();
    return PSL_OK;
}

psl_status sample_batch(const SampleCtx &c, const int64_t *d_batch,
                        hipStream_t st) {
    psl_status s;
    const SampleWs &w = c.w;
    hipLaunchKernelGGL(k_sample_init, dim3(1), dim3(64), 0, st, c.stats,
                       c.q.d_counts);
    if (c.n_hist > 0) {
        ProfScope prof(PSL_PROF_SAMPLE, st);
        const int cu = device_cu_count();
        const int64_t blocks = std::min<int64_t>(
            (c.n_hist + kSampleBlock - 1) / kSampleBlock,
            std::min<int64_t>((int64_t)cu * 16, kSampleMaxBlocks));
        hipLaunchKernelGGL(k_sample, dim3((unsigned)blocks),
                           dim3(kSampleBlock), 0, st, c.sorted, c.offsets,
                           c.n_keys, w.fields, c.geo, w.H, c.n_ranges,
                           w.h_total, w.before, w.T, w.g, c.seed, d_batch,
                           w.slots, c.n_hist, c.q, w.part);
        QueueRegions qr{c.q.ph, c.q.el, 1 + c.q.n_ebuckets,
                        c.q.el.capacity / c.q.n_ebuckets, c.q.d_counts};
        if ((s = compact_slots(w.slots, c.n_hist, nullptr, 0, 0, qr, w.tiles,
                               st)))
            return s;
        if ((s = stats_reduce(w.part, (int)blocks, c.stats, st))) return s;
    }
    PSL_LAUNCHED();
    return PSL_OK;
}

}  // namespace psl

extern "C" psl_status psl_sample(const psl_phsp *sorted,
                                 const int64_t *d_offsets, const psl_grid *g,
                                 const psl_field *fields, int32_t n_fields,
                                 const psl_sample_cfg *cfg, psl_queue *q,
                                 uint8_t *d_mask, int64_t *d_alloc,
                                 psl_stats *d_stats, void *d_ws,
                                 size_t ws_bytes, void *stream) {
    SampleCtx ctx;
    psl_status s = sample_setup(sorted, d_offsets, g, fields, n_fields, cfg,
                                q, d_mask, d_alloc, d_stats, d_ws, ws_bytes,
                                &ctx);
    if (s) return s;
    if ((s = check_device())) return s;
    hipStream_t st = (hipStream_t)stream;
    if ((s = sample_alloc(ctx, st))) return s;
    if ((s = set_i64(ctx.w.batch, cfg->batch, st))) return s;
    return sample_batch(ctx, ctx.w.batch, st);
}

// ------------------------------------------------ allocation-free variant --
// psl_sample with its workspace in a file-scope device array instead of a
// caller buffer.  Each GPU the library runs on holds its own copy of the
// array (kNoAllocScratchBytes) until the process ends; host code reaches it
// only through the address hipGetSymbolAddress returns for the current
// device (the array's name in host code is a host-side stand-in).
namespace {

constexpr size_t kNoAllocScratchBytes = (size_t)64 << 20;
constexpr int kNoAllocMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

std::mutex g_scratch_mu;
void *g_scratch_ptr[kNoAllocMaxDevices] = {};

// The current device's address of `scratch`, looked up once per device.
psl_status scratch_address(void **out) {
    int dev = 0;
    PSL_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kNoAllocMaxDevices) {
        set_error("device %d: psl_sample_noalloc supports devices 0..%d",
                  dev, kNoAllocMaxDevices - 1);
        return PSL_EUNSUPPORTED;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            set_error("hipGetSymbolAddress(scratch) on device %d: %s", dev,
                      hipGetErrorString(e));
            return PSL_EHIP;
        }
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return PSL_OK;
}

}  // namespace

extern "C" size_t psl_sample_noalloc_max_bytes(void) {
    return kNoAllocScratchBytes;
}

extern "C" psl_status psl_sample_noalloc(const psl_phsp *sorted,
                                         const int64_t *d_offsets,
                                         const psl_grid *g,
                                         const psl_field *fields,
                                         int32_t n_fields,
                                         const psl_sample_cfg *cfg,
                                         psl_queue *q, uint8_t *d_mask,
                                         int64_t *d_alloc,
                                         psl_stats *d_stats, void *stream) {
    PSL_REQUIRE(g && cfg, "NULL argument");
    PSL_REQUIRE(n_fields >= 1 && cfg->n_histories >= 0,
                "n_fields = %d, n_histories = %lld", n_fields,
                (long long)cfg->n_histories);
    const size_t need =
        psl_sample_workspace_bytes(g, n_fields, cfg->n_histories);
    if (need == 0 || need > kNoAllocScratchBytes) {
        set_error("psl_sample_noalloc: this grid, %d field(s) and %lld "
                  "histories need %zu bytes of scratch; the static scratch "
                  "holds %zu (use psl_sample with a workspace)",
                  n_fields, (long long)cfg->n_histories, need,
                  kNoAllocScratchBytes);
        return PSL_ENOSPC;
    }
    psl_status s;
    void *ws = nullptr;
    if ((s = check_device())) return s;
    if ((s = scratch_address(&ws))) return s;
    return psl_sample(sorted, d_offsets, g, fields, n_fields, cfg, q, d_mask,
                      d_alloc, d_stats, ws, kNoAllocScratchBytes, stream);
}
