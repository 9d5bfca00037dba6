// transport_batch and psl_physics_init: photon and electron transport with
// per-voxel energy tallies.
//
//   k_photons    persistent grid; each wave takes 64 queued photons at a
//                time.  Woodcock free flights against rho_max, Compton
//                scattering (Butcher-Messel sampling of Klein-Nishina),
//                recoil electrons pushed with one atomic per wave and
//                energy bucket; the attenuation table lives in LDS.
//   k_electrons  persistent grid over the electron buckets from the highest
//                energy down, so a wave holds electrons of similar range.
//                CSDA steps split at voxel faces; the energy after a piece
//                comes from the residual-range table and its inverse in
//                LDS; consecutive deposits into one voxel are merged before
//                the atomic; Highland deflection after each step.
#include "common.hpp"
#include "compact.hpp"

#include <cmath>
#include <vector>

namespace psl {

psl_status validate_queue(const psl_queue *q);

namespace {

constexpr float kME = 0.51099895f;
constexpr float kPI = 3.14159265358979f;
constexpr uint32_t kElectronTag = 0x80000000u;
constexpr int kBlock = 256;
constexpr int kMaxFlights = 1 << 20;
constexpr int kMaxSegments = 1 << 20;

// ------------------------------------------------------------------ tables
double kn_sigma_cm2(double E) {
    const double re = 2.8179403262e-13, me = 0.51099895;
    double k = E / me, a = 1.0 + 2.0 * k, L = std::log(a);
    double s = (1.0 + k) / (k * k) * (2.0 * (1.0 + k) / a - L / k) +
               L / (2.0 * k) - (1.0 + 3.0 * k) / (a * a);
    return 2.0 * M_PI * re * re * s;
}

double bethe_mass_stopping(double T, double n_e, double I_eV) {
    const double re = 2.8179403262e-13, me = 0.51099895;
    double tau = T / me, gam = tau + 1.0, b2 = 1.0 - 1.0 / (gam * gam);
    double ir = I_eV * 1e-6 / me;
    double F = 1.0 - b2 + (tau * tau / 8.0 - (2.0 * tau + 1.0) * M_LN2) /
                              (gam * gam);
    return 2.0 * M_PI * re * re * me * n_e / b2 *
           (std::log(tau * tau * (tau + 2.0) / (2.0 * ir * ir)) + F);
}

// integral of 1/S over [a, b] by 8-point Gauss-Legendre on ln T
double inv_s_integral(double a, double b, double n_e, double I) {
    static const double x[4] = {0.1834346424956498, 0.5255324099163290,
                                0.7966664774136267, 0.9602898564975363};
    static const double w[4] = {0.3626837833783620, 0.3137066458778873,
                                0.2223810344533745, 0.1012285362903763};
    double la = std::log(a), lb = std::log(b);
    double c = 0.5 * (la + lb), h = 0.5 * (lb - la), s = 0.0;
    for (int i = 0; i < 4; ++i)
        for (int sg = -1; sg <= 1; sg += 2) {
            double T = std::exp(c + sg * h * x[i]);
            s += w[i] * T / bethe_mass_stopping(T, n_e, I);
        }
    return s * h;
}

// --------------------------------------------------------------- device ---
struct PhDev {
    int nx, ny, nz;
    float x0, y0, z0, dx, dy, dz, ix_, iy_, iz_;  // inverse voxel sizes
    float rho_max;
    const float *rho;
};

struct PhysDev {
    float step, p_cut, t_cut, X0, pbc_me;
    int flags;
};

__device__ __forceinline__ float lerp_tab(const float *t, int n, float x) {
    x = fminf(fmaxf(x, 0.0f), (float)(n - 1) - 1e-3f);
    int i = (int)x;
    float f = x - (float)i;
    return t[i] + f * (t[i + 1] - t[i]);
}

template <int MODE>
__device__ __forceinline__ void tally(void *acc, int64_t v, float e, float wt,
                                      double scale, uint64_t &n_dep) {
    ++n_dep;
    if (MODE == PSL_ACC_FIXED64) {
        double q = (double)e * (double)wt * scale + 0.5;
        atomicAdd(reinterpret_cast<unsigned long long *>(acc) + v,
                  (unsigned long long)q);
    } else {
        unsafeAtomicAdd(reinterpret_cast<double *>(acc) + v,
                        (double)e * (double)wt);
    }
}

__device__ __forceinline__ void rotate(float &u, float &v, float &w, float ct,
                                       float st, float cp, float sp) {
    float s2 = 1.0f - w * w;
    float nu, nv, nw;
    if (s2 > 1e-10f) {
        float s = sqrtf(s2);
        nu = u * ct + st * (u * w * cp - v * sp) / s;
        nv = v * ct + st * (v * w * cp + u * sp) / s;
        nw = w * ct - st * cp * s;
    } else {
        nu = st * cp;
        nv = st * sp;
        nw = w > 0.0f ? ct : -ct;
    }
    float r = rsqrtf(nu * nu + nv * nv + nw * nw);
    u = nu * r;
    v = nv * r;
    w = nw * r;
}

__device__ __forceinline__ bool voxel_of(const PhDev &P, float x, float y,
                                         float z, int &ix, int &iy, int &iz) {
    ix = (int)floorf((x - P.x0) * P.ix_);
    iy = (int)floorf((y - P.y0) * P.iy_);
    iz = (int)floorf((z - P.z0) * P.iz_);
    return (unsigned)ix < (unsigned)P.nx && (unsigned)iy < (unsigned)P.ny &&
           (unsigned)iz < (unsigned)P.nz;
}

struct Items {
    psl_particles p;
    int32_t n_b;
    int64_t cap_b;
    uint32_t *counts;   // [0] photons, [1 + b] electron buckets
};

// Secondary-electron slots of the photon kernel: photon i owns slots
// spill_cap + i * kSecPerPhoton + j; further secondaries go to the spill
// slots [0, spill_cap) through one counter.
constexpr int kSecPerPhoton = 6;

struct SecSlots {
    Slots s;
    int64_t spill_cap;
    uint32_t *spill_n;
};

__device__ __forceinline__ void put_slot(const Slots &S, int64_t k, float E,
                                         float x, float y, float z, float u,
                                         float v, float w, float wt,
                                         uint64_t uid, uint32_t ctr,
                                         uint8_t code) {
    S.p.E[k] = E; S.p.x[k] = x; S.p.y[k] = y; S.p.z[k] = z;
    S.p.u[k] = u; S.p.v[k] = v; S.p.w[k] = w; S.p.wt[k] = wt;
    S.p.uid[k] = uid; S.p.ctr[k] = ctr;
    S.code[k] = code;
}

template <int MODE>
__global__ void __launch_bounds__(kBlock)
k_photons(Items ph, SecSlots sec, psl_queue qcfg, PhDev P, PhysDev Y,
          const float *__restrict__ tables, uint64_t seed, void *acc,
          double scale, uint32_t *work, uint64_t *part) {
    __shared__ float s_mu[kTabMu];
    __shared__ float s_bk[PSL_MAX_QBUCKETS + 1];
    __shared__ uint64_t s_red[(kBlock / 64) * kStatWords];
    const TableHeader H = *reinterpret_cast<const TableHeader *>(tables);
    const float *gmu = tables + kTabHeaderBytes / 4;
    for (int i = threadIdx.x; i < kTabMu; i += kBlock) s_mu[i] = gmu[i];
    if (threadIdx.x <= PSL_MAX_QBUCKETS)
        s_bk[threadIdx.x] = qcfg.e_bucket_edges[threadIdx.x];
    __syncthreads();
    const int64_t n = (int64_t)ph.counts[0];
    const int64_t n_chunks = (n + 63) / 64;
    StatAcc st;
    st.zero();
    uint64_t n_dep = 0;
    int part_i = (int)((blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6)) %
                       kParts),
        tried = 0;
    for (;;) {
        const int64_t chunk = claim_chunk(work, n_chunks, part_i, tried);
        if (chunk < 0) break;
        const int64_t i = chunk * 64 + __lane_id();
        bool alive = i < n;
        float E = 0, x = 0, y = 0, z = 0, u = 0, v = 0, w = 0, wt = 0;
        uint64_t uid = 0;
        Rng rng;
        if (alive) {
            E = ph.p.E[i]; x = ph.p.x[i]; y = ph.p.y[i]; z = ph.p.z[i];
            u = ph.p.u[i]; v = ph.p.v[i]; w = ph.p.w[i]; wt = ph.p.wt[i];
            uid = ph.p.uid[i];
            rng.init(seed, uid, 0u, 0u, ph.p.ctr[i]);
        }
        float mu1 = alive ? lerp_tab(s_mu, kTabMu,
                                     (__logf(E) - H.mu_lnE0) * H.mu_inv_dlnE)
                          : 0.0f;
        int flights = 0, n_sec = 0;
        while (__ballot(alive)) {
            bool push_e = false;
            float Te = 0, eu = 0, ev = 0, ew = 0;
            uint32_t birth = 0;
            if (alive && E < Y.p_cut) {
                int ix, iy, iz;
                if (voxel_of(P, x, y, z, ix, iy, iz))
                    tally<MODE>(acc, ((int64_t)iz * P.ny + iy) * P.nx + ix, E,
                                wt, scale, n_dep);
                else
                    st.addf(PSL_STAT(e_escaped), (double)E * wt);
                alive = false;
            }
            if (alive) {
                // one free flight against the majorant
                float s = -__logf(rng.next()) / (mu1 * P.rho_max);
                x += s * u; y += s * v; z += s * w;
                st.add(PSL_STAT(flights), 1);
                int ix, iy, iz;
                if (!voxel_of(P, x, y, z, ix, iy, iz)) {
                    st.addf(PSL_STAT(e_escaped), (double)E * wt);
                    alive = false;
                } else {
                    const int64_t vox = ((int64_t)iz * P.ny + iy) * P.nx + ix;
                    if (++flights > kMaxFlights) {
                        st.add(PSL_STAT(runaway), 1);
                        tally<MODE>(acc, vox, E, wt, scale, n_dep);
                        alive = false;
                    } else if (rng.next() * P.rho_max <= P.rho[vox]) {
                        // Compton: Butcher-Messel sampling of eps = E'/E
                        float k = E / kME;
                        float e0 = 1.0f / (1.0f + 2.0f * k);
                        float e0sq = e0 * e0;
                        float a1 = -__logf(e0), a2 = 0.5f * (1.0f - e0sq);
                        float eps, onecost, sint2, phi_u;
                        for (int tries = 0;; ++tries) {
                            float r1 = rng.next(), r2 = rng.next(),
                                  r3 = rng.next();
                            phi_u = rng.next();
                            float epssq;
                            if (r1 * (a1 + a2) < a1) {
                                eps = __expf(-a1 * r2);
                                epssq = eps * eps;
                            } else {
                                epssq = e0sq + (1.0f - e0sq) * r2;
                                eps = sqrtf(epssq);
                            }
                            onecost = (1.0f - eps) / (eps * k);
                            sint2 = onecost * (2.0f - onecost);
                            float gr = 1.0f - eps * sint2 / (1.0f + epssq);
                            if (gr >= r3 || tries > 1000) break;
                        }
                        st.add(PSL_STAT(interactions), 1);
                        float cost = 1.0f - onecost;
                        float sint = sqrtf(fmaxf(sint2, 0.0f));
                        float sp, cp;
                        __sincosf(2.0f * kPI * phi_u, &sp, &cp);
                        float Es = eps * E;
                        float T = E - Es;
                        float pu = u, pv = v, pw = w;
                        rotate(u, v, w, cost, sint, cp, sp);
                        if (T > Y.t_cut &&
                            !(Y.flags & PSL_FLAG_FIRST_COLLISION)) {
                            float qx = E * pu - Es * u, qy = E * pv - Es * v,
                                  qz = E * pw - Es * w;
                            float rq = rsqrtf(qx * qx + qy * qy + qz * qz);
                            push_e = true;
                            Te = T;
                            eu = qx * rq; ev = qy * rq; ew = qz * rq;
                            birth = rng.n;
                        } else {
                            tally<MODE>(acc, vox, T, wt, scale, n_dep);
                        }
                        if (Y.flags & PSL_FLAG_FIRST_COLLISION) {
                            st.addf(PSL_STAT(e_killed), (double)Es * wt);
                            alive = false;
                        } else {
                            E = Es;
                            mu1 = lerp_tab(s_mu, kTabMu,
                                           (__logf(E) - H.mu_lnE0) *
                                               H.mu_inv_dlnE);
                        }
                    }
                }
            }
            // recoil electron: own slot, or a spill slot past kSecPerPhoton
            const bool spill = push_e && n_sec >= kSecPerPhoton;
            uint32_t sslot = wave_reserve(sec.spill_n, 0, spill);
            if (push_e) {
                int b = 0;
                for (int j = 1; j < qcfg.n_ebuckets; ++j)
                    if (Te >= s_bk[j]) b = j;
                int64_t k = -1;
                if (!spill)
                    k = sec.spill_cap + i * kSecPerPhoton + n_sec;
                else if ((int64_t)sslot < sec.spill_cap)
                    k = sslot;
                if (k >= 0) {
                    put_slot(sec.s, k, Te, x, y, z, eu, ev, ew, wt, uid, birth,
                             (uint8_t)(1 + b));
                    st.add(PSL_STAT(secondaries), 1);
                } else {
                    st.add(PSL_STAT(lost), 1);
                }
                ++n_sec;
            }
        }
        // mark this photon's unused secondary slots empty
        if (i < n)
            for (int j = n_sec; j < kSecPerPhoton; ++j)
                sec.s.code[sec.spill_cap + i * kSecPerPhoton + j] = kEmpty;
    }
    st.add(PSL_STAT(photon_deposits), n_dep);
    block_stats_write(st, s_red, part);
}

template <int MODE>
__global__ void __launch_bounds__(kBlock)
k_electrons(Items el, PhDev P, PhysDev Y, const float *__restrict__ tables,
            uint64_t seed, void *acc, double scale, uint32_t *work,
            uint64_t *part) {
    __shared__ float s_rng[kTabRange];
    __shared__ float s_inv[kTabInv];
    __shared__ uint64_t s_red[(kBlock / 64) * kStatWords];
    const TableHeader H = *reinterpret_cast<const TableHeader *>(tables);
    const float *g = tables + kTabHeaderBytes / 4 + kTabMu;
    for (int i = threadIdx.x; i < kTabRange; i += kBlock) s_rng[i] = g[i];
    for (int i = threadIdx.x; i < kTabInv; i += kBlock)
        s_inv[i] = g[kTabRange + i];
    // bucket sizes (clamped to the region capacity), highest energy first
    __shared__ int64_t s_cnt[PSL_MAX_QBUCKETS];
    if (threadIdx.x < PSL_MAX_QBUCKETS) {
        int64_t c = threadIdx.x < el.n_b
                        ? (int64_t)el.counts[1 + threadIdx.x] : 0;
        s_cnt[threadIdx.x] = c < el.cap_b ? c : el.cap_b;
    }
    __syncthreads();
    int64_t total = 0;
    for (int b = 0; b < el.n_b; ++b) total += s_cnt[b];
    const int64_t n_chunks = (total + 63) / 64;
    StatAcc st;
    st.zero();
    uint64_t n_dep = 0;
    int part_i = (int)((blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6)) %
                       kParts),
        tried = 0;
    for (;;) {
        const int64_t chunk = claim_chunk(work, n_chunks, part_i, tried);
        if (chunk < 0) break;
        int64_t t = chunk * 64 + __lane_id();
        if (t >= total) continue;
        int b = el.n_b - 1;
        while (t >= s_cnt[b]) { t -= s_cnt[b]; --b; }
        const int64_t i = (int64_t)b * el.cap_b + t;
        float T = el.p.E[i];
        float x = el.p.x[i], y = el.p.y[i], z = el.p.z[i];
        float u = el.p.u[i], v = el.p.v[i], w = el.p.w[i], wt = el.p.wt[i];
        // entry voxel; a point on the box surface belongs to the voxel
        // inside
        int ix = (int)floorf((x - P.x0) * P.ix_);
        int iy = (int)floorf((y - P.y0) * P.iy_);
        int iz = (int)floorf((z - P.z0) * P.iz_);
        if (ix < -1 || iy < -1 || iz < -1 || ix > P.nx || iy > P.ny ||
            iz > P.nz) {
            st.addf(PSL_STAT(e_escaped), (double)T * wt);
            continue;
        }
        ix = min(max(ix, 0), P.nx - 1);
        iy = min(max(iy, 0), P.ny - 1);
        iz = min(max(iz, 0), P.nz - 1);
        int64_t vox = ((int64_t)iz * P.ny + iy) * P.nx + ix;
        if (T <= Y.t_cut) {
            tally<MODE>(acc, vox, T, wt, scale, n_dep);
            continue;
        }
        Rng rng;
        rng.init(seed, el.p.uid[i], el.p.ctr[i], kElectronTag, 0u);
        float r = lerp_tab(s_rng, kTabRange,
                           (__logf(T) - H.rng_lnT0) * H.rng_inv_dlnT);
        int64_t pv = vox;
        float pe = 0.0f;
        int segs = 0;
        bool done = false;
        while (!done) {
            float rem = Y.step, tm = 0.0f, T0 = T;
            while (rem > 0.0f) {
                float sx = u > 0.0f ? (P.x0 + (ix + 1) * P.dx - x) / u
                         : u < 0.0f ? (P.x0 + ix * P.dx - x) / u : INFINITY;
                float sy = v > 0.0f ? (P.y0 + (iy + 1) * P.dy - y) / v
                         : v < 0.0f ? (P.y0 + iy * P.dy - y) / v : INFINITY;
                float sz = w > 0.0f ? (P.z0 + (iz + 1) * P.dz - z) / w
                         : w < 0.0f ? (P.z0 + iz * P.dz - z) / w : INFINITY;
                int axis = 0;
                float sb = sx;
                if (sy < sb) { sb = sy; axis = 1; }
                if (sz < sb) { sb = sz; axis = 2; }
                sb = fmaxf(sb, 0.0f);
                float seg = fminf(rem, sb);
                float dm = P.rho[vox] * seg;
                st.add(PSL_STAT(segments), 1);
                if (dm >= r || ++segs > kMaxSegments) {
                    if (segs > kMaxSegments) st.add(PSL_STAT(runaway), 1);
                    if (vox != pv) {
                        tally<MODE>(acc, pv, pe, wt, scale, n_dep);
                        pv = vox;
                        pe = 0.0f;
                    }
                    pe += T;
                    T = 0.0f;
                    done = true;
                    break;
                }
                r -= dm;
                float Tn = fminf(lerp_tab(s_inv, kTabInv, r * H.inv_inv_dr), T);
                if (vox != pv) {
                    tally<MODE>(acc, pv, pe, wt, scale, n_dep);
                    pv = vox;
                    pe = 0.0f;
                }
                pe += T - Tn;
                T = Tn;
                tm += dm;
                x += seg * u; y += seg * v; z += seg * w;
                rem -= seg;
                if (seg == sb) {
                    bool in;
                    if (axis == 0) { ix += u > 0.0f ? 1 : -1;
                                     in = (unsigned)ix < (unsigned)P.nx; }
                    else if (axis == 1) { iy += v > 0.0f ? 1 : -1;
                                          in = (unsigned)iy < (unsigned)P.ny; }
                    else { iz += w > 0.0f ? 1 : -1;
                           in = (unsigned)iz < (unsigned)P.nz; }
                    if (!in) {
                        st.addf(PSL_STAT(e_escaped), (double)T * wt);
                        T = 0.0f;
                        done = true;
                        break;
                    }
                    vox = ((int64_t)iz * P.ny + iy) * P.nx + ix;
                }
            }
            if (done) break;
            if (!(Y.flags & PSL_FLAG_NO_MSC) && tm > 0.0f) {
                // Highland angle from the pre-step energy and the step's
                // mass thickness; space angle Rayleigh-distributed with
                // scale theta0, truncated at pi
                float pbc = T0 * (T0 + 2.0f * kME) / (T0 + kME);
                float qq = tm / Y.X0;
                float th0 = 13.6f / pbc * sqrtf(qq) *
                            (1.0f + 0.038f * __logf(qq));
                th0 = fmaxf(th0, 0.0f);
                float th;
                int tries = 0;
                do {
                    th = th0 * sqrtf(-2.0f * __logf(rng.next()));
                } while (th > kPI && ++tries < 64);
                if (th > kPI) th = kPI * rng.next();
                float sth, cth, sp, cp;
                __sincosf(th, &sth, &cth);
                __sincosf(2.0f * kPI * rng.next(), &sp, &cp);
                rotate(u, v, w, cth, sth, cp, sp);
            }
        }
        if (pe > 0.0f) tally<MODE>(acc, pv, pe, wt, scale, n_dep);
    }
    st.add(PSL_STAT(deposits), n_dep);
    block_stats_write(st, s_red, part);
}

__global__ void k_transport_init(uint32_t *work, int n_words,
                                 uint8_t *spill_code, int64_t spill_cap) {
    for (int i = threadIdx.x + blockIdx.x * blockDim.x; i < n_words;
         i += gridDim.x * blockDim.x)
        work[i] = 0;
    for (int64_t i = threadIdx.x + (int64_t)blockIdx.x * blockDim.x;
         i < spill_cap; i += (int64_t)gridDim.x * blockDim.x)
        spill_code[i] = kEmpty;
}

__global__ void k_consume(uint32_t *counts) {
    if (threadIdx.x < PSL_QCOUNTS - 1) counts[threadIdx.x] = 0;
}

struct TransportWs {
    uint32_t *work;        // 2 work-claim arrays + spill counter
    Slots sec;
    uint32_t *tiles;
    uint64_t *part;
    int64_t spill_cap, n_slots;
    size_t bytes;
};

TransportWs carve_transport(void *base, int64_t ph_cap, int grid_blocks) {
    Carver c(base);
    TransportWs w;
    w.work = c.take<uint32_t>(2 * kParts * kPartStride + 64);
    w.spill_cap = std::max<int64_t>(65536, ph_cap / 8);
    w.n_slots = w.spill_cap + std::max<int64_t>(ph_cap, 1) * kSecPerPhoton;
    w.sec.p.capacity = w.n_slots;
    w.sec.p.E = c.take<float>(w.n_slots);
    w.sec.p.x = c.take<float>(w.n_slots);
    w.sec.p.y = c.take<float>(w.n_slots);
    w.sec.p.z = c.take<float>(w.n_slots);
    w.sec.p.u = c.take<float>(w.n_slots);
    w.sec.p.v = c.take<float>(w.n_slots);
    w.sec.p.w = c.take<float>(w.n_slots);
    w.sec.p.wt = c.take<float>(w.n_slots);
    w.sec.p.uid = c.take<uint64_t>(w.n_slots);
    w.sec.p.ctr = c.take<uint32_t>(w.n_slots);
    w.sec.code = c.take<uint8_t>(w.n_slots);
    w.tiles = c.take<uint32_t>((int64_t)kMaxQ * compact_tiles(w.n_slots));
    w.part = c.take<uint64_t>((int64_t)2 * grid_blocks * kStatWords);
    w.bytes = c.used;
    return w;
}

constexpr int kMaxGridBlocks = 64 * 1024;

}  // namespace
}  // namespace psl

using namespace psl;

extern "C" psl_status psl_physics_init(const psl_physics *phys,
                                       void *d_tables, void *stream) {
    PSL_REQUIRE(phys && d_tables, "NULL argument");
    PSL_REQUIRE(phys->p_cut > 0 && phys->t_cut > 0 && phys->e_max > phys->p_cut &&
                    phys->e_max > phys->t_cut,
                "need 0 < cut-offs < e_max");
    PSL_REQUIRE(phys->n_e > 0 && phys->I_eV > 0 && phys->X0 > 0 &&
                    phys->step > 0,
                "physics constants must be positive");
    std::vector<float> blk(PSL_TABLE_BYTES / 4, 0.0f);
    TableHeader *H = reinterpret_cast<TableHeader *>(blk.data());
    float *mu = blk.data() + kTabHeaderBytes / 4;
    float *rng = mu + kTabMu;
    float *inv = rng + kTabRange;
    const double emax = phys->e_max * 1.02;
    // attenuation per unit density on ln E
    double lo = std::log(phys->p_cut * 0.5), hi = std::log(emax);
    double d = (hi - lo) / (kTabMu - 1);
    for (int i = 0; i < kTabMu; ++i)
        mu[i] = (float)(phys->n_e * kn_sigma_cm2(std::exp(lo + i * d)));
    H->n_mu = kTabMu;
    H->mu_lnE0 = (float)lo;
    H->mu_inv_dlnE = (float)(1.0 / d);
    // residual range above t_cut on ln T
    double rlo = std::log(phys->t_cut);
    double rd = (hi - rlo) / (kTabRange - 1);
    std::vector<double> Tn(kTabRange), R(kTabRange);
    R[0] = 0.0;
    Tn[0] = phys->t_cut;
    for (int i = 1; i < kTabRange; ++i) {
        Tn[i] = std::exp(rlo + i * rd);
        R[i] = R[i - 1] + inv_s_integral(Tn[i - 1], Tn[i], phys->n_e,
                                         phys->I_eV);
    }
    for (int i = 0; i < kTabRange; ++i) rng[i] = (float)R[i];
    H->n_rng = kTabRange;
    H->rng_lnT0 = (float)rlo;
    H->rng_inv_dlnT = (float)(1.0 / rd);
    // energy on residual range, uniform in range; Newton on the exact
    // integral from the bracketing node
    const double rmax = R[kTabRange - 1];
    const double dr = rmax / (kTabInv - 1);
    int j = 0;
    for (int i = 0; i < kTabInv; ++i) {
        double r = i * dr;
        while (j + 1 < kTabRange - 1 && R[j + 1] < r) ++j;
        double f = (r - R[j]) / (R[j + 1] - R[j]);
        double T = std::exp(std::log(Tn[j]) + f * rd);
        for (int it = 0; it < 3; ++it) {
            double rt = R[j] + (T > Tn[j] ? inv_s_integral(Tn[j], T, phys->n_e,
                                                           phys->I_eV)
                                          : 0.0);
            T += (r - rt) * bethe_mass_stopping(T, phys->n_e, phys->I_eV);
        }
        inv[i] = (float)(i == 0 ? phys->t_cut : T);
    }
    H->n_inv = kTabInv;
    H->inv_r0 = 0.0f;
    H->inv_inv_dr = (float)(1.0 / dr);
    H->t_cut = (float)phys->t_cut;
    H->p_cut = (float)phys->p_cut;
    H->r_max = (float)rmax;
    H->e_max = (float)emax;
    if (psl_status s = check_device()) return s;
    PSL_HIP(hipMemcpyAsync(d_tables, blk.data(), PSL_TABLE_BYTES,
                           hipMemcpyHostToDevice, (hipStream_t)stream));
    PSL_HIP(hipStreamSynchronize((hipStream_t)stream));
    return PSL_OK;
}

extern "C" size_t transport_batch_workspace_bytes(const psl_queue *q) {
    if (!q) return 0;
    return carve_transport(nullptr, q->ph.capacity, kMaxGridBlocks).bytes;
}

extern "C" psl_status transport_batch(psl_queue *q, const psl_phantom *ph,
                                      const psl_physics *phys,
                                      const void *d_tables, uint64_t seed,
                                      psl_dose_acc *acc, psl_stats *d_stats,
                                      const psl_launch *launch, void *d_ws,
                                      size_t ws_bytes, void *stream) {
    PSL_REQUIRE(q && ph && phys && d_tables && acc && d_stats,
                "NULL argument");
    psl_status s = validate_queue(q);
    if (s) return s;
    PSL_REQUIRE(ph->nx > 0 && ph->ny > 0 && ph->nz > 0 && ph->density,
                "bad phantom");
    PSL_REQUIRE((int64_t)ph->nx * ph->ny * ph->nz < ((int64_t)1 << 40),
                "phantom too large");
    PSL_REQUIRE(ph->dx > 0 && ph->dy > 0 && ph->dz > 0, "bad voxel size");
    PSL_REQUIRE(ph->rho_max > 0, "rho_max must be positive (and >= every "
                                 "voxel density)");
    PSL_REQUIRE(acc->data, "NULL dose accumulator");
    PSL_REQUIRE(acc->mode == PSL_ACC_F64 ||
                    (acc->mode == PSL_ACC_FIXED64 && acc->frac_bits >= 16 &&
                     acc->frac_bits <= 40),
                "bad accumulator mode %d / frac_bits %d", acc->mode,
                acc->frac_bits);
    PSL_REQUIRE(phys->t_cut > 0 && phys->p_cut > 0 && phys->step > 0 &&
                    phys->X0 > 0,
                "bad physics constants");
    psl_launch L{kBlock, 8, 0, 0};
    if (launch) {
        PSL_REQUIRE(launch->block == kBlock,
                    "block must be %d in this build", kBlock);
        PSL_REQUIRE(launch->blocks_per_cu >= 1 && launch->blocks_per_cu <= 64,
                    "blocks_per_cu outside 1..64");
        PSL_REQUIRE(launch->n_cu >= 0 && launch->n_cu <= 1024,
                    "n_cu outside 0..1024");
        L = *launch;
    }
    if (!d_ws || ws_bytes < transport_batch_workspace_bytes(q)) {
        set_error("workspace %zu bytes < %zu required", ws_bytes,
                  transport_batch_workspace_bytes(q));
        return PSL_ENOSPC;
    }
    if ((s = check_device())) return s;
    const int cu = L.n_cu > 0 ? L.n_cu : device_cu_count();
    const int blocks = std::min(cu * L.blocks_per_cu, kMaxGridBlocks);
    hipStream_t st = (hipStream_t)stream;
    TransportWs w = carve_transport(d_ws, q->ph.capacity, kMaxGridBlocks);
    PhDev P{ph->nx, ph->ny, ph->nz, (float)ph->x0, (float)ph->y0,
            (float)ph->z0, (float)ph->dx, (float)ph->dy, (float)ph->dz,
            (float)(1.0 / ph->dx), (float)(1.0 / ph->dy),
            (float)(1.0 / ph->dz), ph->rho_max, ph->density};
    PhysDev Y{(float)phys->step, (float)phys->p_cut, (float)phys->t_cut,
              (float)phys->X0, 0.0f, phys->flags};
    Items iph{q->ph, 1, q->ph.capacity, q->d_counts};
    Items iel{q->el, q->n_ebuckets, q->el.capacity / q->n_ebuckets,
              q->d_counts};
    uint32_t *work_ph = w.work;
    uint32_t *work_el = w.work + kParts * kPartStride;
    uint32_t *spill_n = w.work + 2 * kParts * kPartStride;
    SecSlots sec{w.sec, w.spill_cap, spill_n};
    QueueRegions qr{q->ph, q->el, 1 + q->n_ebuckets,
                    q->el.capacity / q->n_ebuckets, q->d_counts};
    const float *tab = static_cast<const float *>(d_tables);
    const double scale =
        acc->mode == PSL_ACC_FIXED64 ? std::ldexp(1.0, acc->frac_bits) : 1.0;
    const bool fixed = acc->mode == PSL_ACC_FIXED64;
    dim3 grid((unsigned)blocks), block(kBlock);
    hipLaunchKernelGGL(k_transport_init, dim3(256), dim3(256), 0, st, w.work,
                       2 * kParts * kPartStride + 64, w.sec.code,
                       w.spill_cap);
    {
        ProfScope prof(PSL_PROF_PHOTONS, st);
        if (fixed)
            hipLaunchKernelGGL(k_photons<PSL_ACC_FIXED64>, grid, block, 0, st,
                               iph, sec, *q, P, Y, tab, seed, acc->data,
                               scale, work_ph, w.part);
        else
            hipLaunchKernelGGL(k_photons<PSL_ACC_F64>, grid, block, 0, st,
                               iph, sec, *q, P, Y, tab, seed, acc->data,
                               scale, work_ph, w.part);
    }
    {
        ProfScope prof(PSL_PROF_REBUCKET, st);
        if ((s = compact_slots(w.sec, w.n_slots, q->d_counts, kSecPerPhoton,
                               w.spill_cap, qr, w.tiles, st)))
            return s;
    }
    {
        ProfScope prof(PSL_PROF_ELECTRONS, st);
        if (fixed)
            hipLaunchKernelGGL(k_electrons<PSL_ACC_FIXED64>, grid, block, 0,
                               st, iel, P, Y, tab, seed, acc->data, scale,
                               work_el, w.part + (int64_t)blocks * kStatWords);
        else
            hipLaunchKernelGGL(k_electrons<PSL_ACC_F64>, grid, block, 0, st,
                               iel, P, Y, tab, seed, acc->data, scale,
                               work_el, w.part + (int64_t)blocks * kStatWords);
    }
    if ((s = stats_reduce(w.part, 2 * blocks, d_stats, st))) return s;
    hipLaunchKernelGGL(k_consume, dim3(1), dim3(64), 0, st, q->d_counts);
    PSL_LAUNCHED();
    return PSL_OK;
}
