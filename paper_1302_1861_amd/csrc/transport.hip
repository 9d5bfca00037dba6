// transport_batch and psl_physics_init: photon and electron transport with
// per-voxel energy tallies.
//
// Both transport kernels run a persistent grid in which every lane owns one
// particle at a time and refills itself as soon as its particle is done:
// the lanes that need work claim a contiguous run of queue items with one
// atomic per wave on one of 64 counters that split the queue, so waves stay
// full however unequal particle lifetimes are.
//
//   k_photons    Woodcock free flights against rho_max; the Compton energy
//                fraction from an inverse-CDF table of the Klein-Nishina
//                distribution (normalised to its support, in LDS), so one
//                random block drives a whole flight-and-scatter step;
//                recoil electrons above the cut-off go into 64-slot chunks
//                of a pool; each wave keeps one open chunk per energy
//                bucket and tags the chunks it claims (from partitioned
//                counters) with their bucket; the attenuation and Compton
//                tables are staged in LDS.
//   rebucket     (optional) lists the pool's chunks by bucket (one block per
//                claim partition).
//   k_electrons  CSDA steps split at voxel faces; the energy after each
//                piece comes from the residual-range table and its inverse
//                in LDS; deposits into one voxel are merged before the
//                atomic; Highland deflection after each step.  Work is the
//                per bucket from the highest energy down: the source
//                electrons of the bucket, then its listed chunks (or, when
//                not re-bucketed, all source electrons, then the pool).
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

// Klein-Nishina density of the energy fraction eps = E'/E on [eps0, 1],
// unnormalised: eps + 1/eps - sin^2(theta), with 1 - cos(theta) =
// (1 - eps) / (eps k), k = E / m_e c^2.
double kn_eps_density(double eps, double k) {
    const double s = (1.0 - eps) / (eps * k);
    return eps + 1.0 / eps - s * (2.0 - s);
}

// Row of the inverse CDF at energy E, in the normalised variable
// t = (eps - eps0) / (1 - eps0) at quantiles u_m = m / (kKnQ - 1): the CDF
// on a fine grid by Simpson's rule per cell, inverted by linear
// interpolation within the cell.
void kn_inverse_cdf_row(double E, float *row) {
    const double me = 0.51099895, k = E / me, e0 = 1.0 / (1.0 + 2.0 * k);
    constexpr int n = 1 << 14;
    std::vector<double> C(n + 1, 0.0);
    const double h = (1.0 - e0) / n;
    for (int i = 0; i < n; ++i) {
        const double a = e0 + i * h, b = a + h;
        C[i + 1] = C[i] + h / 6.0 *
                              (kn_eps_density(a, k) +
                               4.0 * kn_eps_density(0.5 * (a + b), k) +
                               kn_eps_density(b, k));
    }
    int j = 0;
    for (int m = 0; m < kKnQ; ++m) {
        const double target = C[n] * m / (kKnQ - 1);
        while (j < n - 1 && C[j + 1] < target) ++j;
        const double f = C[j + 1] > C[j] ? (target - C[j]) / (C[j + 1] - C[j])
                                         : 0.0;
        const double t = (j + std::min(std::max(f, 0.0), 1.0)) / n;
        row[m] = (float)(m == 0 ? 0.0 : (m == kKnQ - 1 ? 1.0 : t));
    }
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
    float rho_max, rho_min;
    const float *rho;
};

struct PhysDev {
    float step, p_cut, t_cut, X0;
    int flags;
};

__device__ __forceinline__ float lerp_tab(const float *t, int n, float x) {
    x = fminf(fmaxf(x, 0.0f), (float)(n - 1) - 1e-3f);
    int i = (int)x;
    float f = x - (float)i;
    return t[i] + f * (t[i + 1] - t[i]);
}

// One deposit of e x wt in voxel v.  In PSL_ACC_TRACE mode `scale` holds the
// trace capacity and the voxel index is recorded instead: the lanes of the
// wave that deposit here take consecutive entries (one counter update per
// wave), so the trace keeps the order in which waves issue their deposits.
template <int MODE>
__device__ __forceinline__ void tally(void *acc, int64_t v, float e, float wt,
                                      double scale, uint32_t &n_dep) {
    ++n_dep;
    if (MODE == PSL_ACC_TRACE) {
        const uint64_t active = __ballot(1);
        const int lane = (int)__lane_id();
        const int leader = __ffsll((unsigned long long)active) - 1;
        const uint32_t rank = (uint32_t)__popcll(
            active & ((lane ? ~0ull >> (64 - lane) : 0ull)));
        unsigned long long base = 0;
        if (lane == leader)
            base = atomicAdd(reinterpret_cast<unsigned long long *>(acc),
                             (unsigned long long)__popcll(active));
        base = __shfl(base, leader);
        const uint64_t i = base + rank;
        if (i < (uint64_t)scale)
            (reinterpret_cast<uint32_t *>(acc) + 2)[i] = (uint32_t)v;
    } else if (MODE == PSL_ACC_FIXED64) {
        // the product of two floats is exact in double; rounded to the
        // nearest step, ties to even (rounding ties up biased the sum:
        // sub-p_cut photon deposits at weight 1/4 are exact halves half of
        // the time); two's complement, so a negative value subtracts
        const double q = __builtin_rint((double)e * (double)wt * scale);
        atomicAdd(reinterpret_cast<unsigned long long *>(acc) + v,
                  (unsigned long long)(long long)q);
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
        float s = sqrtf(s2), is = 1.0f / s;
        nu = u * ct + st * (u * w * cp - v * sp) * is;
        nv = v * ct + st * (v * w * cp + u * sp) * is;
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

// ---------------------------------------------------------- work claims ---
// Items [0, n) are split into kParts contiguous partitions with one
// counter each (kPartStride apart).  A wave asks for `want` items from its
// current partition; it gets a contiguous run [*base, *base + got) of at
// most `want`, or moves to the next partition when the current one is
// drained.  Returns false once all partitions are drained.  Wave-uniform.
__device__ __forceinline__ bool claim_items(uint32_t *ctr, int64_t n,
                                            int want, int &part, int &tried,
                                            int64_t &base, int &got) {
    const int64_t len = (n + kParts - 1) / kParts;
    while (tried < kParts) {
        const int64_t p0 = (int64_t)part * len;
        const int64_t p1 = p0 + len < n ? p0 + len : n;
        uint32_t old = 0;
        if (__lane_id() == 0 && p0 < p1)
            old = atomicAdd(&ctr[part * kPartStride], (uint32_t)want);
        old = __shfl(old, 0);
        const int64_t b = p0 + old;
        if (p0 < p1 && b < p1) {
            base = b;
            got = (int)((p1 - b) < want ? (p1 - b) : want);
            return true;
        }
        part = (part + 1) % kParts;
        ++tried;
    }
    return false;
}

// Secondary electrons: a pool of 64-slot chunks claimed per wave from kParts
// partitions of the chunk space.  A wave keeps one open chunk per electron
// energy bucket and tags each chunk it claims with that bucket, so the
// secondaries arrive already bucketed: listing the chunks of each bucket
// replaces moving the particles.
// A secondary in the pool: one 48-byte record, written with three 16-byte
// stores by the lane that creates it and read back the same way, so that
// the lines of a partly filled chunk hold whole records instead of a few
// values of ten separate columns.
struct alignas(16) SecRec {
    float E, x, y, z, u, v, w, wt;
    uint64_t uid;
    uint32_t ctr, pad;
};
static_assert(sizeof(SecRec) == 48, "three 16-byte stores");

struct SecStream {
    Slots s;                 // s.code and s.p.capacity (records in rec)
    SecRec *rec;
    int64_t n_chunks;
    uint32_t *chunk_ctr;     // kParts counters, kPartStride apart
    uint32_t *chunks_used;   // number of chunks claimed (max index + 1),
                             // set by k_chunks_used after the photons
    uint8_t *chunk_bucket;   // bucket of each claimed chunk (kEmpty: none)
};

// A fresh chunk index for the wave, or -1 once the pool is exhausted.
// Wave-uniform; `part` and `tried` are the wave's partition cursor.
__device__ __forceinline__ int64_t new_chunk(const SecStream &S, int &part,
                                             int &tried) {
    const int64_t len = (S.n_chunks + kParts - 1) / kParts;
    while (tried < kParts) {
        const int64_t p0 = (int64_t)part * len;
        const int64_t p1 = p0 + len < S.n_chunks ? p0 + len : S.n_chunks;
        uint32_t old = 0;
        if (__lane_id() == 0 && p0 < p1)
            old = atomicAdd(&S.chunk_ctr[part * kPartStride], 1u);
        old = __shfl(old, 0);
        if (p0 + (int64_t)old < p1) return p0 + old;
        part = (part + 1) % kParts;
        ++tried;
    }
    return -1;
}

// Reserves one slot for each lane with `want` in the wave's open chunk of
// its bucket b (cursors cb[b], cf[b] in LDS: chunk index or -1, slots
// used); -1 when the pool is full.  Lanes of one bucket are served together,
// one bucket per pass.
__device__ __forceinline__ int64_t sec_reserve(const SecStream &S,
                                               int32_t *cb, int32_t *cf,
                                               int &part, int &tried,
                                               bool want, int b) {
    const int lane = __lane_id();
    uint64_t pend = __ballot(want);
    int64_t slot = -1;
    while (pend) {
        const int bb = __shfl(b, __ffsll((unsigned long long)pend) - 1);
        const uint64_t grp = __ballot(want && b == bb) & pend;
        const int cnt = __popcll(grp);
        const int rank = __popcll(grp & lanemask_lt());
        const bool mine = (grp >> lane) & 1ull;
        int32_t base = cb[bb], fill = cf[bb];
        const int left = base >= 0 ? 64 - fill : 0;
        if (cnt <= left) {
            if (mine) slot = (int64_t)base * 64 + fill + rank;
            fill += cnt;
        } else {
            if (mine && rank < left) slot = (int64_t)base * 64 + fill + rank;
            const int64_t nc = new_chunk(S, part, tried);
            if (nc >= 0) {
                if (lane == 0) S.chunk_bucket[nc] = (uint8_t)bb;
                if (mine && rank >= left) slot = nc * 64 + (rank - left);
            }
            base = (int32_t)nc;
            fill = cnt - left;
        }
        if (lane == 0) {
            cb[bb] = base;
            cf[bb] = fill;
        }
        pend &= ~grp;
    }
    return slot;
}

// ---------------------------------------------------------------- photons -
// Lanes are refilled once at least this many are idle.  Vector-memory
// operations retire in issue order, so the wait for refill loads is also a
// wait for the wave's earlier dose atomics and stores; refilling in bursts
// pays that wait on fewer iterations.
#ifndef PSL_PHOTON_REFILL_MIN
#define PSL_PHOTON_REFILL_MIN 24
#endif
constexpr int kRefillMin = PSL_PHOTON_REFILL_MIN;
template <int MODE>
__global__ void __launch_bounds__(kBlock, 5)
k_photons(psl_particles ph, const uint32_t *__restrict__ counts,
          SecStream sec, psl_queue qcfg, PhDev P, PhysDev Y,
          const float *__restrict__ tables, uint64_t seed, void *acc,
          double scale, uint32_t *work, uint64_t *part) {
    __shared__ float s_mu[kTabMu];
    __shared__ float s_kn[kKnE * kKnQ];
    __shared__ float s_bk[PSL_MAX_QBUCKETS + 1];
    __shared__ uint64_t s_red[(kBlock / 64) * kStatWords];
    __shared__ int32_t s_cb[kBlock / 64][PSL_MAX_QBUCKETS];   // open chunks
    __shared__ int32_t s_cf[kBlock / 64][PSL_MAX_QBUCKETS];
    const TableHeader H = *reinterpret_cast<const TableHeader *>(tables);
    const float *gmu = tables + kTabHeaderBytes / 4;
    for (int i = threadIdx.x; i < kTabMu; i += kBlock) s_mu[i] = gmu[i];
    const float *gkn = gmu + kTabMu + kTabRange + kTabInv;
    for (int i = threadIdx.x; i < kKnE * kKnQ; i += kBlock) s_kn[i] = gkn[i];
    if (threadIdx.x <= PSL_MAX_QBUCKETS)
        s_bk[threadIdx.x] = qcfg.e_bucket_edges[threadIdx.x];
    if (threadIdx.x < (kBlock / 64) * PSL_MAX_QBUCKETS) {
        (&s_cb[0][0])[threadIdx.x] = -1;
        (&s_cf[0][0])[threadIdx.x] = 0;
    }
    __syncthreads();
    const int64_t n = (int64_t)counts[0];
    const int wave = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    uint32_t c_int = 0, c_sec = 0, c_fl = 0, c_run = 0, c_lost = 0, c_dep = 0;
    double e_esc = 0.0, e_killed = 0.0;
    int part_i = wave % kParts, tried = 0;
    bool more = true;
    // photons claimed by this wave but not yet given to a lane: the run
    // [pend_b, pend_b + pend_n) (wave-uniform)
    int64_t pend_b = 0;
    int pend_n = 0;
    int32_t *cb = s_cb[threadIdx.x >> 6], *cf = s_cf[threadIdx.x >> 6];
    int sec_part = wave % kParts, sec_tried = 0;
    bool alive = false;
    float E = 0, x = 0, y = 0, z = 0, u = 0, v = 0, w = 0, wt = 0, mu1 = 0;
    uint64_t uid = 0;
    int flights = 0;
    Rng rng;
    rng.init(seed, 0, 0u, 0u, 0u);
    for (;;) {
        // refill the lanes whose photon is done: first from the pending
        // run, then from a fresh claim of 64 (one atomic per several
        // iterations instead of one per iteration)
        const uint64_t need = __ballot(!alive);
        if (need && (pend_n > 0 || more) &&
            (__popcll(need) >= kRefillMin || need == ~0ull)) {
            const int n_need = __popcll(need);
            int64_t nb = 0;
            int ng = 0;
            if (pend_n < n_need && more) {
                more = claim_items(work, n, 64, part_i, tried, nb, ng);
                if (!more) ng = 0;
            }
            const int rank = __popcll(need & lanemask_lt());
            int64_t i = -1;
            if (rank < pend_n)
                i = pend_b + rank;
            else if (rank - pend_n < ng)
                i = nb + (rank - pend_n);
            const int used = min(n_need, pend_n + ng);
            if (used <= pend_n) {
                pend_b += used;
                pend_n -= used;
            } else {
                pend_b = nb + (used - pend_n);
                pend_n = ng - (used - pend_n);
            }
            if (!alive && i >= 0) {
                E = ph.E[i]; x = ph.x[i]; y = ph.y[i]; z = ph.z[i];
                u = ph.u[i]; v = ph.v[i]; w = ph.w[i]; wt = ph.wt[i];
                uid = ph.uid[i];
                const uint32_t c0 = ph.ctr[i];
                // retire the refill loads here (vmcnt 0; expcnt and lgkmcnt
                // left at their maxima), so that no load into the lane's
                // state is outstanding at the loop's back edge, where a
                // conservative wait would also wait for every store and
                // atomic of the iteration
                __builtin_amdgcn_s_waitcnt(0x0F70);
                rng.init(seed, uid, 0u, 0u, c0);
                mu1 = lerp_tab(s_mu, kTabMu,
                               (__logf(E) - H.mu_lnE0) * H.mu_inv_dlnE);
                flights = 0;
                alive = true;
            }
        }
        if (!__ballot(alive)) {
            if (!more && pend_n == 0) break;
            continue;
        }
        bool push_e = false;
        float Te = 0, eu = 0, ev = 0, ew = 0;
        uint32_t birth = 0;
        if (alive && E < Y.p_cut) {
            int ix, iy, iz;
            if (voxel_of(P, x, y, z, ix, iy, iz))
                tally<MODE>(acc, ((int64_t)iz * P.ny + iy) * P.nx + ix, E, wt,
                            scale, c_dep);
            else
                e_esc += (double)E * wt;
            alive = false;
        }
        if (alive) {
            // one free flight against the majorant
            const u32x4 rf = rng.draw();
            const float s = -__logf(u01(rf.x)) / (mu1 * P.rho_max);
            x += s * u; y += s * v; z += s * w;
            ++c_fl;
            int ix, iy, iz;
            if (!voxel_of(P, x, y, z, ix, iy, iz)) {
                e_esc += (double)E * wt;
                alive = false;
            } else {
                const int64_t vox = ((int64_t)iz * P.ny + iy) * P.nx + ix;
                if (++flights > kMaxFlights) {
                    ++c_run;
                    tally<MODE>(acc, vox, E, wt, scale, c_dep);
                    alive = false;
                } else if (const float xi = u01(rf.y) * P.rho_max;
                           xi <= P.rho_min || xi <= P.rho[vox]) {
                    // (rho_min <= every density: the first test implies
                    // the second and spares the gather)
                    // Compton: eps = E'/E from the inverse CDF (bilinear
                    // in ln E and the quantile), then the exact kinematics
                    const float k = E / kME;
                    const float e0 = 1.0f / (1.0f + 2.0f * k);
                    float fe = (__logf(E) - H.kn_lnE0) * H.kn_inv_dlnE;
                    fe = fminf(fmaxf(fe, 0.0f), (float)(kKnE - 1) - 1e-3f);
                    const int ie = (int)fe;
                    const float we = fe - (float)ie;
                    const float fq = u01(rf.z) * (float)(kKnQ - 1);
                    const int iq = min((int)fq, kKnQ - 2);
                    const float wq = fq - (float)iq;
                    const float *r0 = s_kn + ie * kKnQ + iq;
                    const float *r1 = r0 + kKnQ;
                    const float t0 = r0[0] + wq * (r0[1] - r0[0]);
                    const float t1 = r1[0] + wq * (r1[1] - r1[0]);
                    const float t = t0 + we * (t1 - t0);
                    const float eps = e0 + t * (1.0f - e0);
                    const float onecost = (1.0f - eps) / (eps * k);
                    const float sint2 = onecost * (2.0f - onecost);
                    const float phi_u = u01(rf.w);
                    ++c_int;
                    const float cost = 1.0f - onecost;
                    const float sint = sqrtf(fmaxf(sint2, 0.0f));
                    float sp, cp;
                    __sincosf(2.0f * kPI * phi_u, &sp, &cp);
                    const float Es = eps * E;
                    const float T = E - Es;
                    const float pu = u, pv = v, pw = w;
                    rotate(u, v, w, cost, sint, cp, sp);
                    if (T > Y.t_cut && !(Y.flags & PSL_FLAG_FIRST_COLLISION)) {
                        const float qx = E * pu - Es * u, qy = E * pv - Es * v,
                                    qz = E * pw - Es * w;
                        const float rq = rsqrtf(qx * qx + qy * qy + qz * qz);
                        push_e = true;
                        Te = T;
                        eu = qx * rq; ev = qy * rq; ew = qz * rq;
                        birth = rng.n;
                    } else {
                        tally<MODE>(acc, vox, T, wt, scale, c_dep);
                    }
                    if (Y.flags & PSL_FLAG_FIRST_COLLISION) {
                        e_killed += (double)Es * wt;
                        alive = false;
                    } else {
                        E = Es;
                        mu1 = lerp_tab(s_mu, kTabMu,
                                       (__logf(E) - H.mu_lnE0) * H.mu_inv_dlnE);
                    }
                }
            }
        }
        // recoil electrons into the wave's open chunk of their bucket
        int b = 0;
        if (push_e)
            for (int j = 1; j < qcfg.n_ebuckets; ++j)
                if (Te >= s_bk[j]) b = j;
        const int64_t slot =
            sec_reserve(sec, cb, cf, sec_part, sec_tried, push_e, b);
        if (push_e) {
            if (slot >= 0) {
                SecRec r;
                r.E = Te; r.x = x; r.y = y; r.z = z;
                r.u = eu; r.v = ev; r.w = ew; r.wt = wt;
                r.uid = uid; r.ctr = birth; r.pad = 0u;
                const uint4 *q = reinterpret_cast<const uint4 *>(&r);
                uint4 *d = reinterpret_cast<uint4 *>(sec.rec + slot);
                d[0] = q[0]; d[1] = q[1]; d[2] = q[2];
                sec.s.code[slot] = (uint8_t)(1 + b);
                ++c_sec;
            } else {
                ++c_lost;
            }
        }
    }
    StatAcc st;
    st.zero();
    st.add(PSL_STAT(interactions), c_int);
    st.add(PSL_STAT(secondaries), c_sec);
    st.add(PSL_STAT(flights), c_fl);
    st.add(PSL_STAT(runaway), c_run);
    st.add(PSL_STAT(lost), c_lost);
    st.add(PSL_STAT(photon_deposits), c_dep);
    st.addf(PSL_STAT(e_escaped), e_esc);
    st.addf(PSL_STAT(e_killed), e_killed);
    block_stats_write(st, s_red, part);
}

// -------------------------------------------------------------- electrons -
// Work list: the electron bucket regions from the highest bucket down, then
// (optionally) a raw stream of slots whose empty entries are skipped.
struct ElWork {
    psl_particles el;
    int32_t n_b;
    int64_t cap_b;
    const uint32_t *counts;
    Slots sec;                  // secondary chunk pool (code kEmpty: hole)
    const SecRec *rec;          // its records
    const uint32_t *sec_chunks; // chunks used in the pool
    // bucketed: per bucket, the pool chunks tagged with it (list_off[b],
    // list_cnt[b] into list); otherwise the pool in claim order
    int bucketed;
    const int32_t *list;
    const uint32_t *list_off, *list_cnt;
};

template <int MODE>
__global__ void __launch_bounds__(kBlock, 5)
k_electrons(ElWork W, PhDev P, PhysDev Y, const float *__restrict__ tables,
            uint64_t seed, void *acc, double scale, uint32_t *work,
            uint64_t *part) {
    __shared__ float s_rng[kTabRange];
    __shared__ float s_inv[kTabInv];
    __shared__ uint64_t s_red[(kBlock / 64) * kStatWords];
    // work segments in processing order, buckets from high to low energy:
    // bucketed -- (source electrons of b, secondary chunks of b) per bucket;
    // otherwise -- source electrons of every bucket, then the whole pool
    __shared__ int64_t s_cnt[2 * PSL_MAX_QBUCKETS + 1];
    const TableHeader H = *reinterpret_cast<const TableHeader *>(tables);
    const float *g = tables + kTabHeaderBytes / 4 + kTabMu;
    for (int i = threadIdx.x; i < kTabRange; i += kBlock) s_rng[i] = g[i];
    for (int i = threadIdx.x; i < kTabInv; i += kBlock)
        s_inv[i] = g[kTabRange + i];
    const int n_seg = W.bucketed ? 2 * W.n_b : W.n_b + 1;
    if (threadIdx.x < n_seg) {
        const int sg = threadIdx.x;
        int64_t c = 0;
        if (W.bucketed) {
            const int b = W.n_b - 1 - sg / 2;
            if (sg % 2 == 0) {
                c = (int64_t)W.counts[1 + b];
                c = c < W.cap_b ? c : W.cap_b;
            } else {
                c = (int64_t)W.list_cnt[b] * 64;
            }
        } else if (sg < W.n_b) {
            const int b = W.n_b - 1 - sg;
            c = (int64_t)W.counts[1 + b];
            c = c < W.cap_b ? c : W.cap_b;
        } else {
            c = (int64_t)(*W.sec_chunks) * 64;
        }
        s_cnt[sg] = c;
    }
    __syncthreads();
    int64_t total = 0;
    for (int sg = 0; sg < n_seg; ++sg) total += s_cnt[sg];
    const int wave = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    uint32_t c_seg = 0, c_run = 0, c_dep = 0;
    double e_esc = 0.0;
    int part_i = wave % kParts, tried = 0;
    bool more = true;
    int64_t pend_b = 0;   // claimed, not yet given to a lane (wave-uniform)
    int pend_n = 0;
    // the lane's electron
    bool alive = false;
    float T = 0, x = 0, y = 0, z = 0, u = 0, v = 0, w = 0, wt = 0;
    float r = 0;        // residual CSDA range, g/cm^2
    float pe = 0;       // energy deposited in voxel pv, not yet tallied
    float rho_v = 0;    // density of voxel vox
    int ix = 0, iy = 0, iz = 0, segs = 0;
    uint32_t vox = 0, pv = 0;   // voxel indices (< 2^32)
    Rng rng;
    rng.init(seed, 0, 0u, 0u, 0u);
    // Lanes whose electron has ended take a new one between steps, so a
    // wave is not held by its longest track while the deflection code
    // still runs for all live lanes together.
    for (;;) {
        const uint64_t need = __ballot(!alive);
        if (need && (pend_n > 0 || more)) {
            const int n_need = __popcll(need);
            int64_t nb = 0;
            int ng = 0;
            if (pend_n < n_need && more) {
                more = claim_items(work, total, 64, part_i, tried, nb, ng);
                if (!more) ng = 0;
            }
            const int rank = __popcll(need & lanemask_lt());
            int64_t it = -1;
            if (rank < pend_n)
                it = pend_b + rank;
            else if (rank - pend_n < ng)
                it = nb + (rank - pend_n);
            const int used = min(n_need, pend_n + ng);
            if (used <= pend_n) {
                pend_b += used;
                pend_n -= used;
            } else {
                pend_b = nb + (used - pend_n);
                pend_n = ng - (used - pend_n);
            }
            if (!alive && it >= 0) {
                int64_t t = it;
                int sgi = 0;
                while (t >= s_cnt[sgi]) { t -= s_cnt[sgi]; ++sgi; }
                int64_t i;
                bool ok = true;
                uint64_t p_uid = 0;
                uint32_t p_ctr = 0;
                const bool dense = W.bucketed ? sgi % 2 == 0 : sgi < W.n_b;
                if (dense) {
                    const int b = W.n_b - 1 - (W.bucketed ? sgi / 2 : sgi);
                    i = (int64_t)b * W.cap_b + t;
                    T = W.el.E[i];
                    x = W.el.x[i]; y = W.el.y[i]; z = W.el.z[i];
                    u = W.el.u[i]; v = W.el.v[i]; w = W.el.w[i];
                    wt = W.el.wt[i];
                    p_uid = W.el.uid[i];
                    p_ctr = W.el.ctr[i];
                } else {
                    if (W.bucketed) {
                        const int b = W.n_b - 1 - sgi / 2;
                        i = (int64_t)W.list[W.list_off[b] + t / 64] * 64 +
                            t % 64;
                    } else {
                        i = t;
                    }
                    ok = W.sec.code[i] != kEmpty;
                    if (ok) {
                        const uint4 *q =
                            reinterpret_cast<const uint4 *>(W.rec + i);
                        const uint4 a = q[0], bq = q[1], cq = q[2];
                        T = __uint_as_float(a.x);
                        x = __uint_as_float(a.y);
                        y = __uint_as_float(a.z);
                        z = __uint_as_float(a.w);
                        u = __uint_as_float(bq.x);
                        v = __uint_as_float(bq.y);
                        w = __uint_as_float(bq.z);
                        wt = __uint_as_float(bq.w);
                        p_uid = (uint64_t)cq.x | ((uint64_t)cq.y << 32);
                        p_ctr = cq.z;
                    }
                }
                if (ok) {
                    // entry voxel; a point on the box surface belongs to
                    // the voxel inside
                    ix = (int)floorf((x - P.x0) * P.ix_);
                    iy = (int)floorf((y - P.y0) * P.iy_);
                    iz = (int)floorf((z - P.z0) * P.iz_);
                    if (ix < -1 || iy < -1 || iz < -1 || ix > P.nx ||
                        iy > P.ny || iz > P.nz) {
                        e_esc += (double)T * wt;
                    } else {
                        ix = min(max(ix, 0), P.nx - 1);
                        iy = min(max(iy, 0), P.ny - 1);
                        iz = min(max(iz, 0), P.nz - 1);
                        vox = (uint32_t)(((int64_t)iz * P.ny + iy) * P.nx +
                                         ix);
                        if (T <= Y.t_cut) {
                            tally<MODE>(acc, vox, T, wt, scale, c_dep);
                        } else {
                            rng.init(seed, p_uid, p_ctr, kElectronTag, 0u);
                            r = lerp_tab(s_rng, kTabRange,
                                         (__logf(T) - H.rng_lnT0) *
                                             H.rng_inv_dlnT);
                            pv = vox;
                            pe = 0.0f;
                            segs = 0;
                            rho_v = P.rho[vox];
                            alive = true;
                        }
                    }
                }
            }
        }
        if (!__ballot(alive)) {
            if (!more && pend_n == 0) break;
            continue;
        }
        // one step of Y.step cm for every live lane, split at voxel faces
        bool done = false;
        float tm = 0.0f;
        const float T0 = T;
        if (alive) {
            // direction constants of the step: reciprocals, the side of the
            // voxel whose face comes next, the index step across it
            const float iu = u != 0.0f ? 1.0f / u : 0.0f;
            const float iv = v != 0.0f ? 1.0f / v : 0.0f;
            const float iw = w != 0.0f ? 1.0f / w : 0.0f;
            const int fu = u > 0.0f, fv = v > 0.0f, fw = w > 0.0f;
            const int su = u > 0.0f ? 1 : -1, sv = v > 0.0f ? 1 : -1,
                      sw = w > 0.0f ? 1 : -1;
            float rem = Y.step;
            while (rem > 0.0f) {
                const float sx = u != 0.0f
                    ? (P.x0 + (float)(ix + fu) * P.dx - x) * iu : INFINITY;
                const float sy = v != 0.0f
                    ? (P.y0 + (float)(iy + fv) * P.dy - y) * iv : INFINITY;
                const float sz = w != 0.0f
                    ? (P.z0 + (float)(iz + fw) * P.dz - z) * iw : INFINITY;
                int axis = 0;
                float sb = sx;
                if (sy < sb) { sb = sy; axis = 1; }
                if (sz < sb) { sb = sz; axis = 2; }
                sb = fmaxf(sb, 0.0f);
                const float seg = fminf(rem, sb);
                const float dm = rho_v * seg;
                ++c_seg;
                if (dm >= r || ++segs > kMaxSegments) {
                    if (segs > kMaxSegments) ++c_run;
                    pe += T;
                    T = 0.0f;
                    done = true;
                    break;
                }
                r -= dm;
                const float Tn =
                    fminf(lerp_tab(s_inv, kTabInv, r * H.inv_inv_dr), T);
                pe += T - Tn;
                T = Tn;
                tm += dm;
                x += seg * u; y += seg * v; z += seg * w;
                rem -= seg;
                if (seg == sb) {
                    ix += axis == 0 ? su : 0;
                    iy += axis == 1 ? sv : 0;
                    iz += axis == 2 ? sw : 0;
                    if (!((unsigned)ix < (unsigned)P.nx &&
                          (unsigned)iy < (unsigned)P.ny &&
                          (unsigned)iz < (unsigned)P.nz)) {
                        e_esc += (double)T * wt;
                        T = 0.0f;
                        done = true;
                        break;
                    }
                    vox = (uint32_t)(((int64_t)iz * P.ny + iy) * P.nx + ix);
                    // the next density is requested before the deposit of
                    // the voxel just left is sent
                    rho_v = P.rho[vox];
                    if (pe > 0.0f) tally<MODE>(acc, pv, pe, wt, scale, c_dep);
                    pv = vox;
                    pe = 0.0f;
                }
            }
        }
        if (alive && !done && !(Y.flags & PSL_FLAG_NO_MSC) && tm > 0.0f) {
            // Highland angle from the pre-step energy and the step's mass
            // thickness; space angle Rayleigh-distributed with scale
            // theta0, truncated at pi
            const float pbc = T0 * (T0 + 2.0f * kME) / (T0 + kME);
            const float qq = tm / Y.X0;
            float th0 = 13.6f / pbc * sqrtf(qq) * (1.0f + 0.038f * __logf(qq));
            th0 = fmaxf(th0, 0.0f);
            // candidates x, z, w of the first block (y is the azimuth),
            // then four per block, until one is <= pi
            u32x4 q = rng.draw();
            const float phi_u = u01(q.y);
            float th = th0 * sqrtf(-2.0f * __logf(u01(q.x)));
            if (th > kPI) th = th0 * sqrtf(-2.0f * __logf(u01(q.z)));
            if (th > kPI) th = th0 * sqrtf(-2.0f * __logf(u01(q.w)));
            for (int t = 0; t < 15 && th > kPI; ++t) {
                q = rng.draw();
                th = th0 * sqrtf(-2.0f * __logf(u01(q.x)));
                if (th > kPI) th = th0 * sqrtf(-2.0f * __logf(u01(q.y)));
                if (th > kPI) th = th0 * sqrtf(-2.0f * __logf(u01(q.z)));
                if (th > kPI) th = th0 * sqrtf(-2.0f * __logf(u01(q.w)));
            }
            if (th > kPI) th = kPI * u01(rng.draw().x);
            float sth, cth, sp, cp;
            __sincosf(th, &sth, &cth);
            __sincosf(2.0f * kPI * phi_u, &sp, &cp);
            rotate(u, v, w, cth, sth, cp, sp);
        }
        if (alive && done) {
            if (pe > 0.0f) tally<MODE>(acc, pv, pe, wt, scale, c_dep);
            alive = false;
        }
    }
    StatAcc st;
    st.zero();
    st.add(PSL_STAT(segments), c_seg);
    st.add(PSL_STAT(runaway), c_run);
    st.add(PSL_STAT(deposits), c_dep);
    st.addf(PSL_STAT(e_escaped), e_esc);
    block_stats_write(st, s_red, part);
}

// chunks_used = 1 + the highest chunk index claimed: partition p (chunks
// [p len, min((p + 1) len, n))) handed out its first min(ctr[p], its size)
// chunks.  One small kernel instead of a same-address atomic per chunk.
__global__ void k_chunks_used(const uint32_t *__restrict__ ctr,
                              int64_t n_chunks, uint32_t *__restrict__ used) {
    __shared__ uint32_t s[kParts];
    const int p = threadIdx.x;
    const int64_t len = (n_chunks + kParts - 1) / kParts;
    const int64_t p0 = (int64_t)p * len;
    const int64_t p1 = p0 + len < n_chunks ? p0 + len : n_chunks;
    uint32_t top = 0;
    if (p0 < p1) {
        const int64_t got = min((int64_t)ctr[p * kPartStride], p1 - p0);
        if (got > 0) top = (uint32_t)(p0 + got);
    }
    s[p] = top;
    __syncthreads();
    if (p == 0) {
        uint32_t m = 0;
        for (int i = 0; i < kParts; ++i) m = max(m, s[i]);
        *used = m;
    }
}

// Lists the pool chunks of each bucket.  Block p takes the chunks handed
// out by partition p (the first min(ctr[p], size) of its range).  First
// pass: counts per (partition, bucket).  Second pass: every block derives
// its offsets from the whole count table (bucket-major, partition-minor)
// and places its chunks with wave ballots.  The order within a bucket is
// irrelevant: every electron's result depends only on its own state and
// random stream.
__device__ __forceinline__ void partition_range(int64_t n_chunks, int p,
                                                const uint32_t *ctr,
                                                int64_t &a, int64_t &b) {
    const int64_t len = (n_chunks + kParts - 1) / kParts;
    a = (int64_t)p * len;
    const int64_t e = a + len < n_chunks ? a + len : n_chunks;
    b = a;
    if (a < e) b = a + min((int64_t)ctr[p * kPartStride], e - a);
}

__global__ void __launch_bounds__(256)
k_bucket_count(const uint8_t *__restrict__ tag, const uint32_t *ctr,
               int64_t n_chunks, int n_b, uint32_t *__restrict__ pcnt) {
    __shared__ uint32_t s_cnt[PSL_MAX_QBUCKETS];
    const int lane = __lane_id();
    if (threadIdx.x < PSL_MAX_QBUCKETS) s_cnt[threadIdx.x] = 0;
    __syncthreads();
    int64_t a, b;
    partition_range(n_chunks, blockIdx.x, ctr, a, b);
    for (int64_t i0 = a; i0 < b; i0 += 256) {
        const int64_t i = i0 + threadIdx.x;
        const uint32_t t = i < b ? (uint32_t)tag[i] : (uint32_t)kEmpty;
        for (int q = 0; q < n_b; ++q) {
            const uint64_t m = __ballot(t == (uint32_t)q);
            if (lane == 0 && m) atomicAdd(&s_cnt[q], (uint32_t)__popcll(m));
        }
    }
    __syncthreads();
    if (threadIdx.x < PSL_MAX_QBUCKETS)
        pcnt[blockIdx.x * PSL_MAX_QBUCKETS + threadIdx.x] = s_cnt[threadIdx.x];
}

__global__ void __launch_bounds__(256)
k_bucket_list(const uint8_t *__restrict__ tag, const uint32_t *ctr,
              int64_t n_chunks, int n_b,
              const uint32_t *__restrict__ pcnt, int32_t *__restrict__ list,
              uint32_t *__restrict__ off, uint32_t *__restrict__ cnt) {
    __shared__ uint32_t s_cur[PSL_MAX_QBUCKETS];
    __shared__ uint32_t s_p[kParts * PSL_MAX_QBUCKETS];
    const int lane = __lane_id();
    const int p = blockIdx.x;
    for (int i = threadIdx.x; i < kParts * PSL_MAX_QBUCKETS; i += 256)
        s_p[i] = pcnt[i];
    __syncthreads();
    if (threadIdx.x < PSL_MAX_QBUCKETS) {
        const int q = threadIdx.x;
        uint32_t before = 0, total_q = 0;   // earlier buckets; bucket q
        for (int pp = 0; pp < kParts; ++pp)
            for (int qq = 0; qq < n_b; ++qq) {
                const uint32_t c = s_p[pp * PSL_MAX_QBUCKETS + qq];
                if (qq < q) before += c;
                if (qq == q) {
                    total_q += c;
                    if (pp < p) before += c;
                }
            }
        s_cur[q] = before;
        if (p == 0 && q < n_b) {
            cnt[q] = total_q;
            uint32_t o = 0;
            for (int pp = 0; pp < kParts; ++pp)
                for (int qq = 0; qq < q; ++qq)
                    o += s_p[pp * PSL_MAX_QBUCKETS + qq];
            off[q] = o;
        }
    }
    __syncthreads();
    int64_t a, b;
    partition_range(n_chunks, p, ctr, a, b);
    for (int64_t i0 = a; i0 < b; i0 += 256) {
        const int64_t i = i0 + threadIdx.x;
        const uint32_t t = i < b ? (uint32_t)tag[i] : (uint32_t)kEmpty;
        for (int q = 0; q < n_b; ++q) {
            const uint64_t m = __ballot(t == (uint32_t)q);
            uint32_t base = 0;
            if (lane == 0 && m)
                base = atomicAdd(&s_cur[q], (uint32_t)__popcll(m));
            base = __shfl(base, 0);
            if (t == (uint32_t)q)
                list[base + __popcll(m & lanemask_lt())] = (int32_t)i;
        }
    }
}

__global__ void k_transport_init(uint32_t *words, int n_words,
                                 uint32_t *codes, int64_t n_code_words,
                                 uint8_t *tags, int64_t n_tags) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = threadIdx.x + (int64_t)blockIdx.x * blockDim.x;
         i < n_words; i += stride)
        words[i] = 0;
    // every slot of the secondary pool starts empty, every chunk untagged
    const uint32_t e4 = 0x01010101u * kEmpty;
    for (int64_t i = threadIdx.x + (int64_t)blockIdx.x * blockDim.x;
         i < n_code_words; i += stride)
        codes[i] = e4;
    for (int64_t i = threadIdx.x + (int64_t)blockIdx.x * blockDim.x;
         i < n_tags; i += stride)
        tags[i] = kEmpty;
}

__global__ void k_consume(uint32_t *counts, int n_b, psl_stats *stats) {
    if (threadIdx.x == 0) {
        uint32_t peak = 0;
        for (int b = 0; b < n_b; ++b) peak = max(peak, counts[1 + b]);
        if (peak > stats->bucket_peak) stats->bucket_peak = peak;
    }
    __syncthreads();
    if (threadIdx.x < PSL_QCOUNTS - 1) counts[threadIdx.x] = 0;
}

struct TransportWs {
    uint32_t *words;     // photon claims, electron claims, chunk claims,
                         // chunks used
    int n_words;
    SecStream sec;
    int32_t *list;       // pool chunks listed by bucket
    uint32_t *list_off, *list_cnt;
    uint32_t *list_pcnt; // chunks per (partition, bucket)
    uint64_t *part;
    size_t bytes;
};

constexpr int kMaxGridBlocks = 16 * 1024;

TransportWs carve_transport(void *base, int64_t ph_cap) {
    // the secondary stream holds up to 2 secondaries per queued photon
    Carver c(base);
    TransportWs w;
    w.n_words = 3 * kParts * kPartStride + 64;
    w.words = c.take<uint32_t>(w.n_words);
    // secondary stream: one slot per electron-queue entry plus one chunk per
    // wave of the largest grid for partly filled chunks
    const int64_t chunks = (std::max<int64_t>(2 * ph_cap, 64) + 63) / 64 +
                           (int64_t)kMaxGridBlocks * (kBlock / 64);
    const int64_t n = chunks * 64;
    w.sec.n_chunks = chunks;
    w.sec.s.p = psl_particles{};
    w.sec.s.p.capacity = n;
    w.sec.rec = c.take<SecRec>(n);
    w.sec.s.code = c.take<uint8_t>(n);   // n is a multiple of 64
    w.sec.chunk_bucket = c.take<uint8_t>(chunks);
    w.list = c.take<int32_t>(chunks);
    w.list_off = c.take<uint32_t>(PSL_MAX_QBUCKETS);
    w.list_cnt = c.take<uint32_t>(PSL_MAX_QBUCKETS);
    w.list_pcnt = c.take<uint32_t>((int64_t)kParts * PSL_MAX_QBUCKETS);
    w.part = c.take<uint64_t>((int64_t)2 * kMaxGridBlocks * kStatWords);
    w.bytes = c.used;
    return w;
}

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
    // Compton energy fraction: inverse CDF on ln E over [p_cut, emax]
    float *kn = inv + kTabInv;
    const double klo = std::log(phys->p_cut), khi = std::log(emax);
    const double kd = (khi - klo) / (kKnE - 1);
    for (int i = 0; i < kKnE; ++i)
        kn_inverse_cdf_row(std::exp(klo + i * kd), kn + i * kKnQ);
    H->kn_lnE0 = (float)klo;
    H->kn_inv_dlnE = (float)(1.0 / kd);
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
    if (!q || q->n_ebuckets < 1) return 0;
    return carve_transport(nullptr, q->ph.capacity).bytes;
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
    PSL_REQUIRE((int64_t)ph->nx * ph->ny * ph->nz < ((int64_t)1 << 32),
                "phantom too large (at most 2^32 - 1 voxels)");
    PSL_REQUIRE(ph->dx > 0 && ph->dy > 0 && ph->dz > 0, "bad voxel size");
    PSL_REQUIRE(ph->rho_max > 0, "rho_max must be positive (and >= every "
                                 "voxel density)");
    PSL_REQUIRE(ph->rho_min >= 0 && ph->rho_min <= ph->rho_max,
                "rho_min must lie in [0, rho_max] (and be <= every voxel "
                "density)");
    PSL_REQUIRE(acc->data, "NULL dose accumulator");
    PSL_REQUIRE(acc->mode == PSL_ACC_F64 ||
                    (acc->mode == PSL_ACC_FIXED64 && acc->frac_bits >= 16 &&
                     acc->frac_bits <= 40) ||
                    (acc->mode == PSL_ACC_TRACE && acc->trace_capacity >= 0 &&
                     acc->trace_capacity < ((int64_t)1 << 40)),
                "bad accumulator mode %d / frac_bits %d", acc->mode,
                acc->frac_bits);
    PSL_REQUIRE(phys->t_cut > 0 && phys->p_cut > 0 && phys->step > 0 &&
                    phys->X0 > 0,
                "bad physics constants");
    psl_launch L{kBlock, 4, 0, 1};
    if (launch) {
        PSL_REQUIRE(launch->block == kBlock,
                    "block must be %d in this build", kBlock);
        PSL_REQUIRE(launch->blocks_per_cu >= 1 && launch->blocks_per_cu <= 64,
                    "blocks_per_cu outside 1..64");
        PSL_REQUIRE(launch->n_cu >= 0 && launch->n_cu <= 1024,
                    "n_cu outside 0..1024");
        PSL_REQUIRE(launch->rebucket == 0 || launch->rebucket == 1,
                    "rebucket must be 0 or 1");
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
    TransportWs w = carve_transport(d_ws, q->ph.capacity);
    PhDev P{ph->nx, ph->ny, ph->nz, (float)ph->x0, (float)ph->y0,
            (float)ph->z0, (float)ph->dx, (float)ph->dy, (float)ph->dz,
            (float)(1.0 / ph->dx), (float)(1.0 / ph->dy),
            (float)(1.0 / ph->dz), ph->rho_max, ph->rho_min, ph->density};
    PhysDev Y{(float)phys->step, (float)phys->p_cut, (float)phys->t_cut,
              (float)phys->X0, phys->flags};
    uint32_t *work_ph = w.words;
    uint32_t *work_el = w.words + kParts * kPartStride;
    w.sec.chunk_ctr = w.words + 2 * kParts * kPartStride;
    w.sec.chunks_used = w.words + 3 * kParts * kPartStride;
    const int64_t cap_b = q->el.capacity / q->n_ebuckets;
    const float *tab = static_cast<const float *>(d_tables);
    const double scale =
        acc->mode == PSL_ACC_FIXED64 ? std::ldexp(1.0, acc->frac_bits)
        : acc->mode == PSL_ACC_TRACE ? (double)acc->trace_capacity
                                     : 1.0;
    const int mode = acc->mode;
    dim3 grid((unsigned)blocks), block(kBlock);
    hipLaunchKernelGGL(k_transport_init, dim3(1024), dim3(256), 0, st,
                       w.words, w.n_words,
                       reinterpret_cast<uint32_t *>(w.sec.s.code),
                       w.sec.s.p.capacity / 4, w.sec.chunk_bucket,
                       w.sec.n_chunks);
    {
        ProfScope prof(PSL_PROF_PHOTONS, st);
        if (mode == PSL_ACC_FIXED64)
            hipLaunchKernelGGL(k_photons<PSL_ACC_FIXED64>, grid, block, 0, st,
                               q->ph, q->d_counts, w.sec, *q, P, Y, tab, seed,
                               acc->data, scale, work_ph, w.part);
        else if (mode == PSL_ACC_F64)
            hipLaunchKernelGGL(k_photons<PSL_ACC_F64>, grid, block, 0, st,
                               q->ph, q->d_counts, w.sec, *q, P, Y, tab, seed,
                               acc->data, scale, work_ph, w.part);
        else
            hipLaunchKernelGGL(k_photons<PSL_ACC_TRACE>, grid, block, 0, st,
                               q->ph, q->d_counts, w.sec, *q, P, Y, tab, seed,
                               acc->data, scale, work_ph, w.part);
    }
    hipLaunchKernelGGL(k_chunks_used, dim3(1), dim3(kParts), 0, st,
                       w.sec.chunk_ctr, w.sec.n_chunks, w.sec.chunks_used);
    ElWork ew{q->el,   q->n_ebuckets, cap_b,      q->d_counts, w.sec.s,
              w.sec.rec, w.sec.chunks_used, L.rebucket, w.list,
              w.list_off, w.list_cnt};
    if (L.rebucket) {
        ProfScope prof(PSL_PROF_REBUCKET, st);
        hipLaunchKernelGGL(k_bucket_count, dim3(kParts), dim3(256), 0, st,
                           w.sec.chunk_bucket, w.sec.chunk_ctr,
                           w.sec.n_chunks, q->n_ebuckets, w.list_pcnt);
        hipLaunchKernelGGL(k_bucket_list, dim3(kParts), dim3(256), 0, st,
                           w.sec.chunk_bucket, w.sec.chunk_ctr,
                           w.sec.n_chunks, q->n_ebuckets, w.list_pcnt, w.list,
                           w.list_off, w.list_cnt);
    }
    {
        ProfScope prof(PSL_PROF_ELECTRONS, st);
        uint64_t *part_el = w.part + (int64_t)blocks * kStatWords;
        if (mode == PSL_ACC_FIXED64)
            hipLaunchKernelGGL(k_electrons<PSL_ACC_FIXED64>, grid, block, 0,
                               st, ew, P, Y, tab, seed, acc->data, scale,
                               work_el, part_el);
        else if (mode == PSL_ACC_F64)
            hipLaunchKernelGGL(k_electrons<PSL_ACC_F64>, grid, block, 0, st,
                               ew, P, Y, tab, seed, acc->data, scale, work_el,
                               part_el);
        else
            hipLaunchKernelGGL(k_electrons<PSL_ACC_TRACE>, grid, block, 0,
                               st, ew, P, Y, tab, seed, acc->data, scale,
                               work_el, part_el);
    }
    if ((s = stats_reduce(w.part, 2 * blocks, d_stats, st))) return s;
    hipLaunchKernelGGL(k_consume, dim3(1), dim3(64), 0, st, q->d_counts,
                       q->n_ebuckets, d_stats);
    PSL_LAUNCHED();
    return PSL_OK;
}
