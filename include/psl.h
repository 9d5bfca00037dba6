/*
 * psl.h - C ABI of the phase-space-let (PSL) Monte Carlo dose library for
 * AMD Instinct MI355X (gfx950).
 *
 * Method: Townson et al., "GPU-based Monte Carlo radiotherapy dose
 * calculation using phase-space sources" (gDPM v3.0), Method 3.
 *
 * Conventions for every call:
 *  - Units: cm, kinetic MeV, g/cm^3, degrees.  Beam frame: the source is at
 *    the origin, the beam runs along +z, the isocentre is at z = SAD.
 *  - Pointers named d_* and the arrays inside the structs below are DEVICE
 *    pointers unless marked "host".  The caller owns every buffer; the
 *    library never allocates or frees device memory.  Scratch memory comes
 *    from a caller-provided workspace whose size the matching
 *    *_workspace_bytes() query returns.
 *  - Calls only enqueue work on `stream` (a hipStream_t; NULL = the null
 *    stream) and return; none synchronises.  Results that the host needs
 *    (counts, statistics) are written to device memory the caller reads
 *    after synchronising.
 *  - Every call validates its arguments before enqueuing anything and
 *    returns a psl_status; on failure nothing was enqueued and
 *    psl_last_error() (thread-local) describes the problem.  No C++
 *    exception crosses this interface.
 */
#ifndef PSL_H
#define PSL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PSL_ABI_VERSION 1

typedef int32_t psl_status;
#define PSL_OK 0
#define PSL_EINVAL 1         /* bad argument (null pointer, bad size, ...)  */
#define PSL_ENOSPC 2         /* workspace or queue capacity too small       */
#define PSL_EHIP 3           /* HIP runtime or launch error                 */
#define PSL_EUNSUPPORTED 4   /* current device is not gfx950                */

#define PSL_MAX_EBINS 64     /* energy bins of a PSL grid                   */
#define PSL_MAX_POSBINS 128  /* position bins per axis of a PSL grid        */
#define PSL_MAX_QBUCKETS 16  /* energy buckets of the electron queue        */

/* Human-readable description of the last failure on this thread. */
const char *psl_last_error(void);
int32_t psl_version(void);

/* ------------------------------------------------------------------------ */
/* Phase space (structure of arrays, device).                               */
/* ------------------------------------------------------------------------ */
typedef struct psl_phsp {
    int64_t n;          /* particles (input) or capacity (output)           */
    uint8_t *type;      /* 0 photon, 1 electron or positron (merged)        */
    float *E;           /* kinetic energy, MeV                              */
    float *x, *y;       /* position at the grid plane, cm                   */
    float *u, *v, *w;   /* direction cosines                                */
    float *wt;          /* statistical weight                               */
} psl_phsp;

/* PSL bin grid (host struct, passed by pointer, copied by value).  Edges
 * must be strictly increasing.  Bin k of an axis is [edge_k, edge_k+1),
 * the last bin closed on top; values outside [edge_0, edge_n] are outside
 * the grid. */
typedef struct psl_grid {
    int32_t n_e, n_x, n_y, pad;
    double z_plane;                         /* z of the PSL plane, cm       */
    float e_edges[PSL_MAX_EBINS + 1];
    float x_edges[PSL_MAX_POSBINS + 1];
    float y_edges[PSL_MAX_POSBINS + 1];
} psl_grid;

/*
 * psl_build - PSL generation (Sec. 2.3.2): split the phase space by particle
 * type (photons; electrons and positrons merged, Sec. 2.1), by energy bin
 * and by position bin, i.e. a stable sort on
 *     key = ((type * n_e + e) * n_y + iy) * n_x + ix,
 * keeping input order inside each PSL.
 *   in        device SoA of in->n particles (read only); n < 2^31.
 *   out       device SoA with out->n >= in->n; receives the kept particles
 *             in PSL order (entries past the kept count are untouched).
 * Implemented as an LSD radix sort by key whose passes carry the particle
 * columns, so no pass gathers from random positions.
 *   d_offsets device int64[2 * n_e * n_x * n_y + 1]: PSL k holds
 *             out[d_offsets[k] .. d_offsets[k+1]).
 *   d_n_dropped device int64[1]: particles of unknown type (> 1), NaN, or
 *             outside the grid; they are not copied.
 * Errors: PSL_EINVAL for bad sizes or edges, PSL_ENOSPC if ws_bytes <
 * psl_build_workspace_bytes(in->n, g).
 */
size_t psl_build_workspace_bytes(int64_t n, const psl_grid *g);
psl_status psl_build(const psl_phsp *in, const psl_grid *g, psl_phsp *out,
                     int64_t *d_offsets, int64_t *d_n_dropped, void *d_ws,
                     size_t ws_bytes, void *stream);

/*
 * psl_build_apr - PSL generation with azimuthal particle redistribution
 * (Sec. 2.3.1), for a cylindrically symmetric phase space: every particle
 * i is replaced by `copies` copies m = i * copies + j, each turned about
 * the central axis (x = y = 0) by its own uniform azimuth, position and
 * direction cosines alike, weight wt / copies, energy, type and w kept;
 * the PSLs are then built from the copies exactly as psl_build does (so
 * the bins see the turned positions).  The azimuth of copy m: a point
 * (a, b) uniform in the unit disk by rejection from the stream
 * splitmix64(splitmix64(seed ^ m) + t), t = 0, 1, ... (two draws per
 * attempt, the top 53 bits of each scaled to [-1, 1)), and the turn by
 * twice its angle: cos = (a^2 - b^2) / r^2, sin = 2ab / r^2 (no copy is
 * turned after 64 failed attempts, probability < 1e-42).  Double
 * precision without contraction, rounded to float.
 *   copies 1 .. 4096, in->n * copies < 2^31; out->n >= in->n * copies;
 *   workspace psl_build_apr_workspace_bytes(in->n, copies, g).
 * Errors as psl_build.
 */
size_t psl_build_apr_workspace_bytes(int64_t n, int64_t copies,
                                     const psl_grid *g);
psl_status psl_build_apr(const psl_phsp *in, const psl_grid *g,
                         int64_t copies, uint64_t seed, psl_phsp *out,
                         int64_t *d_offsets, int64_t *d_n_dropped,
                         void *d_ws, size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------------ */
/* Source sampling.                                                          */
/* ------------------------------------------------------------------------ */

/* One treatment field or IMRT segment (host struct). */
typedef struct psl_field {
    double X1, X2, Y1, Y2;      /* jaw edges projected to the SAD plane, cm  */
    double gantry_deg;          /* rotation about +y through the isocentre   */
    double MU;                  /* monitor units, > 0                        */
    const float *fluence;       /* device [nfy][nfx] map at the SAD plane,   */
                                /* NULL = no modulation                      */
    int32_t nfx, nfy;
    double f_x0, f_y0, f_pix;   /* map origin (corner) and pixel size, cm   */
    int32_t jaws_on;            /* 0: no jaw model and no ROI for this field */
    int32_t pad;
    double collimator_deg;      /* rotation of the beam about its central    */
                                /* axis (the phase space turns with the      */
                                /* collimator; applied after the jaw test)   */
    double couch_deg;           /* patient rotation about the vertical axis  */
                                /* (z at gantry 0) through the isocentre     */
} psl_field;

#define PSL_ALLOC_COUNTS 0      /* field totals in proportion to the        */
                                /* particles of their selected PSLs (Eq.1-2) */
#define PSL_ALLOC_MU 1          /* field totals in proportion to MU          */

typedef struct psl_sample_cfg {
    uint64_t seed;              /* random starts of the PSLs                 */
    int64_t batch;              /* batch index b >= 0 (cursor and uids)      */
    int64_t n_histories;        /* histories in this batch, all fields       */
    int32_t cull;               /* 1: ROI selection of PSLs (Sec. 2.3.3)     */
    int32_t alloc_mode;         /* PSL_ALLOC_COUNTS or PSL_ALLOC_MU          */
    double sad, z_jaw_x, z_jaw_y;   /* cm; the PSL plane is grid.z_plane     */
    double iso[3];              /* isocentre, world frame, cm                */
    double box_lo[3], box_hi[3];/* phantom bounding box, world frame, cm     */
} psl_sample_cfg;

/* Particle queue entries (structure of arrays, device). */
typedef struct psl_particles {
    int64_t capacity;
    float *E, *x, *y, *z, *u, *v, *w, *wt;
    uint64_t *uid;              /* history id: batch * n_histories + h       */
    uint32_t *ctr;              /* random-number identity (see transport)    */
} psl_particles;

/* Transport queues.  Source electrons are kept in n_ebuckets regions of
 * el.capacity / n_ebuckets entries each, one per kinetic-energy bucket
 * [e_bucket_edges[b], e_bucket_edges[b+1]); secondary electrons live in
 * the transport workspace.  d_counts (device uint32, PSL_QCOUNTS
 * entries): [0] photons queued, [1 + b] electrons in bucket b,
 * [PSL_QCOUNTS - 1] entries lost because a region was full (a batch with a
 * non-zero value here is invalid and must be re-run with more capacity). */
#define PSL_QCOUNTS (PSL_MAX_QBUCKETS + 2)
typedef struct psl_queue {
    psl_particles ph;
    psl_particles el;
    int32_t n_ebuckets, pad;
    float e_bucket_edges[PSL_MAX_QBUCKETS + 1];
    uint32_t *d_counts;
} psl_queue;

/* Device statistics (zeroed by psl_sample, accumulated by the later calls
 * of the same batch). */
typedef struct psl_stats {
    uint64_t histories;         /* sampled histories (Eq. 5 N_simulated)     */
    uint64_t jaw_rejected;
    uint64_t fluence_zero;
    uint64_t missed;            /* accepted but missing the phantom          */
    uint64_t photons;           /* queued source photons                     */
    uint64_t electrons;         /* queued source electrons                   */
    uint64_t lost;              /* queue overflow (batch invalid if > 0)     */
    uint64_t interactions;      /* real photon interactions                  */
    uint64_t secondaries;       /* Compton electrons queued                  */
    uint64_t segments;          /* electron voxel segments                   */
    uint64_t flights;           /* photon free flights (real + virtual)      */
    uint64_t runaway;           /* particles stopped by the loop guard       */
    uint64_t deposits;          /* dose atomics issued by electrons          */
    uint64_t photon_deposits;   /* dose atomics issued by photons            */
    uint64_t bucket_peak;       /* largest electron bucket fill of the batch */
    uint64_t dropped;           /* psl_stream_sample: bad type or NaN energy */
    double e_in;                /* sum E*wt of queued source particles       */
    double e_escaped;           /* sum E*wt leaving the phantom              */
    double e_killed;            /* sum E*wt of photons ended by              */
                                /* PSL_FLAG_FIRST_COLLISION                  */
} psl_stats;

/*
 * psl_sample - the PSL source for one batch (Sec. 2.2, 2.3.3, 2.4).
 *  1. ROI selection: per field, a position bin is selected when its
 *     rectangle overlaps with positive area the ROI obtained by
 *     back-projecting from the field centre at SAD through the jaw edges to
 *     the PSL plane (Sec. 2.3.3, Fig. 1).
 *  2. Histories per (field i, PSL k), Eq. (1)-(4): field totals by
 *     prefix-floor of n_histories over fields (alloc_mode), then
 *     N_ik = floor(N_i S_k / C_i) - floor(N_i S_k-1 / C_i) with S_k the
 *     running selected population; weight factor
 *     g_ik = (MU_i / MU_total) * n_k / N_ik.
 *  3. History r of PSL k reads particle off_k + ((s_k + c + r) mod n_k):
 *     s_k = splitmix64(seed ^ k) mod n_k is the random start of PSL k and c
 *     the particles already read from it by earlier batches and earlier
 *     fields (reading wraps to the start, Sec. 2.3.3).
 *  4. Jaw model (perfect collimators at z_jaw_x / z_jaw_y, Sec. 2.2);
 *     fluence weight of the map pixel the ray crosses at the SAD plane
 *     (Sec. 2.4); w' = w * fluence * g_ik (Eq. 4); gantry rotation; move
 *     along the ray to the phantom box.
 *  5. Accepted photons go to q->ph, electrons to the bucket of q->el that
 *     holds their energy; queue counts are reset first.
 *   grid, fields, cfg are host pointers (copied); fields has n_fields
 *   entries (1 .. 4096).  d_offsets comes from psl_build over `sorted`.
 *   d_mask (optional, device uint8 [n_fields][n_y*n_x]) receives the ROI
 *   selection; d_alloc (optional, device int64 [n_fields][n_keys])
 *   receives N_ik.  d_stats (device) is zeroed and filled.
 * Accepted particles are first written to per-history slots and then
 * compacted into the queues in history order (no contended atomics), so
 * queue contents and order are deterministic.
 * Errors: PSL_EINVAL (sizes, jaws X1 > X2, MU <= 0, z_jaw >= sad, ...),
 * PSL_ENOSPC if the workspace is too small (psl_sample_workspace_bytes for
 * the same grid, field count and n_histories) or the photon queue cannot
 * hold n_histories entries.
 */
size_t psl_sample_workspace_bytes(const psl_grid *g, int32_t n_fields,
                                  int64_t n_histories);
psl_status psl_sample(const psl_phsp *sorted, const int64_t *d_offsets,
                      const psl_grid *g, const psl_field *fields,
                      int32_t n_fields, const psl_sample_cfg *cfg,
                      psl_queue *q, uint8_t *d_mask, int64_t *d_alloc,
                      psl_stats *d_stats, void *d_ws, size_t ws_bytes,
                      void *stream);

/*
 * psl_sample_noalloc - psl_sample without a workspace argument, for callers
 * that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc).  Same arguments, results
 * and errors as psl_sample; the workspace is a static device array of
 * psl_sample_noalloc_max_bytes() (64 MiB) that each GPU holds from the
 * first call on it until the process ends.  That bounds the problem: one
 * field of a 2 x 32 x 22 x 22 grid takes about 1.4M histories per call.
 * Larger requests fail with PSL_ENOSPC before anything is enqueued.  The
 * call allocates nothing (no hipMalloc, no hipFree).
 * Every call on one GPU uses that GPU's one array, which keeps the last
 * call's contents (the sampling writes everything it later reads, so stale
 * contents do not matter): calls that overlap on one GPU (several host
 * threads, or several streams without ordering between them) race, and the
 * caller must order them.
 */
size_t psl_sample_noalloc_max_bytes(void);
psl_status psl_sample_noalloc(const psl_phsp *sorted,
                              const int64_t *d_offsets, const psl_grid *g,
                              const psl_field *fields, int32_t n_fields,
                              const psl_sample_cfg *cfg, psl_queue *q,
                              uint8_t *d_mask, int64_t *d_alloc,
                              psl_stats *d_stats, void *stream);

/*
 * psl_stream_sample - Methods 1 and 2, the paper's sources before PSLs
 * (Sec. 2.1, 2.2): the unsorted phase space is read in file order and
 * sorted on the fly into bins by particle type and energy, each bin
 * flushed to transport when it holds bin_capacity particles, the rest
 * flushed at the end of the batch.
 *  1. History r of batch b reads particle (s + b n_histories + r) mod n,
 *     s = splitmix64(seed) mod n (a random start; reading wraps at the end
 *     of the file).  A particle whose type is not 0 or 1, or whose energy
 *     is NaN, is dropped (stats.dropped).
 *  2. Method 2 passes the particle through the beam model of `field` (jaw
 *     test, fluence weight, as psl_sample); Method 1 takes the phase space
 *     as already collimated (the field's gantry angle applies, its jaws and
 *     fluence map do not).  w' = w * fluence * weight; gantry rotation; move
 *     along the ray to the phantom box.
 *  3. An accepted particle joins bin type * n_e + e, e the largest k with
 *     E >= e_edges[k] clamped to 0 .. n_e-1.  A bin holding bin_capacity
 *     particles is flushed (its particles in arrival order) and starts
 *     empty; after the last history the bins still holding particles are
 *     flushed in bin order.
 *  4. d_flushes receives the flushes in the order they happen: bin, count,
 *     trigger (the history whose arrival filled the bin, -1 for the end of
 *     the batch), first (offset of the flush in the flushed sequence, all
 *     types).  The flushed sequence goes to the queues: photons to q->ph,
 *     electrons to the bucket of q->el that holds their energy, each queue
 *     in flushed-sequence order; uid = b n_histories + r.
 *  phsp: device SoA in file order.  field, cfg: host (copied).
 *  max_flushes must be >= n_histories / bin_capacity + 2 n_e.
 *  d_n_flushes: device int64.  d_stats is zeroed and filled.
 * The result equals the sequential process exactly: bins are ranked by a
 * stable partition of the batch's histories, and a flush's position comes
 * from the stream position of its trigger.
 * Errors: PSL_EINVAL (sizes, edges, method not 1 or 2, capacity < 1,
 * max_flushes too small), PSL_ENOSPC (workspace:
 * psl_stream_workspace_bytes for the same n_histories, n_e and capacity;
 * photon queue smaller than n_histories).
 */
typedef struct psl_stream_cfg {
    uint64_t seed;              /* random start of the file reading          */
    int64_t batch;              /* batch index b                             */
    int64_t n_histories;        /* particles read in this batch              */
    int64_t bin_capacity;       /* N: particles a bin holds before a flush   */
    int32_t method;             /* 1 (collimated phase space) or 2 (jaws)    */
    int32_t n_e;                /* energy bins, 1 .. PSL_MAX_EBINS           */
    const float *e_edges;       /* host [n_e + 1], increasing                */
    double weight;              /* per-history factor g; n / n_histories     */
                                /* gives dose per phase-space particle       */
    double z_plane;             /* phase-space plane (cm)                    */
    double sad, z_jaw_x, z_jaw_y;
    double iso[3];
    double box_lo[3], box_hi[3];
} psl_stream_cfg;

typedef struct psl_flush {
    int32_t bin;                /* type * n_e + energy bin                   */
    int32_t pad;
    int64_t count;
    int64_t trigger;            /* history that filled the bin, -1 at end    */
    int64_t first;              /* offset in the flushed sequence            */
} psl_flush;

size_t psl_stream_workspace_bytes(int64_t n_histories, int32_t n_e,
                                  int64_t bin_capacity);
psl_status psl_stream_sample(const psl_phsp *phsp, const psl_field *field,
                             const psl_stream_cfg *cfg, psl_queue *q,
                             psl_flush *d_flushes, int64_t max_flushes,
                             int64_t *d_n_flushes, psl_stats *d_stats,
                             void *d_ws, size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------------ */
/* Transport.                                                                */
/* ------------------------------------------------------------------------ */

typedef struct psl_phantom {
    int32_t nx, ny, nz, pad;
    double dx, dy, dz;          /* voxel size, cm                             */
    double x0, y0, z0;          /* corner of voxel (0,0,0), world frame, cm   */
    const float *density;       /* device [nz][ny][nx], g/cm^3, x fastest     */
    float rho_max;              /* >= max density (Woodcock majorant)         */
    float rho_min;              /* <= min density, or 0 if unknown: a        */
                                /* tentative collision with xi*rho_max <=    */
                                /* rho_min is real without a density read    */
} psl_phantom;

#define PSL_FLAG_FIRST_COLLISION 1   /* photons stop after one interaction, */
                                     /* recoil energy deposited locally     */
#define PSL_FLAG_NO_MSC 2            /* electrons are not deflected          */

typedef struct psl_physics {
    double n_e;                 /* electrons / cm^3 at 1 g/cm^3 (water)      */
    double I_eV;                /* mean excitation energy                    */
    double X0;                  /* radiation length, g/cm^2                  */
    double step;                /* electron step, cm                         */
    double p_cut, t_cut;        /* kinetic cut-offs, MeV                     */
    double e_max;               /* highest energy the tables cover, MeV      */
    int32_t flags;
    int32_t pad;
} psl_physics;

/* Device tables built by psl_physics_init (opaque, PSL_TABLE_BYTES). */
#define PSL_TABLE_BYTES (64 * 1024)

/*
 * psl_physics_init - builds the transport tables for `phys` into d_tables
 * (device, PSL_TABLE_BYTES): Compton attenuation per unit density
 * n_e sigma_KN(E) on a log energy grid, the CSDA residual range above
 * t_cut of the Bethe collision stopping power with its inverse, and the
 * inverse cumulative distribution of the Klein-Nishina energy fraction
 * (64 log-spaced energies from p_cut x 96 quantiles, in the fraction
 * normalised to its support).  The host computes them in double and
 * enqueues one copy; phys->e_max must cover the highest particle energy.
 */
psl_status psl_physics_init(const psl_physics *phys, void *d_tables,
                            void *stream);

/* Dose accumulator: energy x weight per voxel for the current batch.
 * PSL_ACC_TRACE is a measurement mode, not a tally: the transport kernels
 * record the voxel index of every deposit instead of adding energy, in the
 * order the waves issue them (a wave's deposits of one call site are
 * consecutive).  data then points to a device buffer laid out as a uint64
 * count followed by trace_capacity uint32 voxel indices; the count must be
 * zero before the call and ends as the number of deposits (entries past
 * trace_capacity are counted, not stored).  dose_tally rejects this mode. */
#define PSL_ACC_F64 0           /* double, MeV                               */
#define PSL_ACC_FIXED64 1       /* uint64, MeV * 2^frac_bits                 */
#define PSL_ACC_TRACE 2         /* deposit-address trace (see above)         */
typedef struct psl_dose_acc {
    int32_t mode;
    int32_t frac_bits;          /* FIXED64 only, 16..40                      */
    void *data;                 /* device [nz*ny*nx] (TRACE: see above)      */
    int64_t trace_capacity;     /* TRACE only: voxel indices data can hold   */
} psl_dose_acc;

/* Launch shape.  NULL selects defaults (256, 4, 0, 1); the autotuner
 * chooses values. */
typedef struct psl_launch {
    int32_t block;              /* threads per block (256 in this build)     */
    int32_t blocks_per_cu;      /* transport blocks launched per CU, 1..64   */
    int32_t n_cu;               /* CUs to assume (0 = query the device)      */
    int32_t rebucket;           /* 1: transport electrons bucket by bucket,  */
                                /* highest energy first (secondary chunks    */
                                /* listed by bucket); 0: all source          */
                                /* electrons, then the pool in claim order   */
} psl_launch;

/*
 * transport_batch - transports every queued particle to exhaustion and adds
 * energy x weight per voxel to acc.  Physics (the paper defers to gDPM;
 * this is the model of the workloads): photons undergo Compton scattering
 * only (Klein-Nishina, free electrons at rest, energy fraction drawn from
 * the tabulated inverse distribution), tracked by Woodcock delta tracking
 * with majorant rho_max (and minorant rho_min: a tentative collision below
 * it is real without a density read); a recoil electron above t_cut is
 * queued in
 * its energy bucket, otherwise deposited on the spot; photons below p_cut
 * deposit on the spot.  Electrons slow down continuously (CSDA, Bethe
 * collision stopping power, I = I_eV, no density effect) in steps of
 * `step` cm split at voxel faces, each piece depositing its energy loss in
 * its voxel, deflected after each step by Highland's angle; at t_cut the
 * remainder is deposited.  Particles leaving the box are tallied in
 * stats.e_escaped.  FP32 arithmetic; tallies in FP64 or 64-bit fixed point.
 * Random numbers: Philox4x32-10 keyed by seed, counter (uid, ctr, tag), so
 * results do not depend on scheduling.  Photons are processed first, then
 * electron buckets from the highest energy down.  Queues are consumed
 * (counts zeroed).
 * Secondary electrons go to a workspace pool of 64-slot chunks (room for
 * 2 x ph.capacity of them; beyond that they are counted in stats.lost),
 * each chunk holding one energy bucket.
 * Errors: PSL_EINVAL (sizes, null pointers, bad acc mode), PSL_ENOSPC
 * (workspace too small).
 */
size_t transport_batch_workspace_bytes(const psl_queue *q);
psl_status transport_batch(psl_queue *q, const psl_phantom *ph,
                           const psl_physics *phys, const void *d_tables,
                           uint64_t seed, psl_dose_acc *acc,
                           psl_stats *d_stats, const psl_launch *launch,
                           void *d_ws, size_t ws_bytes, void *stream);

/*
 * dose_tally - batch statistics and normalisation (Sec. 2.3.3, Eq. 5).
 *  PSL_TALLY_FOLD: s1 += a, s2 += a^2 (double, per voxel) for the batch
 *    tally a (MeV), then a = 0.
 *  PSL_TALLY_FINALIZE: over n_batches >= 2 folded batches,
 *    dose  = (s1 / B) * c_v,
 *    sigma = sqrt(max(0, s2 - s1^2 / B) / (B - 1) / B) * c_v,
 *    c_v = 1.602176634e-10 / (rho_v dx dy dz) * norm  [Gy per MeV];
 *    norm = 1 / N_incident (dose per incident particle, Eq. 5 with the
 *    history weights g_ik already carrying N_total / N_simulated).
 *    Voxels of zero density get 0.
 * d_s1, d_s2: device double [voxels]; d_dose, d_sigma: device float
 * [voxels] (FINALIZE only).
 */
/*
 * dose_point - the dose at a reference point, for absolute calibration and
 * relative output factors (Sec. 2.5): the mean of d_dose over the voxels
 * whose centres lie within `radius` cm of (x, y, z) (the voxel holding the
 * point when no centre does), with the standard error of that mean from
 * d_sigma, sqrt(sum sigma^2) / count.  d_dose, d_sigma: device float
 * [nz][ny][nx] as dose_tally FINALIZE writes them.  d_out: device double
 * [3] = {mean dose, its standard error, voxel count} (all 0 when the point
 * lies outside the phantom and no centre is within the radius).  The sum
 * runs in a fixed order, so repeated calls agree bit for bit.
 * Errors: PSL_EINVAL (NULL, bad phantom, negative radius, a sphere over
 * more than 2^26 voxels).
 */
psl_status dose_point(const float *d_dose, const float *d_sigma,
                      const psl_phantom *ph, double x, double y, double z,
                      double radius, double *d_out, void *stream);

#define PSL_TALLY_FOLD 0
#define PSL_TALLY_FINALIZE 1
psl_status dose_tally(psl_dose_acc *acc, double *d_s1, double *d_s2,
                      int32_t op, int32_t n_batches, const psl_phantom *ph,
                      double norm, float *d_dose, float *d_sigma,
                      void *stream);

/*
 * dose_gamma - 3D global gamma index of an evaluated dose against a
 * reference (the dose-difference / distance-to-agreement test behind the
 * pass rates of Table 1; Low et al. 1998).  For every reference voxel with
 * ref >= ref_min:
 *   gamma^2 = min over offsets o of |o|^2 / dta^2
 *                                   + (E(r + o) - ref(r))^2 / dd^2,
 * the offsets being the points (-dta + i step, -dta + j step, -dta + k step),
 * i, j, k = 0 .. ceil((2 dta + 1e-12) / step) - 1, with |o|^2 <= dta^2 +
 * 1e-12, and E the trilinear interpolation of d_eval with indices clamped
 * to the volume.  Arithmetic in double.  dd is the absolute dose criterion
 * (global gamma: a fraction of the reference maximum).
 * d_ref, d_eval: device float [nz][ny][nx]; dx, dy, dz and dta in one
 * length unit.  d_gamma2 (optional): device float [voxels], gamma^2 of the
 * evaluated voxels and -1 elsewhere.  d_counts: device uint64 [2], to which
 * the call adds the number of evaluated voxels and of those with
 * gamma^2 <= 1 (the caller clears it).  PSL_EINVAL for non-positive
 * criteria or more than 64 offsets per axis.
 */
psl_status dose_gamma(const float *d_ref, const float *d_eval, int32_t nx,
                      int32_t ny, int32_t nz, double dx, double dy, double dz,
                      double dd, double dta, double step, double ref_min,
                      float *d_gamma2, uint64_t *d_counts, void *stream);

/* ------------------------------------------------------------------------ */
/* Kernel timing for benchmarks.                                             */
/* ------------------------------------------------------------------------ */
#define PSL_PROF_BUILD 0        /* psl_build: all kernels                    */
#define PSL_PROF_SAMPLE 1       /* psl_sample: the per-history kernel        */
#define PSL_PROF_ALLOC 2        /* psl_sample: cull, allocation, scans       */
#define PSL_PROF_PHOTONS 3      /* transport_batch: photon kernel            */
#define PSL_PROF_ELECTRONS 4    /* transport_batch: electron kernel          */
#define PSL_PROF_FOLD 5         /* dose_tally: fold                          */
#define PSL_PROF_FINALIZE 6     /* dose_tally: finalize                      */
#define PSL_PROF_REBUCKET 7     /* transport_batch: secondary re-bucketing   */
#define PSL_PROF_N 8

/*
 * psl_profile_enable - while on, the calls above bracket the kernels of each
 * PSL_PROF_* group with hipEvents recorded on the call's own stream.
 * psl_profile_read waits for the recorded events, returns the accumulated
 * milliseconds and launch counts per group (arrays of PSL_PROF_N, either may
 * be NULL) and, if reset != 0, clears them.  Host-side state shared by all
 * threads; not meant for concurrent use.
 */
psl_status psl_profile_enable(int32_t on);
psl_status psl_profile_read(double *ms, int64_t *launches, int32_t reset);

/* ------------------------------------------------------------------------ */
/* Batched plans (many fields or segments, batch after batch).              */
/* ------------------------------------------------------------------------ */
typedef struct psl_plan psl_plan;   /* opaque, host-side */

typedef struct psl_tune_result {
    psl_launch launch;              /* chosen transport launch shape         */
    int32_t n_ebuckets;             /* chosen electron bucket count          */
    int32_t configs_tried;
    float e_bucket_edges[PSL_MAX_QBUCKETS + 1];
    double ms_per_batch;            /* sample + transport time of the choice */
    int64_t el_capacity_suggested;  /* electron queue capacity that holds    */
                                    /* the observed peak bucket with 25%     */
                                    /* margin, for n_ebuckets buckets        */
    int64_t bucket_peak;            /* observed peak bucket fill             */
} psl_tune_result;

/*
 * psl_plan_create - a plan over n_fields fields or segments (for an IMRT
 * plan: the segments of all beams, Sec. 2.3.3 and 2.4 treat each as a field
 * with its jaws, MU and fluence map).  ROI selection and the allocation of
 * Eq. (1)-(4) are computed once here, on `stream`; each batch of
 * psl_plan_run is then psl_sample's per-history step, transport_batch and
 * dose_tally(FOLD) into d_s1/d_s2, all in one persistent launch per kernel
 * whatever the number of segments.  Buffers are as for the individual
 * calls; d_ws holds psl_plan_workspace_bytes() and is owned by the plan
 * until psl_plan_destroy.  launch NULL: 256-thread blocks, 4 per CU,
 * re-bucketing on.  *out receives a host handle.
 */
size_t psl_plan_workspace_bytes(const psl_grid *g, int32_t n_fields,
                                int64_t n_histories, const psl_queue *q);
psl_status psl_plan_create(psl_plan **out, const psl_phsp *sorted,
                           const int64_t *d_offsets, const psl_grid *g,
                           const psl_field *fields, int32_t n_fields,
                           const psl_sample_cfg *cfg, const psl_queue *q,
                           const psl_phantom *ph, const psl_physics *phys,
                           const void *d_tables, uint64_t seed,
                           const psl_dose_acc *acc, double *d_s1,
                           double *d_s2, psl_stats *d_stats,
                           const psl_launch *launch, void *d_ws,
                           size_t ws_bytes, void *stream);
/*
 * psl_plan_run - enqueues batches first_batch .. first_batch + n_batches - 1.
 * With use_graph != 0 the batch is captured once into a hipGraph (on this
 * stream, which must not be the null stream) and replayed per batch; the
 * batch index lives in device memory and each replay advances it, so the
 * result is identical to the eager path.
 */
psl_status psl_plan_run(psl_plan *p, int64_t first_batch, int32_t n_batches,
                        int32_t use_graph, void *stream);
/*
 * psl_autotune - times `trials` batches (after one warm-up) of sampling and
 * transport for electron bucket counts {1, 4, 8, 16} (edges log-spaced from
 * t_cut to e_max), with and without re-bucketing, at 2, 4, 8 and 16 blocks
 * per CU; configurations that overflow a queue region are rejected.  The
 * fastest is applied to the plan and returned with the queue capacity it
 * needs.  The tallies d_s1/d_s2 are not touched; the batch accumulator is
 * left zero.  Synchronises the stream.
 */
psl_status psl_autotune(psl_plan *p, int32_t trials, psl_tune_result *out,
                        void *stream);
/* Current queue layout and launch shape of a plan (after tuning). */
psl_status psl_plan_get(const psl_plan *p, psl_queue *q, psl_launch *launch);
/*
 * psl_plan_run_pair - batches first_batch .. first_batch + n_batches - 1 of
 * one plan split over two plans a and b of the same fields (Sec. 2.3.3,
 * 2.4: many fields sharing one phase space, batch after batch) that fold
 * into the same d_s1/d_s2 but each own their queues, accumulator,
 * statistics and workspace: batches first + 2k run on a, first + 2k + 1 on
 * b, the two of a pair in flight at once (b's on a stream a holds, each
 * plan's transport with half its blocks per CU), a's fold before b's.
 * With an odd count the last batch runs on a alone.  The histories and,
 * with the fixed-point tally, the sums equal those of psl_plan_run of
 * either plan over the same batches.  use_graph != 0 captures one pair into
 * a hipGraph (kept by a, captured again when b's tuning changes) and
 * replays it.  PSL_EINVAL if the plans share buffers they must not share
 * or fold into different sums.  Calls on one pair must not overlap.
 */
psl_status psl_plan_run_pair(psl_plan *a, psl_plan *b, int64_t first_batch,
                             int32_t n_batches, int32_t use_graph,
                             void *stream);
/*
 * psl_plan_run_set - batches first_batch .. first_batch + n_batches - 1 of
 * one job (Sec. 2.3.3, 2.4: many fields sharing one phase space, batch
 * after batch) over n_plans plans of the same fields, 1 <= n_plans <= 8,
 * any two of which meet psl_plan_run_pair's requirements (the same
 * d_s1/d_s2 and accumulator mode, their own queues, accumulator,
 * statistics and workspace): batch first + i runs on plans[i mod n_plans],
 * plans[0] on `stream` and each other plan on a stream it holds, so that
 * n_plans batches are in flight at once (one sampled while others are
 * transported); with more than one plan each transport runs with half its
 * plan's blocks per CU.  The folds keep batch order.  Enqueued eagerly (no
 * graph); `stream` waits for every plan's stream before the call returns,
 * so work enqueued on it afterwards sees the sums.  The histories and,
 * with the fixed-point tally, the sums equal those of psl_plan_run over the
 * same batches.  PSL_EINVAL for a NULL or repeated plan, a count outside
 * 1..8 or buffers the plans must not share.  Calls on plans of one set
 * must not overlap.
 */
psl_status psl_plan_run_set(psl_plan *const *plans, int32_t n_plans,
                            int64_t first_batch, int32_t n_batches,
                            void *stream);
/* Gives dst the transport launch shape and electron bucketing of src (for
 * example after psl_autotune on src), so that two plans of a pair run the
 * same configuration. */
psl_status psl_plan_copy_tuning(psl_plan *dst, const psl_plan *src);
psl_status psl_plan_destroy(psl_plan *p);

/* ------------------------------------------------------------------------ */
/* Learned dose denoiser (not part of the paper's method).                   */
/* ------------------------------------------------------------------------ */
/* A 3D U-Net: 4 levels of 16/32/64/128 channels, two 3x3x3 convolutions
 * (zero padding, ReLU) per level and side, 2x2x2 average pooling, nearest
 * up-sampling with concatenated skips, and a 1x1 head added to the input
 * dose (residual).  Inputs per sample are the noisy dose and the density,
 * both [nz][ny][nx]; the dose is normalised by its maximum.  BF16 weights
 * and activations on MFMA with FP32 accumulation; FP32 master weights.
 * Parameter blob layout (floats): for each of the 14 convolutions in the
 * order enc0a enc0b enc1a enc1b enc2a enc2b enc3a enc3b dec2a dec2b dec1a
 * dec1b dec0a dec0b: W[Cout][Kp] with K = offset * Cin + ci (offset =
 * (dz+1)*9 + (dy+1)*3 + (dx+1)) zero-padded to Kp = roundup(27 Cin, 32),
 * then b[Cout]; then the head w[16] and b[1] (plus 7 padding floats).
 * enc0a reads 16 input channels: dose, density and 14 zeros. */
typedef struct psl_unet {
    int32_t levels, base;       /* 4 and 16 in this build                  */
    int64_t n_params;           /* unet_param_count(4, 16)                 */
    float *params;              /* device fp32 master weights              */
    uint16_t *params_bf16;      /* device bf16 copy used by the kernels    */
} psl_unet;

int64_t unet_param_count(int32_t levels, int32_t base);
size_t unet_workspace_bytes(const psl_unet *u, int32_t n, int32_t nz,
                            int32_t ny, int32_t nx, int32_t training);
/* He-normal weights (counter-based, from seed), zero biases, zero head. */
psl_status unet_init(psl_unet *u, uint64_t seed, void *stream);
/* Refreshes the bf16 copy from the fp32 master weights (round to nearest
 * even), after the caller has written u->params (for example weights loaded
 * from a file in the blob layout above). */
psl_status unet_set_params(psl_unet *u, void *stream);
/* d_out [n][nz][ny][nx] = denoised dose (same units as d_dose).  Each axis
 * must be a multiple of 8. */
psl_status unet_forward(const psl_unet *u, const float *d_dose,
                        const float *d_density, int32_t n, int32_t nz,
                        int32_t ny, int32_t nx, float *d_out, void *d_ws,
                        size_t ws_bytes, void *stream);
/* Forward with saved activations, then the mean squared error against
 * d_target (in normalised units) added into *d_loss (device double) and
 * its gradient added into d_grads (n_params floats, same layout). */
psl_status unet_backward(const psl_unet *u, const float *d_dose,
                         const float *d_density, const float *d_target,
                         int32_t n, int32_t nz, int32_t ny, int32_t nx,
                         float *d_grads, double *d_loss, void *d_ws,
                         size_t ws_bytes, void *stream);
/* Adam on the fp32 weights (step counts from 1), refreshes the bf16 copy
 * and zeroes d_grads. */
psl_status unet_adam_step(psl_unet *u, float *d_grads, float *d_m, float *d_v,
                          float lr, float beta1, float beta2, float eps,
                          int32_t step, void *stream);
/* Caps the grid of the finest-level convolution (16 -> 16 channels), which
 * runs as a loop over 16x4x4-voxel bricks: at most max_blocks blocks, each
 * walking its share of the bricks, instead of as many as are resident at
 * once (max_blocks = 0, the default).  Process-wide; the results do not
 * depend on it (tests use it to put many bricks on each block at small
 * volumes).  PSL_EINVAL for max_blocks < 0. */
psl_status unet_set_brick_blocks(int32_t max_blocks);
/* dose_denoise - one volume through the trained network (unet_forward with
 * n = 1); plain Monte Carlo stays the reference the result is judged by. */
psl_status dose_denoise(const float *d_dose, const float *d_density,
                        int32_t nx, int32_t ny, int32_t nz,
                        const psl_unet *net, float *d_out, void *d_ws,
                        size_t ws_bytes, void *stream);

/*
 * psl_bench_atomics - measures the atomic roofs the dose tally works
 * against, on the current device: rates[0] = 64-bit atomic adds per second
 * scattered over n_addresses (>= 1024) 8-byte counters, the access pattern
 * of the tally; rates[1] = atomic adds per second that all target one
 * address.  Needs psl_bench_atomics_workspace_bytes(n_addresses) of device
 * workspace (contents destroyed).  Synchronises the stream.
 */
size_t psl_bench_atomics_workspace_bytes(int64_t n_addresses);
psl_status psl_bench_atomics(int64_t n_addresses, double *rates, void *d_ws,
                             size_t ws_bytes, void *stream);

/*
 * psl_bench_atomics_replay - the atomic roof of the tally's own address
 * pattern: replays d_trace (device uint32 [n_trace] voxel indices below
 * n_addresses, as recorded by transport_batch in PSL_ACC_TRACE mode) as
 * 64-bit atomic adds on an n_addresses-entry array in the workspace, entry
 * j on thread j mod (grid size), `reps` times per launch, for each launch
 * shape blocks_per_cu[0 .. n_shapes-1] (256-thread blocks per CU, 1..64).
 * rates[i] receives atomic adds per second for shape i.  Workspace:
 * psl_bench_atomics_workspace_bytes(n_addresses), contents destroyed.
 * Entries at or above n_addresses are skipped (still counted in the
 * rate).  Synchronises the stream.
 */
psl_status psl_bench_atomics_replay(const uint32_t *d_trace, int64_t n_trace,
                                    int64_t n_addresses,
                                    const int32_t *blocks_per_cu,
                                    int32_t n_shapes, int32_t reps,
                                    double *rates, void *d_ws,
                                    size_t ws_bytes, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* PSL_H */
