/*
 * CPU oracle for the phase-space-let (PSL) dose path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark load this code.  The product (the HIP
 * library) never calls it, and the two share no code: the only thing both
 * see is the seeded synthetic input.
 *
 * Plain, slow, obviously correct: double precision throughout, scalar loops,
 * built with -ffp-contract=off.  Each function cites the part of the paper it
 * follows (Townson et al., "GPU-based Monte Carlo radiotherapy dose
 * calculation using phase-space sources").
 *
 *   oracle_build      PSL generation: split by type, energy bin, position bin
 *                     (Sec. 2.3.2), stable counting sort.
 *   oracle_cull       ROI selection of PSLs per field (Sec. 2.3.3, Fig. 1).
 *   oracle_alloc      histories per (field, PSL), Eq. (1)-(4) (Sec. 2.3.3).
 *   oracle_sample     cyclic reading with a random start, jaw accept/reject
 *                     (Sec. 2.2), fluence weight (Sec. 2.4), MU weight
 *                     (Eq. 4), gantry rotation and projection to the phantom
 *                     (Sec. 2.3.3).
 *   oracle_transport  photon (Klein-Nishina Compton) and electron (CSDA,
 *                     Bethe stopping power, Highland scattering) transport
 *                     with a per-voxel energy tally.  The paper defers its
 *                     physics to gDPM; this model is the one the workloads
 *                     prescribe.  The algorithms here (exact voxel ray march,
 *                     naive rejection for the Compton angle, Runge-Kutta for
 *                     the energy loss, quadrature for the range, Gaussian
 *                     projected angles) are deliberately independent of the
 *                     GPU kernels', so agreement there is statistical.
 *
 * Every function here is pinned by tests against closed forms, library
 * routines or brute force; see tests/test_oracle_*.py.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define ME 0.51099895            /* electron rest energy, MeV */
#define RE 2.8179403262e-13      /* classical electron radius, cm */
#define PI 3.14159265358979323846

/* ------------------------------------------------------------------------ */
/* Random numbers (oracle only).                                             */
/* splitmix64 (Steele, Lea & Flood 2014) and xoshiro256** (Blackman & Vigna   */
/* 2018), written from their published definitions.                          */
/* ------------------------------------------------------------------------ */
uint64_t oracle_splitmix64(uint64_t x)
{
    uint64_t z = x + 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

typedef struct { uint64_t s[4]; } xrng;

static uint64_t rotl(uint64_t x, int k) { return (x << k) | (x >> (64 - k)); }

static uint64_t xnext(xrng *r)
{
    uint64_t *s = r->s;
    uint64_t res = rotl(s[1] * 5, 7) * 9;
    uint64_t t = s[1] << 17;
    s[2] ^= s[0];
    s[3] ^= s[1];
    s[1] ^= s[2];
    s[0] ^= s[3];
    s[2] ^= t;
    s[3] = rotl(s[3], 45);
    return res;
}

static void xseed(xrng *r, uint64_t seed, uint64_t stream)
{
    uint64_t x = seed ^ oracle_splitmix64(stream);
    for (int i = 0; i < 4; ++i) {
        x = oracle_splitmix64(x);
        r->s[i] = x;
    }
}

/* uniform in [0, 1) with 53 random bits */
static double urand(xrng *r) { return (double)(xnext(r) >> 11) * 0x1.0p-53; }

/* ------------------------------------------------------------------------ */
/* PSL generation (Sec. 2.3.2).                                              */
/* ------------------------------------------------------------------------ */

/* Bin of v on edges[0..n]: the largest k with v >= edges[k], the top edge
 * closed.  Values outside [edges[0], edges[n]] (and NaN) give -1. */
static int bin_of(float v, const float *edges, int n)
{
    if (!(v >= edges[0]) || !(v <= edges[n])) return -1;
    int k = 0;
    for (int j = 1; j <= n; ++j)
        if (v >= edges[j]) k = j;
    if (k > n - 1) k = n - 1;
    return k;
}

/* Split the phase space by type (photon / electron+positron), energy bin
 * and position bin, keeping input order inside each PSL.
 *   key = ((type * n_e + e) * n_y + iy) * n_x + ix
 * perm[j] is the input index of the j-th particle in PSL order; offsets has
 * n_keys + 1 entries.  Particles of unknown type or outside the grid are
 * dropped and counted.  Returns the number kept. */
int64_t oracle_build(int64_t n, const uint8_t *type, const float *E,
                     const float *x, const float *y,
                     int n_e, const float *e_edges,
                     int n_x, const float *x_edges,
                     int n_y, const float *y_edges,
                     int64_t *perm, int64_t *offsets, int64_t *n_dropped)
{
    int64_t n_keys = 2LL * n_e * n_x * n_y;
    int64_t *key = (int64_t *)malloc(sizeof(int64_t) * (n > 0 ? n : 1));
    int64_t *run = (int64_t *)calloc((size_t)n_keys, sizeof(int64_t));
    int64_t dropped = 0;
    for (int64_t k = 0; k <= n_keys; ++k) offsets[k] = 0;
    for (int64_t i = 0; i < n; ++i) {
        int t = type[i];
        int e = bin_of(E[i], e_edges, n_e);
        int ix = bin_of(x[i], x_edges, n_x);
        int iy = bin_of(y[i], y_edges, n_y);
        if (t > 1 || e < 0 || ix < 0 || iy < 0) {
            key[i] = -1;
            ++dropped;
            continue;
        }
        key[i] = (((int64_t)t * n_e + e) * n_y + iy) * n_x + ix;
        offsets[key[i] + 1] += 1;
    }
    for (int64_t k = 0; k < n_keys; ++k) offsets[k + 1] += offsets[k];
    for (int64_t i = 0; i < n; ++i) {
        if (key[i] < 0) continue;
        perm[offsets[key[i]] + run[key[i]]] = i;
        run[key[i]] += 1;
    }
    free(key);
    free(run);
    *n_dropped = dropped;
    return n - dropped;
}

/* Azimuthal particle redistribution (Sec. 2.3.1).  Copy m of the expanded
 * phase space turns about the central axis by an azimuth drawn uniformly:
 * a point (a, b) uniform in the unit disk by rejection from the stream
 * splitmix64(key + t), key = splitmix64(seed ^ m), two draws per attempt,
 * each the top 53 bits scaled to [-1, 1); the angle of (a, b) is uniform
 * and so is twice it, whose cosine and sine are (a^2 - b^2) / r^2 and
 * 2ab / r^2 (no square root or trigonometry, so the value is exact IEEE
 * arithmetic on any machine).  After 64 failed attempts (probability
 * below 1e-42) the copy is not turned. */
void oracle_apr_rotation(uint64_t seed, uint64_t m, double *c, double *s)
{
    const uint64_t key = oracle_splitmix64(seed ^ m);
    for (uint64_t t = 0; t < 64; ++t) {
        double a = (double)(oracle_splitmix64(key + 2 * t) >> 11) *
                   0x1.0p-53 * 2.0 - 1.0;
        double b = (double)(oracle_splitmix64(key + 2 * t + 1) >> 11) *
                   0x1.0p-53 * 2.0 - 1.0;
        double r2 = a * a + b * b;
        if (r2 > 0.0 && r2 <= 1.0) {
            *c = (a * a - b * b) / r2;
            *s = 2.0 * a * b / r2;
            return;
        }
    }
    *c = 1.0;
    *s = 0.0;
}

/* The APR-expanded phase space: particle i gives copies i*k .. i*k+k-1,
 * each turned about the central axis (x = y = 0) by its own azimuth,
 * position and direction alike (the direction cosines follow the turn, so
 * a cylindrically symmetric phase space stays so), with weight wt / k;
 * type, energy and w are kept.  Arithmetic in double, rounded to float. */
void oracle_apr_expand(int64_t n, int64_t k, uint64_t seed,
                       const uint8_t *type, const float *E, const float *x,
                       const float *y, const float *u, const float *v,
                       const float *w, const float *wt, uint8_t *otype,
                       float *oE, float *ox, float *oy, float *ou, float *ov,
                       float *ow, float *owt)
{
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < k; ++j) {
            const int64_t m = i * k + j;
            double c, s;
            oracle_apr_rotation(seed, (uint64_t)m, &c, &s);
            double px = x[i], py = y[i], du = u[i], dv = v[i];
            otype[m] = type[i];
            oE[m] = E[i];
            ox[m] = (float)(c * px - s * py);
            oy[m] = (float)(s * px + c * py);
            ou[m] = (float)(c * du - s * dv);
            ov[m] = (float)(s * du + c * dv);
            ow[m] = w[i];
            owt[m] = (float)((double)wt[i] / (double)k);
        }
}

/* ------------------------------------------------------------------------ */
/* ROI selection (Sec. 2.3.3, Fig. 1).                                       */
/* ------------------------------------------------------------------------ */

/* The ROI at the PSL plane: from the open-field centre at SAD, back-project
 * through each jaw edge (the edge sits at jaw_edge_at_SAD * z_jaw / SAD) to
 * z_psl.  A position bin is kept when its rectangle overlaps the ROI with
 * positive area; the ROI is the intersection of the X- and Y-jaw
 * exposures.  mask is [n_fields][n_y * n_x], 1 = kept.  With cull == 0 or a
 * field without jaws every bin is kept. */
void oracle_roi(double lo_at_sad, double hi_at_sad, double z_jaw, double sad,
                double z_psl, double *lo, double *hi)
{
    double c = (lo_at_sad + hi_at_sad) * 0.5;
    double f = (sad - z_psl) / (sad - z_jaw);
    double a_lo = lo_at_sad * z_jaw / sad;
    double a_hi = hi_at_sad * z_jaw / sad;
    *lo = c + (a_lo - c) * f;
    *hi = c + (a_hi - c) * f;
}

void oracle_cull(int n_fields, const double *X1, const double *X2,
                 const double *Y1, const double *Y2, const int32_t *jaws_on,
                 int cull, double sad, double z_x, double z_y, double z_psl,
                 int n_x, const float *x_edges, int n_y, const float *y_edges,
                 uint8_t *mask)
{
    for (int f = 0; f < n_fields; ++f) {
        uint8_t *m = mask + (int64_t)f * n_x * n_y;
        if (!cull || !jaws_on[f]) {
            for (int b = 0; b < n_x * n_y; ++b) m[b] = 1;
            continue;
        }
        double xlo, xhi, ylo, yhi;
        oracle_roi(X1[f], X2[f], z_x, sad, z_psl, &xlo, &xhi);
        oracle_roi(Y1[f], Y2[f], z_y, sad, z_psl, &ylo, &yhi);
        for (int iy = 0; iy < n_y; ++iy)
            for (int ix = 0; ix < n_x; ++ix) {
                int keep = ((double)x_edges[ix] < xhi) &&
                           ((double)x_edges[ix + 1] > xlo) &&
                           ((double)y_edges[iy] < yhi) &&
                           ((double)y_edges[iy + 1] > ylo);
                m[iy * n_x + ix] = (uint8_t)keep;
            }
    }
}

/* ------------------------------------------------------------------------ */
/* Histories per (field, PSL): Eq. (1)-(4) (Sec. 2.3.3).                      */
/* ------------------------------------------------------------------------ */

/* Field totals N_i: mode 0 splits n_sim in proportion to the particles in
 * each field's selected PSLs (Eq. 1-2, C_i = sum of selected populations),
 * mode 1 in proportion to MU_i.  Within a field, PSL k receives
 *   N_ik = floor(N_i S_k / C_i) - floor(N_i S_{k-1} / C_i),
 * S_k the running selected population in key order, so N_ik is the floor or
 * ceiling of N_i n_k / C_i and the N_ik sum to N_i exactly (Eq. 2-3: each
 * typed PSL gets a count proportional to its population).  The history
 * weight factor is g_ik = (MU_i / MU_total) n_k / N_ik (Eq. 4 times the
 * recycling factor), 0 where N_ik = 0.  A field whose selected PSLs hold no
 * particles gets N_ik = 0 everywhere (its histories are lost).  Returns 0,
 * or -1 if no field selects any particle in mode 0. */
int oracle_alloc(int n_fields, const double *MU, int mode, int64_t n_sim,
                 int64_t n_keys, int n_pos, const int64_t *offsets,
                 const uint8_t *mask, int64_t *N, double *g,
                 int64_t *N_field)
{
    int64_t *C = (int64_t *)calloc((size_t)n_fields, sizeof(int64_t));
    double mu_tot = 0.0;
    for (int f = 0; f < n_fields; ++f) mu_tot += MU[f];
    int64_t c_all = 0;
    for (int f = 0; f < n_fields; ++f) {
        for (int64_t k = 0; k < n_keys; ++k)
            if (mask[(int64_t)f * n_pos + k % n_pos])
                C[f] += offsets[k + 1] - offsets[k];
        c_all += C[f];
    }
    /* field totals by prefix-floor */
    int64_t prev = 0;
    if (mode == 0) {
        if (c_all == 0) { free(C); return -1; }
        __int128 acc = 0;
        for (int f = 0; f < n_fields; ++f) {
            acc += C[f];
            int64_t F = (f == n_fields - 1)
                            ? n_sim
                            : (int64_t)(((__int128)n_sim * acc) / c_all);
            N_field[f] = F - prev;
            prev = F;
        }
    } else {
        double m = 0.0;
        for (int f = 0; f < n_fields; ++f) {
            m += MU[f];
            int64_t F = (f == n_fields - 1)
                            ? n_sim
                            : (int64_t)floor((double)n_sim * m / mu_tot);
            N_field[f] = F - prev;
            prev = F;
        }
    }
    for (int f = 0; f < n_fields; ++f) {
        int64_t Ni = N_field[f];
        __int128 S = 0;
        int64_t prevk = 0;
        for (int64_t k = 0; k < n_keys; ++k) {
            int64_t idx = (int64_t)f * n_keys + k;
            int64_t nk = offsets[k + 1] - offsets[k];
            int sel = mask[(int64_t)f * n_pos + k % n_pos];
            if (!sel || C[f] == 0) {
                N[idx] = 0;
                g[idx] = 0.0;
                continue;
            }
            S += nk;
            int64_t Fk = (int64_t)(((__int128)Ni * S) / C[f]);
            N[idx] = Fk - prevk;
            prevk = Fk;
            g[idx] = N[idx] > 0
                         ? (MU[f] / mu_tot) * ((double)nk / (double)N[idx])
                         : 0.0;
        }
    }
    free(C);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Source sampling (Sec. 2.2, 2.3.3, 2.4).                                    */
/* ------------------------------------------------------------------------ */

typedef struct {
    double X1, X2, Y1, Y2;      /* jaw edges at SAD, cm */
    double cos_g, sin_g;        /* gantry rotation about +y through iso */
    double MU;
    int32_t jaws_on;
    int32_t nfx, nfy;           /* fluence map size, 0 = none */
    int32_t pad;
    double f_x0, f_y0, f_pix;   /* fluence map origin and pixel at SAD */
    const float *fluence;       /* [nfy][nfx] */
    double cos_c, sin_c;        /* collimator: about the central axis */
    double cos_t, sin_t;        /* couch: patient about the vertical axis */
} ofield;

typedef struct {
    double sad, z_x, z_y, z_psl;
    double iso[3];              /* isocentre, world frame */
    double box_lo[3], box_hi[3];/* phantom AABB, world frame */
} ogeom;

/* One phase-space particle through the beam model (Sec. 2.2, 2.4), from
 * its position (x, y) at the phase-space plane and direction (u, v, w):
 * the jaw model (perfect collimators at z_x and z_y, zero transmission,
 * edges given at SAD, closed interval), the fluence weight of the map pixel
 * its ray crosses at the SAD plane (nearest pixel; outside the map or zero
 * rejects), the weight w' = wt * fluence * gk, the collimator, gantry
 * and couch rotations and the straight-line move to the phantom box.
 * Returns 0 jaw-rejected, 1 accepted, 2 zero fluence, 3 misses the phantom;
 * S = E x y z u v w w' on acceptance, zeros otherwise. */
static int beam_particle(const ofield *F, const ogeom *G, float x, float y,
                         float u, float v, float w, float wt, float E,
                         double gk, double S[8])
{
    for (int q = 0; q < 8; ++q) S[q] = 0.0;
    double px = x, py = y, pz = G->z_psl;
    double du = u, dv = v, dw = w;
    /* jaw model: test the crossing of each jaw plane */
    if (F->jaws_on) {
        if (!(dw > 0.0)) return 0;
        double tx = du / dw, ty = dv / dw;
        double xj = px + tx * (G->z_x - pz);
        double yj = py + ty * (G->z_y - pz);
        double xlo = F->X1 * G->z_x / G->sad;
        double xhi = F->X2 * G->z_x / G->sad;
        double ylo = F->Y1 * G->z_y / G->sad;
        double yhi = F->Y2 * G->z_y / G->sad;
        if (!(xj >= xlo && xj <= xhi && yj >= ylo && yj <= yhi)) return 0;
    }
    /* fluence weight at the SAD plane, nearest pixel */
    double fl = 1.0;
    if (F->nfx > 0) {
        if (!(dw > 0.0)) return 2;
        double xs = px + (du / dw) * (G->sad - pz);
        double ys = py + (dv / dw) * (G->sad - pz);
        double fx = floor((xs - F->f_x0) / F->f_pix);
        double fy = floor((ys - F->f_y0) / F->f_pix);
        if (!(fx >= 0.0 && fy >= 0.0 && fx < (double)F->nfx &&
              fy < (double)F->nfy))
            fl = 0.0;
        else
            fl = (double)F->fluence[(int64_t)fy * F->nfx + (int64_t)fx];
        if (!(fl > 0.0)) return 2;
    }
    double wgt = (double)wt * fl * gk;
    /* the rotations of the field, applied to the position about the
     * isocentre and to the direction: collimator (the phase space turns
     * with it about the central axis, z through the isocentre; the jaw
     * test above is in its frame), then gantry about +y, then couch (the
     * patient turns by +angle about the vertical, z at gantry 0, so the
     * beam turns by -angle).  Collimator and couch act only when one of
     * them is not zero, so the unturned case is the gantry alone, term for
     * term. */
    const int turned = F->cos_c != 1.0 || F->sin_c != 0.0 ||
                       F->cos_t != 1.0 || F->sin_t != 0.0;
    double rx = px - G->iso[0], ry = py - G->iso[1], rz = pz - G->iso[2];
    double au = du, av = dv;
    if (turned) {
        double x1 = F->cos_c * rx - F->sin_c * ry;
        double y1 = F->sin_c * rx + F->cos_c * ry;
        double u1 = F->cos_c * au - F->sin_c * av;
        double v1 = F->sin_c * au + F->cos_c * av;
        rx = x1; ry = y1; au = u1; av = v1;
    }
    double qx = F->cos_g * rx + F->sin_g * rz + G->iso[0];
    double qy = ry + G->iso[1];
    double qz = -F->sin_g * rx + F->cos_g * rz + G->iso[2];
    double eu = F->cos_g * au + F->sin_g * dw;
    double ev = av;
    double ew = -F->sin_g * au + F->cos_g * dw;
    if (turned) {
        double sx = qx - G->iso[0], sy = qy - G->iso[1];
        qx = F->cos_t * sx + F->sin_t * sy + G->iso[0];
        qy = -F->sin_t * sx + F->cos_t * sy + G->iso[1];
        double u2 = F->cos_t * eu + F->sin_t * ev;
        double v2 = -F->sin_t * eu + F->cos_t * ev;
        eu = u2; ev = v2;
    }
    /* straight-line projection to the phantom box (slab test) */
    double pos[3] = {qx, qy, qz}, dir[3] = {eu, ev, ew};
    double tn = -INFINITY, tf = INFINITY;
    int miss = 0;
    for (int a = 0; a < 3; ++a) {
        if (dir[a] != 0.0) {
            double t1 = (G->box_lo[a] - pos[a]) / dir[a];
            double t2 = (G->box_hi[a] - pos[a]) / dir[a];
            double lo = t1 < t2 ? t1 : t2, hi = t1 < t2 ? t2 : t1;
            if (lo > tn) tn = lo;
            if (hi < tf) tf = hi;
        } else if (pos[a] < G->box_lo[a] || pos[a] > G->box_hi[a]) {
            miss = 1;
        }
    }
    if (miss || tn > tf || tf <= 0.0) return 3;
    double t = tn > 0.0 ? tn : 0.0;
    S[0] = E;
    S[1] = pos[0] + t * dir[0];
    S[2] = pos[1] + t * dir[1];
    S[3] = pos[2] + t * dir[2];
    S[4] = eu;
    S[5] = ev;
    S[6] = ew;
    S[7] = wgt;
    return 1;
}

/* Histories of one batch, in canonical order: field-major, then key, then r.
 * History r of PSL k in field i reads the particle at
 *   off_k + ((s_k + c + r) mod n_k),
 * s_k = splitmix64(seed ^ k) mod n_k the random start of PSL k (chosen the
 * first time it is opened) and c the number of particles already read from
 * it by earlier batches and earlier fields of this batch (reading wraps to
 * the start at the end of the PSL).  The particle passes the jaw model
 * (perfect collimators, zero transmission), picks up the fluence weight of
 * the map pixel its ray crosses at the SAD plane and the factor g_ik, is
 * rotated by the gantry and moved along its ray to the phantom surface.
 * status: 0 jaw-rejected, 1 accepted, 2 zero fluence, 3 misses the phantom.
 * Outputs are per history (n_hist = sum N_ik). */
void oracle_sample(int n_fields, const ofield *fields, const ogeom *G,
                   int64_t n_keys, const int64_t *offsets, const int64_t *N,
                   const double *g, int64_t batch, uint64_t seed,
                   const uint8_t *type, const float *E, const float *x,
                   const float *y, const float *u, const float *v,
                   const float *w, const float *wt,
                   int64_t *src, int32_t *field, int32_t *keyo, uint8_t *status,
                   double *state /* [n_hist][8]: E x y z u v w wt */)
{
    /* T_k = histories per batch from PSL k over all fields */
    int64_t h = 0;
    for (int f = 0; f < n_fields; ++f) {
        const ofield *F = &fields[f];
        for (int64_t k = 0; k < n_keys; ++k) {
            int64_t Nik = N[(int64_t)f * n_keys + k];
            if (Nik == 0) continue;
            int64_t nk = offsets[k + 1] - offsets[k];
            int64_t Tk = 0, before = 0;
            for (int ff = 0; ff < n_fields; ++ff) {
                Tk += N[(int64_t)ff * n_keys + k];
                if (ff < f) before += N[(int64_t)ff * n_keys + k];
            }
            uint64_t sk = oracle_splitmix64(seed ^ (uint64_t)k) % (uint64_t)nk;
            uint64_t c = (uint64_t)batch * (uint64_t)Tk + (uint64_t)before;
            double gk = g[(int64_t)f * n_keys + k];
            for (int64_t r = 0; r < Nik; ++r, ++h) {
                int64_t p = offsets[k] +
                            (int64_t)((sk + c + (uint64_t)r) % (uint64_t)nk);
                src[h] = p;
                field[h] = f;
                keyo[h] = (int32_t)k;
                status[h] = (uint8_t)beam_particle(F, G, x[p], y[p], u[p],
                                                   v[p], w[p], wt[p], E[p],
                                                   gk, state + 8 * h);
            }
        }
    }
    (void)type;
}

/* Methods 1 and 2 (Sec. 2.1, 2.2): the phase space is read in file order
 * and sorted on the fly into bins by particle type (photon; electron or
 * positron) and energy.  History r of batch b reads particle
 *   (s + b * n_hist + r) mod n,  s = splitmix64(seed) mod n,
 * (a random start, as the PSLs get in Sec. 2.3.3; reading wraps at the end
 * of the file).  Method 2 passes each particle through the beam model of
 * field F with weight factor gk; Method 1 (a phase space already
 * collimated) passes the jaw and fluence tests by construction (F without
 * jaws or map).  A particle whose type is neither 0 nor 1, or whose energy
 * is NaN, is dropped (status 4).  An accepted particle joins the bin of its
 * type and energy (largest k with E >= e_edges[k], clamped to the n_e bins);
 * when a bin holds cap particles it is flushed: its particles leave as one
 * transport batch in the order they arrived, and the bin starts empty.
 * After the last history the bins still holding particles are flushed in
 * bin order.  Outputs: status and state (E x y z u v w w') per history;
 * the flushes in order: bin (type * n_e + e), count, trigger (the history
 * whose arrival filled the bin; -1 at the end) and first (the flush's
 * offset in the flushed sequence); seq, the history index of every flushed
 * particle, flushes concatenated.  Returns the number of flushes. */
int64_t oracle_stream(const ofield *F, const ogeom *G, int method, int64_t n,
                      const uint8_t *type, const float *E, const float *x,
                      const float *y, const float *u, const float *v,
                      const float *w, const float *wt, int n_e,
                      const float *e_edges, int64_t n_hist, int64_t batch,
                      uint64_t seed, double gk, int64_t cap, uint8_t *status,
                      double *state, int32_t *fl_bin, int64_t *fl_count,
                      int64_t *fl_trigger, int64_t *fl_first, int64_t *seq)
{
    ofield open = *F;
    if (method == 1) { open.jaws_on = 0; open.nfx = 0; open.nfy = 0; }
    const int n_bins = 2 * n_e;
    int64_t **bin = (int64_t **)calloc((size_t)n_bins, sizeof(int64_t *));
    int64_t *fill = (int64_t *)calloc((size_t)n_bins, sizeof(int64_t));
    int64_t *room = (int64_t *)calloc((size_t)n_bins, sizeof(int64_t));
    int64_t n_fl = 0, n_seq = 0;
    const uint64_t s0 = n > 0 ? oracle_splitmix64(seed) % (uint64_t)n : 0;
    for (int64_t r = 0; r < n_hist; ++r) {
        const int64_t p = (int64_t)((s0 + (uint64_t)batch * (uint64_t)n_hist +
                                     (uint64_t)r) % (uint64_t)n);
        double *S = state + 8 * r;
        if (type[p] > 1 || E[p] != E[p]) {
            for (int q = 0; q < 8; ++q) S[q] = 0.0;
            status[r] = 4;
            continue;
        }
        status[r] = (uint8_t)beam_particle(&open, G, x[p], y[p], u[p], v[p],
                                           w[p], wt[p], E[p], gk, S);
        if (status[r] != 1) continue;
        int e = 0;
        for (int k = 1; k < n_e; ++k)
            if (E[p] >= e_edges[k]) e = k;
        const int b = (int)type[p] * n_e + e;
        if (fill[b] == room[b]) {
            room[b] = room[b] ? 2 * room[b] : 64;
            bin[b] = (int64_t *)realloc(bin[b], (size_t)room[b] * 8);
        }
        bin[b][fill[b]++] = r;
        if (fill[b] == cap) {
            fl_bin[n_fl] = b;
            fl_count[n_fl] = cap;
            fl_trigger[n_fl] = r;
            fl_first[n_fl] = n_seq;
            ++n_fl;
            for (int64_t i = 0; i < cap; ++i) seq[n_seq++] = bin[b][i];
            fill[b] = 0;
        }
    }
    for (int b = 0; b < n_bins; ++b) {
        if (fill[b] == 0) continue;
        fl_bin[n_fl] = b;
        fl_count[n_fl] = fill[b];
        fl_trigger[n_fl] = -1;
        fl_first[n_fl] = n_seq;
        ++n_fl;
        for (int64_t i = 0; i < fill[b]; ++i) seq[n_seq++] = bin[b][i];
        fill[b] = 0;
    }
    for (int b = 0; b < n_bins; ++b) free(bin[b]);
    free(bin);
    free(fill);
    free(room);
    return n_fl;
}

/* ------------------------------------------------------------------------ */
/* Transport physics.                                                        */
/* ------------------------------------------------------------------------ */

typedef struct {
    int32_t nx, ny, nz, pad;
    double dx, dy, dz, x0, y0, z0;
    const float *rho;           /* [nz][ny][nx] g/cm^3 */
} ophantom;

typedef struct {
    double n_e;                 /* electrons / cm^3 at 1 g/cm^3 */
    double I_eV;                /* mean excitation energy */
    double X0;                  /* radiation length, g/cm^2 */
    double step;                /* electron step, cm */
    double p_cut, t_cut;        /* kinetic cut-offs, MeV */
    int32_t flags;              /* 1 first collision only, 2 no scattering */
    int32_t pad;
} ophys;

#define FLAG_FIRST_COLLISION 1
#define FLAG_NO_MSC 2

/* Klein-Nishina total cross section per electron (cm^2), closed form. */
double oracle_kn_sigma(double E)
{
    double k = E / ME;
    double a = 1.0 + 2.0 * k;
    double l = log(a);
    double t1 = (1.0 + k) / (k * k) * (2.0 * (1.0 + k) / a - l / k);
    double t2 = l / (2.0 * k);
    double t3 = (1.0 + 3.0 * k) / (a * a);
    return 2.0 * PI * RE * RE * (t1 + t2 - t3);
}

/* Bethe collision stopping power of electrons, Rohrlich-Carlson form,
 * no density effect, per unit density (MeV cm^2 / g) for a medium with
 * n_e electrons per gram. */
double oracle_stopping_power(double T, double n_e, double I_eV)
{
    double tau = T / ME;
    double gam = tau + 1.0;
    double beta2 = 1.0 - 1.0 / (gam * gam);
    double ir = I_eV * 1.0e-6 / ME;
    double F = 1.0 - beta2 +
               (tau * tau / 8.0 - (2.0 * tau + 1.0) * log(2.0)) / (gam * gam);
    double L = log(tau * tau * (tau + 2.0) / (2.0 * ir * ir));
    return 2.0 * PI * RE * RE * ME * n_e / beta2 * (L + F);
}

/* CSDA residual range from t_lo to T, integral of dT / S(T) (g/cm^2), by
 * adaptive Simpson quadrature. */
static double simpson_inv_s(double a, double b, double fa, double fm, double fb,
                            double whole, double tol, int depth,
                            double n_e, double I)
{
    double m = 0.5 * (a + b);
    double lm = 0.5 * (a + m), rm = 0.5 * (m + b);
    double flm = 1.0 / oracle_stopping_power(lm, n_e, I);
    double frm = 1.0 / oracle_stopping_power(rm, n_e, I);
    double left = (m - a) / 6.0 * (fa + 4.0 * flm + fm);
    double right = (b - m) / 6.0 * (fm + 4.0 * frm + fb);
    if (depth <= 0 || fabs(left + right - whole) <= 15.0 * tol)
        return left + right + (left + right - whole) / 15.0;
    return simpson_inv_s(a, m, fa, flm, fm, left, tol / 2, depth - 1, n_e, I) +
           simpson_inv_s(m, b, fm, frm, fb, right, tol / 2, depth - 1, n_e, I);
}

double oracle_csda_range(double t_lo, double T, double n_e, double I_eV)
{
    if (T <= t_lo) return 0.0;
    double fa = 1.0 / oracle_stopping_power(t_lo, n_e, I_eV);
    double fb = 1.0 / oracle_stopping_power(T, n_e, I_eV);
    double m = 0.5 * (t_lo + T);
    double fm = 1.0 / oracle_stopping_power(m, n_e, I_eV);
    double whole = (T - t_lo) / 6.0 * (fa + 4.0 * fm + fb);
    return simpson_inv_s(t_lo, T, fa, fm, fb, whole, 1e-12, 40, n_e, I_eV);
}

/* Energy after a mass thickness dm (g/cm^2) of CSDA slowing down, by
 * integrating dT/dm = -S(T) with classical Runge-Kutta, sub-steps of at
 * most 0.005 g/cm^2. */
static double csda_slow(double T, double dm, double n_e, double I)
{
    int n = (int)ceil(dm / 0.005);
    if (n < 1) n = 1;
    double h = dm / n;
    for (int i = 0; i < n; ++i) {
        double k1 = oracle_stopping_power(T, n_e, I);
        double k2 = oracle_stopping_power(T - 0.5 * h * k1, n_e, I);
        double k3 = oracle_stopping_power(T - 0.5 * h * k2, n_e, I);
        double k4 = oracle_stopping_power(T - h * k3, n_e, I);
        T -= h / 6.0 * (k1 + 2.0 * k2 + 2.0 * k3 + k4);
    }
    return T;
}

/* Highland characteristic angle (rad) for an electron of kinetic energy T
 * crossing a mass thickness t (g/cm^2), radiation length X0 (g/cm^2). */
double oracle_highland(double T, double t, double X0)
{
    double pbc = T * (T + 2.0 * ME) / (T + ME);
    double r = t / X0;
    double th = 13.6 / pbc * sqrt(r) * (1.0 + 0.038 * log(r));
    return th > 0.0 ? th : 0.0;
}

static double dot3(const double a[3], const double b[3])
{
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

static void cross3(const double a[3], const double b[3], double c[3])
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

/* New direction after deflection by polar angle theta and azimuth phi about
 * d, built from an explicit orthonormal frame (e1, e2, d). */
static void deflect(double d[3], double cth, double sth, double phi)
{
    double a[3] = {0, 0, 0};
    if (fabs(d[0]) < 0.6) a[0] = 1.0; else a[1] = 1.0;
    double e1[3] = {a[1] * d[2] - a[2] * d[1], a[2] * d[0] - a[0] * d[2],
                    a[0] * d[1] - a[1] * d[0]};
    double n1 = sqrt(e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2]);
    for (int i = 0; i < 3; ++i) e1[i] /= n1;
    double e2[3] = {d[1] * e1[2] - d[2] * e1[1], d[2] * e1[0] - d[0] * e1[2],
                    d[0] * e1[1] - d[1] * e1[0]};
    double cp = cos(phi), sp = sin(phi), nd[3];
    for (int i = 0; i < 3; ++i)
        nd[i] = cth * d[i] + sth * (cp * e1[i] + sp * e2[i]);
    double nn = sqrt(nd[0] * nd[0] + nd[1] * nd[1] + nd[2] * nd[2]);
    for (int i = 0; i < 3; ++i) d[i] = nd[i] / nn;
}

/* Multiple-scattering deflection after one electron step: two independent
 * Gaussian projected angles of width theta0 = Highland(T0, t_mass) (Box-
 * Muller), T0 the kinetic energy at the start of the step and t_mass the
 * mass thickness it crossed; the polar angle is resampled while it exceeds
 * pi.  d is turned by that polar angle at the azimuth of the pair. */
static void msc_deflect(xrng *R, double T0, double t_mass, double X0,
                        double d[3])
{
    double th0 = oracle_highland(T0, t_mass, X0), th, ax, ay;
    do {
        double u1 = 1.0 - urand(R), u2 = urand(R);
        double rr = sqrt(-2.0 * log(u1));
        ax = th0 * rr * cos(2.0 * PI * u2);
        ay = th0 * rr * sin(2.0 * PI * u2);
        th = sqrt(ax * ax + ay * ay);
    } while (th > PI);
    deflect(d, cos(th), sin(th), atan2(ay, ax));
}

typedef struct {
    const ophantom *P;
    const ophys *Y;
    double *acc;                /* [voxels] energy (MeV x weight) */
    double dep, esc, killed;    /* per-history ledger (MeV, unweighted) */
    int64_t n_interactions;     /* photon interactions */
    int64_t n_segments;         /* electron voxel segments */
    double *trace;              /* optional: per-particle trace (TRACE_N) */
} octx;

/* Per-particle trace columns (optional output of oracle_transport). */
#define TRACE_N 10
#define TR_Z 0          /* photon: depth z of the first interaction        */
#define TR_COS 1        /*         its scattering cosine                   */
#define TR_T 2          /*         recoil kinetic energy                   */
#define TR_E 3          /*         photon energy before the interaction    */
#define TR_COSE 4       /*         cosine of the recoil electron's         */
                        /*         direction to the incident photon's      */
#define TR_SIDE 5       /*         normalised (d0 x d') . (d0 x p_e): -1   */
                        /*         when photon and electron leave on       */
                        /*         opposite sides of the incident axis     */
#define TR_PNORM 6      /*         |E d0 - E' d'| / sqrt(T (T + 2 m))      */
#define TR_EXIT 7       /* both: direction (3) of the primary at escape    */

static int voxel_of(const ophantom *P, const double p[3], int ijk[3])
{
    double lo[3] = {P->x0, P->y0, P->z0};
    double dd[3] = {P->dx, P->dy, P->dz};
    int nn[3] = {P->nx, P->ny, P->nz};
    for (int a = 0; a < 3; ++a) {
        double f = floor((p[a] - lo[a]) / dd[a]);
        if (f < 0.0 || f >= (double)nn[a]) return 0;
        ijk[a] = (int)f;
    }
    return 1;
}

/* Same, but a point on the box surface is assigned to the adjacent voxel
 * inside the box. */
static int voxel_of_clamped(const ophantom *P, const double p[3], int ijk[3])
{
    double lo[3] = {P->x0, P->y0, P->z0};
    double dd[3] = {P->dx, P->dy, P->dz};
    int nn[3] = {P->nx, P->ny, P->nz};
    for (int a = 0; a < 3; ++a) {
        double f = floor((p[a] - lo[a]) / dd[a]);
        if (f < -1.0 || f > (double)nn[a]) return 0;
        if (f < 0.0) f = 0.0;
        if (f > nn[a] - 1) f = nn[a] - 1;
        ijk[a] = (int)f;
    }
    return 1;
}

/* Energy leaving the phantom; the primary (trace row given) also records
 * its direction at escape. */
static void escape(octx *C, double e, const double d[3], double *tr)
{
    C->esc += e;
    if (tr)
        for (int a = 0; a < 3; ++a) tr[TR_EXIT + a] = d[a];
}

static int64_t vindex(const ophantom *P, const int ijk[3])
{
    return ((int64_t)ijk[2] * P->ny + ijk[1]) * P->nx + ijk[0];
}

static void deposit(octx *C, const int ijk[3], double e, double wgt)
{
    double *a = &C->acc[vindex(C->P, ijk)];
#pragma omp atomic
    *a += e * wgt;
    C->dep += e;
}

/* Distance from p along d to the boundary of voxel ijk, and the axis whose
 * face is crossed first. */
static double exit_distance(const ophantom *P, const double p[3],
                            const double d[3], const int ijk[3], int *axis)
{
    double lo[3] = {P->x0, P->y0, P->z0};
    double dd[3] = {P->dx, P->dy, P->dz};
    double best = INFINITY;
    *axis = -1;
    for (int a = 0; a < 3; ++a) {
        double s;
        if (d[a] > 0.0)
            s = (lo[a] + (ijk[a] + 1) * dd[a] - p[a]) / d[a];
        else if (d[a] < 0.0)
            s = (lo[a] + ijk[a] * dd[a] - p[a]) / d[a];
        else
            continue;
        if (s < 0.0) s = 0.0;
        if (s < best) { best = s; *axis = a; }
    }
    return best;
}

static int step_voxel(const ophantom *P, int ijk[3], int axis,
                      const double d[3])
{
    int nn[3] = {P->nx, P->ny, P->nz};
    ijk[axis] += d[axis] > 0.0 ? 1 : -1;
    return ijk[axis] >= 0 && ijk[axis] < nn[axis];
}

/* Electron: CSDA in steps of Y->step cm.  Within a step the straight
 * segment is split at voxel faces; the energy lost in each piece is
 * deposited in that voxel.  The electron stops where its residual CSDA
 * range above the cut-off runs out, depositing what is left there.  After
 * each complete step the direction is deflected by Highland's Gaussian
 * projected angles for the pre-step energy and the step's mass
 * thickness. */
static void transport_electron(octx *C, xrng *R, double T, double p[3],
                               double d[3], double wgt, double *tr)
{
    const ophantom *P = C->P;
    const ophys *Y = C->Y;
    double n_e = Y->n_e;
    int ijk[3];
    if (!voxel_of_clamped(P, p, ijk)) { escape(C, T, d, tr); return; }
    if (T <= Y->t_cut) { deposit(C, ijk, T, wgt); return; }
    double r_left = oracle_csda_range(Y->t_cut, T, n_e, Y->I_eV);
    for (;;) {
        double remaining = Y->step, t_mass = 0.0, T0 = T;
        while (remaining > 0.0) {
            int axis;
            double sb = exit_distance(P, p, d, ijk, &axis);
            double seg = remaining < sb ? remaining : sb;
            double rho = P->rho[vindex(P, ijk)];
            double dm = rho * seg;
            C->n_segments++;
            if (dm >= r_left) {     /* residual range runs out here */
                deposit(C, ijk, T, wgt);
                return;
            }
            double Tn = csda_slow(T, dm, n_e, Y->I_eV);
            if (Tn < Y->t_cut) Tn = Y->t_cut;
            deposit(C, ijk, T - Tn, wgt);
            T = Tn;
            r_left -= dm;
            t_mass += dm;
            for (int a = 0; a < 3; ++a) p[a] += seg * d[a];
            remaining -= seg;
            if (seg == sb && axis >= 0) {
                if (!step_voxel(P, ijk, axis, d)) {
                    escape(C, T, d, tr);
                    return;
                }
            }
        }
        if (!(Y->flags & FLAG_NO_MSC) && t_mass > 0.0)
            msc_deflect(R, T0, t_mass, Y->X0, d);
    }
}

/* Photon: exact ray march through the voxels.  The optical depth to the
 * next interaction is -ln(xi); each voxel crossed consumes
 * rho n_e sigma_KN(E) times its chord.  At an interaction the Compton
 * scattering angle is drawn by naive rejection from the Klein-Nishina
 * differential cross section; the recoil electron takes the energy and
 * momentum difference.  Electrons above the cut-off are transported at
 * once, others deposit locally; photons below the cut-off deposit
 * locally. */
static void transport_photon(octx *C, xrng *R, double E, double p[3],
                             double d[3], double wgt, int first_only)
{
    const ophantom *P = C->P;
    const ophys *Y = C->Y;
    double *tr = C->trace;
    int ijk[3];
    if (!voxel_of_clamped(P, p, ijk)) { escape(C, E, d, tr); return; }
    int first = 1;
    for (;;) {
        if (E < Y->p_cut) { deposit(C, ijk, E, wgt); return; }
        double tau = -log(1.0 - urand(R));
        double mu1 = Y->n_e * oracle_kn_sigma(E);
        for (;;) {
            int axis;
            double sb = exit_distance(P, p, d, ijk, &axis);
            double mu = P->rho[vindex(P, ijk)] * mu1;
            if (mu > 0.0 && tau <= mu * sb) {
                double s = tau / mu;
                for (int a = 0; a < 3; ++a) p[a] += s * d[a];
                break;
            }
            tau -= mu * sb;
            for (int a = 0; a < 3; ++a) p[a] += sb * d[a];
            if (axis < 0 || !step_voxel(P, ijk, axis, d)) {
                escape(C, E, d, tr);
                return;
            }
        }
        /* Compton interaction: naive rejection on cos(theta) ~ U[-1,1]
         * against the Klein-Nishina differential cross section, whose
         * maximum over angle is at theta = 0. */
        double k = E / ME, ct, Pr;
        for (;;) {
            ct = 2.0 * urand(R) - 1.0;
            Pr = 1.0 / (1.0 + k * (1.0 - ct));
            double f = 0.5 * Pr * Pr * (Pr + 1.0 / Pr - (1.0 - ct * ct));
            if (urand(R) < f) break;
        }
        double Es = E * Pr, T = E - Es;
        double phi = 2.0 * PI * urand(R);
        double st = sqrt(fmax(0.0, 1.0 - ct * ct));
        double dold[3] = {d[0], d[1], d[2]};
        deflect(d, ct, st, phi);
        C->n_interactions++;
        /* recoil electron: momentum conservation, p_e = p_photon - p'
         * (in MeV/c, photon momentum = its energy) */
        double pe[3];
        for (int a = 0; a < 3; ++a) pe[a] = E * dold[a] - Es * d[a];
        double pn = sqrt(pe[0] * pe[0] + pe[1] * pe[1] + pe[2] * pe[2]);
        for (int a = 0; a < 3; ++a) pe[a] /= pn;
        if (tr && first) {
            double c1[3], c2[3];
            cross3(dold, d, c1);
            cross3(dold, pe, c2);
            double n1 = sqrt(dot3(c1, c1)), n2 = sqrt(dot3(c2, c2));
            tr[TR_Z] = p[2];
            tr[TR_COS] = ct;
            tr[TR_T] = T;
            tr[TR_E] = E;
            tr[TR_COSE] = dot3(dold, pe);
            tr[TR_SIDE] = n1 > 0.0 && n2 > 0.0 ? dot3(c1, c2) / (n1 * n2)
                                               : NAN;
            tr[TR_PNORM] = pn / sqrt(T * (T + 2.0 * ME));
        }
        first = 0;
        if (first_only) {
            deposit(C, ijk, T, wgt);
            C->killed += Es;
            return;
        }
        if (T > Y->t_cut) {
            double pp[3] = {p[0], p[1], p[2]};
            transport_electron(C, R, T, pp, pe, wgt, NULL);
        } else {
            deposit(C, ijk, T, wgt);
        }
        E = Es;
    }
}

/* Transport n particles (state rows E x y z u v w wt) of the given types
 * and accumulate energy x weight per voxel into acc (MeV).  The random
 * stream of particle i is keyed by (seed, uid[i]).  ledger, if given,
 * receives per particle (E0, deposited, escaped, killed) unweighted;
 * trace, if given, receives TRACE_N values per particle: the kinematics of
 * the first photon interaction and the primary's direction at escape (the
 * TR_* columns; NaN where they do not apply).  counts[0] += photon interactions,
 * counts[1] += electron voxel segments. */
void oracle_transport(int64_t n, const uint8_t *type, const double *state,
                      const uint64_t *uid, uint64_t seed, const ophantom *P,
                      const ophys *Y, double *acc, double *ledger,
                      double *trace, int64_t *counts, int n_threads)
{
    int64_t ni = 0, ns = 0;
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#else
    (void)n_threads;
#endif
#pragma omp parallel for schedule(dynamic, 256) reduction(+ : ni, ns)
    for (int64_t i = 0; i < n; ++i) {
        octx C;
        C.P = P;
        C.Y = Y;
        C.acc = acc;
        C.dep = C.esc = C.killed = 0.0;
        C.n_interactions = C.n_segments = 0;
        double tr[TRACE_N];
        for (int a = 0; a < TRACE_N; ++a) tr[a] = NAN;
        C.trace = trace ? tr : NULL;
        xrng R;
        xseed(&R, seed, uid[i]);
        const double *S = state + 8 * i;
        double p[3] = {S[1], S[2], S[3]}, d[3] = {S[4], S[5], S[6]};
        double dn = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        for (int a = 0; a < 3; ++a) d[a] /= dn;
        if (type[i] == 0)
            transport_photon(&C, &R, S[0], p, d, S[7],
                             Y->flags & FLAG_FIRST_COLLISION);
        else
            transport_electron(&C, &R, S[0], p, d, S[7], C.trace);
        if (ledger) {
            ledger[4 * i + 0] = S[0];
            ledger[4 * i + 1] = C.dep;
            ledger[4 * i + 2] = C.esc;
            ledger[4 * i + 3] = C.killed;
        }
        if (trace)
            for (int a = 0; a < TRACE_N; ++a) trace[TRACE_N * i + a] = tr[a];
        ni += C.n_interactions;
        ns += C.n_segments;
    }
    counts[0] += ni;
    counts[1] += ns;
}

/* Sample the Highland deflection of the oracle n times for (T, t) and
 * return the projected angles on the two axes perpendicular to an initial
 * direction along +z (for the pin of the scattering sampler). */
void oracle_msc_samples(int64_t n, double T, double t, double X0,
                        uint64_t seed, double *proj)
{
    xrng R;
    xseed(&R, seed, 0);
    for (int64_t i = 0; i < n; ++i) {
        double d[3] = {0.0, 0.0, 1.0};
        msc_deflect(&R, T, t, X0, d);
        proj[2 * i + 0] = atan2(d[0], d[2]);
        proj[2 * i + 1] = atan2(d[1], d[2]);
    }
}
