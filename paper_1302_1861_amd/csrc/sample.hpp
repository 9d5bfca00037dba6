// Internal interface of the PSL source, shared by psl_sample and the
// batched plan: host-side setup (validation, workspace carving, field
// descriptors), the allocation kernels (run once per plan) and the
// per-batch sampling kernels (capturable in a graph: kernels only, batch
// index read from device memory).
#pragma once

#include <cmath>
#include <vector>

#include "common.hpp"
#include "compact.hpp"

namespace psl {

struct FieldDev {
    double X1, X2, Y1, Y2;
    double cos_g, sin_g, MU;
    const float *fluence;
    int32_t nfx, nfy, jaws_on, turned;   // turned: collimator or couch != 0
    double f_x0, f_y0, f_pix;
    double cos_c, sin_c, cos_t, sin_t;   // collimator, couch (table)
};

// Host: the device descriptor of a field (angles in degrees).
inline FieldDev make_field_dev(const psl_field &f, bool jaws,
                               bool fluence) {
    const double g = f.gantry_deg * (M_PI / 180.0);
    const double c = f.collimator_deg * (M_PI / 180.0);
    const double t = f.couch_deg * (M_PI / 180.0);
    return FieldDev{f.X1, f.X2, f.Y1, f.Y2, std::cos(g), std::sin(g), f.MU,
                    fluence ? f.fluence : nullptr,
                    fluence ? f.nfx : 0, fluence ? f.nfy : 0, jaws ? 1 : 0,
                    (f.collimator_deg != 0.0 || f.couch_deg != 0.0) ? 1 : 0,
                    f.f_x0, f.f_y0, f.f_pix, std::cos(c), std::sin(c),
                    std::cos(t), std::sin(t)};
}

struct Geo {
    double sad, z_x, z_y, z_psl;
    double iso[3], lo[3], hi[3];
};

// One phase-space particle through the beam model (Sec. 2.2, 2.4), from its
// position (x, y) at the phase-space plane and direction (u, v, w): the
// jaws as perfect collimators (edges given at SAD, closed interval), the
// weight of the fluence-map pixel its ray crosses at the SAD plane (outside
// the map or zero rejects), w' = wt * fluence * g, the gantry rotation about
// +y through the isocentre and the straight move onto the phantom box.
// Returns 0 jaw-rejected, 1 accepted, 2 zero fluence, 3 misses the phantom;
// on acceptance o = x y z u v w w', each rounded to float from its double
// value.  Double precision, no contraction, so every decision is
// reproducible operation by operation.
__device__ __forceinline__ int beam_model(const FieldDev &F, const Geo &geo,
                                          float fx_, float fy_, float fu,
                                          float fv, float fw, float fwt,
                                          double g, float o[7]) {
#pragma clang fp contract(off)
    const double px = fx_, py = fy_, pz = geo.z_psl;
    const double du = fu, dv = fv, dw = fw;
    if (F.jaws_on) {
        if (!(dw > 0.0)) return 0;
        double tx = du / dw, ty = dv / dw;
        double xj = px + tx * (geo.z_x - pz);
        double yj = py + ty * (geo.z_y - pz);
        double xlo = F.X1 * geo.z_x / geo.sad;
        double xhi = F.X2 * geo.z_x / geo.sad;
        double ylo = F.Y1 * geo.z_y / geo.sad;
        double yhi = F.Y2 * geo.z_y / geo.sad;
        if (!(xj >= xlo && xj <= xhi && yj >= ylo && yj <= yhi)) return 0;
    }
    double fl = 1.0;
    if (F.nfx > 0) {
        if (!(dw > 0.0)) return 2;
        double xs = px + (du / dw) * (geo.sad - pz);
        double ys = py + (dv / dw) * (geo.sad - pz);
        double fx = floor((xs - F.f_x0) / F.f_pix);
        double fy = floor((ys - F.f_y0) / F.f_pix);
        if (!(fx >= 0.0 && fy >= 0.0 && fx < (double)F.nfx &&
              fy < (double)F.nfy))
            fl = 0.0;
        else
            fl = (double)F.fluence[(int64_t)fy * F.nfx + (int64_t)fx];
        if (!(fl > 0.0)) return 2;
    }
    const double wgt = (double)fwt * fl * g;
    double rx = px - geo.iso[0], ry = py - geo.iso[1], rz = pz - geo.iso[2];
    double au = du, av = dv;
    if (F.turned) {
        // collimator: about the central axis (z through the isocentre)
        const double x1 = F.cos_c * rx - F.sin_c * ry;
        const double y1 = F.sin_c * rx + F.cos_c * ry;
        const double u1 = F.cos_c * au - F.sin_c * av;
        const double v1 = F.sin_c * au + F.cos_c * av;
        rx = x1; ry = y1; au = u1; av = v1;
    }
    // gantry: about +y through the isocentre
    double qx = F.cos_g * rx + F.sin_g * rz + geo.iso[0];
    double qy = ry + geo.iso[1];
    double qz = -F.sin_g * rx + F.cos_g * rz + geo.iso[2];
    double eu = F.cos_g * au + F.sin_g * dw;
    double ev = av;
    double ew = -F.sin_g * au + F.cos_g * dw;
    if (F.turned) {
        // couch: the patient turns by +angle about the vertical (z at
        // gantry 0) through the isocentre, so the beam turns by -angle
        const double sx = qx - geo.iso[0], sy = qy - geo.iso[1];
        qx = F.cos_t * sx + F.sin_t * sy + geo.iso[0];
        qy = -F.sin_t * sx + F.cos_t * sy + geo.iso[1];
        const double u2 = F.cos_t * eu + F.sin_t * ev;
        const double v2 = -F.sin_t * eu + F.cos_t * ev;
        eu = u2; ev = v2;
    }
    double pos[3] = {qx, qy, qz}, dir[3] = {eu, ev, ew};
    double tn = -INFINITY, tf = INFINITY;
    bool miss = false;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (dir[a] != 0.0) {
            double t1 = (geo.lo[a] - pos[a]) / dir[a];
            double t2 = (geo.hi[a] - pos[a]) / dir[a];
            double l = t1 < t2 ? t1 : t2, u = t1 < t2 ? t2 : t1;
            if (l > tn) tn = l;
            if (u < tf) tf = u;
        } else if (pos[a] < geo.lo[a] || pos[a] > geo.hi[a]) {
            miss = true;
        }
    }
    if (miss || tn > tf || tf <= 0.0) return 3;
    const double t = tn > 0.0 ? tn : 0.0;
    o[0] = (float)(pos[0] + t * dir[0]);
    o[1] = (float)(pos[1] + t * dir[1]);
    o[2] = (float)(pos[2] + t * dir[2]);
    o[3] = (float)eu;
    o[4] = (float)ev;
    o[5] = (float)ew;
    o[6] = (float)wgt;
    return 1;
}

struct SampleWs {
    FieldDev *fields;
    uint8_t *mask;
    int64_t *C, *NF, *N, *H, *before, *T;
    double *g, *mu_tot;
    uint64_t *chunks, *h_total, *part;
    int64_t *batch;
    Slots slots;
    uint32_t *tiles;
    size_t bytes;
};

SampleWs carve_sample_impl(void *base, int64_t n_keys, int P, int F,
                           int64_t n_hist);

struct SampleCtx {
    SampleWs w;
    psl_phsp sorted;
    const int64_t *offsets;
    psl_grid g;
    Geo geo;
    int n_fields, P, cull, alloc_mode;
    int64_t n_keys, n_ranges, n_hist;
    uint64_t seed;
    psl_queue q;
    psl_stats *stats;
    uint8_t *mask;
    int64_t *N;
    std::vector<FieldDev> fd;
};

// Validates the arguments and fills ctx (host only, nothing enqueued).
psl_status sample_setup(const psl_phsp *sorted, const int64_t *d_offsets,
                        const psl_grid *g, const psl_field *fields,
                        int32_t n_fields, const psl_sample_cfg *cfg,
                        const psl_queue *q, uint8_t *d_mask, int64_t *d_alloc,
                        psl_stats *d_stats, void *d_ws, size_t ws_bytes,
                        SampleCtx *ctx);
// Uploads the field descriptors and enqueues ROI selection and allocation.
psl_status sample_alloc(const SampleCtx &ctx, hipStream_t st);
// Enqueues one batch (index read from *d_batch): statistics and queue reset,
// the per-history kernel, compaction into the queues.
psl_status sample_batch(const SampleCtx &ctx, const int64_t *d_batch,
                        hipStream_t st);
// Writes v into *p / adds 1 / adds v to *p (device int64), as kernels.
psl_status set_i64(int64_t *p, int64_t v, hipStream_t st);
psl_status inc_i64(int64_t *p, hipStream_t st);
psl_status add_i64(int64_t *p, int64_t v, hipStream_t st);

psl_status validate_queue(const psl_queue *q);

}  // namespace psl
