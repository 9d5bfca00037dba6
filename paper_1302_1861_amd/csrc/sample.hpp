// Internal interface of the PSL source, shared by psl_sample and the
// batched plan: host-side setup (validation, workspace carving, field
// descriptors), the allocation kernels (run once per plan) and the
// per-batch sampling kernels (capturable in a graph: kernels only, batch
// index read from device memory).
#pragma once

#include <vector>

#include "common.hpp"
#include "compact.hpp"

namespace psl {

struct FieldDev {
    double X1, X2, Y1, Y2;
    double cos_g, sin_g, MU;
    const float *fluence;
    int32_t nfx, nfy, jaws_on, pad;
    double f_x0, f_y0, f_pix;
};

struct Geo {
    double sad, z_x, z_y, z_psl;
    double iso[3], lo[3], hi[3];
};

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
// Writes v into *p / adds 1 to *p (device int64), as kernels.
psl_status set_i64(int64_t *p, int64_t v, hipStream_t st);
psl_status inc_i64(int64_t *p, hipStream_t st);

psl_status validate_queue(const psl_queue *q);

}  // namespace psl
