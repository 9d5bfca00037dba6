// Gamma index of one dose against another: one thread per reference voxel
// searches a fixed lattice of offsets inside the distance-to-agreement
// sphere, interpolating the evaluated dose trilinearly (indices clamped),
// and keeps the smallest gamma^2.  Double arithmetic, so that pass/fail
// decisions agree with any other double implementation of the definition
// up to ties.
#include "common.hpp"

#include <cmath>

namespace psl {
namespace {

struct GammaArgs {
    int nx, ny, nz, n_off;
    double dx, dy, dz;        // voxel size
    double inv_dd2, inv_dta2, lim2, dta, step, ref_min;
};

__device__ __forceinline__ double tri(const float *__restrict__ e,
                                      const GammaArgs &A, double cz,
                                      double cy, double cx) {
    const double fz = floor(cz), fy = floor(cy), fx = floor(cx);
    const double wz = cz - fz, wy = cy - fy, wx = cx - fx;
    const int z0 = min(max((int)fz, 0), A.nz - 1),
              z1 = min(max((int)fz + 1, 0), A.nz - 1);
    const int y0 = min(max((int)fy, 0), A.ny - 1),
              y1 = min(max((int)fy + 1, 0), A.ny - 1);
    const int x0 = min(max((int)fx, 0), A.nx - 1),
              x1 = min(max((int)fx + 1, 0), A.nx - 1);
    auto at = [&](int z, int y, int x) {
        return (double)e[((int64_t)z * A.ny + y) * A.nx + x];
    };
    const double c00 = at(z0, y0, x0) * (1 - wx) + at(z0, y0, x1) * wx;
    const double c01 = at(z0, y1, x0) * (1 - wx) + at(z0, y1, x1) * wx;
    const double c10 = at(z1, y0, x0) * (1 - wx) + at(z1, y0, x1) * wx;
    const double c11 = at(z1, y1, x0) * (1 - wx) + at(z1, y1, x1) * wx;
    const double c0 = c00 * (1 - wy) + c01 * wy;
    const double c1 = c10 * (1 - wy) + c11 * wy;
    return c0 * (1 - wz) + c1 * wz;
}

__global__ void __launch_bounds__(256)
k_gamma(const float *__restrict__ ref, const float *__restrict__ ev,
        GammaArgs A, float *__restrict__ g2out,
        unsigned long long *__restrict__ counts) {
    const int64_t nvox = (int64_t)A.nx * A.ny * A.nz;
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool eval = false, pass = false;
    if (v < nvox) {
        const double r = ref[v];
        eval = r >= A.ref_min;
        if (eval) {
            const int x = (int)(v % A.nx);
            const int y = (int)((v / A.nx) % A.ny);
            const int z = (int)(v / ((int64_t)A.nx * A.ny));
            double best = INFINITY;
            for (int k = 0; k < A.n_off; ++k) {
                const double oz = -A.dta + k * A.step;
                for (int j = 0; j < A.n_off; ++j) {
                    const double oy = -A.dta + j * A.step;
                    for (int i = 0; i < A.n_off; ++i) {
                        const double ox = -A.dta + i * A.step;
                        const double d2 = ox * ox + oy * oy + oz * oz;
                        if (d2 > A.lim2) continue;
                        const double e = tri(ev, A, z + oz / A.dz,
                                             y + oy / A.dy, x + ox / A.dx);
                        const double dd = e - r;
                        const double g2 = d2 * A.inv_dta2 + dd * dd * A.inv_dd2;
                        best = fmin(best, g2);
                    }
                }
            }
            pass = best <= 1.0;
            if (g2out) g2out[v] = (float)best;
        } else if (g2out) {
            g2out[v] = -1.0f;
        }
    }
    const uint64_t ne = __popcll(__ballot(eval));
    const uint64_t np = __popcll(__ballot(pass));
    if (__lane_id() == 0 && ne) {
        atomicAdd(&counts[0], (unsigned long long)ne);
        if (np) atomicAdd(&counts[1], (unsigned long long)np);
    }
}

}  // namespace
}  // namespace psl

using namespace psl;

extern "C" psl_status dose_gamma(const float *d_ref, const float *d_eval,
                                 int32_t nx, int32_t ny, int32_t nz,
                                 double dx, double dy, double dz, double dd,
                                 double dta, double step, double ref_min,
                                 float *d_gamma2, uint64_t *d_counts,
                                 void *stream) {
    PSL_REQUIRE(d_ref && d_eval && d_counts, "NULL argument");
    PSL_REQUIRE(nx > 0 && ny > 0 && nz > 0, "empty volume");
    PSL_REQUIRE(dx > 0 && dy > 0 && dz > 0, "voxel sizes must be positive");
    PSL_REQUIRE(dd > 0 && dta > 0 && step > 0,
                "dose criterion, DTA and step must be positive");
    const double n_off = std::ceil((2.0 * dta + 1e-12) / step);
    PSL_REQUIRE(n_off >= 1 && n_off <= 64,
                "%g offsets per axis (2 dta / step) outside 1..64", n_off);
    if (psl_status s = check_device()) return s;
    GammaArgs A{nx, ny, nz, (int)n_off, dx, dy, dz,
                1.0 / (dd * dd), 1.0 / (dta * dta), dta * dta + 1e-12, dta,
                step, ref_min};
    const int64_t nvox = (int64_t)nx * ny * nz;
    hipLaunchKernelGGL(k_gamma, dim3((unsigned)((nvox + 255) / 256)),
                       dim3(256), 0, (hipStream_t)stream, d_ref, d_eval, A,
                       d_gamma2,
                       reinterpret_cast<unsigned long long *>(d_counts));
    PSL_LAUNCHED();
    return PSL_OK;
}
