// dose_tally: per-batch fold of the energy tally into running sums of the
// tally and its square, and the final dose with its batch standard error
// (Sec. 2.3.3) normalised per incident particle (Eq. 5).  Both passes are
// streaming and bound by HBM bandwidth.
#include "common.hpp"

#include <cmath>

namespace psl {
namespace {

constexpr int kBlock = 256;

template <int MODE>
__global__ void __launch_bounds__(kBlock)
k_fold(void *acc, double inv_scale, double *__restrict__ s1,
       double *__restrict__ s2, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += stride) {
        double a;
        if (MODE == PSL_ACC_FIXED64) {
            uint64_t *p = reinterpret_cast<uint64_t *>(acc) + i;
            a = (double)*p * inv_scale;
            *p = 0;
        } else {
            double *p = reinterpret_cast<double *>(acc) + i;
            a = *p;
            *p = 0.0;
        }
        s1[i] += a;
        s2[i] += a * a;
    }
}

__global__ void __launch_bounds__(kBlock)
k_finalize(const double *__restrict__ s1, const double *__restrict__ s2,
           const float *__restrict__ rho, double inv_mass_unit, double norm,
           int B, float *__restrict__ dose, float *__restrict__ sigma,
           int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    const double invB = 1.0 / B;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += stride) {
        double r = rho[i];
        double c = r > 0.0 ? 1.602176634e-10 * inv_mass_unit / r * norm : 0.0;
        double a = s1[i], q = s2[i];
        double var = fmax(q - a * a * invB, 0.0) / (B - 1);
        dose[i] = (float)(a * invB * c);
        sigma[i] = (float)(sqrt(var * invB) * c);
    }
}

// Reference-point dose (Sec. 2.5): one block sums, over the voxels of the
// sphere's bounding box whose centres lie within the radius, the dose, the
// squared standard errors and the count, in a fixed order (thread-strided
// partial sums, then a tree in LDS).
constexpr int kPointBlock = 256;
__global__ void __launch_bounds__(kPointBlock)
k_dose_point(const float *__restrict__ dose, const float *__restrict__ sigma,
             int nx, int ny, int nz, double x0, double y0, double z0,
             double dx, double dy, double dz, double px, double py,
             double pz, double radius, int ilo, int ihi, int jlo, int jhi,
             int klo, int khi, int fi, int fj, int fk, double *out) {
#pragma clang fp contract(off)
    __shared__ double s_d[kPointBlock], s_v[kPointBlock], s_n[kPointBlock];
    const int64_t wi = ihi - ilo + 1, wj = jhi - jlo + 1, wk = khi - klo + 1;
    const int64_t m = wi * wj * wk;
    double sd = 0.0, sv = 0.0, sn = 0.0;
    const double r2 = radius < 0.0 ? -1.0 : radius * radius;  // < 0: none
    for (int64_t t = threadIdx.x; t < m; t += kPointBlock) {
        const int i = ilo + (int)(t % wi);
        const int j = jlo + (int)((t / wi) % wj);
        const int k = klo + (int)(t / (wi * wj));
        const double cx = x0 + ((double)i + 0.5) * dx - px;
        const double cy = y0 + ((double)j + 0.5) * dy - py;
        const double cz = z0 + ((double)k + 0.5) * dz - pz;
        const bool in = cx * cx + cy * cy + cz * cz <= r2;
        if (in) {
            const int64_t v = ((int64_t)k * ny + j) * nx + i;
            const double s = sigma[v];
            sd += (double)dose[v];
            sv += s * s;
            sn += 1.0;
        }
    }
    s_d[threadIdx.x] = sd;
    s_v[threadIdx.x] = sv;
    s_n[threadIdx.x] = sn;
    __syncthreads();
    for (int h = kPointBlock / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            s_d[threadIdx.x] += s_d[threadIdx.x + h];
            s_v[threadIdx.x] += s_v[threadIdx.x + h];
            s_n[threadIdx.x] += s_n[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        double d = s_d[0], v = s_v[0], n = s_n[0];
        if (n == 0.0 && fi >= 0) {
            // no voxel centre inside the sphere: the voxel holding the point
            const int64_t c = ((int64_t)fk * ny + fj) * nx + fi;
            const double s = sigma[c];
            d = dose[c];
            v = s * s;
            n = 1.0;
        }
        out[0] = n > 0.0 ? d / n : 0.0;
        out[1] = n > 0.0 ? sqrt(v) / n : 0.0;
        out[2] = n;
    }
}

}  // namespace
}  // namespace psl

using namespace psl;

extern "C" psl_status dose_point(const float *d_dose, const float *d_sigma,
                                 const psl_phantom *ph, double x, double y,
                                 double z, double radius, double *d_out,
                                 void *stream) {
    PSL_REQUIRE(d_dose && d_sigma && ph && d_out, "NULL argument");
    PSL_REQUIRE(ph->nx > 0 && ph->ny > 0 && ph->nz > 0, "bad phantom");
    PSL_REQUIRE(ph->dx > 0 && ph->dy > 0 && ph->dz > 0, "bad voxel size");
    PSL_REQUIRE(radius >= 0 && std::isfinite(radius) && std::isfinite(x) &&
                    std::isfinite(y) && std::isfinite(z),
                "bad point or radius");
    // index range of the voxels whose centres can lie in the sphere
    auto lo_hi = [](double c, double r, double o, double d, int n, int *lo,
                    int *hi) {
        double a = std::ceil((c - r - o) / d - 0.5);
        double b = std::floor((c + r - o) / d - 0.5);
        *lo = (int)std::max(0.0, a);
        *hi = (int)std::min((double)(n - 1), b);
    };
    int ilo, ihi, jlo, jhi, klo, khi;
    lo_hi(x, radius, ph->x0, ph->dx, ph->nx, &ilo, &ihi);
    lo_hi(y, radius, ph->y0, ph->dy, ph->ny, &jlo, &jhi);
    lo_hi(z, radius, ph->z0, ph->dz, ph->nz, &klo, &khi);
    if (ihi < ilo || jhi < jlo || khi < klo) {   // nothing in the box
        ilo = ihi = jlo = jhi = klo = khi = 0;
        radius = -1.0;                            // no centre qualifies
    }
    PSL_REQUIRE((int64_t)(ihi - ilo + 1) * (jhi - jlo + 1) * (khi - klo + 1) <=
                    ((int64_t)1 << 26),
                "radius spans more than 2^26 voxels");
    // the voxel holding the point, if the point is inside the phantom
    const double fx = std::floor((x - ph->x0) / ph->dx);
    const double fy = std::floor((y - ph->y0) / ph->dy);
    const double fz = std::floor((z - ph->z0) / ph->dz);
    int fi = -1, fj = -1, fk = -1;
    if (fx >= 0 && fx < ph->nx && fy >= 0 && fy < ph->ny && fz >= 0 &&
        fz < ph->nz) {
        fi = (int)fx; fj = (int)fy; fk = (int)fz;
    }
    if (psl_status s = check_device()) return s;
    hipLaunchKernelGGL(k_dose_point, dim3(1), dim3(kPointBlock), 0,
                       (hipStream_t)stream, d_dose, d_sigma, ph->nx, ph->ny,
                       ph->nz, ph->x0, ph->y0, ph->z0, ph->dx, ph->dy, ph->dz,
                       x, y, z, radius, ilo, ihi, jlo, jhi, klo, khi, fi, fj,
                       fk, d_out);
    PSL_LAUNCHED();
    return PSL_OK;
}

extern "C" psl_status dose_tally(psl_dose_acc *acc, double *d_s1,
                                 double *d_s2, int32_t op, int32_t n_batches,
                                 const psl_phantom *ph, double norm,
                                 float *d_dose, float *d_sigma,
                                 void *stream) {
    PSL_REQUIRE(ph && d_s1 && d_s2, "NULL argument");
    PSL_REQUIRE(ph->nx > 0 && ph->ny > 0 && ph->nz > 0, "bad phantom");
    const int64_t n = (int64_t)ph->nx * ph->ny * ph->nz;
    hipStream_t st = (hipStream_t)stream;
    const int cu = device_cu_count();
    const int64_t blocks = std::min<int64_t>((n + kBlock - 1) / kBlock,
                                             (int64_t)cu * 16);
    if (op == PSL_TALLY_FOLD) {
        PSL_REQUIRE(acc && acc->data, "NULL accumulator");
        PSL_REQUIRE(acc->mode == PSL_ACC_F64 ||
                        (acc->mode == PSL_ACC_FIXED64 &&
                         acc->frac_bits >= 16 && acc->frac_bits <= 40),
                    "bad accumulator mode");
        if (psl_status s = check_device()) return s;
        ProfScope prof(PSL_PROF_FOLD, st);
        if (acc->mode == PSL_ACC_FIXED64)
            hipLaunchKernelGGL(k_fold<PSL_ACC_FIXED64>, dim3((unsigned)blocks),
                               dim3(kBlock), 0, st, acc->data,
                               std::ldexp(1.0, -acc->frac_bits), d_s1, d_s2, n);
        else
            hipLaunchKernelGGL(k_fold<PSL_ACC_F64>, dim3((unsigned)blocks),
                               dim3(kBlock), 0, st, acc->data, 1.0, d_s1,
                               d_s2, n);
    } else if (op == PSL_TALLY_FINALIZE) {
        PSL_REQUIRE(n_batches >= 2, "need at least 2 batches");
        PSL_REQUIRE(d_dose && d_sigma && ph->density, "NULL output");
        PSL_REQUIRE(ph->dx > 0 && ph->dy > 0 && ph->dz > 0, "bad voxel size");
        if (psl_status s = check_device()) return s;
        double inv_vol = 1.0 / (ph->dx * ph->dy * ph->dz);
        ProfScope prof(PSL_PROF_FINALIZE, st);
        hipLaunchKernelGGL(k_finalize, dim3((unsigned)blocks), dim3(kBlock), 0,
                           st, d_s1, d_s2, ph->density, inv_vol, norm,
                           n_batches, d_dose, d_sigma, n);
    } else {
        PSL_REQUIRE(false, "op = %d", op);
    }
    PSL_LAUNCHED();
    return PSL_OK;
}
