// dose_tally: per-batch fold of the energy tally into running sums of the
// tally and its square, and the final dose with its batch standard error
// (Sec. 2.3.3) normalised per incident particle (Eq. 5).  Both passes are
// streaming and bound by HBM bandwidth.
#include "common.hpp"

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

}  // namespace
}  // namespace psl

using namespace psl;

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
