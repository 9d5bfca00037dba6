// Error reporting, version and device checks of the C ABI.
#include "common.hpp"

#include <cstring>
#include <mutex>
#include <vector>

namespace psl {

static thread_local char g_err[1024] = "";

void set_error(const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
}

psl_status check_device() {
    int dev = 0;
    PSL_HIP(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    PSL_HIP(hipGetDeviceProperties(&prop, dev));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
        set_error("device %d is %s; this library is built for gfx950", dev,
                  prop.gcnArchName);
        return PSL_EUNSUPPORTED;
    }
    return PSL_OK;
}

int device_cu_count() {
    static thread_local int cached_dev = -1, cached_cu = 0;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (dev != cached_dev) {
        int cu = 0;
        if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount,
                                  dev) != hipSuccess || cu <= 0)
            cu = 256;
        cached_dev = dev;
        cached_cu = cu;
    }
    return cached_cu;
}

// ------------------------------------------------------- stats reduction --
namespace {
constexpr int kRedBlock = 256;
__global__ void __launch_bounds__(kRedBlock)
k_stats_reduce(const uint64_t *__restrict__ part, int n_blocks,
               psl_stats *out) {
    __shared__ uint64_t s[kRedBlock];
    uint64_t *o = reinterpret_cast<uint64_t *>(out);
    const int i = blockIdx.x;   // one statistics word per block
    const bool is_int = i < kStatFirstDouble;
    uint64_t v = 0;
    double d = 0.0;
    for (int b = threadIdx.x; b < n_blocks; b += kRedBlock) {
        uint64_t x = part[(int64_t)b * kStatWords + i];
        if (is_int) v += x;
        else d += __longlong_as_double(x);
    }
    s[threadIdx.x] = is_int ? v : (uint64_t)__double_as_longlong(d);
    __syncthreads();
    for (int h = kRedBlock / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h) {
            if (is_int)
                s[threadIdx.x] += s[threadIdx.x + h];
            else
                s[threadIdx.x] = __double_as_longlong(
                    __longlong_as_double(s[threadIdx.x]) +
                    __longlong_as_double(s[threadIdx.x + h]));
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (is_int) o[i] += s[0];
        else o[i] = __double_as_longlong(__longlong_as_double(o[i]) +
                                         __longlong_as_double(s[0]));
    }
}
}  // namespace

psl_status stats_reduce(const uint64_t *part, int n_blocks, psl_stats *out,
                        hipStream_t st) {
    hipLaunchKernelGGL(k_stats_reduce, dim3(kStatWords), dim3(kRedBlock), 0,
                       st, part, n_blocks, out);
    PSL_LAUNCHED();
    return PSL_OK;
}

// ------------------------------------------------------------- profiler --
namespace {
struct Pending {
    int group;
    hipEvent_t a, b;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<Pending> g_pending;
double g_ms[PSL_PROF_N] = {0};
int64_t g_launches[PSL_PROF_N] = {0};
}  // namespace

ProfScope::ProfScope(int group, hipStream_t st) : group_(group), st_(st) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (!g_prof_on) return;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st_, &cs) != hipSuccess ||
        cs != hipStreamCaptureStatusNone)
        return;   // no timing events inside a graph being captured
    if (hipEventCreate(&a_) != hipSuccess) return;
    if (hipEventCreate(&b_) != hipSuccess) {
        (void)hipEventDestroy(a_);
        return;
    }
    if (hipEventRecord(a_, st_) != hipSuccess) {
        (void)hipEventDestroy(a_);
        (void)hipEventDestroy(b_);
        return;
    }
    active_ = true;
}

ProfScope::~ProfScope() {
    if (!active_) return;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (hipEventRecord(b_, st_) != hipSuccess) {
        (void)hipEventDestroy(a_);
        (void)hipEventDestroy(b_);
        return;
    }
    g_pending.push_back(Pending{group_, a_, b_});
}

}  // namespace psl

extern "C" psl_status psl_profile_enable(int32_t on) {
    std::lock_guard<std::mutex> lk(psl::g_prof_mu);
    psl::g_prof_on = on != 0;
    return PSL_OK;
}

extern "C" psl_status psl_profile_read(double *ms, int64_t *launches,
                                       int32_t reset) {
    std::lock_guard<std::mutex> lk(psl::g_prof_mu);
    psl_status st = PSL_OK;
    for (auto &p : psl::g_pending) {
        float t = 0.0f;
        if (hipEventSynchronize(p.b) == hipSuccess &&
            hipEventElapsedTime(&t, p.a, p.b) == hipSuccess) {
            psl::g_ms[p.group] += t;
            psl::g_launches[p.group] += 1;
        } else {
            psl::set_error("profiling event failed");
            st = PSL_EHIP;
        }
        (void)hipEventDestroy(p.a);
        (void)hipEventDestroy(p.b);
    }
    psl::g_pending.clear();
    for (int i = 0; i < PSL_PROF_N; ++i) {
        if (ms) ms[i] = psl::g_ms[i];
        if (launches) launches[i] = psl::g_launches[i];
        if (reset) {
            psl::g_ms[i] = 0.0;
            psl::g_launches[i] = 0;
        }
    }
    return st;
}

extern "C" const char *psl_last_error(void) { return psl::g_err; }
extern "C" int32_t psl_version(void) { return PSL_ABI_VERSION; }
