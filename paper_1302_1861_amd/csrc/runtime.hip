// Error reporting, version and device checks of the C ABI.
#include "common.hpp"

#include <cstring>

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

}  // namespace psl

extern "C" const char *psl_last_error(void) { return psl::g_err; }
extern "C" int32_t psl_version(void) { return PSL_ABI_VERSION; }
