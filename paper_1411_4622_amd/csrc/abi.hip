// Host plumbing shared by every entry point: error messages, geometry
// validation, exact trig at multiples of 90 degrees, device information.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>

#include "common.hpp"

namespace pila {

static thread_local char g_err[512] = "";

int32_t fail(int32_t code, const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

int32_t hip_fail(hipError_t e, const char* what, const char* file, int line)
{
    return fail(PILA_EHIP, "%s failed: %s (%s:%d)", what, hipGetErrorString(e), file, line);
}

void clear_error() { g_err[0] = 0; }

void trig_of(double deg, double* c, double* s)
{
    if (std::fmod(deg, 90.0) == 0.0) {
        long q = (long)(deg / 90.0) % 4;
        if (q < 0) q += 4;
        static const double tc[4] = {1.0, 0.0, -1.0, 0.0};
        static const double ts[4] = {0.0, 1.0, 0.0, -1.0};
        *c = tc[q];
        *s = ts[q];
    } else {
        const double a = deg * (M_PI / 180.0);
        *c = std::cos(a);
        *s = std::sin(a);
    }
}

int32_t check_geom(const pila_geom* g)
{
    if (!g) return fail(PILA_EINVAL, "geometry is NULL");
    if (g->n < 1 || g->n_angles < 1 || g->n_bins < 1)
        return fail(PILA_EINVAL, "bad sizes n=%d U=%d K=%d", g->n, g->n_angles, g->n_bins);
    if ((int64_t)g->n * g->n > (int64_t)1 << 30 || (int64_t)g->n_angles * g->n_bins > (int64_t)1 << 30)
        return fail(PILA_EINVAL, "geometry too large (n=%d U=%d K=%d)", g->n, g->n_angles, g->n_bins);
    if (g->len_dtype != PILA_F64 && g->len_dtype != PILA_F32 && g->len_dtype != PILA_U8)
        return fail(PILA_EINVAL, "len_dtype must be PILA_F64, PILA_F32 or PILA_U8 (got %d)", g->len_dtype);
    if (!g->angles_deg) return fail(PILA_EINVAL, "angles_deg is NULL");
    for (int u = 0; u < g->n_angles; ++u)
        if (!std::isfinite(g->angles_deg[u]))
            return fail(PILA_EINVAL, "angle %d is not finite", u);
    return PILA_OK;
}

}  // namespace pila

extern "C" const char* pila_last_error(void) { return pila::g_err; }

extern "C" int32_t pila_get_device_info(pila_device_info* info)
{
    if (!info) return pila::fail(PILA_EINVAL, "info is NULL");
    int dev = 0;
    PILA_HIP(hipGetDevice(&dev));
    hipDeviceProp_t p;
    PILA_HIP(hipGetDeviceProperties(&p, dev));
    std::memset(info, 0, sizeof(*info));
    info->cu_count = p.multiProcessorCount;
    info->lds_per_block = (int32_t)p.sharedMemPerBlock;
    info->clock_khz = p.clockRate;
    info->warp_size = p.warpSize;
    info->hbm_bytes = p.totalGlobalMem;
    std::snprintf(info->name, sizeof(info->name), "%s", p.gcnArchName);
    int wc = 0;
    PILA_HIP(hipDeviceGetAttribute(&wc, hipDeviceAttributeWallClockRate, dev));
    info->wallclock_khz = wc;
    return PILA_OK;
}
