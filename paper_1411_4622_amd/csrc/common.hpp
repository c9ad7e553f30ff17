// Shared device helpers and host error plumbing for the gfx950 PILA library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "pila.h"

namespace pila {

// ---------------------------------------------------------------------------
// host-side error reporting (thread-local message, status codes of pila.h)
// ---------------------------------------------------------------------------
int32_t fail(int32_t code, const char* fmt, ...);
int32_t hip_fail(hipError_t e, const char* what, const char* file, int line);
void clear_error();

#define PILA_HIP(call)                                                          \
    do {                                                                        \
        hipError_t e_ = (call);                                                 \
        if (e_ != hipSuccess) return ::pila::hip_fail(e_, #call, __FILE__, __LINE__); \
    } while (0)

#define PILA_TRY(expr)                      \
    do {                                    \
        int32_t rc_ = (expr);               \
        if (rc_ != PILA_OK) return rc_;     \
    } while (0)

constexpr double kTau = 1e-9;  // lengths at or below this (corner touches) are not stored
constexpr int kWave = 64;

// One-byte intersection length (section II-B: the length times 180,
// rounded; halves away from zero).  It stands for the float q / 180,
// correctly rounded, which for every byte value equals q * fl(1/180) with
// one fused multiply-add correction of its residual (three instructions
// instead of a division; the identity is checked exhaustively by the test
// suite).  Kernels templated on the length type read it through this float
// conversion; the PILA build stores it through the constructor.
struct LenQ {
    uint8_t q;
    LenQ() = default;
    __host__ __device__ explicit LenQ(double l) : q((uint8_t)round(180.0 * l)) {}
    __host__ __device__ operator float() const
    {
        const float x = (float)q, c = 1.0f / 180.0f;
        const float r = x * c;
        return fmaf(fmaf(-r, 180.0f, x), c, r);
    }
};
static_assert(sizeof(LenQ) == 1, "one byte per length");

// host: (cos, sin) of degrees, exact at multiples of 90 degrees
void trig_of(double deg, double* c, double* s);
// host: validate a geometry (sizes, finite angles, dtype)
int32_t check_geom(const pila_geom* g);
// host: bytes of one stored length of a len_dtype
inline int len_bytes(int32_t dtype) { return dtype == PILA_F64 ? 8 : dtype == PILA_F32 ? 4 : 1; }

// ---------------------------------------------------------------------------
// device: Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11)
// ---------------------------------------------------------------------------
struct Words4 {
    uint64_t w0, w1, w2, w3;
};

__device__ __forceinline__ Words4 philox4x64(uint64_t k0, uint64_t k1, uint64_t c0, uint64_t c1,
                                             uint64_t c2, uint64_t c3)
{
    constexpr uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    constexpr uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += W0;
            k1 += W1;
        }
        const uint64_t hi0 = __umul64hi(M0, c0), lo0 = M0 * c0;
        const uint64_t hi1 = __umul64hi(M1, c2), lo1 = M1 * c2;
        const uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    return {c0, c1, c2, c3};
}

__device__ __forceinline__ double unit53(uint64_t w) { return (double)(w >> 11) * 0x1p-53; }

// ---------------------------------------------------------------------------
// device: wavefront reductions (64 lanes)
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T wave_sum(T v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

__device__ __forceinline__ int wave_isum(int v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

// exclusive prefix over the lanes of a wave (lane order)
__device__ __forceinline__ int wave_excl_scan(int v, int lane)
{
    int x = v;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        int y = __shfl_up(x, o, kWave);
        if (lane >= o) x += y;
    }
    return x - v;
}

// ---------------------------------------------------------------------------
// device: intersection length of one ray with one pixel (closed form)
//
// The chord of the line  x c + y s = s_k  through a unit square, as a
// function of the signed offset t between the line and the square's centre,
// is a trapezoid: constant 1 / max(|c|,|s|) for |t| <= (hi - lo)/2, falling
// linearly to 0 at |t| = (hi + lo)/2, with hi/lo = max/min(|c|, |s|).
// Near-axis rays make the ramp steep (slope 1 / (hi lo)), so t is formed
// with error-free products and sums (FMA-based) to keep the length error
// near 1e-14 even on 1024-pixel grids.
// Axis-parallel rays (c or s exactly 0) go to the pixel whose half-open
// interval [left, left + 1) or [bottom, bottom + 1) contains them.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double sum_err(double a, double b, double s)
{
    const double bb = s - a;
    return (a - (s - bb)) + (b - bb);
}

// t = sk - (xc c + yc s) as an unevaluated sum hi + *lo (error-free
// products and sums: the pair is exact to about 1e-32)
__device__ __forceinline__ double ray_offset(double sk, double xc, double yc, double c, double s,
                                             double* lo)
{
    const double p = xc * c, ep = fma(xc, c, -p);
    const double q = yc * s, eq = fma(yc, s, -q);
    const double a = sk - p, ea = sum_err(sk, -p, a);
    const double b = a - q, eb = sum_err(a, -q, b);
    *lo = (ea + eb) - (ep + eq);
    return b;
}

__device__ __forceinline__ double pixel_ray_length(double xl, double yb, double c, double s,
                                                   double sk)
{
    if (s == 0.0) {
        const double x = sk * c;
        return (x >= xl && x < xl + 1.0) ? 1.0 : 0.0;
    }
    if (c == 0.0) {
        const double y = sk * s;
        return (y >= yb && y < yb + 1.0) ? 1.0 : 0.0;
    }
    double th_lo;
    const double th = ray_offset(sk, xl + 0.5, yb + 0.5, c, s, &th_lo);
    const double t = fabs(th + th_lo);
    const double a = fabs(c), b = fabs(s);
    const double hi = fmax(a, b), lo = fmin(a, b);
    const double flat = 0.5 * (hi - lo), edge = 0.5 * (hi + lo);
    double l = 0.0;
    if (t <= flat) {
        l = 1.0 / hi;
    } else if (t < edge) {
        // 2 (edge - |t|) = (E - 2|th|) + (E_err - 2 sgn th_lo) with E = hi + lo
        // split error-free; on the ramp the first difference is exact
        // (Sterbenz) whenever the slope 1 / (hi lo) is large
        const double sg = th < 0.0 ? -1.0 : 1.0;
        const double E = hi + lo, Ee = sum_err(hi, lo, E);
        const double u = 0.5 * ((E - 2.0 * sg * th) + (Ee - 2.0 * sg * th_lo));
        l = u / (hi * lo);
    }
    return l > kTau ? l : 0.0;
}

}  // namespace pila
