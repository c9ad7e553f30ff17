// PILA-driven projection (Eq. 1), its transpose, and simultaneous SIRT
// (section III-D, Eq. 10-11) on gfx950.
//
// Both directions are gathers, never scatters: the forward projection walks
// the ray-major copy of the PILA (one wavefront per ray, lanes stride over
// the ray's entries, FP64 accumulation, shuffle reduction), the back
// projection walks the pixel-major copy (one wavefront per pixel).  Every
// output is produced by exactly one wavefront in a fixed order, so results
// are deterministic and need no atomics.  Both stream the PILA from HBM
// once per call (the image / sinogram being gathered stays in L2 / MALL):
// these are HBM-bound kernels.
#include <cmath>
#include <vector>

#include "common.hpp"

namespace pila {

namespace {

constexpr int kGatherBlocks = 4096;  // fixed grid: reduction order does not depend on sizes
constexpr int kWPB = 4;              // wavefronts per block

enum { kFwd = 0, kResW = 1, kW = 2 };

// This lane's share of one CSR row's dot product with a gathered vector x
// (or, SQUARES, of the row's squared lengths): entries q = b + lane + 64 i in
// ascending i, fused multiply-add in FP64.  kU entries are loaded before any
// is used, so each lane keeps kU row loads and kU gathers in flight.
constexpr int kU = 8;

template <typename LenT, bool SQUARES>
__device__ __forceinline__ double row_dot(int64_t b, int64_t e, int lane,
                                          const int32_t* __restrict__ ci,
                                          const LenT* __restrict__ ln,
                                          const double* __restrict__ x)
{
    double acc = 0.0;
    for (int64_t q0 = b + lane; q0 < e; q0 += 64 * kU) {
        double l[kU], v[kU];
        int32_t c[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const int64_t q = q0 + 64 * u < e ? q0 + 64 * u : b;
            l[u] = (double)ln[q];
            if (!SQUARES) c[u] = ci[q];
        }
        if (!SQUARES) {
#pragma unroll
            for (int u = 0; u < kU; ++u) v[u] = x[c[u]];
        }
#pragma unroll
        for (int u = 0; u < kU; ++u)
            if (q0 + 64 * u < e) acc = fma(l[u], SQUARES ? l[u] : v[u], acc);
    }
    return acc;
}

template <typename LenT, int MODE>
__global__ __launch_bounds__(256) void ray_gather_kernel(int64_t G, const int64_t* __restrict__ rp,
                                                         const int32_t* __restrict__ ci,
                                                         const LenT* __restrict__ ln,
                                                         const double* __restrict__ f,
                                                         const double* __restrict__ sino,
                                                         const double* __restrict__ W,
                                                         double* __restrict__ out,
                                                         double* __restrict__ partial)
{
    __shared__ double wpart[kWPB];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    double sq = 0.0;  // lane 0: this wavefront's sum of squared residuals
    for (int64_t g = (int64_t)blockIdx.x * kWPB + w; g < G; g += (int64_t)gridDim.x * kWPB) {
        const int64_t b = rp[g], e = rp[g + 1];
        const double acc = wave_sum(row_dot<LenT, MODE == kW>(b, e, lane, ci, ln, f));
        if (lane == 0) {
            if (MODE == kResW) {
                const double res = sino[g] - acc;
                const double wg = W[g];
                out[g] = wg > 0.0 ? res / wg : 0.0;
                sq += res * res;
            } else {
                out[g] = acc;
            }
        }
    }
    if (MODE == kResW) {
        if (lane == 0) wpart[w] = sq;
        __syncthreads();
        if (threadIdx.x == 0) {
            double s = 0.0;
            for (int q = 0; q < kWPB; ++q) s += wpart[q];
            partial[blockIdx.x] = s;
        }
    }
}

// one workgroup: out[0] = sum of partial[0..n) in a fixed order
__global__ __launch_bounds__(256) void reduce_kernel(const double* __restrict__ partial, int n,
                                                     double* __restrict__ out)
{
    __shared__ double ws[4];
    double s = 0.0;
    for (int q = threadIdx.x; q < n; q += 256) s += partial[q];
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) out[0] = (ws[0] + ws[1]) + (ws[2] + ws[3]);
}

enum { kBack = 0, kSirt = 1 };

template <typename LenT, int MODE>
__global__ __launch_bounds__(256) void pixel_gather_kernel(int64_t NP, const int64_t* __restrict__ rp,
                                                           const int32_t* __restrict__ ci,
                                                           const LenT* __restrict__ ln,
                                                           const double* __restrict__ y,
                                                           double* __restrict__ out, double scale)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int64_t p = (int64_t)blockIdx.x * kWPB + w; p < NP; p += (int64_t)gridDim.x * kWPB) {
        const int64_t b = rp[p], e = rp[p + 1];
        if (MODE == kSirt && b == e) continue;
        const double acc = wave_sum(row_dot<LenT, false>(b, e, lane, ci, ln, y));
        if (lane == 0) {
            if (MODE == kSirt)
                out[p] = out[p] + scale * acc;
            else
                out[p] = acc;
        }
    }
}

unsigned gather_blocks(int64_t rows)
{
    const int64_t b = (rows + kWPB - 1) / kWPB;
    return (unsigned)(b < kGatherBlocks ? (b > 0 ? b : 1) : kGatherBlocks);
}

int32_t check_csr(const pila_geom* g, const pila_csr* c, bool need_rays, bool need_pixels)
{
    PILA_TRY(check_geom(g));
    if (!c) return fail(PILA_EINVAL, "csr is NULL");
    if (need_pixels && (!c->row_ptr || !c->col || !c->len))
        return fail(PILA_EINVAL, "pixel-major PILA arrays missing");
    if (need_rays && (!c->t_row_ptr || !c->t_col || !c->t_len))
        return fail(PILA_EINVAL, "ray-major PILA arrays missing");
    return PILA_OK;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

}  // namespace pila

using namespace pila;

extern "C" int32_t pila_forward(const pila_geom* geom, const pila_csr* csr, const double* d_image,
                                double* d_out, void* stream)
{
    clear_error();
    PILA_TRY(check_csr(geom, csr, true, false));
    if (!d_image || !d_out) return fail(PILA_EINVAL, "image or output is NULL");
    const int64_t G = (int64_t)geom->n_angles * geom->n_bins;
    hipStream_t st = (hipStream_t)stream;
    if (geom->len_dtype == PILA_F64)
        ray_gather_kernel<double, kFwd><<<gather_blocks(G), 256, 0, st>>>(
            G, csr->t_row_ptr, csr->t_col, (const double*)csr->t_len, d_image, nullptr, nullptr, d_out, nullptr);
    else
        ray_gather_kernel<float, kFwd><<<gather_blocks(G), 256, 0, st>>>(
            G, csr->t_row_ptr, csr->t_col, (const float*)csr->t_len, d_image, nullptr, nullptr, d_out, nullptr);
    PILA_HIP(hipGetLastError());
    return PILA_OK;
}

extern "C" int32_t pila_backproject(const pila_geom* geom, const pila_csr* csr, const double* d_sino,
                                    double* d_out, void* stream)
{
    clear_error();
    PILA_TRY(check_csr(geom, csr, false, true));
    if (!d_sino || !d_out) return fail(PILA_EINVAL, "sinogram or output is NULL");
    const int64_t NP = (int64_t)geom->n * geom->n;
    hipStream_t st = (hipStream_t)stream;
    if (geom->len_dtype == PILA_F64)
        pixel_gather_kernel<double, kBack><<<gather_blocks(NP), 256, 0, st>>>(
            NP, csr->row_ptr, csr->col, (const double*)csr->len, d_sino, d_out, 0.0);
    else
        pixel_gather_kernel<float, kBack><<<gather_blocks(NP), 256, 0, st>>>(
            NP, csr->row_ptr, csr->col, (const float*)csr->len, d_sino, d_out, 0.0);
    PILA_HIP(hipGetLastError());
    return PILA_OK;
}

extern "C" int32_t sirt_workspace_size(const pila_geom* geom, const sirt_params* params, size_t* bytes)
{
    clear_error();
    PILA_TRY(check_geom(geom));
    if (!params || !bytes) return fail(PILA_EINVAL, "params or bytes is NULL");
    if (params->n_iter < 0) return fail(PILA_EINVAL, "n_iter < 0");
    const size_t G = (size_t)geom->n_angles * geom->n_bins;
    *bytes = 2 * align256(sizeof(double) * G) + align256(sizeof(double) * kGatherBlocks) +
             align256(sizeof(double) * (size_t)(params->n_iter > 0 ? params->n_iter : 1));
    return PILA_OK;
}

template <typename LenT>
static int32_t sirt_impl(const pila_geom* geom, const pila_csr* csr, const double* d_sino,
                         const sirt_params* prm, double* d_image, char* ws, double* h_cost,
                         hipStream_t st)
{
    const int64_t G = (int64_t)geom->n_angles * geom->n_bins;
    const int64_t NP = (int64_t)geom->n * geom->n;
    double* W = (double*)ws;
    double* q = (double*)(ws + align256(sizeof(double) * G));
    double* partial = (double*)(ws + 2 * align256(sizeof(double) * G));
    double* sse = (double*)(ws + 2 * align256(sizeof(double) * G) + align256(sizeof(double) * kGatherBlocks));
    const unsigned gb = gather_blocks(G), pb = gather_blocks(NP);
    // factor matrix: W_g = sum of squared lengths of ray g over the support
    ray_gather_kernel<LenT, kW><<<gb, 256, 0, st>>>(G, csr->t_row_ptr, csr->t_col,
                                                    (const LenT*)csr->t_len, nullptr, nullptr,
                                                    nullptr, W, nullptr);
    const double scale = prm->lambda / (double)geom->n_angles;
    for (int32_t it = 0; it < prm->n_iter; ++it) {
        ray_gather_kernel<LenT, kResW><<<gb, 256, 0, st>>>(G, csr->t_row_ptr, csr->t_col,
                                                           (const LenT*)csr->t_len, d_image, d_sino,
                                                           W, q, partial);
        reduce_kernel<<<1, 256, 0, st>>>(partial, (int)gb, sse + it);
        pixel_gather_kernel<LenT, kSirt><<<pb, 256, 0, st>>>(NP, csr->row_ptr, csr->col,
                                                             (const LenT*)csr->len, q, d_image, scale);
    }
    PILA_HIP(hipGetLastError());
    if (h_cost && prm->n_iter > 0) {
        std::vector<double> s((size_t)prm->n_iter);
        PILA_HIP(hipMemcpyAsync(s.data(), sse, sizeof(double) * s.size(), hipMemcpyDeviceToHost, st));
        PILA_HIP(hipStreamSynchronize(st));
        const double KU = (double)geom->n_bins * (double)geom->n_angles;
        for (size_t i = 0; i < s.size(); ++i) h_cost[i] = std::sqrt(s[i] / KU);
    }
    return PILA_OK;
}

extern "C" int32_t sirt_run(const pila_geom* geom, const pila_csr* csr, const double* d_sino,
                            const sirt_params* params, double* d_image, void* d_ws, size_t ws_bytes,
                            double* h_cost, void* stream)
{
    clear_error();
    PILA_TRY(check_csr(geom, csr, true, true));
    if (!params || !d_sino || !d_image) return fail(PILA_EINVAL, "params, sinogram or image is NULL");
    if (!std::isfinite(params->lambda)) return fail(PILA_EINVAL, "lambda is not finite");
    size_t need = 0;
    PILA_TRY(sirt_workspace_size(geom, params, &need));
    if (!d_ws || ws_bytes < need)
        return fail(PILA_ENOMEM, "workspace of %zu bytes is below the %zu needed", ws_bytes, need);
    hipStream_t st = (hipStream_t)stream;
    if (geom->len_dtype == PILA_F64)
        return sirt_impl<double>(geom, csr, d_sino, params, d_image, (char*)d_ws, h_cost, st);
    return sirt_impl<float>(geom, csr, d_sino, params, d_image, (char*)d_ws, h_cost, st);
}
