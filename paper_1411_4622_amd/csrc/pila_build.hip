// PILA build on gfx950 (section II-B, Eq. 5).
//
// The paper runs Siddon's ray trace for one pixel at a time; here every
// (pixel, angle) pair is independent work: a wavefront owns one pixel and
// its lanes walk the angles, each lane evaluating the closed-form chord of
// the (at most two) rays that cross the pixel at its angle.  The ray-major
// copy is produced the same way from the ray side (a wavefront per ray,
// lanes over image rows), calling the same length function, so both copies
// hold bit-identical lengths.  Offsets come from a count pass, an in-place
// single-workgroup scan, and a fill pass that places each wavefront's
// entries with a lane prefix sum, giving rows in ascending ray (pixel-major)
// or pixel (ray-major) order without sorting.
#include <algorithm>
#include <cmath>
#include <vector>

#include "common.hpp"
#include "sat_host.hpp"

namespace pila {

namespace {

constexpr int kWavesPerBlock = 4;

template <bool FILL, typename LenT>
__global__ __launch_bounds__(256) void pixel_rows_kernel(int32_t N, int32_t U, int32_t K,
                                                         const double* __restrict__ trig,
                                                         const uint8_t* __restrict__ mask,
                                                         int64_t* __restrict__ row_ptr,
                                                         int32_t* __restrict__ col,
                                                         LenT* __restrict__ len)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t p = (int64_t)blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
    if (p >= (int64_t)N * N) return;
    const bool inside = !mask || mask[p];
    const int i = (int)(p / N), j = (int)(p % N);
    const double h = 0.5 * N, cK = 0.5 * (K - 1);
    const double xl = j - h, yb = h - 1.0 - i;
    int64_t base = 0;
    if (FILL) base = row_ptr[p];
    int64_t total = 0;
    if (inside) {
        for (int u0 = 0; u0 < U; u0 += kWave) {
            const int u = u0 + lane;
            int cnt = 0;
            int32_t g[3] = {0, 0, 0};
            double l[3] = {0.0, 0.0, 0.0};
            if (u < U) {
                const double c = trig[2 * u], s = trig[2 * u + 1];
                const double t0 = (xl + 0.5) * c + (yb + 0.5) * s;
                const int klo = (int)floor(t0 + cK - 1.0);
                for (int k = klo < 0 ? 0 : klo; k <= klo + 3 && k < K; ++k) {
                    const double lk = pixel_ray_length(xl, yb, c, s, k - cK);
                    if (lk > 0.0 && cnt < 3) {
                        g[cnt] = u * K + k;
                        l[cnt] = lk;
                        ++cnt;
                    }
                }
            }
            if (FILL) {
                const int64_t q = base + total + wave_excl_scan(cnt, lane);
                for (int e = 0; e < cnt; ++e) {
                    col[q + e] = g[e];
                    len[q + e] = (LenT)l[e];
                }
            }
            total += wave_isum(cnt);
        }
    }
    if (!FILL && lane == 0) row_ptr[p + 1] = total;
}

// candidate columns of image row i for ray (c, s, sk): a superset of the
// pixels the ray crosses in that row
__device__ __forceinline__ void row_candidates(int32_t N, double h, double c, double s, double sk,
                                               double yb, int* jlo, int* jhi)
{
    *jlo = 0;
    *jhi = -1;
    if (s == 0.0) {
        const double jf = floor(sk * c + h);
        if (jf >= 0.0 && jf < (double)N) *jlo = *jhi = (int)jf;
        return;
    }
    if (c == 0.0) {
        const double y = sk * s;
        if (y >= yb && y < yb + 1.0) {
            *jlo = 0;
            *jhi = N - 1;
        }
        return;
    }
    const double yc = yb + 0.5, edge = 0.5 * (fabs(c) + fabs(s));
    const double a1 = (sk - yc * s - edge) / c, a2 = (sk - yc * s + edge) / c;
    double lo = floor(fmin(a1, a2) + h - 0.5) - 1.0;
    double hi = ceil(fmax(a1, a2) + h - 0.5) + 1.0;
    lo = fmax(lo, 0.0);
    hi = fmin(hi, (double)(N - 1));
    if (hi >= lo) {
        *jlo = (int)lo;
        *jhi = (int)hi;
    }
}

template <bool FILL, typename LenT>
__global__ __launch_bounds__(256) void ray_rows_kernel(int32_t N, int32_t U, int32_t K,
                                                       const double* __restrict__ trig,
                                                       const uint8_t* __restrict__ mask,
                                                       int64_t* __restrict__ t_row_ptr,
                                                       int32_t* __restrict__ t_col,
                                                       LenT* __restrict__ t_len)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t g = (int64_t)blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
    if (g >= (int64_t)U * K) return;
    const int u = (int)(g / K), k = (int)(g % K);
    const double c = trig[2 * u], s = trig[2 * u + 1];
    const double h = 0.5 * N, sk = k - 0.5 * (K - 1);
    int64_t base = 0;
    if (FILL) base = t_row_ptr[g];
    int64_t total = 0;
    for (int i0 = 0; i0 < N; i0 += kWave) {
        const int i = i0 + lane;
        int cnt = 0, jlo = 0, jhi = -1;
        const double yb = h - 1.0 - i;
        if (i < N) {
            row_candidates(N, h, c, s, sk, yb, &jlo, &jhi);
            for (int j = jlo; j <= jhi; ++j) {
                const int64_t p = (int64_t)i * N + j;
                if (mask && !mask[p]) continue;
                if (pixel_ray_length(j - h, yb, c, s, sk) > 0.0) ++cnt;
            }
        }
        if (FILL) {
            int64_t q = base + total + wave_excl_scan(cnt, lane);
            for (int j = jlo; j <= jhi && cnt > 0; ++j) {
                const int64_t p = (int64_t)i * N + j;
                if (mask && !mask[p]) continue;
                const double l = pixel_ray_length(j - h, yb, c, s, sk);
                if (l > 0.0) {
                    t_col[q] = (int32_t)p;
                    t_len[q] = (LenT)l;
                    ++q;
                }
            }
        }
        total += wave_isum(cnt);
    }
    if (!FILL && lane == 0) t_row_ptr[g + 1] = total;
}

// out[0] = max of a[1..n) (the row counts before the scan), one workgroup
__global__ __launch_bounds__(1024) void max_count_kernel(const int64_t* __restrict__ a, int64_t n,
                                                         int64_t* __restrict__ out)
{
    __shared__ int64_t wmax[16];
    int64_t m = 0;
    for (int64_t q = 1 + threadIdx.x; q < n; q += 1024) m = a[q] > m ? a[q] : m;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const int64_t y = __shfl_xor(m, o, 64);
        m = y > m ? y : m;
    }
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t r = 0;
        for (int w = 0; w < 16; ++w) r = wmax[w] > r ? wmax[w] : r;
        out[0] = r;
    }
}

// In-place inclusive scan of a[0..n) by one workgroup of 1024 threads.
// a[0] is 0 and a[x+1] holds the count of row x, so the result is the CSR
// offset array.
__global__ __launch_bounds__(1024) void scan_kernel(int64_t* __restrict__ a, int64_t n)
{
    constexpr int IT = 8;
    __shared__ int64_t wsum[16];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    int64_t carry = 0;
    for (int64_t base = 0; base < n; base += 1024 * IT) {
        int64_t v[IT];
        int64_t loc = 0;
#pragma unroll
        for (int q = 0; q < IT; ++q) {
            const int64_t idx = base + (int64_t)t * IT + q;
            loc += idx < n ? a[idx] : 0;
            v[q] = loc;
        }
        int64_t x = loc;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int64_t y = __shfl_up(x, o, 64);
            if (lane >= o) x += y;
        }
        if (lane == 63) wsum[w] = x;
        __syncthreads();
        if (w == 0) {
            int64_t z = lane < 16 ? wsum[lane] : 0;
#pragma unroll
            for (int o = 1; o < 16; o <<= 1) {
                const int64_t y = __shfl_up(z, o, 64);
                if (lane >= o) z += y;
            }
            if (lane < 16) wsum[lane] = z;
        }
        __syncthreads();
        const int64_t pre = carry + (w > 0 ? wsum[w - 1] : 0) + (x - loc);
#pragma unroll
        for (int q = 0; q < IT; ++q) {
            const int64_t idx = base + (int64_t)t * IT + q;
            if (idx < n) a[idx] = v[q] + pre;
        }
        carry += wsum[15];
        __syncthreads();
    }
}

unsigned blocks_for(int64_t items) { return (unsigned)((items + kWavesPerBlock - 1) / kWavesPerBlock); }

template <typename LenT>
void launch_fill(const pila_geom* g, pila_csr* csr, const uint8_t* dmask, hipStream_t st)
{
    const int64_t NP = (int64_t)g->n * g->n, G = (int64_t)g->n_angles * g->n_bins;
    pixel_rows_kernel<true, LenT><<<blocks_for(NP), 256, 0, st>>>(
        g->n, g->n_angles, g->n_bins, csr->trig, dmask, csr->row_ptr, csr->col, (LenT*)csr->len);
    ray_rows_kernel<true, LenT><<<blocks_for(G), 256, 0, st>>>(g->n, g->n_angles, g->n_bins,
                                                                csr->trig, dmask, csr->t_row_ptr,
                                                                csr->t_col, (LenT*)csr->t_len);
}

}  // namespace

}  // namespace pila

using namespace pila;

size_t pila::pila_build_scratch(const pila_geom* geom) { return 256 + (size_t)geom->n * (size_t)geom->n; }

extern "C" int32_t pila_build_scratch_size(const pila_geom* geom, size_t* bytes)
{
    clear_error();
    PILA_TRY(check_geom(geom));
    if (!bytes) return fail(PILA_EINVAL, "bytes is NULL");
    *bytes = pila_build_scratch(geom);
    return PILA_OK;
}

extern "C" int32_t pila_build(const pila_geom* geom, pila_csr* csr, void* d_scratch, size_t scratch_bytes,
                              void* stream)
{
    clear_error();
    PILA_TRY(check_geom(geom));
    if (!csr) return fail(PILA_EINVAL, "csr is NULL");
    if (!csr->row_ptr || !csr->trig || !csr->t_row_ptr)
        return fail(PILA_EINVAL, "row_ptr, trig and t_row_ptr must be allocated");
    if (!d_scratch) return fail(PILA_EINVAL, "scratch is NULL");
    if (scratch_bytes < pila_build_scratch(geom))
        return fail(PILA_ENOMEM, "scratch of %zu bytes is below the %zu needed", scratch_bytes,
                    pila_build_scratch(geom));
    return pila_build_with(geom, csr, d_scratch, (hipStream_t)stream);
}

int32_t pila::pila_build_with(const pila_geom* geom, pila_csr* csr, void* d_scratch, hipStream_t st)
{
    PILA_TRY(check_geom(geom));
    if (!csr || !d_scratch) return fail(PILA_EINVAL, "csr or scratch is NULL");
    if (!csr->row_ptr || !csr->trig || !csr->t_row_ptr)
        return fail(PILA_EINVAL, "row_ptr, trig and t_row_ptr must be allocated");
    const int32_t N = geom->n, U = geom->n_angles, K = geom->n_bins;
    const int64_t NP = (int64_t)N * N, G = (int64_t)U * K;

    std::vector<int32_t> support;
    support.reserve((size_t)NP);
    double rmax2 = -1.0;  // largest squared distance of a support pixel centre from the axis
    for (int64_t p = 0; p < NP; ++p)
        if (!geom->mask || geom->mask[p]) {
            support.push_back((int32_t)p);
            const double xc = (double)(p % N) - 0.5 * N + 0.5, yc = 0.5 * N - 0.5 - (double)(p / N);
            rmax2 = std::max(rmax2, xc * xc + yc * yc);
        }

    // scratch: [0, 256) small results, [256, 256 + N*N) the mask
    int64_t* d_small = (int64_t*)d_scratch;
    const uint8_t* mk = nullptr;
    if (geom->mask) {
        PILA_HIP(hipMemcpyAsync((char*)d_scratch + 256, geom->mask, (size_t)NP, hipMemcpyHostToDevice, st));
        mk = (const uint8_t*)d_scratch + 256;
    }

    if (!csr->col) {  // phase 1: trig, offsets, sizes
        std::vector<double> cs(2 * (size_t)U);
        for (int u = 0; u < U; ++u) trig_of(geom->angles_deg[u], &cs[2 * u], &cs[2 * u + 1]);
        PILA_HIP(hipMemcpyAsync(csr->trig, cs.data(), sizeof(double) * cs.size(),
                                hipMemcpyHostToDevice, st));
        PILA_HIP(hipMemsetAsync(csr->row_ptr, 0, sizeof(int64_t), st));
        PILA_HIP(hipMemsetAsync(csr->t_row_ptr, 0, sizeof(int64_t), st));
        pixel_rows_kernel<false, double><<<blocks_for(NP), 256, 0, st>>>(
            N, U, K, csr->trig, mk, csr->row_ptr, nullptr, nullptr);
        PILA_HIP(hipGetLastError());
        max_count_kernel<<<1, 1024, 0, st>>>(csr->row_ptr, NP + 1, d_small);
        scan_kernel<<<1, 1024, 0, st>>>(csr->row_ptr, NP + 1);
        ray_rows_kernel<false, double><<<blocks_for(G), 256, 0, st>>>(N, U, K, csr->trig, mk,
                                                                     csr->t_row_ptr, nullptr, nullptr);
        PILA_HIP(hipGetLastError());
        scan_kernel<<<1, 1024, 0, st>>>(csr->t_row_ptr, G + 1);
        PILA_HIP(hipGetLastError());
        int64_t tot[3] = {0, 0, 0};
        PILA_HIP(hipMemcpyAsync(&tot[0], csr->row_ptr + NP, sizeof(int64_t), hipMemcpyDeviceToHost, st));
        PILA_HIP(hipMemcpyAsync(&tot[1], csr->t_row_ptr + G, sizeof(int64_t), hipMemcpyDeviceToHost, st));
        PILA_HIP(hipMemcpyAsync(&tot[2], d_small, sizeof(int64_t), hipMemcpyDeviceToHost, st));
        PILA_HIP(hipStreamSynchronize(st));
        if (tot[0] != tot[1])
            return fail(PILA_EHIP, "pixel-major (%lld) and ray-major (%lld) entry counts differ",
                        (long long)tot[0], (long long)tot[1]);
        csr->nnz = tot[0];
        csr->n_support = (int32_t)support.size();
        csr->max_row = (int32_t)tot[2];
        // a ray reaches a pixel only within 0.71 of its centre's projection, so
        // every bin used by the support lies within R + 1 of the detector centre
        if (rmax2 < 0.0) {
            csr->k_lo = 0;
            csr->k_hi = -1;
        } else {
            const double R = std::sqrt(rmax2), cK = 0.5 * (K - 1);
            csr->k_lo = (int32_t)std::max(0.0, std::floor(cK - R - 1.0));
            csr->k_hi = (int32_t)std::min((double)(K - 1), std::ceil(cK + R + 1.0));
        }
        return PILA_OK;
    }

    // phase 2: entries
    if (!csr->len || !csr->support || !csr->t_col || !csr->t_len)
        return fail(PILA_EINVAL, "phase 2 needs col, len, support, t_col and t_len");
    int64_t tot = -1;
    PILA_HIP(hipMemcpyAsync(&tot, csr->row_ptr + NP, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    PILA_HIP(hipStreamSynchronize(st));
    if (tot != csr->nnz)
        return fail(PILA_ESIZE, "row_ptr holds %lld entries but csr->nnz is %lld", (long long)tot,
                    (long long)csr->nnz);
    if (csr->n_support != (int32_t)support.size())
        return fail(PILA_ESIZE, "n_support %d does not match the mask (%zu)", csr->n_support,
                    support.size());
    if (geom->len_dtype == PILA_F64)
        launch_fill<double>(geom, csr, mk, st);
    else if (geom->len_dtype == PILA_F32)
        launch_fill<float>(geom, csr, mk, st);
    else
        launch_fill<LenQ>(geom, csr, mk, st);
    PILA_HIP(hipGetLastError());
    if (!support.empty())
        PILA_HIP(hipMemcpyAsync(csr->support, support.data(), sizeof(int32_t) * support.size(),
                                hipMemcpyHostToDevice, st));
    PILA_HIP(hipStreamSynchronize(st));
    return PILA_OK;
}
