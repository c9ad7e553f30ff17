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

// Rows [0, n) in 8 contiguous chunks, one per XCD: the dispatcher hands
// workgroups to the 8 XCDs round robin (workgroup b to XCD b mod 8), so the
// workgroups of one XCD take neighbouring rays (or pixels), whose gathers
// touch the same image (or sinogram) lines and hit that XCD's L2.  Within a
// chunk the XCD's wavefronts stride over the rows.  The grid is a multiple
// of 8; each row still has exactly one wavefront.
struct XcdRows {
    int64_t first, end, stride;
};

__device__ __forceinline__ XcdRows xcd_rows(int64_t n, int w)
{
    constexpr int kXcd = 8;
    const int x = blockIdx.x % kXcd;
    const int64_t nb = gridDim.x / kXcd;
    const int64_t chunk = (n + kXcd - 1) / kXcd;
    const int64_t lo = x * chunk;
    const int64_t hi = lo + chunk < n ? lo + chunk : n;
    return {lo + (int64_t)(blockIdx.x / kXcd) * kWPB + w, hi, nb * kWPB};
}

// The same dot product for a ray closer to the image's columns than to its
// rows (|cos| > |sin|): its consecutive entries are pixels of consecutive
// image rows, so the image is read transposed (fT[j N + i] = f[i N + j]),
// where they are neighbours.  Same entries, lanes and order as row_dot.
template <typename LenT>
__device__ __forceinline__ double row_dot_t(int64_t b, int64_t e, int lane,
                                            const int32_t* __restrict__ ci,
                                            const LenT* __restrict__ ln,
                                            const double* __restrict__ fT, int N, double invN)
{
    double acc = 0.0;
    for (int64_t q0 = b + lane; q0 < e; q0 += 64 * kU) {
        double l[kU], v[kU];
        int32_t c[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const int64_t q = q0 + 64 * u < e ? q0 + 64 * u : b;
            l[u] = (double)ln[q];
            c[u] = ci[q];
        }
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            int i = (int)((double)c[u] * invN);  // c / N, then corrected
            int j = c[u] - i * N;
            if (j < 0) {
                --i;
                j += N;
            } else if (j >= N) {
                ++i;
                j -= N;
            }
            v[u] = fT[j * N + i];
        }
#pragma unroll
        for (int u = 0; u < kU; ++u)
            if (q0 + 64 * u < e) acc = fma(l[u], v[u], acc);
    }
    return acc;
}

// fT = f transposed (N x N), 32 x 32 tiles through LDS
__global__ __launch_bounds__(256) void transpose_kernel(int N, const double* __restrict__ f,
                                                        double* __restrict__ fT)
{
    __shared__ double tile[32][33];
    const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8 threads
    for (int r = ty; r < 32; r += 8) {
        const int i = by + r, j = bx + tx;
        if (i < N && j < N) tile[r][tx] = f[(int64_t)i * N + j];
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        const int j = bx + r, i = by + tx;
        if (i < N && j < N) fT[(int64_t)j * N + i] = tile[tx][r];
    }
}

template <typename LenT, int MODE>
__global__ __launch_bounds__(256) void ray_gather_kernel(int64_t G, const int64_t* __restrict__ rp,
                                                         const int32_t* __restrict__ ci,
                                                         const LenT* __restrict__ ln,
                                                         const double* __restrict__ f,
                                                         const double* __restrict__ sino,
                                                         const double* __restrict__ W,
                                                         double* __restrict__ out,
                                                         double* __restrict__ partial,
                                                         const double* __restrict__ fT = nullptr,
                                                         const double* __restrict__ trig = nullptr,
                                                         int N = 0, int K = 1)
{
    __shared__ double wpart[kWPB];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    double sq = 0.0;  // lane 0: this wavefront's sum of squared residuals
    const XcdRows xr = xcd_rows(G, w);
    const double invN = N > 0 ? 1.0 / (double)N : 0.0;
    for (int64_t g = xr.first; g < xr.end; g += xr.stride) {
        const int64_t b = rp[g], e = rp[g + 1];
        bool cols = false;
        if (MODE != kW && fT) {
            const int64_t u = g / K;
            cols = fabs(trig[2 * u]) > fabs(trig[2 * u + 1]);
        }
        const double acc = wave_sum(cols ? row_dot_t<LenT>(b, e, lane, ci, ln, fT, N, invN)
                                         : row_dot<LenT, MODE == kW>(b, e, lane, ci, ln, f));
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
    const XcdRows xr = xcd_rows(NP, w);
    for (int64_t p = xr.first; p < xr.end; p += xr.stride) {
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

// ---------------------------------------------------------------------------
// SIRT back projection by pixel tiles.  The PILA row of a pixel holds, per
// angle, one or two rays of adjacent bins (a unit pixel's shadow is at most
// sqrt 2 bins wide).  For a tile of 8 x 8 pixels the tile layout stores, per
// angle and pixel, the lower bin k and the lengths l0 (bin k) and l1 (bin
// k + 1), zero where absent, angle-major: element (t, u, lane) at
// (t U + u) 64 + lane.  A wavefront takes a tile (lane = pixel); at angle u
// its 64 pixels read 64 consecutive words and gather sinogram values from a
// span of about 12 bins of one sinogram row.  Each pixel adds its terms in
// the row's order (angle, then bin), as a sequential walk of the row would.
// ---------------------------------------------------------------------------
constexpr int kTile = 8;

__device__ __forceinline__ int64_t tile_pixel(const int32_t* tiles, int t, int lane, int N)
{
    const int tt = tiles[t];
    const int ti = tt >> 16, tj = tt & 0xFFFF;
    const int i = ti * kTile + (lane >> 3), j = tj * kTile + (lane & 7);
    return (i < N && j < N) ? (int64_t)i * N + j : -1;
}

template <typename LenT>
__global__ __launch_bounds__(64) void tile_build_kernel(int N, int U, int K, const int32_t* __restrict__ tiles,
                                                       const int64_t* __restrict__ rp,
                                                       const int32_t* __restrict__ ci,
                                                       const LenT* __restrict__ ln,
                                                       int32_t* __restrict__ tk, LenT* __restrict__ t0,
                                                       LenT* __restrict__ t1)
{
    const int t = blockIdx.x, lane = threadIdx.x;
    const int64_t base = (int64_t)t * U * 64;
    for (int u = 0; u < U; ++u) {
        tk[base + (int64_t)u * 64 + lane] = 0;
        t0[base + (int64_t)u * 64 + lane] = (LenT)0;
        t1[base + (int64_t)u * 64 + lane] = (LenT)0;
    }
    const int64_t p = tile_pixel(tiles, t, lane, N);
    if (p < 0) return;
    int prev = -1;
    for (int64_t q = rp[p]; q < rp[p + 1]; ++q) {
        const int g = ci[q];
        const int u = g / K, k = g - u * K;
        const int64_t at = base + (int64_t)u * 64 + lane;
        if (u == prev) {
            t1[at] = ln[q];
        } else {
            tk[at] = k;
            t0[at] = ln[q];
            prev = u;
        }
    }
}

template <typename LenT>
__global__ __launch_bounds__(256) void tile_back_kernel(int N, int U, int K, int n_tiles,
                                                       const int32_t* __restrict__ tiles,
                                                       const int64_t* __restrict__ rp,
                                                       const int32_t* __restrict__ tk,
                                                       const LenT* __restrict__ t0,
                                                       const LenT* __restrict__ t1,
                                                       const double* __restrict__ y,
                                                       double* __restrict__ f, double scale)
{
    constexpr int kA = 8;  // angles in flight
    const int lane = threadIdx.x & 63;
    const int t = blockIdx.x * kWPB + (threadIdx.x >> 6);
    if (t >= n_tiles) return;
    const int64_t base = (int64_t)t * U * 64 + lane;
    double acc = 0.0;
    for (int u0 = 0; u0 < U; u0 += kA) {
        int32_t kk[kA];
        double a0[kA], a1[kA], y0[kA], y1[kA];
#pragma unroll
        for (int a = 0; a < kA; ++a) {
            const int u = u0 + a < U ? u0 + a : U - 1;
            kk[a] = tk[base + (int64_t)u * 64];
            a0[a] = (double)t0[base + (int64_t)u * 64];
            a1[a] = (double)t1[base + (int64_t)u * 64];
        }
#pragma unroll
        for (int a = 0; a < kA; ++a) {
            const int u = u0 + a < U ? u0 + a : U - 1;
            const int64_t g = (int64_t)u * K + kk[a];
            y0[a] = y[g];
            y1[a] = y[kk[a] + 1 < K ? g + 1 : g];
        }
#pragma unroll
        for (int a = 0; a < kA; ++a) {
            if (u0 + a < U) {
                acc = fma(a0[a], y0[a], acc);
                acc = fma(a1[a], y1[a], acc);
            }
        }
    }
    const int64_t p = tile_pixel(tiles, t, lane, N);
    if (p >= 0 && rp[p + 1] > rp[p]) f[p] = f[p] + scale * acc;
}

// ---------------------------------------------------------------------------
// SIRT forward projection by ray tiles: 64 rays of consecutive bins at one
// angle (lane = bin).  A ray whose direction is closer to the image columns
// (|cos| > |sin|) crosses each image row at one or two adjacent pixels, one
// closer to the rows crosses each column so; the layout stores, per step
// (row, or column) and ray, the lower column (or row) index and the two
// lengths, zero where absent: element (t, step, lane) at (t N + step) 64 +
// lane, with each tile's used step range [s_lo, s_hi].  At a step the 64
// rays read consecutive words and gather image values from one image row
// (or, through the transposed image, one column) about 64-90 pixels wide.
// Ray-major entries come by ascending row, then column, so the first entry
// of a step is the lower pixel.  A step crossing holds at most two pixels
// (the ray moves less than one pixel sideways per step); should rounding
// give a corner-touching third one, or two that are not neighbours, the
// tile is marked irregular (hi = -2) and its rays are summed from the CSR.
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool ray_cols(const double* trig, int u)
{
    return fabs(trig[2 * u]) > fabs(trig[2 * u + 1]);
}

template <typename LenT>
__global__ __launch_bounds__(64) void ray_tile_build_kernel(int N, int U, int K, int nkt,
                                                           const double* __restrict__ trig,
                                                           const int64_t* __restrict__ rp,
                                                           const int32_t* __restrict__ ci,
                                                           const LenT* __restrict__ ln,
                                                           int32_t* __restrict__ tk, LenT* __restrict__ t0,
                                                           LenT* __restrict__ t1,
                                                           int32_t* __restrict__ range)
{
    const int t = blockIdx.x, lane = threadIdx.x;
    const int u = t / nkt, k = (t - u * nkt) * 64 + lane;
    const bool cols = ray_cols(trig, u);
    const int64_t base = (int64_t)t * N * 64 + lane;
    for (int st = 0; st < N; ++st) {
        tk[base + (int64_t)st * 64] = -1;
        t0[base + (int64_t)st * 64] = (LenT)0;
        t1[base + (int64_t)st * 64] = (LenT)0;
    }
    int lo = N, hi = -1;
    bool odd = false;
    if (k < K) {
        const int64_t g = (int64_t)u * K + k;
        for (int64_t q = rp[g]; q < rp[g + 1]; ++q) {
            const int p = ci[q];
            const int i = p / N, j = p - i * N;
            const int st = cols ? i : j, idx = cols ? j : i;
            const int64_t at = base + (int64_t)st * 64;
            if (tk[at] < 0) {
                tk[at] = idx;
                t0[at] = ln[q];
            } else if (idx == tk[at] + 1 && t1[at] == (LenT)0) {
                t1[at] = ln[q];
            } else {
                odd = true;
            }
            lo = st < lo ? st : lo;
            hi = st > hi ? st : hi;
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        lo = min(lo, __shfl_xor(lo, o, 64));
        hi = max(hi, __shfl_xor(hi, o, 64));
    }
    odd = __any(odd);
    if (lane == 0) {
        range[2 * t] = odd ? 0 : lo;
        range[2 * t + 1] = odd ? -2 : hi;
    }
}

// res = Pm - A f per ray, q = res / W (0 where W = 0), and per-block sums of res^2
template <typename LenT>
__global__ __launch_bounds__(256) void ray_tile_res_kernel(int N, int U, int K, int nkt, int n_tiles,
                                                          const double* __restrict__ trig,
                                                          const int32_t* __restrict__ tk,
                                                          const LenT* __restrict__ t0,
                                                          const LenT* __restrict__ t1,
                                                          const int32_t* __restrict__ range,
                                                          const int64_t* __restrict__ rp,
                                                          const int32_t* __restrict__ ci,
                                                          const LenT* __restrict__ ln,
                                                          const double* __restrict__ f,
                                                          const double* __restrict__ fT,
                                                          const double* __restrict__ sino,
                                                          const double* __restrict__ W,
                                                          double* __restrict__ out,
                                                          double* __restrict__ partial)
{
    constexpr int kS = 8;  // steps in flight
    __shared__ double wpart[kWPB];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    double sq = 0.0;
    const XcdRows xr = xcd_rows(n_tiles, w);
    for (int64_t t = xr.first; t < xr.end; t += xr.stride) {
        const int u = (int)(t / nkt), k = (int)(t - (int64_t)u * nkt) * 64 + lane;
        const double* img = ray_cols(trig, u) ? f : fT;
        const int lo = range[2 * t], hi = range[2 * t + 1];
        const int64_t base = t * N * 64 + lane;
        double acc = 0.0;
        if (hi == -2 && k < K) {  // irregular tile: each lane walks its ray's entries
            const int64_t g = (int64_t)u * K + k;
            for (int64_t q = rp[g]; q < rp[g + 1]; ++q) acc = fma((double)ln[q], f[ci[q]], acc);
        }
        for (int s0 = lo; s0 <= hi; s0 += kS) {
            int32_t ii[kS];
            double a0[kS], a1[kS], v0[kS], v1[kS];
#pragma unroll
            for (int a = 0; a < kS; ++a) {
                const int st = s0 + a <= hi ? s0 + a : hi;
                ii[a] = tk[base + (int64_t)st * 64];
                a0[a] = (double)t0[base + (int64_t)st * 64];
                a1[a] = (double)t1[base + (int64_t)st * 64];
            }
#pragma unroll
            for (int a = 0; a < kS; ++a) {
                const int st = s0 + a <= hi ? s0 + a : hi;
                const int i0 = ii[a] < 0 ? 0 : ii[a];
                const int64_t at = (int64_t)st * N + i0;
                v0[a] = img[at];
                v1[a] = img[i0 + 1 < N ? at + 1 : at];
            }
#pragma unroll
            for (int a = 0; a < kS; ++a) {
                if (s0 + a <= hi) {
                    acc = fma(a0[a], v0[a], acc);
                    acc = fma(a1[a], v1[a], acc);
                }
            }
        }
        if (k < K) {
            const int64_t g = (int64_t)u * K + k;
            const double res = sino[g] - acc;
            const double wg = W[g];
            out[g] = wg > 0.0 ? res / wg : 0.0;
            sq += res * res;
        }
    }
    sq = wave_sum(sq);
    if (lane == 0) wpart[w] = sq;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int q = 0; q < kWPB; ++q) s += wpart[q];
        partial[blockIdx.x] = s;
    }
}

// 8 x 8 tiles holding at least one support pixel, as (tile row << 16 | tile column)
std::vector<int32_t> support_tiles(const pila_geom* g)
{
    const int N = g->n, nt = (N + kTile - 1) / kTile;
    std::vector<int32_t> out;
    for (int ti = 0; ti < nt; ++ti)
        for (int tj = 0; tj < nt; ++tj) {
            bool any = false;
            for (int a = 0; a < kTile && !any; ++a)
                for (int b = 0; b < kTile && !any; ++b) {
                    const int i = ti * kTile + a, j = tj * kTile + b;
                    if (i < N && j < N && (!g->mask || g->mask[(int64_t)i * N + j])) any = true;
                }
            if (any) out.push_back((ti << 16) | tj);
        }
    return out;
}

// SIRT workspace: factor matrix, scaled residual, block partials, costs,
// the transposed image and the tile layout
struct SirtLayout {
    size_t W, q, partial, sse, fT, tiles, tk, t0, t1, rk, r0, r1, range, total;
};

SirtLayout sirt_layout(const pila_geom* g, int32_t n_iter, size_t n_tiles)
{
    const size_t G = (size_t)g->n_angles * g->n_bins, NP = (size_t)g->n * g->n;
    const size_t ls = g->len_dtype == PILA_F32 ? 4 : 8;
    const size_t cells = n_tiles * (size_t)g->n_angles * 64;
    SirtLayout L;
    size_t at = 0;
    auto take = [&](size_t bytes) {
        const size_t o = at;
        at += (bytes + 255) & ~(size_t)255;
        return o;
    };
    L.W = take(sizeof(double) * G);
    L.q = take(sizeof(double) * G);
    L.partial = take(sizeof(double) * kGatherBlocks);
    L.sse = take(sizeof(double) * (size_t)(n_iter > 0 ? n_iter : 1));
    L.fT = take(sizeof(double) * NP);
    L.tiles = take(sizeof(int32_t) * (n_tiles ? n_tiles : 1));
    L.tk = take(sizeof(int32_t) * cells);
    L.t0 = take(ls * cells);
    L.t1 = take(ls * cells);
    const size_t nrt = (size_t)g->n_angles * ((g->n_bins + 63) / 64);
    const size_t rcells = nrt * (size_t)g->n * 64;
    L.rk = take(sizeof(int32_t) * rcells);
    L.r0 = take(ls * rcells);
    L.r1 = take(ls * rcells);
    L.range = take(sizeof(int32_t) * 2 * nrt);
    L.total = at;
    return L;
}

unsigned gather_blocks(int64_t rows)
{
    int64_t b = (rows + kWPB - 1) / kWPB;
    b = b < kGatherBlocks ? b : kGatherBlocks;
    return (unsigned)((b + 7) / 8 * 8);  // a multiple of the 8 XCDs, at least 8
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
    *bytes = sirt_layout(geom, params->n_iter, support_tiles(geom).size()).total;
    return PILA_OK;
}

template <typename LenT>
static int32_t sirt_impl(const pila_geom* geom, const pila_csr* csr, const double* d_sino,
                         const sirt_params* prm, double* d_image, char* ws, double* h_cost,
                         hipStream_t st)
{
    const int N = geom->n, U = geom->n_angles, K = geom->n_bins;
    const int64_t G = (int64_t)U * K;
    const std::vector<int32_t> tiles = support_tiles(geom);
    const int n_tiles = (int)tiles.size();
    const SirtLayout L = sirt_layout(geom, prm->n_iter, tiles.size());
    double* W = (double*)(ws + L.W);
    double* q = (double*)(ws + L.q);
    double* partial = (double*)(ws + L.partial);
    double* sse = (double*)(ws + L.sse);
    double* fT = (double*)(ws + L.fT);
    int32_t* d_tiles = (int32_t*)(ws + L.tiles);
    int32_t* tk = (int32_t*)(ws + L.tk);
    LenT* t0 = (LenT*)(ws + L.t0);
    LenT* t1 = (LenT*)(ws + L.t1);
    const unsigned gb = gather_blocks(G);
    // factor matrix: W_g = sum of squared lengths of ray g over the support
    ray_gather_kernel<LenT, kW><<<gb, 256, 0, st>>>(G, csr->t_row_ptr, csr->t_col,
                                                    (const LenT*)csr->t_len, nullptr, nullptr,
                                                    nullptr, W, nullptr);
    if (n_tiles > 0) {
        PILA_HIP(hipMemcpyAsync(d_tiles, tiles.data(), sizeof(int32_t) * tiles.size(),
                                hipMemcpyHostToDevice, st));
        tile_build_kernel<LenT><<<n_tiles, 64, 0, st>>>(N, U, K, d_tiles, csr->row_ptr, csr->col,
                                                        (const LenT*)csr->len, tk, t0, t1);
    }
    const int nkt = (K + 63) / 64, n_rt = U * nkt;
    int32_t* rk = (int32_t*)(ws + L.rk);
    LenT* r0 = (LenT*)(ws + L.r0);
    LenT* r1 = (LenT*)(ws + L.r1);
    int32_t* range = (int32_t*)(ws + L.range);
    ray_tile_build_kernel<LenT><<<n_rt, 64, 0, st>>>(N, U, K, nkt, csr->trig, csr->t_row_ptr, csr->t_col,
                                                     (const LenT*)csr->t_len, rk, r0, r1, range);
    const unsigned rtb = gather_blocks(n_rt);
    const double scale = prm->lambda / (double)geom->n_angles;
    const dim3 tgrid((unsigned)((N + 31) / 32), (unsigned)((N + 31) / 32));
    for (int32_t it = 0; it < prm->n_iter; ++it) {
        transpose_kernel<<<tgrid, 256, 0, st>>>(N, d_image, fT);
        ray_tile_res_kernel<LenT><<<rtb, 256, 0, st>>>(N, U, K, nkt, n_rt, csr->trig, rk, r0, r1, range,
                                                      csr->t_row_ptr, csr->t_col, (const LenT*)csr->t_len,
                                                      d_image, fT, d_sino, W, q, partial);
        reduce_kernel<<<1, 256, 0, st>>>(partial, (int)rtb, sse + it);
        if (n_tiles > 0)
            tile_back_kernel<LenT><<<(unsigned)((n_tiles + kWPB - 1) / kWPB), 256, 0, st>>>(
                N, U, K, n_tiles, d_tiles, csr->row_ptr, tk, t0, t1, q, d_image, scale);
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
    if (!csr->trig) return fail(PILA_EINVAL, "trig (from pila_build) is NULL");
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
