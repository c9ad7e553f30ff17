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
#include <climits>
#include <cmath>
#include <cstdlib>
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
// Tile layouts for SIRT.  Both projections run one wavefront per tile of 64
// PILA rows (lane = row) and walk the tile's rows in step: at one step each
// lane holds at most two entries, at neighbouring indices, stored as an
// 8-bit offset from the step's smallest index (one base per step) and two
// lengths, zero where absent.  Element (t, s, lane) sits at (t S + s) 64 +
// lane, so the 64 lanes of a step read consecutive bytes and words.  A tile
// whose rows break that shape (a third entry at one step, a pair that is
// not neighbours, an offset above 255) is flagged and its rows are summed
// straight from the CSR.
//
// Back projection: tiles of 8 x 8 pixels, steps = angles.  A pixel's shadow
// on the detector is at most sqrt 2 bins wide, so at one angle it meets one
// or two rays of neighbouring bins, and the tile's 64 pixels meet about 12
// bins of one sinogram row.  Each pixel adds its terms in its row's order
// (angle, then bin), as a walk of the row would.
//
// Forward projection: tiles of 64 rays of consecutive bins at one angle;
// steps are image rows for rays closer to the columns (|cos| > |sin|), image
// columns for the others.  Such a ray moves less than one pixel sideways per
// step, so it meets one or two neighbouring pixels there, and the tile's 64
// rays meet about 64-91 pixels of one image row (read from the image) or
// column (read from its transpose).  Steps run over the tile's used range.
// ---------------------------------------------------------------------------
constexpr int kTile = 8;
constexpr int kOdd = -2;  // flag of a tile summed from its CSR rows

__device__ __forceinline__ int64_t tile_pixel(const int32_t* tiles, int t, int lane, int N)
{
    const int tt = tiles[t];
    const int ti = tt >> 16, tj = tt & 0xFFFF;
    const int i = ti * kTile + (lane >> 3), j = tj * kTile + (lane & 7);
    return (i < N && j < N) ? (int64_t)i * N + j : -1;
}

__device__ __forceinline__ bool ray_cols(const double* trig, int u)
{
    return fabs(trig[2 * u]) > fabs(trig[2 * u + 1]);
}

// A lane's window of kWin consecutive PILA entries (index and length) in
// LDS, aligned to kWin entries.  A tile build walks 64 rows at once, one per
// lane, a few entries per step; read straight from memory each entry would
// cost a cache line that is evicted again before the lane's next step.
// Through the window each 64-byte segment is fetched once.
constexpr int kWin = 16;

template <typename LenT>
struct EntryWindow {
    int32_t* wc;  // LDS, kWin indices of this lane
    LenT* wl;     // LDS, kWin lengths
    int64_t w;    // first entry held
    const int32_t* __restrict__ ci;
    const LenT* __restrict__ ln;
    int64_t nnz;
    bool vec;  // ci and ln 16-byte aligned: fill with 16-byte loads
    __device__ void fill(int64_t q)
    {
        w = q & ~(int64_t)(kWin - 1);
        if (vec && w + kWin <= nnz) {
            const int4* c4 = reinterpret_cast<const int4*>(ci + w);
#pragma unroll
            for (int a = 0; a < kWin / 4; ++a) {
                const int4 v = c4[a];
                wc[4 * a] = v.x;
                wc[4 * a + 1] = v.y;
                wc[4 * a + 2] = v.z;
                wc[4 * a + 3] = v.w;
            }
            constexpr int kPer = 16 / (int)sizeof(LenT);
            const int4* l4 = reinterpret_cast<const int4*>(ln + w);
#pragma unroll
            for (int a = 0; a < kWin / kPer; ++a) {
                const int4 v = l4[a];
                __builtin_memcpy(wl + a * kPer, &v, 16);
            }
        } else {
            for (int a = 0; a < kWin && w + a < nnz; ++a) {
                wc[a] = ci[w + a];
                wl[a] = ln[w + a];
            }
        }
    }
    __device__ int32_t col(int64_t q)
    {
        if (q < w || q >= w + kWin) fill(q);
        return wc[q - w];
    }
    __device__ LenT len(int64_t q)
    {
        if (q < w || q >= w + kWin) fill(q);
        return wl[q - w];
    }
};

// LDS of the 64 lanes' windows (rows padded by one word against bank conflicts)
template <typename LenT>
struct WindowLds {
    int32_t c[64][kWin + 1];
    LenT l[64][kWin + 1];
};

template <typename LenT>
__device__ __forceinline__ EntryWindow<LenT> entry_window(WindowLds<LenT>& lds, int lane,
                                                          const int32_t* ci, const LenT* ln,
                                                          int64_t nnz, bool vec)
{
    return EntryWindow<LenT>{lds.c[lane], lds.l[lane], -(int64_t)kWin - 1, ci, ln, nnz, vec};
}

// Walk of a PILA row in its stored order.
struct RowWalk {
    int64_t q, e;
    __device__ bool more() const { return q < e; }
    template <typename Win>
    __device__ void next(Win&) { ++q; }
};

// Walk of a ray's entries in ascending step order.  Entries are stored by
// ascending image row, then column.  Where the steps are image rows, or are
// columns that rise with the rows, that order already is the step order;
// for a ray whose columns fall as its rows rise, the walk takes the row
// groups (entries of one image row) last to first, each first to last.
struct RayWalk {
    int N;
    int64_t b, q, gs, ge;
    bool rev;
    template <typename Win>
    __device__ int64_t group_start(Win& win, int64_t x) const
    {
        const int r = win.col(x) / N;
        while (x > b && win.col(x - 1) / N == r) --x;
        return x;
    }
    template <typename Win>
    __device__ RayWalk(Win& win, int n, int64_t b0, int64_t e0, bool reverse)
        : N(n), b(b0), q(b0), gs(b0), ge(e0), rev(reverse && e0 > b0)
    {
        if (rev) q = gs = group_start(win, e0 - 1);
    }
    __device__ bool more() const { return q < ge; }
    template <typename Win>
    __device__ void next(Win& win)
    {
        if (++q == ge && rev && gs > b) {
            ge = gs;
            gs = group_start(win, gs - 1);
            q = gs;
        }
    }
};

// One step of a tile build: each lane takes the entries of its row at step
// st from its walk, and the wave writes the step's cells and base.  False
// where the entries break the tile shape.  Every lane of the wavefront calls
// it with the same st.
template <typename LenT, typename Walk, typename Key>
__device__ __forceinline__ bool tile_step(int st, int R, Walk& wk, EntryWindow<LenT>& win, const Key& key,
                                          int64_t cell, int64_t bcell, uint8_t* __restrict__ off,
                                          LenT* __restrict__ l0, LenT* __restrict__ l1,
                                          int32_t* __restrict__ base)
{
    int ia = -1, ib = -1;
    LenT la = (LenT)0, lb = (LenT)0;
    bool ok = true;
    for (int c = 0; c < 3 && wk.more(); ++c) {
        int s, idx;
        key(win.col(wk.q), &s, &idx);
        if (s != st) break;
        if (c == 0) {
            ia = idx;
            la = win.len(wk.q);
        } else if (c == 1) {
            ib = idx;
            lb = win.len(wk.q);
        } else {
            ok = false;
        }
        wk.next(win);
    }
    if (ib >= 0 && ib < ia) {
        const int ti = ia;
        ia = ib;
        ib = ti;
        const LenT tl = la;
        la = lb;
        lb = tl;
    }
    if (ib >= 0 && ib != ia + 1) ok = false;
    if (ia >= R || (ia < 0 && ib >= 0)) {  // not an index of this step's line
        ok = false;
        ia = ib = -1;
    }
    int m = ia >= 0 ? ia : INT_MAX;
    for (int o = 32; o > 0; o >>= 1) m = min(m, __shfl_xor(m, o, 64));
    const int d = ia >= 0 ? ia - m : 0;
    if (d > 255) ok = false;
    off[cell] = (uint8_t)(d > 255 ? 0 : d);
    l0[cell] = la;
    l1[cell] = lb;
    if ((threadIdx.x & 63) == 0) base[bcell] = m == INT_MAX ? 0 : m;
    return ok;
}

// Sum over the steps lo..hi of one lane's tile cells: l0 src[s R + x] +
// l1 src[s R + x + 1] with x = base[s] + offset, S steps at a time.  The
// next group's cells are loaded after this group's gathers are issued, so
// they are in flight while the gathers are waited for (loads complete in
// issue order).  Terms are added by ascending step, l0 before l1.
template <typename LenT, int S>
__device__ __forceinline__ double tile_sum(int lo, int hi, int R, const int32_t* __restrict__ tb,
                                           const uint8_t* __restrict__ off, const LenT* __restrict__ l0,
                                           const LenT* __restrict__ l1, int64_t cb,
                                           const double* __restrict__ src)
{
    double acc = 0.0;
    if (lo > hi) return acc;
    int32_t ii[S];
    LenT a0[S], a1[S];
    auto load = [&](int s0) {
#pragma unroll
        for (int a = 0; a < S; ++a) {
            const int st = s0 + a <= hi ? s0 + a : hi;
            ii[a] = tb[st] + (int32_t)off[cb + (int64_t)st * 64];
            a0[a] = l0[cb + (int64_t)st * 64];
            a1[a] = l1[cb + (int64_t)st * 64];
        }
    };
    load(lo);
    for (int s0 = lo; s0 <= hi; s0 += S) {
        double v0[S], v1[S];
        LenT c0[S], c1[S];
#pragma unroll
        for (int a = 0; a < S; ++a) {
            const int st = s0 + a <= hi ? s0 + a : hi;
            const int64_t at = (int64_t)st * R + ii[a];
            v0[a] = src[at];
            v1[a] = src[ii[a] + 1 < R ? at + 1 : at];
            c0[a] = a0[a];
            c1[a] = a1[a];
        }
        __builtin_amdgcn_sched_barrier(0);
        if (s0 + S <= hi) load(s0 + S);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int a = 0; a < S; ++a) {
            if (s0 + a <= hi) {
                acc = fma((double)c0[a], v0[a], acc);
                acc = fma((double)c1[a], v1[a], acc);
            }
        }
    }
    return acc;
}

template <typename LenT>
__global__ __launch_bounds__(64) void tile_build_kernel(int N, int U, int K, const int32_t* __restrict__ tiles,
                                                       const int64_t* __restrict__ rp,
                                                       const int32_t* __restrict__ ci,
                                                       const LenT* __restrict__ ln,
                                                       uint8_t* __restrict__ off, LenT* __restrict__ l0,
                                                       LenT* __restrict__ l1, int32_t* __restrict__ base,
                                                       int32_t* __restrict__ flag, int64_t nnz, bool vec,
                                                       bool force_csr)
{
    __shared__ WindowLds<LenT> lds;
    const int t = blockIdx.x, lane = threadIdx.x;
    const int64_t p = tile_pixel(tiles, t, lane, N);
    auto key = [&](int g, int* s, int* idx) {
        const int u = g / K;
        *s = u;
        *idx = g - u * K;
    };
    EntryWindow<LenT> win = entry_window(lds, lane, ci, ln, nnz, vec);
    RowWalk wk{p >= 0 ? rp[p] : 0, p >= 0 ? rp[p + 1] : 0};
    bool ok = true;
    for (int u = 0; u < U; ++u) {
        const int64_t bc = (int64_t)t * U + u;
        ok &= tile_step<LenT>(u, K, wk, win, key, bc * 64 + lane, bc, off, l0, l1, base);
    }
    if (wk.more() || force_csr) ok = false;
    const bool odd = __any(!ok);
    if (lane == 0) flag[t] = odd ? kOdd : 0;
}

// Workgroup b's tile: workgroups go to the 8 XCDs round robin, so XCD x
// takes the x-th eighth of the tiles (neighbouring tiles, shared L2 lines);
// -1 for the padding of the grid to a multiple of 8.
__device__ __forceinline__ int64_t xcd_tile(int64_t n)
{
    constexpr int kXcd = 8;
    const int64_t chunk = (n + kXcd - 1) / kXcd;
    const int64_t t = (int64_t)(blockIdx.x % kXcd) * chunk + blockIdx.x / kXcd;
    return (int64_t)(blockIdx.x / kXcd) < chunk && t < n ? t : -1;
}

unsigned xcd_grid(int64_t n)
{
    return (unsigned)(8 * ((n + 7) / 8));
}

// The steps lo..hi split in kWPB nearly equal parts, wavefront w taking part w
__device__ __forceinline__ void wave_part(int lo, int hi, int w, int* a, int* b)
{
    const int64_t n = (int64_t)hi - lo + 1;
    *a = lo + (int)(n * w / kWPB);
    *b = lo + (int)(n * (w + 1) / kWPB) - 1;
}

// One workgroup per pixel tile; its 4 wavefronts take a quarter of the
// angles each, and their sums are added in wavefront order.
template <typename LenT>
__global__ __launch_bounds__(256) void tile_back_kernel(int N, int U, int K, int n_tiles,
                                                       const int32_t* __restrict__ tiles,
                                                       const int64_t* __restrict__ rp,
                                                       const int32_t* __restrict__ ci,
                                                       const LenT* __restrict__ ln,
                                                       const int32_t* __restrict__ flag,
                                                       const uint8_t* __restrict__ off,
                                                       const LenT* __restrict__ l0,
                                                       const LenT* __restrict__ l1,
                                                       const int32_t* __restrict__ base,
                                                       const double* __restrict__ y,
                                                       double* __restrict__ f, double scale)
{
    constexpr int kA = 8;  // angles in flight
    __shared__ double part[kWPB][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t t = xcd_tile(n_tiles);
    if (t < 0) return;
    const int64_t p = tile_pixel(tiles, (int)t, lane, N);
    double acc = 0.0;
    if (flag[t] == kOdd) {
        if (w == 0 && p >= 0)
            for (int64_t q = rp[p]; q < rp[p + 1]; ++q) acc = fma((double)ln[q], y[ci[q]], acc);
    } else {
        int a, b;
        wave_part(0, U - 1, w, &a, &b);
        acc = tile_sum<LenT, kA>(a, b, K, base + t * U, off, l0, l1, t * U * 64 + lane, y);
    }
    part[w][lane] = acc;
    __syncthreads();
    if (w == 0) {
        const double sum = ((part[0][lane] + part[1][lane]) + part[2][lane]) + part[3][lane];
        if (p >= 0 && rp[p + 1] > rp[p]) f[p] = f[p] + scale * sum;
    }
}

template <typename LenT>
__global__ __launch_bounds__(64) void ray_tile_build_kernel(int N, int U, int K, int nkt,
                                                           const double* __restrict__ trig,
                                                           const int64_t* __restrict__ rp,
                                                           const int32_t* __restrict__ ci,
                                                           const LenT* __restrict__ ln,
                                                           uint8_t* __restrict__ off, LenT* __restrict__ l0,
                                                           LenT* __restrict__ l1, int32_t* __restrict__ base,
                                                           int32_t* __restrict__ range, int64_t nnz, bool vec,
                                                           bool force_csr)
{
    __shared__ WindowLds<LenT> lds;
    const int t = blockIdx.x, lane = threadIdx.x;
    const int u = t / nkt, k = (t - u * nkt) * 64 + lane;
    const bool cols = ray_cols(trig, u);
    auto key = [&](int p, int* s, int* idx) {
        const int i = p / N, j = p - i * N;
        *s = cols ? i : j;
        *idx = cols ? j : i;
    };
    EntryWindow<LenT> win = entry_window(lds, lane, ci, ln, nnz, vec);
    const int64_t g = (int64_t)u * K + k;
    const int64_t b = k < K ? rp[g] : 0, e = k < K ? rp[g + 1] : 0;
    int lo = N, hi = -1;
    bool bad = false;
    for (int64_t q = b; q < e; ++q) {
        int s, x;
        key(win.col(q), &s, &x);
        if (s < 0 || s >= N) {  // not a pixel index: the tile is summed from the CSR
            bad = true;
            continue;
        }
        lo = min(lo, s);
        hi = max(hi, s);
    }
    for (int o = 32; o > 0; o >>= 1) {
        lo = min(lo, __shfl_xor(lo, o, 64));
        hi = max(hi, __shfl_xor(hi, o, 64));
    }
    // a row of the image is one pixel high, and the ray moves s / c pixels
    // along it per row: its columns fall as its rows rise where c s < 0
    RayWalk wk(win, N, b, e, !cols && trig[2 * u] * trig[2 * u + 1] < 0.0);
    bool ok = true;
    for (int st = lo; st <= hi; ++st) {
        const int64_t bc = (int64_t)t * N + st;
        ok &= tile_step<LenT>(st, N, wk, win, key, bc * 64 + lane, bc, off, l0, l1, base);
    }
    if (wk.more() || bad || force_csr) ok = false;
    const bool odd = __any(!ok);
    if (lane == 0) {
        range[2 * t] = odd ? 0 : lo;
        range[2 * t + 1] = odd ? kOdd : hi;
    }
}

// Forward projection by bands: the steps of all ray tiles are cut into bands
// of B image rows (or transposed-image rows), B N doubles of each image about
// a megabyte, and the work items (tile, band) of an XCD run band by band, so
// that the XCD's L2 holds the image lines its gathers need.  An item writes
// its 64 partial sums; ray_tile_res_kernel adds them in band order.
int ray_band(int N)
{
    int b = 131072 / (N > 0 ? N : 1);
    b = b < 8 ? 8 : (b > 256 ? 256 : b);
    return b & ~7;
}

template <typename LenT>
__global__ __launch_bounds__(64) void ray_tile_part_kernel(int N, int K, int nkt, int n_tiles, int band,
                                                           int n_bands, const double* __restrict__ trig,
                                                           const uint8_t* __restrict__ off,
                                                           const LenT* __restrict__ l0,
                                                           const LenT* __restrict__ l1,
                                                           const int32_t* __restrict__ base,
                                                           const int32_t* __restrict__ range,
                                                           const int64_t* __restrict__ rp,
                                                           const int32_t* __restrict__ ci,
                                                           const LenT* __restrict__ ln,
                                                           const double* __restrict__ f,
                                                           const double* __restrict__ fT,
                                                           double* __restrict__ part)
{
    constexpr int kS = 8;  // steps in flight
    const int lane = threadIdx.x;
    // item j of XCD x (workgroups go to the XCDs round robin): band j / chunk
    // of tile x chunk + j mod chunk
    const int64_t chunk = (n_tiles + 7) / 8, j = blockIdx.x / 8;
    const int64_t bnd = j / chunk, t = (int64_t)(blockIdx.x % 8) * chunk + j % chunk;
    if (bnd >= n_bands || t >= n_tiles) return;
    const int u = (int)(t / nkt), k = (int)(t - (int64_t)u * nkt) * 64 + lane;
    const double* img = ray_cols(trig, u) ? f : fT;
    const int lo = range[2 * t], hi = range[2 * t + 1];
    double acc = 0.0;
    if (hi == kOdd) {
        if (bnd == 0 && k < K) {
            const int64_t g = (int64_t)u * K + k;
            for (int64_t q = rp[g]; q < rp[g + 1]; ++q) acc = fma((double)ln[q], f[ci[q]], acc);
        }
    } else {
        const int b0 = (int)bnd * band;
        const int a = lo > b0 ? lo : b0, b = hi < b0 + band - 1 ? hi : b0 + band - 1;
        acc = tile_sum<LenT, kS>(a, b, N, base + t * N, off, l0, l1, t * N * 64 + lane, img);
    }
    part[(bnd * n_tiles + t) * 64 + lane] = acc;
}

// res = Pm - A f per ray (A f the band sums added in band order), q = res / W
// (0 where W = 0), and per ray tile the sum of res^2.  A wavefront per tile.
__global__ __launch_bounds__(256) void ray_tile_res_kernel(int K, int nkt, int n_tiles, int n_bands,
                                                           const double* __restrict__ part,
                                                           const double* __restrict__ sino,
                                                           const double* __restrict__ W,
                                                           double* __restrict__ out,
                                                           double* __restrict__ partial)
{
    const int lane = threadIdx.x & 63;
    const int64_t t = (int64_t)blockIdx.x * kWPB + (threadIdx.x >> 6);
    if (t >= n_tiles) return;
    const int u = (int)(t / nkt), k = (int)(t - (int64_t)u * nkt) * 64 + lane;
    double sum = 0.0;
    for (int b = 0; b < n_bands; ++b) sum += part[((int64_t)b * n_tiles + t) * 64 + lane];
    double sq = 0.0;
    if (k < K) {
        const int64_t g = (int64_t)u * K + k;
        const double res = sino[g] - sum;
        const double wg = W[g];
        out[g] = wg > 0.0 ? res / wg : 0.0;
        sq = res * res;
    }
    sq = wave_sum(sq);
    if (lane == 0) partial[t] = sq;
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
    size_t W, q, partial, sse, fT, tiles, flag, off, l0, l1, base, roff, r0, r1, rbase, range, bpart, total;
};

SirtLayout sirt_layout(const pila_geom* g, int32_t n_iter, size_t n_tiles)
{
    const size_t G = (size_t)g->n_angles * g->n_bins, NP = (size_t)g->n * g->n;
    const size_t ls = (size_t)len_bytes(g->len_dtype);
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
    const size_t nrt0 = (size_t)g->n_angles * ((g->n_bins + 63) / 64);
    L.partial = take(sizeof(double) * (nrt0 > (size_t)kGatherBlocks ? nrt0 : (size_t)kGatherBlocks));
    L.fT = take(sizeof(double) * NP);
    L.tiles = take(sizeof(int32_t) * (n_tiles ? n_tiles : 1));
    L.flag = take(sizeof(int32_t) * (n_tiles ? n_tiles : 1));
    L.off = take(cells);
    L.l0 = take(ls * cells);
    L.l1 = take(ls * cells);
    L.base = take(sizeof(int32_t) * (cells / 64));
    const size_t nrt = (size_t)g->n_angles * ((g->n_bins + 63) / 64);
    const size_t rcells = nrt * (size_t)g->n * 64;
    L.roff = take(rcells);
    L.r0 = take(ls * rcells);
    L.r1 = take(ls * rcells);
    L.rbase = take(sizeof(int32_t) * (rcells / 64));
    L.range = take(sizeof(int32_t) * 2 * nrt);
    const int band = ray_band(g->n);
    const size_t n_bands = (size_t)((g->n + band - 1) / band);
    L.bpart = take(sizeof(double) * n_bands * nrt * 64);
    // last, so that the layouts above sit at the same offsets for any n_iter
    L.sse = take(sizeof(double) * (size_t)(n_iter > 0 ? n_iter : 1));
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
    else if (geom->len_dtype == PILA_F32)
        ray_gather_kernel<float, kFwd><<<gather_blocks(G), 256, 0, st>>>(
            G, csr->t_row_ptr, csr->t_col, (const float*)csr->t_len, d_image, nullptr, nullptr, d_out, nullptr);
    else
        ray_gather_kernel<LenQ, kFwd><<<gather_blocks(G), 256, 0, st>>>(
            G, csr->t_row_ptr, csr->t_col, (const LenQ*)csr->t_len, d_image, nullptr, nullptr, d_out, nullptr);
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
    else if (geom->len_dtype == PILA_F32)
        pixel_gather_kernel<float, kBack><<<gather_blocks(NP), 256, 0, st>>>(
            NP, csr->row_ptr, csr->col, (const float*)csr->len, d_sino, d_out, 0.0);
    else
        pixel_gather_kernel<LenQ, kBack><<<gather_blocks(NP), 256, 0, st>>>(
            NP, csr->row_ptr, csr->col, (const LenQ*)csr->len, d_sino, d_out, 0.0);
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

static bool aligned16(const void* a, const void* b)
{
    return ((uintptr_t)a % 16) == 0 && ((uintptr_t)b % 16) == 0;
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
    int32_t* flag = (int32_t*)(ws + L.flag);
    uint8_t* off = (uint8_t*)(ws + L.off);
    LenT* l0 = (LenT*)(ws + L.l0);
    LenT* l1 = (LenT*)(ws + L.l1);
    int32_t* base = (int32_t*)(ws + L.base);
    const unsigned gb = gather_blocks(G);
    // PILA_SIRT_CSR=1 sums every tile from its CSR rows (the path a tile of
    // irregular shape takes), for tests of that path
    const char* env = std::getenv("PILA_SIRT_CSR");
    const bool force_csr = env && env[0] == '1';
    const bool reuse = (prm->flags & PILA_SIRT_REUSE_LAYOUT) != 0;
    // factor matrix: W_g = sum of squared lengths of ray g over the support
    if (!reuse)
        ray_gather_kernel<LenT, kW><<<gb, 256, 0, st>>>(G, csr->t_row_ptr, csr->t_col,
                                                        (const LenT*)csr->t_len, nullptr, nullptr,
                                                        nullptr, W, nullptr);
    if (n_tiles > 0 && !reuse) {
        PILA_HIP(hipMemcpyAsync(d_tiles, tiles.data(), sizeof(int32_t) * tiles.size(),
                                hipMemcpyHostToDevice, st));
        tile_build_kernel<LenT><<<n_tiles, 64, 0, st>>>(N, U, K, d_tiles, csr->row_ptr, csr->col,
                                                        (const LenT*)csr->len, off, l0, l1, base, flag,
                                                        csr->nnz, aligned16(csr->col, csr->len), force_csr);
    }
    const int nkt = (K + 63) / 64, n_rt = U * nkt;
    uint8_t* roff = (uint8_t*)(ws + L.roff);
    LenT* r0 = (LenT*)(ws + L.r0);
    LenT* r1 = (LenT*)(ws + L.r1);
    int32_t* rbase = (int32_t*)(ws + L.rbase);
    int32_t* range = (int32_t*)(ws + L.range);
    double* bpart = (double*)(ws + L.bpart);
    const int band = ray_band(N), n_bands = (N + band - 1) / band;
    if (!reuse)
        ray_tile_build_kernel<LenT><<<n_rt, 64, 0, st>>>(N, U, K, nkt, csr->trig, csr->t_row_ptr, csr->t_col,
                                                         (const LenT*)csr->t_len, roff, r0, r1, rbase, range,
                                                         csr->nnz, aligned16(csr->t_col, csr->t_len), force_csr);

    const double scale = prm->lambda / (double)geom->n_angles;
    const dim3 tgrid((unsigned)((N + 31) / 32), (unsigned)((N + 31) / 32));
    for (int32_t it = 0; it < prm->n_iter; ++it) {
        transpose_kernel<<<tgrid, 256, 0, st>>>(N, d_image, fT);
        ray_tile_part_kernel<LenT><<<(unsigned)(8 * ((n_rt + 7) / 8) * n_bands), 64, 0, st>>>(
            N, K, nkt, n_rt, band, n_bands, csr->trig, roff, r0, r1, rbase, range, csr->t_row_ptr, csr->t_col,
            (const LenT*)csr->t_len, d_image, fT, bpart);
        ray_tile_res_kernel<<<(unsigned)((n_rt + kWPB - 1) / kWPB), 256, 0, st>>>(K, nkt, n_rt, n_bands, bpart,
                                                                                d_sino, W, q, partial);
        reduce_kernel<<<1, 256, 0, st>>>(partial, n_rt, sse + it);
        if (n_tiles > 0)
            tile_back_kernel<LenT><<<xcd_grid(n_tiles), 256, 0, st>>>(
                N, U, K, n_tiles, d_tiles, csr->row_ptr, csr->col, (const LenT*)csr->len, flag, off, l0, l1,
                base, q, d_image, scale);
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
    if (params->flags & ~PILA_SIRT_REUSE_LAYOUT) return fail(PILA_EINVAL, "unknown flags %d", params->flags);
    size_t need = 0;
    PILA_TRY(sirt_workspace_size(geom, params, &need));
    if (!d_ws || ws_bytes < need)
        return fail(PILA_ENOMEM, "workspace of %zu bytes is below the %zu needed", ws_bytes, need);
    hipStream_t st = (hipStream_t)stream;
    if (geom->len_dtype == PILA_F64)
        return sirt_impl<double>(geom, csr, d_sino, params, d_image, (char*)d_ws, h_cost, st);
    if (geom->len_dtype == PILA_F32)
        return sirt_impl<float>(geom, csr, d_sino, params, d_image, (char*)d_ws, h_cost, st);
    return sirt_impl<LenQ>(geom, csr, d_sino, params, d_image, (char*)d_ws, h_cost, st);
}
