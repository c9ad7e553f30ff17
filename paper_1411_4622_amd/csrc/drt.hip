// The comparison method of section III-A: simulated annealing whose
// evaluation step computes the projections of each estimate's whole image by
// the discrete Radon transform with bilinear interpolation (no PILA), and its
// cost from Eq. 4.  It exists to measure what the PILA saves on this
// hardware; it is not on the reconstruction path.
//
// Ray (u, k) is sampled at unit steps t = -T .. T (T = ceil(N / sqrt 2) + 1)
// at the points (s c - t sn, s sn + t c); each sample interpolates the image
// bilinearly between pixel centres, zero outside the grid.  Per step one
// kernel computes, for every estimate m and every ray, (DRT_m - Pm)^2 and
// per-block sums (fixed order); a one-wavefront kernel adds each estimate's
// block sums in block order, takes the first estimate of least cost (BoME),
// and applies Step 4 with the estimates, temperatures and acceptance
// uniforms the PILA chain uses (Philox4x64-10 counters (s, m, 0, 0) and
// (s, 0, 1, 0)).
#include <algorithm>
#include <cmath>
#include <vector>

#include "sat_chain.hpp"
#include "sat_host.hpp"

namespace pila {
namespace {

constexpr int kDrtThreads = 256;

struct DrtArgs {
    int32_t N, U, K, P, M, T, n_stages, schedule, proposal, n_blocks;
    int64_t n_steps;
    uint64_t seed, chain_id;
    double T0, TN, delta_max, f_min, f_max;
    const double* trig;
    const int32_t* support;
    const double* sino;
    double* f;
    double* part;   // [M][n_blocks] block sums of squared residuals
    int32_t* cand_p;
    double* cand_fn;  // [M] the step's estimates
    double* state;  // [0]: C of the current image
    int32_t* tr_m;
    uint8_t* tr_acc;
    double* tr_dc;
};

// bilinear value of the image at (x, y), pixel ov_p reading ov_v
__device__ __forceinline__ double bilinear(const DrtArgs& A, double x, double y, int32_t ov_p, double ov_v)
{
    const double h = A.N / 2.0;
    const double cx = x + h - 0.5, cy = h - 0.5 - y;
    const double j0 = floor(cx), i0 = floor(cy);
    const double ax = cx - j0, ay = cy - i0;
    double v = 0.0;
    for (int di = 0; di < 2; ++di)
        for (int dj = 0; dj < 2; ++dj) {
            const double i = i0 + di, j = j0 + dj;
            if (i < 0 || j < 0 || i >= A.N || j >= A.N) continue;
            const int32_t p = (int32_t)i * A.N + (int32_t)j;
            const double fv = p == ov_p ? ov_v : A.f[p];
            const double wgt = (di ? ay : 1.0 - ay) * (dj ? ax : 1.0 - ax);
            v += wgt * fv;
        }
    return v;
}

// Step s's estimates (Step 2, Eq. 3), computed once per step by one wave
__global__ __launch_bounds__(64) void drt_draw_kernel(DrtArgs A, int64_t s)
{
    const int m = threadIdx.x;
    if (m >= A.M) return;
    const Words4 w = philox4x64(A.seed, A.chain_id, (uint64_t)s, (uint64_t)m, 0, 0);
    const int32_t p = A.support[__umul64hi(w.w0, (uint64_t)A.P)];
    const double fo = A.f[p];
    double fn = fo + A.delta_max * (2.0 * unit53(w.w1) - 1.0);
    if (A.proposal == PILA_PROP_REDRAW) {
        for (uint64_t j = 1; (fn < A.f_min || fn > A.f_max) && j <= kRedrawMax; ++j)
            fn = fo + A.delta_max *
                          (2.0 * unit53(philox4x64(A.seed, A.chain_id, (uint64_t)s, (uint64_t)m, 0, j).w1) - 1.0);
        if (fn < A.f_min || fn > A.f_max) fn = fo;
    } else {
        if (fn < A.f_min) fn = A.f_min;
        if (fn > A.f_max) fn = A.f_max;
    }
    A.cand_p[m] = p;
    A.cand_fn[m] = fn;
}

// (DRT - Pm)^2 of every ray for estimate blockIdx.y (or the current image
// when cand is false), summed per block in a fixed order
__global__ __launch_bounds__(kDrtThreads) void drt_cost_kernel(DrtArgs A, int cand)
{
    __shared__ double red[kDrtThreads / kWave];
    const int m = blockIdx.y;
    const int32_t ov_p = cand ? A.cand_p[m] : -1;
    const double ov_v = cand ? A.cand_fn[m] : 0.0;
    const int64_t G = (int64_t)A.U * A.K;
    const int64_t g = (int64_t)blockIdx.x * kDrtThreads + threadIdx.x;
    double sq = 0.0;
    if (g < G) {
        const int u = (int)(g / A.K), k = (int)(g - (int64_t)u * A.K);
        const double c = A.trig[2 * u], sn = A.trig[2 * u + 1];
        const double sk = k - (A.K - 1) / 2.0;
        double acc = 0.0;
        for (int32_t t = -A.T; t <= A.T; ++t) acc += bilinear(A, sk * c - t * sn, sk * sn + t * c, ov_p, ov_v);
        const double d = acc - A.sino[g];
        sq = d * d;
    }
    sq = wave_canon_sum(sq);
    if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = sq;
    __syncthreads();
    if (threadIdx.x == 0) {
        double b = 0.0;
        for (int i = 0; i < kDrtThreads / kWave; ++i) b += red[i];
        A.part[(int64_t)m * A.n_blocks + blockIdx.x] = b;
    }
}

// sum of estimate m's block sums, lane-strided then the canonical butterfly
__device__ double block_total(const DrtArgs& A, int m, int lane)
{
    double a = 0.0;
    for (int b = lane; b < A.n_blocks; b += kWave) a += A.part[(int64_t)m * A.n_blocks + b];
    return wave_canon_sum(a);
}

__global__ __launch_bounds__(64) void drt_init_kernel(DrtArgs A)
{
    const double sse = block_total(A, 0, threadIdx.x);
    if (threadIdx.x == 0) A.state[0] = sqrt(sse / ((double)A.K * (double)A.U));
}

// BoME over the step's estimates and Step 4
__global__ __launch_bounds__(64) void drt_decide_kernel(DrtArgs A, int64_t s)
{
    const int lane = threadIdx.x;
    const double KU = (double)A.K * (double)A.U;
    int best = -1;
    double bestC = INFINITY;
    for (int m = 0; m < A.M; ++m) {
        const double Cm = sqrt(block_total(A, m, lane) / KU);
        if (Cm < bestC || best < 0) {
            bestC = Cm;
            best = m;
        }
    }
    if (lane != 0) return;
    const double C = A.state[0];
    const double dC = bestC - C;
    const int64_t n = (s * (int64_t)A.n_stages) / A.n_steps;
    const double x = (double)n, NN = (double)A.n_stages;
    double T;
    if (A.schedule == PILA_SCHED_EXP)
        T = A.T0 * pow(A.TN / A.T0, x / NN);
    else if (A.schedule == PILA_SCHED_CUBIC)
        T = A.T0 - (x * x * x) * ((A.T0 - A.TN) / (NN * NN * NN));
    else
        T = A.T0 - x * ((A.T0 - A.TN) / NN);
    const double N1 = unit53(philox4x64(A.seed, A.chain_id, (uint64_t)s, 0, 1, 0).w0);
    const bool accept = dC <= 0.0 || N1 < exp(-dC / T);
    if (A.tr_m) A.tr_m[s] = best;
    if (A.tr_acc) A.tr_acc[s] = accept ? 1 : 0;
    if (A.tr_dc) A.tr_dc[s] = dC;
    if (accept) {
        A.f[A.cand_p[best]] = A.cand_fn[best];
        A.state[0] = bestC;
    }
}

size_t drt_bytes(const pila_geom* g, const sat_params* p)
{
    const int64_t G = (int64_t)g->n_angles * g->n_bins;
    const size_t nb = (size_t)((G + kDrtThreads - 1) / kDrtThreads);
    const size_t M = (size_t)(p->m_cand > 0 ? p->m_cand : 1);
    return align256(8 * M * nb) + align256(4 * M) + align256(8 * M) + align256(8 * 2) +
           align256(8 * 2 * (size_t)g->n_angles) + align256(4 * (size_t)g->n * g->n);
}

}  // namespace
}  // namespace pila

using namespace pila;

extern "C" int32_t sat_drt_workspace_size(const pila_geom* geom, const sat_params* params, size_t* bytes)
{
    clear_error();
    PILA_TRY(check_geom(geom));
    if (!params || !bytes) return fail(PILA_EINVAL, "params or bytes is NULL");
    *bytes = drt_bytes(geom, params);
    return PILA_OK;
}

extern "C" int32_t sat_drt_run(const pila_geom* geom, const double* d_sino, const sat_params* params,
                               double* d_image, void* d_ws, size_t ws_bytes, double* h_cost_final,
                               const sat_trace* trace, void* stream)
{
    clear_error();
    PILA_TRY(check_geom(geom));
    if (!params || !d_sino || !d_image) return fail(PILA_EINVAL, "params, sinogram or image is NULL");
    const sat_params* p = params;
    if (p->m_cand < 1 || p->m_cand > 64) return fail(PILA_EINVAL, "m_cand must be in 1..64");
    if (p->n_steps < 0 || p->n_stages < 1) return fail(PILA_EINVAL, "bad n_steps / n_stages");
    if (!(p->T0 > 0.0 && p->TN > 0.0 && std::isfinite(p->T0) && std::isfinite(p->TN)))
        return fail(PILA_EINVAL, "the DRT chain needs T0 and TN given (positive, finite)");
    if (!(p->delta_max >= 0.0) || !std::isfinite(p->delta_max) || !(p->f_max >= p->f_min))
        return fail(PILA_EINVAL, "bad delta_max / value range");
    if (p->schedule < PILA_SCHED_LINEAR || p->schedule > PILA_SCHED_CUBIC)
        return fail(PILA_EINVAL, "schedule must be PILA_SCHED_LINEAR, _EXP or _CUBIC");
    if (p->proposal != PILA_PROP_CLAMP && p->proposal != PILA_PROP_REDRAW)
        return fail(PILA_EINVAL, "proposal must be PILA_PROP_CLAMP or PILA_PROP_REDRAW");
    const size_t need = drt_bytes(geom, p);
    if (!d_ws || ws_bytes < need)
        return fail(PILA_ENOMEM, "workspace of %zu bytes is below the %zu needed", ws_bytes, need);
    hipStream_t st = (hipStream_t)stream;
    const int32_t N = geom->n, U = geom->n_angles, K = geom->n_bins;
    const int64_t NP = (int64_t)N * N, G = (int64_t)U * K;
    std::vector<int32_t> support;
    for (int64_t q = 0; q < NP; ++q)
        if (!geom->mask || geom->mask[q]) support.push_back((int32_t)q);
    if (support.empty()) return fail(PILA_EINVAL, "empty support");
    std::vector<double> cs(2 * (size_t)U);
    for (int u = 0; u < U; ++u) trig_of(geom->angles_deg[u], &cs[2 * u], &cs[2 * u + 1]);
    DrtArgs A;
    A.N = N;
    A.U = U;
    A.K = K;
    A.P = (int32_t)support.size();
    A.M = p->m_cand;
    A.T = (int32_t)std::ceil(N / std::sqrt(2.0)) + 1;
    A.n_stages = p->n_stages;
    A.schedule = p->schedule;
    A.proposal = p->proposal;
    A.n_blocks = (int32_t)((G + kDrtThreads - 1) / kDrtThreads);
    A.n_steps = p->n_steps;
    A.seed = p->seed;
    A.chain_id = p->chain_id;
    A.T0 = p->T0;
    A.TN = p->TN;
    A.delta_max = p->delta_max;
    A.f_min = p->f_min;
    A.f_max = p->f_max;
    char* ws = (char*)d_ws;
    const size_t M = (size_t)A.M, nb = (size_t)A.n_blocks;
    A.part = (double*)ws;
    ws += align256(8 * M * nb);
    A.cand_p = (int32_t*)ws;
    ws += align256(4 * M);
    A.cand_fn = (double*)ws;
    ws += align256(8 * M);
    A.state = (double*)ws;
    ws += align256(8 * 2);
    double* d_trig = (double*)ws;
    ws += align256(8 * 2 * (size_t)U);
    int32_t* d_support = (int32_t*)ws;
    A.trig = d_trig;
    A.support = d_support;
    A.sino = d_sino;
    A.f = d_image;
    A.tr_m = trace ? trace->m_star : nullptr;
    A.tr_acc = trace ? trace->accept : nullptr;
    A.tr_dc = trace ? trace->dC : nullptr;
    // geometry to the workspace (the host arrays end with this call)
    PILA_HIP(hipMemcpyAsync(d_trig, cs.data(), sizeof(double) * cs.size(), hipMemcpyHostToDevice, st));
    PILA_HIP(hipMemcpyAsync(d_support, support.data(), sizeof(int32_t) * support.size(), hipMemcpyHostToDevice,
                            st));
    const dim3 grid1((unsigned)A.n_blocks, 1), gridM((unsigned)A.n_blocks, (unsigned)A.M);
    drt_cost_kernel<<<grid1, kDrtThreads, 0, st>>>(A, 0);
    drt_init_kernel<<<1, 64, 0, st>>>(A);
    for (int64_t s = 0; s < p->n_steps; ++s) {
        drt_draw_kernel<<<1, 64, 0, st>>>(A, s);
        drt_cost_kernel<<<gridM, kDrtThreads, 0, st>>>(A, 1);
        drt_decide_kernel<<<1, 64, 0, st>>>(A, s);
    }
    PILA_HIP(hipGetLastError());
    if (h_cost_final) {
        PILA_HIP(hipMemcpyAsync(h_cost_final, A.state, sizeof(double), hipMemcpyDeviceToHost, st));
    }
    // the geometry upload reads host memory owned by this call
    PILA_HIP(hipStreamSynchronize(st));
    return PILA_OK;
}
