// Simulated annealing tomography chains on gfx950: kernels and the host
// entry points sat_run / sat_run_batch.  The chain bodies and their
// algorithm are in sat_chain.hpp.
#include <algorithm>
#include <cstdlib>
#include <cmath>
#include <memory>
#include <mutex>
#include <vector>

#include "sat_chain.hpp"
#include "sat_host.hpp"

namespace pila {

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// values of a chain's global residual: its tiled layout (tiles of 4 angles x
// 8 bins) pads the angles to a multiple of 4 and the bins to a multiple of 8
size_t residual_values(const pila_geom* g)
{
    return (size_t)((g->n_angles + 3) / 4) * 4 * (size_t)((g->n_bins + 7) / 8) * 8;
}

size_t chain_bytes(const pila_geom* g, const sat_params* p)
{
    const size_t G = (size_t)g->n_angles * g->n_bins;
    const size_t T = (G + 63) / 64;
    const size_t rs = p->precision == PILA_F32 ? 4 : 8;
    return align256(rs * residual_values(g)) + 2 * align256(8 * T) + align256(sizeof(ChainCarry)) +
           align256(sizeof(sat_stats));
}

int32_t check_params(const pila_geom* g, const pila_csr* c, const sat_params* p)
{
    PILA_TRY(check_geom(g));
    if (!c || !p) return fail(PILA_EINVAL, "csr or params is NULL");
    if (!c->row_ptr || !c->col || !c->len || !c->t_row_ptr || !c->t_col || !c->t_len || !c->support)
        return fail(PILA_EINVAL, "PILA arrays (pixel-major, ray-major and support) are required");
    if (c->n_support < 1) return fail(PILA_EINVAL, "empty support");
    if (c->nnz > 0 && (c->max_row < 1 || c->max_row > 2 * g->n_angles))
        return fail(PILA_EINVAL, "max_row %d is not the longest row from pila_build", c->max_row);
    if (p->m_cand < 1 || p->m_cand > kMaxCand) return fail(PILA_EINVAL, "m_cand must be in 1..64");
    if (p->n_steps < 0 || p->n_stages < 1) return fail(PILA_EINVAL, "bad n_steps / n_stages");
    if (p->precision != PILA_F64 && p->precision != PILA_F32)
        return fail(PILA_EINVAL, "precision must be PILA_F64 or PILA_F32");
    if (g->len_dtype != PILA_U8 && p->precision != g->len_dtype)
        return fail(PILA_EINVAL, "the residual precision must match the PILA length type (or the lengths be one byte)");
    if (!(p->T0 > 0.0) && (p->q_auto < 1 || !(p->tn_ratio > 0.0)))
        return fail(PILA_EINVAL, "automatic T0 needs q_auto >= 1 and tn_ratio > 0");
    if (p->T0 > 0.0 && !(p->TN > 0.0 && std::isfinite(p->T0) && std::isfinite(p->TN)))
        return fail(PILA_EINVAL, "T0 and TN must be positive and finite");
    if (!(p->delta_max >= 0.0) || !std::isfinite(p->delta_max) || !(p->f_max >= p->f_min))
        return fail(PILA_EINVAL, "bad delta_max / value range");
    if (p->resync_every < 0) return fail(PILA_EINVAL, "resync_every < 0");
    if (p->schedule != PILA_SCHED_LINEAR && p->schedule != PILA_SCHED_EXP && p->schedule != PILA_SCHED_CUBIC)
        return fail(PILA_EINVAL, "schedule must be PILA_SCHED_LINEAR, _EXP or _CUBIC");
    if (p->proposal != PILA_PROP_CLAMP && p->proposal != PILA_PROP_REDRAW)
        return fail(PILA_EINVAL, "proposal must be PILA_PROP_CLAMP or PILA_PROP_REDRAW");
    return PILA_OK;
}

ChainJob make_job(const pila_geom* g, const pila_csr* c, const double* sino, const sat_params* p,
                  double* image, char* ws)
{
    const size_t G = (size_t)g->n_angles * g->n_bins;
    const size_t rs = p->precision == PILA_F32 ? 4 : 8;
    ChainJob J;
    J.N = g->n;
    J.U = g->n_angles;
    J.K = g->n_bins;
    J.P = c->n_support;
    J.precision = p->precision;
    J.m_cand = p->m_cand;
    J.n_stages = p->n_stages;
    J.q_auto = p->q_auto;
    J.n_steps = p->n_steps;
    J.resync_every = p->precision == PILA_F32 ? p->resync_every : 0;
    J.seed = p->seed;
    J.chain_id = p->chain_id;
    J.T0 = p->T0 > 0.0 ? p->T0 : 0.0;
    J.TN = p->T0 > 0.0 ? p->TN : 0.0;
    J.tn_ratio = p->tn_ratio;
    J.delta_max = p->delta_max;
    J.f_min = p->f_min;
    J.f_max = p->f_max;
    J.ln09 = std::log(0.9);
    J.row_ptr = c->row_ptr;
    J.col = c->col;
    J.len = c->len;
    J.t_row_ptr = c->t_row_ptr;
    J.t_col = c->t_col;
    J.t_len = c->t_len;
    J.support = c->support;
    J.sino = sino;
    J.f = image;
    J.max_row = c->max_row;
    J.schedule = p->schedule;
    J.k_lo = c->k_lo;
    J.Kc = c->k_hi >= c->k_lo ? c->k_hi - c->k_lo + 1 : 0;
    J.UL = 0;
    J.proposal = p->proposal;
    // g / K for g < 2^24 as (g * m) >> (24 + L), L = ceil(log2 K), m = ceil(2^(24+L) / K):
    // the error g (m - 2^(24+L)/K) / 2^(24+L) stays below 2^-L <= 1/K; larger
    // geometries divide (kdiv_s = 0)
    J.kdiv_s = 0;
    J.kdiv_m = 0;
    if (G < ((size_t)1 << 24)) {
        uint32_t L = 0;
        while ((1u << L) < (uint32_t)J.K) ++L;
        const uint64_t den = (uint64_t)1 << (24 + L);
        J.kdiv_s = 24 + L;
        J.kdiv_m = (uint32_t)((den + (uint64_t)J.K - 1) / (uint64_t)J.K);
    }
    J.rkb = (J.K + 7) / 8;
    J.lenq = g->len_dtype == PILA_U8 ? 1 : 0;
    const size_t T = (G + 63) / 64;
    const size_t rb = align256(rs * residual_values(g));
    J.r = ws;
    J.tsum = (double*)(ws + rb);
    J.tdrift = (double*)(ws + rb + align256(8 * T));
    J.carry = (ChainCarry*)(ws + rb + 2 * align256(8 * T));
    J.stats = (sat_stats*)(ws + rb + 2 * align256(8 * T) + align256(sizeof(ChainCarry)));
    J.tr_m = nullptr;
    J.tr_acc = nullptr;
    J.tr_dc = nullptr;
    J.tcol = nullptr;
    J.cancel = nullptr;
    J.cancel_tag = 0;
    return J;
}

int device_props(hipDeviceProp_t* prop)
{
    int dev = 0;
    PILA_HIP(hipGetDevice(&dev));
    PILA_HIP(hipGetDeviceProperties(prop, dev));
    return PILA_OK;
}

bool piped_allowed(const pila_geom* g, const pila_csr* c)
{
    // ray index g = u K + k below 2^24 (the multiply-shift split), bins
    // below 8192 (the patch-table tag), and 32-bit byte offsets into the rows
    const int64_t G = (int64_t)g->n_angles * g->n_bins;
    const int64_t lb = len_bytes(g->len_dtype);
    return c->nnz >= 1 && c->max_row >= 1 && g->n_bins < 8192 && G < (1 << 24) &&
           c->nnz * lb <= ((int64_t)1 << 32);
}

// LDS of a pipelined chain whose residual is not wholly in LDS: the patch
// table, then as many angles of the residual (over the bins the support
// reaches) as fit in 'budget'.  Sets J->UL; returns the bytes to request.
int64_t hybrid_lds(ChainJob* J, int64_t budget)
{
    const int64_t rs = J->precision == PILA_F32 ? 4 : 8;
    const int64_t table = (16 * (int64_t)J->U + 2 * rs * J->U + 15) & ~(int64_t)15;
    J->UL = 0;
    if (table > budget) return table;
    if (J->Kc > 0) {
        const int64_t ul = (budget - table) / (J->Kc * rs);
        J->UL = (int32_t)std::min<int64_t>(ul, J->U);
    }
    return table + (int64_t)J->UL * J->Kc * rs;
}

bool long_allowed(const pila_geom* g, const pila_csr* c, const sat_params* p)
{
    return piped_allowed(g, c) && c->max_row <= kWave * (kLongE + kLongOver) &&
           p->m_cand <= kPipedThreads / kWave;
}

int64_t long_lds(ChainJob* J, int64_t budget)
{
    const int64_t rs = J->precision == PILA_F32 ? 4 : 8;
    J->UL = 0;
    if (J->Kc > 0 && budget > 0) J->UL = (int32_t)std::min<int64_t>(budget / (J->Kc * rs), J->U);
    return (int64_t)J->UL * J->Kc * rs;
}

int32_t set_lds(const void* k, int bytes)
{
    PILA_HIP(hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, bytes));
    return PILA_OK;
}

namespace {

// one chain, pipelined body (rows in registers); TK: slot words from job.tcol
template <typename Real, bool RLDS, int CPW, int E, bool TK = false, typename LenT = Real>
__global__ __launch_bounds__(kPipedThreads) void sat_piped_kernel(ChainJob job)
{
    extern __shared__ __align__(16) char lds[];
    __shared__ ChainShared sh;
    run_chain_piped<Real, RLDS, CPW, E, false, TK, LenT, true>(job, lds, sh, false);
}

// one segment of a chain whose FP64 resyncs run grid-wide between segments
template <int CPW, int E, bool TK = false, typename LenT = float>
__global__ __launch_bounds__(kPipedThreads) void sat_segment_kernel(ChainJob job)
{
    extern __shared__ __align__(16) char lds[];
    __shared__ ChainShared sh;
    if (job.carry->done || job.carry->status != PILA_OK) return;
    run_chain_piped<float, false, CPW, E, false, TK, LenT, true>(job, lds, sh, true);
}

// the slot word (ray_slot) of every PILA entry, for the TK kernels
__global__ __launch_bounds__(256) void tcol_kernel(ChainJob J, int64_t nnz, int32_t* __restrict__ tcol)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < nnz; q += stride)
        tcol[q] = ray_slot(J, J.col[q]);
}

// one chain, long-row body (64 E entries per row in registers, one estimate per wavefront)
template <typename Real, bool RLDS, int E, typename LenT = Real>
__global__ __launch_bounds__(kPipedThreads) void sat_long_kernel(ChainJob job)
{
    extern __shared__ __align__(16) char lds[];
    __shared__ ChainShared sh;
    run_chain_long<Real, RLDS, E, false, LenT, true>(job, lds, sh, false);
}

// one segment of a long-row chain whose FP64 resyncs run grid-wide between segments
template <int E, typename LenT = float>
__global__ __launch_bounds__(kPipedThreads) void sat_long_segment_kernel(ChainJob job)
{
    extern __shared__ __align__(16) char lds[];
    __shared__ ChainShared sh;
    if (job.carry->done || job.carry->status != PILA_OK) return;
    run_chain_long<float, false, E, false, LenT, true>(job, lds, sh, true);
}

// one segment of a general-body chain (FP32, residual in global memory)
// whose FP64 resyncs run grid-wide between segments
template <typename LenT = float>
__global__ __launch_bounds__(1024) void sat_simple_segment_kernel(ChainJob job)
{
    extern __shared__ __align__(16) char lds[];
    __shared__ ChainShared sh;
    if (job.carry->done || job.carry->status != PILA_OK) return;
    run_chain_simple<float, false, LenT>(job, lds, sh, true);
}

// one chain, general body
template <typename Real, typename LenT = Real>
__global__ __launch_bounds__(1024) void sat_simple_kernel(ChainJob job, int lds_bytes)
{
    extern __shared__ __align__(16) char lds[];
    __shared__ ChainShared sh;
    run_chain_simple_dispatch<Real, LenT>(job, lds, lds_bytes, sh);
}

// at most 8 wavefronts per workgroup of a split chain (256 registers per lane)
constexpr int kSplitThreads = 512;

// one segment of a chain split over gridDim.x workgroups; workgroup g > 0
// works on its own copies of the residual and the image
template <typename Real, typename LenT = Real>
__global__ __launch_bounds__(kSplitThreads) void sat_split_kernel(ChainJob job, SplitX X)
{
    __shared__ SplitShared sp;
    if (job.carry->done || job.carry->status != PILA_OK) return;
    const int g = blockIdx.x;
    if (g > 0) {
        char* base = X.copies + (int64_t)(g - 1) * (X.r_bytes + X.f_bytes);
        job.r = base;
        job.f = (double*)(base + X.r_bytes);
        job.tr_m = nullptr;
        job.tr_acc = nullptr;
        job.tr_dc = nullptr;
        job.stats = nullptr;
    }
    run_chain_split<Real, LenT>(job, X, g, sp);
}

// A split chain's copies: at the start (start = 1) the residual and the
// image, with the exchange words cleared; after a resync (start = 0, only
// when the segment asked for one) the residual.
__global__ __launch_bounds__(256) void sat_split_copy_kernel(ChainJob job, SplitX X, int64_t n_image, int start)
{
    if (!start && !job.carry->resync_due) return;
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nt = (int64_t)gridDim.x * blockDim.x;
    if (start && tid < 2 * kMaxCand * 2) X.word[tid] = 0;
    const int64_t nr = X.r_bytes / 16;
    const uint4* rs = (const uint4*)job.r;
    for (int k = 1; k < X.groups; ++k) {
        char* base = X.copies + (int64_t)(k - 1) * (X.r_bytes + X.f_bytes);
        uint4* rd = (uint4*)base;
        for (int64_t i = tid; i < nr; i += nt) rd[i] = rs[i];
        if (start) {
            double* fd = (double*)(base + X.r_bytes);
            for (int64_t i = tid; i < n_image; i += nt) fd[i] = job.f[i];
        }
    }
}

// Grid-wide FP64 rebuild of a chain's residual, one wavefront per 64-ray
// tile.  measure: a resync (runs only when the segment asked for one).
template <typename Real, typename LenT = Real>
__global__ __launch_bounds__(256) void sat_rebuild_kernel(ChainJob job, int measure)
{
    if (measure && !job.carry->resync_due) return;
    const int lane = threadIdx.x & 63;
    const int G = job.U * job.K, T = (G + kWave - 1) / kWave;
    const int waves = gridDim.x * (blockDim.x >> 6);
    for (int t = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); t < T; t += waves)
        rebuild_tile<Real, true, LenT>(job, (Real*)job.r, G, t, measure != 0, lane);
}

// After the initial rebuild: sum of squares and Eq. 8, then the carry.
template <typename Real, typename LenT = Real>
__global__ __launch_bounds__(512) void sat_setup_kernel(ChainJob job)
{
    __shared__ ChainShared sh;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, NW = blockDim.x >> 6;
    const int G = job.U * job.K;
    if (wave == 0) {
        double s, d;
        tile_totals(job, G, false, lane, &s, &d);
        if (lane == 0) sh.scalar[0] = s;
    }
    __syncthreads();
    const double sse = uniform_f64(sh.scalar[0]);
    __syncthreads();
    double T0 = job.T0, TN = job.TN;
    int32_t status = PILA_OK;
    if (!(T0 > 0.0))
        auto_temperature<Real, true, LenT>(job, (const Real*)job.r, sse, sh, lane, wave, NW, &T0, &TN, &status);
    if (threadIdx.x == 0) {
        ChainCarry& c = *job.carry;
        c.s_next = 0;
        c.accepts = c.accepts_nz = c.since = 0;
        c.resyncs = 0;
        c.status = status;
        c.resync_due = 0;
        c.done = (status != PILA_OK || job.n_steps == 0) ? 1 : 0;
        c.sse = sse;
        c.T0 = T0;
        c.TN = TN;
        c.drift_r = c.drift_sse = 0.0;
    }
}

// After a grid-wide resync: new sum of squares and the drift figures.
__global__ __launch_bounds__(64) void sat_resync_finish_kernel(ChainJob job)
{
    ChainCarry& c = *job.carry;
    if (!c.resync_due) return;
    double sse64, drift;
    tile_totals(job, job.U * job.K, true, threadIdx.x, &sse64, &drift);
    if (threadIdx.x == 0) {
        c.drift_r = fmax(c.drift_r, drift);
        const double ds = sse64 > 0.0 ? fabs(c.sse - sse64) / sse64 : fabs(c.sse - sse64);
        c.drift_sse = fmax(c.drift_sse, ds);
        c.sse = sse64;
        c.since = 0;
        c.resyncs += 1;
        c.resync_due = 0;
    }
}

__global__ void sat_final_kernel(ChainJob job)
{
    const ChainCarry& c = *job.carry;
    const double KU = (double)job.K * (double)job.U;
    sat_stats st;
    st.steps = c.status == PILA_OK ? job.n_steps : 0;
    st.accepts = c.accepts;
    st.accepts_nonzero = c.accepts_nz;
    st.resyncs = c.resyncs;
    st.status = c.status;
    st.T0_used = c.T0;
    st.TN_used = c.TN;
    st.sse_final = c.sse;
    st.cost_final = sqrt(fmax(c.sse, 0.0) / KU);
    st.max_drift_r = c.drift_r;
    st.max_drift_sse = c.drift_sse;
    st.chain_launches = 0;
    st.body = 0;
    st.chain_kernel_ms = 0.0;
    st.t_begin = st.t_end = 0;
    *job.stats = st;
}

// Persistent batch: each workgroup takes chains from a ticket counter until
// the tickets run out, so every workgroup reaches the exit.  The pipelined
// kernel runs chains whose rows and estimates fit its (CPW, E) shape; FP32
// chains read the slot words of their PILA's entries (computed once per PILA
// and batch), FP64 chains form them per entry.  The long-row and general
// kernels run the others.  All give the result the chain would give alone.
// Thread 0 stamps the device wall clock when the chain is taken and when it
// is done into the chain's statistics.
__device__ __forceinline__ void stamp_chain(const ChainJob& J, int64_t t0)
{
    if (threadIdx.x == 0 && J.stats) {
        J.stats->t_begin = t0;
        J.stats->t_end = (int64_t)wall_clock64();
    }
}

template <typename Real, int CPW, int E, typename LenT = Real>
__global__ __launch_bounds__(kPipedThreads) void sat_batch_kernel(
    const ChainJob* __restrict__ jobs, const int* __restrict__ order, int n_jobs,
    int* __restrict__ ticket, int lds_bytes)
{
    extern __shared__ __align__(16) char lds[];
    __shared__ ChainShared sh;
    (void)lds_bytes;
    for (;;) {
        if (threadIdx.x == 0) sh.ticket = atomicAdd(ticket, 1);
        __syncthreads();
        const int j = sh.ticket;
        __syncthreads();
        if (j >= n_jobs) break;
        const int64_t t0 = (int64_t)wall_clock64();
        // the descriptor stays in memory, read by scalar loads where a field
        // is used (a copy in registers holds every field live: spills)
        const ChainJob& J = jobs[__builtin_amdgcn_readfirstlane(order[j])];
        run_chain_piped<Real, false, CPW, E, false, sizeof(Real) == 4, LenT>(J, lds, sh, false);
        stamp_chain(J, t0);
    }
}

// Persistent batch of long-row chains (one estimate per wavefront)
template <typename Real, int E, typename LenT = Real>
__global__ __launch_bounds__(kPipedThreads) void sat_batch_long_kernel(
    const ChainJob* __restrict__ jobs, const int* __restrict__ order, int n_jobs,
    int* __restrict__ ticket, int lds_bytes)
{
    extern __shared__ __align__(16) char lds[];
    __shared__ ChainShared sh;
    (void)lds_bytes;
    for (;;) {
        if (threadIdx.x == 0) sh.ticket = atomicAdd(ticket, 1);
        __syncthreads();
        const int j = sh.ticket;
        __syncthreads();
        if (j >= n_jobs) break;
        const int64_t t0 = (int64_t)wall_clock64();
        const ChainJob J = uniform_job(jobs[order[j]]);  // fields in scalar registers
        run_chain_long<Real, false, E, false, LenT>(J, lds, sh, false);
        stamp_chain(J, t0);
    }
}

// Persistent batch for the general body (any row length, M or proposal
// rule), one kernel per residual precision and length type
template <typename Real, typename LenT = Real>
__global__ __launch_bounds__(1024) void sat_batch_simple_kernel(const ChainJob* __restrict__ jobs,
                                                                const int* __restrict__ order,
                                                                int n_jobs, int* __restrict__ ticket,
                                                                int lds_bytes)
{
    extern __shared__ __align__(16) char lds[];
    __shared__ ChainShared sh;
    for (;;) {
        if (threadIdx.x == 0) sh.ticket = atomicAdd(ticket, 1);
        __syncthreads();
        const int j = sh.ticket;
        __syncthreads();
        if (j >= n_jobs) break;
        const int64_t t0 = (int64_t)wall_clock64();
        const ChainJob J = uniform_job(jobs[order[j]]);  // fields in scalar registers
        run_chain_simple_dispatch<Real, LenT>(J, lds, lds_bytes, sh);
        stamp_chain(J, t0);
    }
}

__global__ void zero_ints_kernel(int* p, int n)
{
    for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0;
}

// ---------------------------------------------------------------------------
// launch tables
// ---------------------------------------------------------------------------
typedef void (*ChainKernel)(ChainJob);

struct PipedShape {
    int cpw, e;
    ChainKernel k_lds, k_glob, k_seg;
    ChainKernel k_glob_tk, k_seg_tk;  // FP32: the same with precomputed slot words
};

template <typename Real, int CPW, int E>
PipedShape piped_shape()
{
    ChainKernel seg = nullptr, glob_tk = nullptr, seg_tk = nullptr;
    if constexpr (sizeof(Real) == 4) {
        seg = sat_segment_kernel<CPW, E>;
        glob_tk = sat_piped_kernel<float, false, CPW, E, true>;
        seg_tk = sat_segment_kernel<CPW, E, true>;
    }
    return {CPW, E, sat_piped_kernel<Real, true, CPW, E>, sat_piped_kernel<Real, false, CPW, E>, seg, glob_tk,
            seg_tk};
}

// one-byte lengths (FP32 only): the LDS-residual kernel and the global ones
// with precomputed slot words
template <int CPW, int E>
PipedShape piped_shape_q()
{
    return {CPW,
            E,
            sat_piped_kernel<float, true, CPW, E, false, LenQ>,
            nullptr,
            nullptr,
            sat_piped_kernel<float, false, CPW, E, true, LenQ>,
            sat_segment_kernel<CPW, E, true, LenQ>};
}

const std::vector<PipedShape>& piped_shapes(int precision, bool lenq)
{
    static const std::vector<PipedShape> f64 = {
        piped_shape<double, 1, 2>(), piped_shape<double, 1, 4>(), piped_shape<double, 2, 4>(),
        piped_shape<double, 2, 8>(), piped_shape<double, 4, 8>()};
    static const std::vector<PipedShape> f32 = {
        piped_shape<float, 1, 4>(), piped_shape<float, 1, 8>(), piped_shape<float, 2, 8>(),
        piped_shape<float, 4, 8>()};
    static const std::vector<PipedShape> q32 = {piped_shape_q<1, 4>(), piped_shape_q<1, 8>(),
                                                piped_shape_q<2, 8>()};
    static const std::vector<PipedShape> none;
    if (lenq) return precision == PILA_F32 ? q32 : none;
    return precision == PILA_F64 ? f64 : f32;
}

// Pick the pipelined shape for one chain: the fewest estimates per
// wavefront (most lanes per row) whose registers hold the longest row and
// whose wavefront count fits the kernel.  Returns nullptr when none fits.
const PipedShape* choose_piped(int precision, bool lenq, int m_cand, int max_row, int* waves)
{
    for (int cpw : {1, 2, 4}) {
        const int nw = (m_cand + cpw - 1) / cpw;
        if (nw * kWave > kPipedThreads) continue;
        for (const PipedShape& ps : piped_shapes(precision, lenq)) {
            if (ps.cpw != cpw || max_row > (kWave / cpw) * ps.e) continue;
            *waves = nw;
            return &ps;
        }
    }
    return nullptr;
}

typedef void (*BatchKernel)(const ChainJob*, const int*, int, int*, int);

struct BatchShape {
    int cpw, e;
    BatchKernel k;
};

// the pipelined shapes of the batch kernels, per precision (FP64 rows hold
// at most 256 entries in registers; longer FP64 rows take the long-row body)
const std::vector<BatchShape>& batch_shapes(int precision, bool lenq)
{
    static const std::vector<BatchShape> f32 = {
        {1, 4, sat_batch_kernel<float, 1, 4>}, {1, 8, sat_batch_kernel<float, 1, 8>},
        {2, 8, sat_batch_kernel<float, 2, 8>}, {4, 8, sat_batch_kernel<float, 4, 8>}};
    static const std::vector<BatchShape> f64 = {{1, 4, sat_batch_kernel<double, 1, 4>},
                                                {2, 8, sat_batch_kernel<double, 2, 8>}};
    static const std::vector<BatchShape> q32 = {{1, 4, sat_batch_kernel<float, 1, 4, LenQ>},
                                                {1, 8, sat_batch_kernel<float, 1, 8, LenQ>},
                                                {2, 8, sat_batch_kernel<float, 2, 8, LenQ>}};
    static const std::vector<BatchShape> none;
    if (lenq) return precision == PILA_F32 ? q32 : none;
    return precision == PILA_F64 ? f64 : f32;
}

// HIP events around each chain-kernel launch of one sat_run, summed after
// the final synchronisation; inactive when no statistics are requested
struct LaunchTimer {
    bool on = false;
    std::vector<hipEvent_t> ev;
    ~LaunchTimer()
    {
        for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    }
    int32_t mark(hipStream_t st)
    {
        if (!on) return PILA_OK;
        hipEvent_t e;
        PILA_HIP(hipEventCreate(&e));
        ev.push_back(e);
        PILA_HIP(hipEventRecord(e, st));
        return PILA_OK;
    }
    int32_t total_ms(double* ms) const
    {
        double t = 0.0;
        for (size_t i = 0; i + 1 < ev.size(); i += 2) {
            float x = 0.0f;
            PILA_HIP(hipEventElapsedTime(&x, ev[i], ev[i + 1]));
            t += x;
        }
        *ms = t;
        return PILA_OK;
    }
};

// A chain split over several workgroups (run_chain_split) when its residual
// lives in global memory and a step scores at least kSplitMinEntries row
// entries (M times the mean row): below that one compute unit's gathers
// take less time than the exchange of the sums.  Four estimates per
// workgroup (M / 4 workgroups, 2 to kSplitGroups) measured best at 1024^2 x
// 720 for M = 16, 32 and 64 (two per workgroup: more exchange per step,
// eight: more gathers per compute unit).
constexpr int kSplitGroups = 16;
constexpr int kSplitMinM = 4;
// how long (ms) a workgroup of a split chain waits for the others' sums
constexpr int64_t kSplitWaitMs = 10000;
constexpr int64_t kSplitMinEntries = 12288;
constexpr size_t kSplitWordBytes = 2 * kMaxCand * 2 * sizeof(unsigned long long);

bool split_wanted(const pila_csr* c, const sat_params* p)
{
    return p->m_cand >= kSplitMinM && c->n_support > 0 &&
           (int64_t)p->m_cand * (c->nnz / c->n_support) >= kSplitMinEntries;
}

int split_groups(int m_cand)
{
    return std::max(2, std::min(kSplitGroups, m_cand / 4));
}

// the exchange words, then per workgroup after the first a residual copy
// and an image copy
size_t split_bytes(const pila_geom* g, const sat_params* p)
{
    const size_t rs = p->precision == PILA_F32 ? 4 : 8;
    return align256(kSplitWordBytes) + (size_t)(kSplitGroups - 1) * (align256(rs * residual_values(g)) +
                                                                     align256(8 * (size_t)g->n * g->n));
}

// the launches of a split chain: initial rebuild, Eq. 8 and the copies, then
// one segment per resync (rebuilt grid-wide on group 0's residual and copied
// to the others), then the statistics
template <typename Real, typename LenT>
int32_t enqueue_split(ChainJob& J, SplitX& X, int nw, int64_t n_image, int64_t n_seg, bool resync, unsigned rb,
                      hipStream_t st, LaunchTimer* tm)
{
    const unsigned cb = (unsigned)std::max<int64_t>(1, std::min<int64_t>((X.r_bytes / 16 + 255) / 256, 2048));
    sat_rebuild_kernel<Real, LenT><<<rb, 256, 0, st>>>(J, 0);
    sat_setup_kernel<Real, LenT><<<1, kPipedThreads, 0, st>>>(J);
    sat_split_copy_kernel<<<cb, 256, 0, st>>>(J, X, n_image, 1);
    for (int64_t k = 0; k < n_seg; ++k) {
        void* args[] = {&J, (void*)&X};
        PILA_TRY(tm->mark(st));
        PILA_HIP(hipLaunchKernel((const void*)sat_split_kernel<Real, LenT>, dim3(X.groups), dim3(nw * kWave), args,
                                 0, st));
        PILA_TRY(tm->mark(st));
        if (resync) {
            sat_rebuild_kernel<Real, LenT><<<rb, 256, 0, st>>>(J, 1);
            sat_split_copy_kernel<<<cb, 256, 0, st>>>(J, X, n_image, 0);
            sat_resync_finish_kernel<<<1, 64, 0, st>>>(J);
        }
    }
    sat_final_kernel<<<1, 1, 0, st>>>(J);
    PILA_HIP(hipGetLastError());
    return PILA_OK;
}

int32_t launch1(ChainKernel k, ChainJob* J, int threads, int lds, hipStream_t st, LaunchTimer* tm)
{
    PILA_TRY(set_lds((const void*)k, lds));
    void* args[] = {J};
    PILA_TRY(tm->mark(st));
    PILA_HIP(hipLaunchKernel((const void*)k, dim3(1), dim3(threads), args, (size_t)lds, st));
    PILA_TRY(tm->mark(st));
    return PILA_OK;
}

}  // namespace

}  // namespace pila

using namespace pila;

// Room for the slot words of every PILA entry (one int32 each) that the
// pipelined FP32 body takes precomputed (without them its 8-entry shapes run
// out of registers); offered for geometries of at most 512 angles (rows of
// at most 512 entries, the pipelined body's limit, need U <= 512), sized by
// the bound of two rays per support pixel and angle.
size_t tcol_bytes(const pila_geom* g, const sat_params* p)
{
    if (p->precision != PILA_F32 || g->n_angles > 512) return 0;
    int64_t sup = (int64_t)g->n * g->n;
    if (g->mask) {
        sup = 0;
        for (int64_t i = 0; i < (int64_t)g->n * g->n; ++i) sup += g->mask[i] != 0;
    }
    return align256((size_t)sup * 2 * (size_t)g->n_angles * sizeof(int32_t));
}

int32_t pila::launch_tcol(const ChainJob& J, int64_t nnz, int32_t* dst, hipStream_t st)
{
    if (nnz > 0) tcol_kernel<<<(unsigned)std::min<int64_t>((nnz + 255) / 256, 8192), 256, 0, st>>>(J, nnz, dst);
    PILA_HIP(hipGetLastError());
    return PILA_OK;
}

extern "C" int32_t sat_workspace_size(const pila_geom* geom, const sat_params* params, size_t* bytes)
{
    clear_error();
    PILA_TRY(check_geom(geom));
    if (!params || !bytes) return fail(PILA_EINVAL, "params or bytes is NULL");
    // room for a split chain's copies wherever the residual may not fit in
    // LDS (it always does below 64 KB)
    const size_t rv = (size_t)geom->n_angles * geom->n_bins * (params->precision == PILA_F32 ? 4 : 8);
    const size_t sb = params->m_cand >= kSplitMinM && rv > 65536 ? split_bytes(geom, params) : 0;
    *bytes = chain_bytes(geom, params) + std::max(tcol_bytes(geom, params), sb);
    return PILA_OK;
}

extern "C" int32_t sat_workspace_min(const pila_geom* geom, const sat_params* params, size_t* bytes)
{
    clear_error();
    PILA_TRY(check_geom(geom));
    if (!params || !bytes) return fail(PILA_EINVAL, "params or bytes is NULL");
    *bytes = chain_bytes(geom, params);
    return PILA_OK;
}

// One chain on the workspace d_ws (ws_bytes, at least chain_bytes; the
// slot words go after the chain state when there is room).  timed: HIP
// events around each chain-kernel launch (they are created per call).
static int32_t sat_run_impl(const pila_geom* geom, const pila_csr* csr, const double* d_sino,
                            const sat_params* params, double* d_image, void* d_ws, size_t ws_bytes,
                            sat_stats* h_stats, const sat_trace* trace, void* stream, bool timed,
                            int* body_out = nullptr)
{
    PILA_TRY(check_params(geom, csr, params));
    if (!d_sino || !d_image) return fail(PILA_EINVAL, "sinogram or image is NULL");
    const size_t need = chain_bytes(geom, params);
    if (!d_ws || ws_bytes < need)
        return fail(PILA_ENOMEM, "workspace of %zu bytes is below the %zu needed", ws_bytes, need);
    hipStream_t st = (hipStream_t)stream;
    ChainJob J = make_job(geom, csr, d_sino, params, d_image, (char*)d_ws);
    LaunchTimer tm;
    tm.on = h_stats != nullptr && timed;
    if (trace) {
        J.tr_m = trace->m_star;
        J.tr_acc = trace->accept;
        J.tr_dc = trace->dC;
    }
    hipDeviceProp_t prop;
    PILA_TRY(device_props(&prop));
    const int64_t G = (int64_t)geom->n_angles * geom->n_bins;
    const int rs = params->precision == PILA_F32 ? 4 : 8;
    const int64_t budget = (int64_t)prop.sharedMemPerBlock - (int64_t)sizeof(ChainShared) - 1024;
    const bool r_in_lds = G * rs <= budget;
    const int table_lds = (int)hybrid_lds(&J, budget);
    int waves = 0;
    // redrawn proposals depend on the image value at the step: general body only
    const bool ahead = params->proposal == PILA_PROP_CLAMP;
    const bool lenq = J.lenq != 0;
    const PipedShape* ps = ahead && piped_allowed(geom, csr)
                               ? choose_piped(params->precision, lenq, params->m_cand, csr->max_row, &waves)
                               : nullptr;
    const bool resync = params->precision == PILA_F32 && params->resync_every > 0;
    // the pipelined body in global mode takes the entries' slot words
    // precomputed when the workspace has room for them (one-byte lengths:
    // only then)
    const size_t tcb = align256((size_t)csr->nnz * sizeof(int32_t));
    const bool tk = ps && !r_in_lds && table_lds <= budget && ps->k_glob_tk && tcol_bytes(geom, params) > 0 &&
                    ws_bytes >= need + tcb;
    if (ps && !r_in_lds && !tk && !ps->k_glob) ps = nullptr;
    // the global mode's slot words hold the angle in 9 bits
    if (ps && !r_in_lds && geom->n_angles > kSlotMaxAngles) ps = nullptr;
    // rows too long for the pipelined body's registers: the long-row body
    // (one-byte lengths: FP32 only)
    const bool lng = ahead && !ps && long_allowed(geom, csr, params) && !(lenq && params->precision == PILA_F64);
    const bool piped_seg = ps && !r_in_lds && table_lds <= budget && resync && (tk ? ps->k_seg_tk : ps->k_seg);
    if (tk) {
        J.tcol = (const int32_t*)((char*)d_ws + need);
        if (csr->nnz > 0)
            tcol_kernel<<<(unsigned)std::min<int64_t>((csr->nnz + 255) / 256, 8192), 256, 0, st>>>(
                J, csr->nnz, (int32_t*)((char*)d_ws + need));
    }
    const bool long_seg = lng && !r_in_lds && resync;
    // long rows and many estimates with the residual in global memory: the
    // chain split over several workgroups, when the workspace has room for
    // their copies after the chain state
    const bool split = !ps && !lng && !r_in_lds && split_wanted(csr, params) &&
                       !(lenq && params->precision == PILA_F64) && ws_bytes >= need + split_bytes(geom, params) &&
                       ((uintptr_t)d_ws & 255) == 0;
    const bool simple_seg = !ps && !lng && !r_in_lds && resync && !split;
    const int glob = r_in_lds ? 0 : PILA_BODY_GLOBAL_R;
    int body = 0;
    if (split) {
        const int M = params->m_cand;
        const int ng = split_groups(M);
        const int nw = std::min(kSplitThreads / kWave, (M + ng - 1) / ng);
        SplitX X;
        X.word = (unsigned long long*)((char*)d_ws + need);
        X.copies = (char*)d_ws + need + align256(kSplitWordBytes);
        X.r_bytes = (int64_t)align256((size_t)rs * residual_values(geom));
        X.f_bytes = (int64_t)align256(8 * (size_t)geom->n * geom->n);
        X.groups = ng;
        X.pad = 0;
        int khz = 0;
        int dev = 0;
        PILA_HIP(hipGetDevice(&dev));
        PILA_HIP(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
        // PILA_SPLIT_WAIT_MS (environment) shortens or lengthens the wait
        int64_t wait_ms = kSplitWaitMs;
        if (const char* e = std::getenv("PILA_SPLIT_WAIT_MS")) wait_ms = std::max<int64_t>(0, std::atoll(e));
        X.wait_ticks = (int64_t)(khz > 0 ? khz : 100000) * wait_ms;
        body = PILA_BODY_SPLIT | PILA_BODY_GLOBAL_R | PILA_BODY_SEGMENTED | (ng << 8);
        const int T = (int)((G + 63) / 64);
        const unsigned rb = (unsigned)std::min<int64_t>((T + 3) / 4, 4096);
        const int64_t n_seg = resync ? params->n_steps / params->resync_every + 1 : 1;
        const int64_t n_image = (int64_t)geom->n * geom->n;
        const int32_t rc = params->precision == PILA_F64
                               ? enqueue_split<double, double>(J, X, nw, n_image, n_seg, false, rb, st, &tm)
                           : lenq ? enqueue_split<float, LenQ>(J, X, nw, n_image, n_seg, resync, rb, st, &tm)
                                  : enqueue_split<float, float>(J, X, nw, n_image, n_seg, resync, rb, st, &tm);
        PILA_TRY(rc);
    } else if (piped_seg || long_seg || simple_seg) {
        body = (piped_seg ? PILA_BODY_PIPED | (ps->cpw << 8) | (ps->e << 16)
                          : long_seg ? PILA_BODY_LONG : PILA_BODY_GENERAL) |
               PILA_BODY_GLOBAL_R | PILA_BODY_SEGMENTED;
        // FP32 residual in global memory: chain segments end at each resync,
        // which runs grid-wide; the host only enqueues, it never waits
        const int T = (int)((G + 63) / 64);
        const unsigned rb = (unsigned)std::min<int64_t>((T + 3) / 4, 4096);
        const int long_bytes = long_seg ? (int)long_lds(&J, budget) : 0;
        if (lenq) {
            sat_rebuild_kernel<float, LenQ><<<rb, 256, 0, st>>>(J, 0);
            sat_setup_kernel<float, LenQ><<<1, kPipedThreads, 0, st>>>(J);
        } else {
            sat_rebuild_kernel<float><<<rb, 256, 0, st>>>(J, 0);
            sat_setup_kernel<float><<<1, kPipedThreads, 0, st>>>(J);
        }
        const int64_t n_seg = params->n_steps / params->resync_every + 1;
        const int sw = params->m_cand < kMaxWaves ? params->m_cand : kMaxWaves;
        for (int64_t k = 0; k < n_seg; ++k) {
            if (piped_seg) {
                PILA_TRY(launch1(tk ? ps->k_seg_tk : ps->k_seg, &J, waves * kWave, table_lds, st, &tm));
            } else if (long_seg) {
                PILA_TRY(launch1(lenq ? sat_long_segment_kernel<kLongE, LenQ> : sat_long_segment_kernel<kLongE>,
                                 &J, params->m_cand * kWave, long_bytes, st, &tm));
            } else {
                PILA_TRY(tm.mark(st));
                if (lenq)
                    sat_simple_segment_kernel<LenQ><<<1, sw * kWave, 0, st>>>(J);
                else
                    sat_simple_segment_kernel<float><<<1, sw * kWave, 0, st>>>(J);
                PILA_TRY(tm.mark(st));
            }
            if (lenq)
                sat_rebuild_kernel<float, LenQ><<<rb, 256, 0, st>>>(J, 1);
            else
                sat_rebuild_kernel<float><<<rb, 256, 0, st>>>(J, 1);
            sat_resync_finish_kernel<<<1, 64, 0, st>>>(J);
        }
        sat_final_kernel<<<1, 1, 0, st>>>(J);
    } else if (ps && (r_in_lds || table_lds <= budget)) {
        body = PILA_BODY_PIPED | glob | (ps->cpw << 8) | (ps->e << 16);
        const int lds = r_in_lds ? (int)(G * rs) : table_lds;
        PILA_TRY(launch1(r_in_lds ? ps->k_lds : (tk ? ps->k_glob_tk : ps->k_glob), &J, waves * kWave, lds, st,
                         &tm));
    } else if (lng) {
        body = PILA_BODY_LONG | glob;
        const int lds = r_in_lds ? (int)(G * rs) : (int)long_lds(&J, budget);
        ChainKernel k;
        if (params->precision == PILA_F64)
            k = r_in_lds ? sat_long_kernel<double, true, kLongE> : sat_long_kernel<double, false, kLongE>;
        else if (lenq)
            k = r_in_lds ? sat_long_kernel<float, true, kLongE, LenQ> : sat_long_kernel<float, false, kLongE, LenQ>;
        else
            k = r_in_lds ? sat_long_kernel<float, true, kLongE> : sat_long_kernel<float, false, kLongE>;
        PILA_TRY(launch1(k, &J, params->m_cand * kWave, lds, st, &tm));
    } else {
        body = PILA_BODY_GENERAL | glob;
        waves = params->m_cand < kMaxWaves ? params->m_cand : kMaxWaves;
        const int lds = r_in_lds ? (int)(G * rs) : 0;
        const void* k = params->precision == PILA_F64
                            ? (lenq ? (const void*)sat_simple_kernel<double, LenQ>
                                    : (const void*)sat_simple_kernel<double>)
                            : (lenq ? (const void*)sat_simple_kernel<float, LenQ>
                                    : (const void*)sat_simple_kernel<float>);
        PILA_TRY(set_lds(k, lds));
        PILA_TRY(tm.mark(st));
        void* args[] = {&J, (void*)&lds};
        PILA_HIP(hipLaunchKernel(k, dim3(1), dim3(waves * kWave), args, (size_t)lds, st));
        PILA_TRY(tm.mark(st));
    }
    PILA_HIP(hipGetLastError());
    if (body_out) *body_out = body;
    if (h_stats) {
        PILA_HIP(hipMemcpyAsync(h_stats, J.stats, sizeof(sat_stats), hipMemcpyDeviceToHost, st));
        PILA_HIP(hipStreamSynchronize(st));
        h_stats->chain_launches = (int32_t)(tm.ev.size() / 2);
        h_stats->body = body;
        PILA_TRY(tm.total_ms(&h_stats->chain_kernel_ms));
    }
    return PILA_OK;
}

extern "C" int32_t sat_run(const pila_geom* geom, const pila_csr* csr, const double* d_sino,
                           const sat_params* params, double* d_image, void* d_ws, size_t ws_bytes,
                           sat_stats* h_stats, const sat_trace* trace, void* stream)
{
    clear_error();
    return sat_run_impl(geom, csr, d_sino, params, d_image, d_ws, ws_bytes, h_stats, trace, stream, true);
}

// ---------------------------------------------------------------------------
// sat_run_static: sat_run on a workspace the library holds in a file-scope
// device array, for callers that cannot allocate.  In host code the array's
// name is only a stand-in for the symbol; its device address (one per GPU)
// comes from hipGetSymbolAddress, taken once per device with that device
// current, and only that address is passed to kernels.
// ---------------------------------------------------------------------------
static __device__ __align__(256) char scratch[PILA_STATIC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;

namespace {
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

int32_t scratch_address(void** out)
{
    int dev = 0;
    PILA_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(PILA_EINVAL, "device %d out of range", dev);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)", __FILE__, __LINE__);
        if (!ptr) return fail(PILA_EHIP, "hipGetSymbolAddress(scratch) gave a NULL address");
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return PILA_OK;
}
}  // namespace

extern "C" int32_t sat_run_static(const pila_geom* geom, const pila_csr* csr, const double* d_sino,
                                  const sat_params* params, double* d_image, sat_stats* h_stats,
                                  const sat_trace* trace, void* stream)
{
    clear_error();
    PILA_TRY(check_geom(geom));
    if (!params) return fail(PILA_EINVAL, "params is NULL");
    const size_t need = chain_bytes(geom, params);
    if (need > PILA_STATIC_SCRATCH_BYTES)
        return fail(PILA_ENOMEM,
                    "the chain needs %zu bytes of workspace, above the %zu of the library's static scratch "
                    "(use sat_run with a caller workspace)",
                    need, (size_t)PILA_STATIC_SCRATCH_BYTES);
    void* ws = nullptr;
    PILA_TRY(scratch_address(&ws));
    return sat_run_impl(geom, csr, d_sino, params, d_image, ws, PILA_STATIC_SCRATCH_BYTES, h_stats, trace,
                        stream, false);
}

// A batch runs its chains in groups, one persistent kernel per group: the
// pipelined body at each register shape its chains need, the long-row body
// and the general body.  The groups' kernels run side by side on forked
// streams, so no chain waits for another group's kernel to end.
constexpr int kMaxGroups = 8;
constexpr int kMaxAux = kMaxGroups - 1;

// Streams that the groups after the first run on, per device, created on
// first use at the default priority and kept until the process ends.
static int32_t aux_streams(int n, hipStream_t* out)
{
    static std::mutex mu;
    static hipStream_t streams[kMaxDevices][kMaxAux] = {};
    int dev = 0;
    PILA_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(PILA_EINVAL, "device %d out of range", dev);
    std::lock_guard<std::mutex> lk(mu);
    for (int i = 0; i < n; ++i) {
        if (!streams[dev][i]) PILA_HIP(hipStreamCreateWithFlags(&streams[dev][i], hipStreamNonBlocking));
        out[i] = streams[dev][i];
    }
    return PILA_OK;
}

// The PILAs of a batch whose FP32 chains may take the pipelined body (rows
// of at most 512 entries): each gets one slot word per entry, shared by the
// batch's chains on it (their LDS layouts are the same).
std::vector<const pila_csr*> batch_tcol_pilas(int32_t n_jobs, const sat_job* jobs)
{
    std::vector<const pila_csr*> v;
    for (int32_t j = 0; j < n_jobs; ++j) {
        const pila_csr* c = jobs[j].csr;
        if (!c || jobs[j].params.precision != PILA_F32 || c->max_row > 512 || c->nnz <= 0) continue;
        bool seen = false;
        for (const pila_csr* o : v) seen = seen || o->col == c->col;
        if (!seen) v.push_back(c);
    }
    return v;
}

extern "C" int32_t sat_batch_workspace_size(int32_t n_jobs, const sat_job* jobs, size_t* bytes)
{
    clear_error();
    if (n_jobs < 0 || (n_jobs > 0 && !jobs) || !bytes) return fail(PILA_EINVAL, "bad batch arguments");
    size_t total = align256(sizeof(ChainJob) * (size_t)(n_jobs > 0 ? n_jobs : 1)) +
                   align256(sizeof(int) * (kMaxGroups + (size_t)(n_jobs > 0 ? n_jobs : 1)));
    for (int32_t j = 0; j < n_jobs; ++j) {
        PILA_TRY(check_geom(jobs[j].geom));
        total += chain_bytes(jobs[j].geom, &jobs[j].params);
    }
    for (const pila_csr* c : batch_tcol_pilas(n_jobs, jobs)) total += align256(sizeof(int32_t) * (size_t)c->nnz);
    *bytes = total;
    return PILA_OK;
}

struct BatchGroup {
    int kind;                       // PILA_BODY_PIPED, _LONG or _GENERAL (+256: FP64)
    const BatchShape* shape;        // the pipelined register shape (kind PIPED)
    int waves;                      // wavefronts per chain
    std::vector<int> ids;           // its chains, longest first
    double longest = 0.0;           // estimated work of its longest chain
};

// What the host decides about a batch: chain descriptors, groups and their
// order, the slot words to compute, and where each lives in the workspace.
struct BatchPlan {
    int32_t n_jobs = 0;
    std::vector<ChainJob> host;
    std::vector<BatchGroup> groups;
    std::vector<int> order;
    struct Tcol {
        ChainJob J;
        int64_t nnz;
        int32_t* dst;
    };
    std::vector<Tcol> tcols;
    ChainJob* d_jobs = nullptr;
    int* d_ticket = nullptr;
    int* d_order = nullptr;
    int lds = 0, n_cu = 0, per_cu = 1;
};

static int32_t batch_plan(int32_t n_jobs, const sat_job* jobs, const sat_launch* launch, void* d_ws,
                          size_t ws_bytes, BatchPlan* bp)
{
    size_t need = 0;
    PILA_TRY(sat_batch_workspace_size(n_jobs, jobs, &need));
    if (!d_ws || ws_bytes < need)
        return fail(PILA_ENOMEM, "workspace of %zu bytes is below the %zu needed", ws_bytes, need);
    bp->n_jobs = n_jobs;
    if (n_jobs == 0) return PILA_OK;
    char* ws = (char*)d_ws;
    bp->d_jobs = (ChainJob*)ws;
    bp->d_ticket = (int*)(ws + align256(sizeof(ChainJob) * (size_t)n_jobs));
    bp->d_order = bp->d_ticket + kMaxGroups;
    char* cur = ws + align256(sizeof(ChainJob) * (size_t)n_jobs) + align256(sizeof(int) * (kMaxGroups + (size_t)n_jobs));
    std::vector<ChainJob>& host = bp->host;
    host.resize((size_t)n_jobs);
    for (int32_t j = 0; j < n_jobs; ++j) {
        const sat_job& jb = jobs[j];
        PILA_TRY(check_params(jb.geom, jb.csr, &jb.params));
        if (!jb.d_sino || !jb.d_image) return fail(PILA_EINVAL, "job %d: sinogram or image is NULL", j);
        host[j] = make_job(jb.geom, jb.csr, jb.d_sino, &jb.params, jb.d_image, cur);
        cur += chain_bytes(jb.geom, &jb.params);
    }
    int launch_waves = 4, per_cu = 2, use_lds = 1;
    if (launch) {
        launch_waves = launch->waves_per_chain;
        per_cu = launch->chains_per_cu;
        use_lds = launch->lds_residual;
    }
    auto waves_ok = [](int w) { return w == 1 || w == 2 || w == 4 || w == 8 || w == 16; };
    if (!waves_ok(launch_waves)) return fail(PILA_EINVAL, "waves_per_chain must be 1, 2, 4, 8 or 16");
    for (int32_t j = 0; j < n_jobs; ++j)
        if (jobs[j].waves_per_chain != 0 && !waves_ok(jobs[j].waves_per_chain))
            return fail(PILA_EINVAL, "job %d: waves_per_chain must be 0, 1, 2, 4, 8 or 16", j);
    if (per_cu < 1 || per_cu > 32) return fail(PILA_EINVAL, "chains_per_cu must be in 1..32");
    hipDeviceProp_t prop;
    PILA_TRY(device_props(&prop));
    int lds = 0;
    if (use_lds) {
        const int per_wg = (int)(prop.sharedMemPerBlock / (size_t)per_cu) - (int)sizeof(ChainShared) - 512;
        lds = per_wg > 0 ? (per_wg & ~255) : 0;
    }
    bp->lds = lds;
    bp->n_cu = prop.multiProcessorCount;
    bp->per_cu = per_cu;
    // estimated work of a chain: steps x estimates x mean row length
    auto work = [&](int j) {
        const double row = jobs[j].csr->n_support > 0
                               ? (double)jobs[j].csr->nnz / (double)jobs[j].csr->n_support
                               : 1.0;
        return (double)jobs[j].params.n_steps * (double)jobs[j].params.m_cand * (row + 8.0);
    };
    // each chain's body: the pipelined body at the smallest register shape
    // that holds its rows (the fewest estimates per wavefront first), else
    // the long-row body, else the general body
    std::vector<BatchGroup>& groups = bp->groups;
    auto group_of = [&](int kind, const BatchShape* shape, int w) -> BatchGroup& {
        for (BatchGroup& g : groups)
            if (g.kind == kind && g.shape == shape && g.waves == w) return g;
        groups.push_back(BatchGroup{kind, shape, w, {}, 0.0});
        return groups.back();
    };
    for (int32_t j = 0; j < n_jobs; ++j) {
        ChainJob& J = host[j];
        const int waves = jobs[j].waves_per_chain ? jobs[j].waves_per_chain : launch_waves;
        const bool ahead = J.proposal == PILA_PROP_CLAMP;
        const bool fits = ahead && waves * kWave <= kPipedThreads;
        const BatchShape* bs = nullptr;
        if (fits && piped_allowed(jobs[j].geom, jobs[j].csr) && jobs[j].geom->n_angles <= kSlotMaxAngles) {
            for (int cpw : {1, 2, 4}) {
                if (J.m_cand > waves * cpw) continue;
                for (const BatchShape& sp : batch_shapes(J.precision, J.lenq != 0))
                    if (sp.cpw == cpw && J.max_row <= (kWave / cpw) * sp.e) {
                        bs = &sp;
                        break;
                    }
                if (bs) break;
            }
            if (bs && hybrid_lds(&J, lds) > lds) bs = nullptr;  // LDS part of the residual
        }
        int kind = PILA_BODY_GENERAL;
        if (bs) {
            kind = PILA_BODY_PIPED;
        } else if (fits && J.m_cand <= waves && long_allowed(jobs[j].geom, jobs[j].csr, &jobs[j].params) &&
                   !(J.lenq && J.precision == PILA_F64)) {
            long_lds(&J, lds);
            kind = PILA_BODY_LONG;
        } else {
            J.UL = 0;
        }
        const int lq = kind != PILA_BODY_PIPED && J.lenq ? 512 : 0;  // (the piped shape says it)
        BatchGroup& g = group_of(kind | (J.precision == PILA_F64 ? 256 : 0) | lq, bs, waves);
        g.ids.push_back(j);
        g.longest = std::max(g.longest, work(j));
    }
    if ((int)groups.size() > kMaxGroups) return fail(PILA_EINVAL, "too many chain groups");
    // longest chains first within a group, so that no long chain starts late
    // behind short ones and sets the makespan (results do not depend on the
    // order); the group holding the batch's longest chain launches first
    for (BatchGroup& g : groups)
        std::stable_sort(g.ids.begin(), g.ids.end(), [&](int a, int b) { return work(a) > work(b); });
    std::stable_sort(groups.begin(), groups.end(),
                     [](const BatchGroup& a, const BatchGroup& b) { return a.longest > b.longest; });
    // slot words of the pipelined chains' PILAs (the pipelined kernels read them)
    const std::vector<const pila_csr*> tp = batch_tcol_pilas(n_jobs, jobs);
    std::vector<int32_t*> where(tp.size(), nullptr);
    for (const BatchGroup& g : groups) {
        if (g.kind != PILA_BODY_PIPED) continue;  // FP32 pipelined groups only
        for (int j : g.ids) {
            size_t i = 0;
            while (i < tp.size() && tp[i]->col != jobs[j].csr->col) ++i;
            if (i == tp.size()) return fail(PILA_EINVAL, "job %d: no slot-word room for its PILA", j);
            if (!where[i]) {
                where[i] = (int32_t*)cur;
                cur += align256(sizeof(int32_t) * (size_t)tp[i]->nnz);
                bp->tcols.push_back({host[j], tp[i]->nnz, where[i]});
            }
            host[j].tcol = where[i];
        }
    }
    for (const BatchGroup& g : groups) bp->order.insert(bp->order.end(), g.ids.begin(), g.ids.end());
    return PILA_OK;
}

// The device work of a planned batch on stream st (descriptors and order
// already in the workspace): ticket counters, slot words, then each group's
// persistent kernel on its own stream forked from st and joined back into
// it.  Capturable into a HIP graph (kernels and event dependencies only).
// t_ev (nullable, 2 per group): events recorded around each group's kernel.
static int32_t batch_enqueue(const BatchPlan& bp, hipStream_t st, hipEvent_t* t_ev)
{
    const std::vector<BatchGroup>& groups = bp.groups;
    zero_ints_kernel<<<1, 64, 0, st>>>(bp.d_ticket, kMaxGroups);
    PILA_HIP(hipGetLastError());
    for (const BatchPlan::Tcol& t : bp.tcols) PILA_TRY(launch_tcol(t.J, t.nnz, t.dst, st));
    // fork: every group after the first waits for the work above on its own stream
    const int n_aux = (int)groups.size() - 1;
    hipStream_t aux[kMaxAux] = {};
    hipEvent_t fork = nullptr, join[kMaxAux] = {};
    struct Events {
        hipEvent_t* f;
        hipEvent_t* j;
        int n;
        ~Events()
        {
            if (*f) (void)hipEventDestroy(*f);
            for (int i = 0; i < n; ++i)
                if (j[i]) (void)hipEventDestroy(j[i]);
        }
    } cleanup{&fork, join, n_aux > 0 ? n_aux : 0};
    if (n_aux > 0) {
        PILA_TRY(aux_streams(n_aux, aux));
        PILA_HIP(hipEventCreateWithFlags(&fork, hipEventDisableTiming));
        PILA_HIP(hipEventRecord(fork, st));
        for (int i = 0; i < n_aux; ++i) {
            PILA_HIP(hipStreamWaitEvent(aux[i], fork, 0));
            PILA_HIP(hipEventCreateWithFlags(&join[i], hipEventDisableTiming));
        }
    }
    const ChainJob* jobs_arg = bp.d_jobs;
    int lds_arg = bp.lds;
    size_t first = 0;
    for (size_t gi = 0; gi < groups.size(); ++gi) {
        const BatchGroup& g = groups[gi];
        hipStream_t gs = gi == 0 ? st : aux[gi - 1];
        int n_arg = (int)g.ids.size();
        const int* order_arg = bp.d_order + first;
        int* ticket_arg = bp.d_ticket + gi;
        first += g.ids.size();
        void* args[] = {&jobs_arg, &order_arg, &n_arg, &ticket_arg, &lds_arg};
        const int grid = std::min(n_arg, bp.n_cu * bp.per_cu);
        const int kind = g.kind & 255;
        const bool f64 = (g.kind & 256) != 0;
        const bool lq = (g.kind & 512) != 0;
        const void* k = kind == PILA_BODY_PIPED ? (const void*)g.shape->k
                        : kind == PILA_BODY_LONG
                            ? (f64  ? (const void*)sat_batch_long_kernel<double, kLongE>
                               : lq ? (const void*)sat_batch_long_kernel<float, kLongE, LenQ>
                                    : (const void*)sat_batch_long_kernel<float, kLongE>)
                        : f64 ? (lq ? (const void*)sat_batch_simple_kernel<double, LenQ>
                                    : (const void*)sat_batch_simple_kernel<double>)
                              : (lq ? (const void*)sat_batch_simple_kernel<float, LenQ>
                                    : (const void*)sat_batch_simple_kernel<float>);
        PILA_TRY(set_lds(k, bp.lds));
        if (t_ev) PILA_HIP(hipEventRecord(t_ev[2 * gi], gs));
        PILA_HIP(hipLaunchKernel(k, dim3(grid), dim3(g.waves * kWave), args, (size_t)bp.lds, gs));
        if (t_ev) PILA_HIP(hipEventRecord(t_ev[2 * gi + 1], gs));
        if (gi > 0) PILA_HIP(hipEventRecord(join[gi - 1], gs));
    }
    for (int i = 0; i < n_aux; ++i) PILA_HIP(hipStreamWaitEvent(st, join[i], 0));
    PILA_HIP(hipGetLastError());
    return PILA_OK;
}

// the body code of each chain of a planned batch (PILA_BODY_* | shape | width)
static void batch_bodies(const BatchPlan& bp, std::vector<int32_t>* body)
{
    body->assign((size_t)bp.n_jobs, 0);
    for (const BatchGroup& g : bp.groups)
        for (int j : g.ids) {
            const ChainJob& J = bp.host[j];
            const int64_t rb = (int64_t)J.U * J.K * (J.precision == PILA_F32 ? 4 : 8);
            const int kind = g.kind & 255;
            const bool glob = kind != PILA_BODY_GENERAL || rb > bp.lds;
            (*body)[j] = kind | (glob ? PILA_BODY_GLOBAL_R : 0) |
                         (g.shape ? (g.shape->cpw << 8) | (g.shape->e << 16) : 0) | (g.waves << 24);
        }
}

extern "C" int32_t sat_run_batch(int32_t n_jobs, const sat_job* jobs, const sat_launch* launch,
                                 void* d_ws, size_t ws_bytes, sat_stats* h_stats, void* stream)
{
    clear_error();
    BatchPlan bp;
    PILA_TRY(batch_plan(n_jobs, jobs, launch, d_ws, ws_bytes, &bp));
    if (n_jobs == 0) return PILA_OK;
    hipStream_t st = (hipStream_t)stream;
    PILA_HIP(hipMemcpyAsync(bp.d_jobs, bp.host.data(), sizeof(ChainJob) * bp.host.size(), hipMemcpyHostToDevice,
                            st));
    PILA_HIP(hipMemcpyAsync(bp.d_order, bp.order.data(), sizeof(int) * bp.order.size(), hipMemcpyHostToDevice,
                            st));
    // HIP events around each group's kernel on its stream, when asked for
    const bool timed = launch && launch->max_groups > 0 && launch->h_group_ms;
    hipEvent_t t_ev[2 * kMaxGroups] = {};
    struct TimingEvents {
        hipEvent_t* e;
        ~TimingEvents()
        {
            for (int i = 0; i < 2 * kMaxGroups; ++i)
                if (e[i]) (void)hipEventDestroy(e[i]);
        }
    } t_cleanup{t_ev};
    if (timed)
        for (size_t i = 0; i < 2 * bp.groups.size(); ++i) PILA_HIP(hipEventCreate(&t_ev[i]));
    PILA_TRY(batch_enqueue(bp, st, timed ? t_ev : nullptr));
    if (h_stats) {
        for (int32_t j = 0; j < n_jobs; ++j)
            PILA_HIP(hipMemcpyAsync(&h_stats[j], bp.host[j].stats, sizeof(sat_stats), hipMemcpyDeviceToHost, st));
    }
    // the descriptor upload reads host memory owned by this call
    PILA_HIP(hipStreamSynchronize(st));
    if (h_stats) {
        std::vector<int32_t> body;
        batch_bodies(bp, &body);
        for (int32_t j = 0; j < n_jobs; ++j) h_stats[j].body = body[j];
    }
    if (launch && launch->max_groups > 0) {
        for (int i = 0; i < launch->max_groups; ++i) {
            const bool have = i < (int)bp.groups.size();
            const BatchGroup* g = have ? &bp.groups[i] : nullptr;
            if (launch->h_group_ms) {
                float ms = 0.0f;
                if (have && timed) PILA_HIP(hipEventElapsedTime(&ms, t_ev[2 * i], t_ev[2 * i + 1]));
                launch->h_group_ms[i] = ms;
            }
            if (launch->h_group_desc)
                launch->h_group_desc[i] =
                    have ? (g->kind & 255) | (g->shape ? (g->shape->cpw << 8) | (g->shape->e << 16) : 0) |
                               (g->waves << 24)
                         : 0;
            if (launch->h_group_chains) launch->h_group_chains[i] = have ? (int)g->ids.size() : 0;
        }
    }
    return PILA_OK;
}

// ---------------------------------------------------------------------------
// HIP graphs: a chain's or a batch's launches captured once and replayed
// ---------------------------------------------------------------------------
struct sat_graph_s {
    hipGraphExec_t exec = nullptr;
    std::vector<sat_stats*> stats;  // where each chain's statistics land in the workspace
    std::vector<int32_t> body;
};

// capture what enqueue() puts on a private stream into an instantiated graph
template <typename F>
static int32_t capture_graph(F enqueue, hipGraphExec_t* exec)
{
    hipStream_t cap = nullptr;
    PILA_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    struct StreamGuard {
        hipStream_t s;
        ~StreamGuard() { (void)hipStreamDestroy(s); }
    } guard{cap};
    PILA_HIP(hipStreamBeginCapture(cap, hipStreamCaptureModeRelaxed));
    const int32_t rc = enqueue(cap);
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(cap, &graph);
    if (rc != PILA_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture", __FILE__, __LINE__);
    const hipError_t ei = hipGraphInstantiate(exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ei != hipSuccess) return hip_fail(ei, "hipGraphInstantiate", __FILE__, __LINE__);
    return PILA_OK;
}

extern "C" int32_t sat_graph_create(const pila_geom* geom, const pila_csr* csr, const double* d_sino,
                                    const sat_params* params, double* d_image, void* d_ws, size_t ws_bytes,
                                    const sat_trace* trace, sat_graph** out)
{
    clear_error();
    if (!out) return fail(PILA_EINVAL, "out is NULL");
    *out = nullptr;
    PILA_TRY(check_params(geom, csr, params));
    auto g = std::make_unique<sat_graph_s>();
    int body = 0;
    PILA_TRY(capture_graph(
        [&](hipStream_t cap) {
            return sat_run_impl(geom, csr, d_sino, params, d_image, d_ws, ws_bytes, nullptr, trace, cap, false,
                                &body);
        },
        &g->exec));
    const ChainJob J = make_job(geom, csr, d_sino, params, d_image, (char*)d_ws);
    g->stats.push_back(J.stats);
    g->body.push_back(body);
    *out = g.release();
    return PILA_OK;
}

extern "C" int32_t sat_batch_graph_create(int32_t n_jobs, const sat_job* jobs, const sat_launch* launch,
                                          void* d_ws, size_t ws_bytes, sat_graph** out)
{
    clear_error();
    if (!out) return fail(PILA_EINVAL, "out is NULL");
    *out = nullptr;
    if (n_jobs < 1) return fail(PILA_EINVAL, "a batch graph needs at least one job");
    BatchPlan bp;
    PILA_TRY(batch_plan(n_jobs, jobs, launch, d_ws, ws_bytes, &bp));
    // descriptors and order go to the workspace once, before the capture
    PILA_HIP(hipMemcpy(bp.d_jobs, bp.host.data(), sizeof(ChainJob) * bp.host.size(), hipMemcpyHostToDevice));
    PILA_HIP(hipMemcpy(bp.d_order, bp.order.data(), sizeof(int) * bp.order.size(), hipMemcpyHostToDevice));
    auto g = std::make_unique<sat_graph_s>();
    PILA_TRY(capture_graph([&](hipStream_t cap) { return batch_enqueue(bp, cap, nullptr); }, &g->exec));
    for (const ChainJob& J : bp.host) g->stats.push_back(J.stats);
    batch_bodies(bp, &g->body);
    *out = g.release();
    return PILA_OK;
}

extern "C" int32_t sat_graph_launch(sat_graph* g, void* stream)
{
    clear_error();
    if (!g || !g->exec) return fail(PILA_EINVAL, "graph is NULL");
    PILA_HIP(hipGraphLaunch(g->exec, (hipStream_t)stream));
    return PILA_OK;
}

extern "C" int32_t sat_graph_stats(sat_graph* g, sat_stats* h_stats, void* stream)
{
    clear_error();
    if (!g || !h_stats) return fail(PILA_EINVAL, "graph or stats is NULL");
    hipStream_t st = (hipStream_t)stream;
    for (size_t i = 0; i < g->stats.size(); ++i)
        PILA_HIP(hipMemcpyAsync(&h_stats[i], g->stats[i], sizeof(sat_stats), hipMemcpyDeviceToHost, st));
    PILA_HIP(hipStreamSynchronize(st));
    for (size_t i = 0; i < g->stats.size(); ++i) h_stats[i].body = g->body[i];
    return PILA_OK;
}

extern "C" int32_t sat_graph_destroy(sat_graph* g)
{
    clear_error();
    if (!g) return PILA_OK;
    hipError_t e = hipSuccess;
    if (g->exec) e = hipGraphExecDestroy(g->exec);
    delete g;
    return e == hipSuccess ? PILA_OK : hip_fail(e, "hipGraphExecDestroy", __FILE__, __LINE__);
}
