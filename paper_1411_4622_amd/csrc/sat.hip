// Simulated annealing tomography chains on gfx950 (section II-A Steps 1-4,
// section II-B Eq. 6-7, section III Eq. 8, section III-B BoME).
//
// One workgroup runs one chain from start to end in a persistent loop; the
// host is not involved between steps.  Per step:
//   * each wavefront draws its estimates (Philox, a pure function of the step
//     and estimate index), gathers the estimate pixel's PILA row, and reduces
//     Eq. 7's inner sum S_m = sum l d (2 r + l d) with a shuffle reduction;
//   * after one barrier every wavefront takes the same argmin over the
//     M sums (ties to the lowest index) and the same Metropolis decision on
//     Delta C = sqrt(C^2 + S/KU) - C written cancellation-free;
//   * on acceptance the wavefront that owns the winner scatters Eq. 6 into
//     the residual (the row's rays are distinct, so no atomics), and a
//     second barrier publishes it.
// The residual lives in LDS when U*K values fit the workgroup's LDS budget,
// else in global memory (L2 / MALL resident).  In FP32 mode the residual
// and the row sums are FP32 and the residual is rebuilt from scratch in FP64
// (ray-major forward projection inside the workgroup) every resync_every
// accepted nonzero changes.  Every sum that feeds a decision is formed in an
// order that does not depend on the number of wavefronts, so a chain's
// result does not depend on the launch shape or on other chains.
#include <cmath>
#include <vector>

#include "common.hpp"

namespace pila {

struct ChainJob {
    int32_t N, U, K, P;
    int32_t precision, m_cand, n_stages, q_auto;
    int64_t n_steps, resync_every;
    uint64_t seed, chain_id;
    double T0, TN, tn_ratio, delta_max, f_min, f_max, ln09;
    const int64_t* row_ptr;
    const int32_t* col;
    const void* len;
    const int64_t* t_row_ptr;
    const int32_t* t_col;
    const void* t_len;
    const int32_t* support;
    const double* sino;
    double* f;
    void* r;      // residual, U*K values of the chain's precision (global mode)
    double* sq;   // U*K doubles: per-ray squared residuals for ordered sums
    sat_stats* stats;
    int32_t* tr_m;
    uint8_t* tr_acc;
    double* tr_dc;
};

namespace {

constexpr int kMaxCand = 64;
constexpr int kMaxWaves = 16;

struct ChainShared {
    double S[kMaxCand];
    double fn[kMaxCand];
    double d[kMaxCand];
    int32_t p[kMaxCand];
    double red[kMaxWaves];
    double scalar[4];
    int32_t ticket;
};

__device__ __forceinline__ double cost_change(double sse, double dS, double KU)
{
    const double cn = sqrt(fmax(sse + dS, 0.0) / KU);
    const double co = sqrt(sse / KU);
    const double den = cn + co;
    if (den == 0.0) return 0.0;
    return (dS / KU) / den;
}

// Draw one estimate (Step 2, Eq. 3 with a clamp to [f_min, f_max]) and return
// this lane's part of Eq. 7's inner sum over the pixel's PILA row.
template <typename Real>
__device__ __forceinline__ Real estimate_partial(const ChainJob& J, const Real* __restrict__ r,
                                                 uint64_t c0, uint64_t c1, uint64_t c2, int lane,
                                                 int32_t* p_out, double* fn_out, double* d_out)
{
    const Words4 w = philox4x64(J.seed, J.chain_id, c0, c1, c2, 0);
    const int32_t p = J.support[__umul64hi(w.w0, (uint64_t)J.P)];
    const double delta = J.delta_max * (2.0 * unit53(w.w1) - 1.0);
    const double fo = J.f[p];
    double fn = fo + delta;
    if (fn < J.f_min) fn = J.f_min;
    if (fn > J.f_max) fn = J.f_max;
    const double d = fn - fo;
    const Real* len = (const Real*)J.len;
    const int64_t b = J.row_ptr[p], e = J.row_ptr[p + 1];
    const Real dr = (Real)d;
    Real acc = 0;
    for (int64_t q = b + lane; q < e; q += kWave) {
        const Real t = dr * len[q];
        acc = fma(t, (Real)2 * r[J.col[q]] + t, acc);
    }
    *p_out = p;
    *fn_out = fn;
    *d_out = d;
    return acc;
}

// From-scratch FP64 residual r = A f - Pm over the ray-major PILA (Eq. 1,
// Eq. 4).  Wavefront w handles rays w, w + NW, ...; each ray's sum is formed
// by one wavefront in lane order.  Writes r (in the chain's precision) and
// sq[g] = r64^2, and returns this wavefront's max |r_old - r64| (lane 0).
template <typename Real>
__device__ double rebuild_residual(const ChainJob& J, Real* __restrict__ r, int G, bool measure,
                                   int lane, int wave, int NW)
{
    const Real* tl = (const Real*)J.t_len;
    double drift = 0.0;
    for (int g = wave; g < G; g += NW) {
        const int64_t b = J.t_row_ptr[g], e = J.t_row_ptr[g + 1];
        double acc = 0.0;
        for (int64_t q = b + lane; q < e; q += kWave) acc = fma((double)tl[q], J.f[J.t_col[q]], acc);
        acc = wave_sum(acc);
        if (lane == 0) {
            const double r64 = acc - J.sino[g];
            if (measure) drift = fmax(drift, fabs((double)r[g] - r64));
            r[g] = (Real)r64;
            J.sq[g] = r64 * r64;
        }
    }
    return drift;
}

// sum of sq[0..G) in a fixed order (lane-strided partial sums, then a
// shuffle tree), independent of the workgroup size; result to every thread
__device__ double ordered_sum(const double* __restrict__ sq, int G, ChainShared& sh, int lane, int wave)
{
    __syncthreads();
    if (wave == 0) {
        double a = 0.0;
        for (int g = lane; g < G; g += kWave) a += sq[g];
        a = wave_sum(a);
        if (lane == 0) sh.scalar[0] = a;
    }
    __syncthreads();
    const double v = sh.scalar[0];
    __syncthreads();
    return v;
}

__device__ double block_max(double v, ChainShared& sh, int lane, int wave, int NW)
{
    if (lane == 0) sh.red[wave] = v;
    __syncthreads();
    double m = 0.0;
    for (int w = 0; w < NW; ++w) m = fmax(m, sh.red[w]);
    __syncthreads();
    return m;
}

template <typename Real, bool LDS>
__device__ void run_chain(const ChainJob& J, char* lds, ChainShared& sh)
{
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x >> 6, NW = blockDim.x >> 6;
    const int G = J.U * J.K;
    const double KU = (double)J.K * (double)J.U;
    const int M = J.m_cand;
    Real* r = LDS ? (Real*)lds : (Real*)J.r;

    // Step 1: residual of the starting image and its sum of squares
    rebuild_residual<Real>(J, r, G, false, lane, wave, NW);
    double sse = ordered_sum(J.sq, G, sh, lane, wave);

    // temperatures: given, or Eq. 8 from uphill estimates of the start image
    double T0 = J.T0, TN = J.TN;
    int32_t status = PILA_OK;
    if (!(T0 > 0.0)) {
        const int64_t limit = 1000 * (int64_t)J.q_auto;
        int64_t found = 0;
        double sum = 0.0;
        for (int64_t q0 = 0; q0 < limit && found < J.q_auto; q0 += NW) {
            const int64_t q = q0 + wave;
            if (q < limit) {
                int32_t p;
                double fn, d;
                Real part = estimate_partial<Real>(J, r, (uint64_t)q, 0, 2, lane, &p, &fn, &d);
                const double S = (double)wave_sum(part);
                if (lane == 0) sh.S[wave] = cost_change(sse, S, KU);
            }
            __syncthreads();
            if (threadIdx.x == 0) {
                for (int w = 0; w < NW && q0 + w < limit && found < J.q_auto; ++w) {
                    const double dC = sh.S[w];
                    if (dC > 0.0) {
                        sum += dC;
                        ++found;
                    }
                }
                sh.scalar[1] = sum;
                sh.scalar[2] = (double)found;
            }
            __syncthreads();
            sum = sh.scalar[1];
            found = (int64_t)sh.scalar[2];
            __syncthreads();
        }
        if (found < J.q_auto) {
            status = PILA_EINVAL;
            T0 = TN = 0.0;
        } else {
            T0 = -sum / ((double)J.q_auto * J.ln09);
            TN = T0 / J.tn_ratio;
        }
    }

    int64_t accepts = 0, accepts_nz = 0, since = 0;
    int32_t resyncs = 0;
    double drift_r = 0.0, drift_sse = 0.0;
    const int64_t n_steps = status == PILA_OK ? J.n_steps : 0;
    const bool f32 = sizeof(Real) == 4;

    for (int64_t s = 0; s < n_steps; ++s) {
        const int64_t n = (s * (int64_t)J.n_stages) / J.n_steps;
        const double T = T0 - (double)n * ((T0 - TN) / (double)J.n_stages);
        for (int m = wave; m < M; m += NW) {
            int32_t p;
            double fn, d;
            Real part = estimate_partial<Real>(J, r, (uint64_t)s, (uint64_t)m, 0, lane, &p, &fn, &d);
            const Real S = wave_sum(part);
            if (lane == 0) {
                sh.S[m] = (double)S;
                sh.p[m] = p;
                sh.fn[m] = fn;
                sh.d[m] = d;
            }
        }
        __syncthreads();
        // BoME: first minimal S (every wavefront computes the same answer)
        double v = lane < M ? sh.S[lane] : INFINITY;
        if (v != v) v = INFINITY;  // a NaN sum never wins; the index stays wave-uniform
        int idx = lane < M ? lane : kMaxCand;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const double ov = __shfl_xor(v, o, kWave);
            const int oi = __shfl_xor(idx, o, kWave);
            if (ov < v || (ov == v && oi < idx)) {
                v = ov;
                idx = oi;
            }
        }
        const int ms = idx < M ? idx : 0;
        const double dC = cost_change(sse, v, KU);
        const double N1 = unit53(philox4x64(J.seed, J.chain_id, (uint64_t)s, 0, 1, 0).w0);
        const bool accept = (dC <= 0.0) || (N1 < exp(-dC / T));
        const double dstar = sh.d[ms];
        if (accept) {
            if (wave == ms % NW) {  // the owner of the winner applies Eq. 6
                const int32_t p = sh.p[ms];
                const Real* len = (const Real*)J.len;
                const int64_t b = J.row_ptr[p], e = J.row_ptr[p + 1];
                const Real dr = (Real)dstar;
                for (int64_t q = b + lane; q < e; q += kWave) {
                    const int32_t g = J.col[q];
                    r[g] = r[g] + dr * len[q];
                }
                if (lane == 0) J.f[p] = sh.fn[ms];
            }
            sse += v;
            ++accepts;
            if (dstar != 0.0) {
                ++accepts_nz;
                ++since;
            }
        }
        if (threadIdx.x == 0) {
            if (J.tr_m) J.tr_m[s] = ms;
            if (J.tr_acc) J.tr_acc[s] = accept ? 1 : 0;
            if (J.tr_dc) J.tr_dc[s] = dC;
        }
        if (f32 && J.resync_every > 0 && since >= J.resync_every) {
            __syncthreads();
            const double dr = rebuild_residual<Real>(J, r, G, true, lane, wave, NW);
            drift_r = fmax(drift_r, block_max(dr, sh, lane, wave, NW));
            const double sse64 = ordered_sum(J.sq, G, sh, lane, wave);
            const double ds = sse64 > 0.0 ? fabs(sse - sse64) / sse64 : fabs(sse - sse64);
            drift_sse = fmax(drift_sse, ds);
            sse = sse64;
            since = 0;
            ++resyncs;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0 && J.stats) {
        sat_stats st;
        st.steps = n_steps;
        st.accepts = accepts;
        st.accepts_nonzero = accepts_nz;
        st.resyncs = resyncs;
        st.status = status;
        st.T0_used = T0;
        st.TN_used = TN;
        st.sse_final = sse;
        st.cost_final = sqrt(fmax(sse, 0.0) / KU);
        st.max_drift_r = drift_r;
        st.max_drift_sse = drift_sse;
        *J.stats = st;
    }
    __syncthreads();
}

__device__ void dispatch_chain(const ChainJob& J, char* lds, int lds_bytes, ChainShared& sh)
{
    const int64_t G = (int64_t)J.U * J.K;
    if (J.precision == PILA_F64) {
        if (G * 8 <= lds_bytes)
            run_chain<double, true>(J, lds, sh);
        else
            run_chain<double, false>(J, lds, sh);
    } else {
        if (G * 4 <= lds_bytes)
            run_chain<float, true>(J, lds, sh);
        else
            run_chain<float, false>(J, lds, sh);
    }
}

__global__ __launch_bounds__(1024) void sat_chain_kernel(ChainJob job, int lds_bytes)
{
    extern __shared__ __align__(16) char lds[];
    __shared__ ChainShared sh;
    dispatch_chain(job, lds, lds_bytes, sh);
}

// Persistent batch: each workgroup takes chains from a ticket counter until
// the tickets run out, so every workgroup reaches the exit.
__global__ __launch_bounds__(1024) void sat_batch_kernel(const ChainJob* __restrict__ jobs, int n_jobs,
                                                         int* __restrict__ ticket, int lds_bytes)
{
    extern __shared__ __align__(16) char lds[];
    __shared__ ChainShared sh;
    for (;;) {
        if (threadIdx.x == 0) sh.ticket = atomicAdd(ticket, 1);
        __syncthreads();
        const int j = sh.ticket;
        __syncthreads();
        if (j >= n_jobs) break;
        const ChainJob J = jobs[j];
        dispatch_chain(J, lds, lds_bytes, sh);
    }
}

__global__ void zero_int_kernel(int* p) { *p = 0; }

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

size_t chain_bytes(const pila_geom* g, const sat_params* p)
{
    const size_t G = (size_t)g->n_angles * g->n_bins;
    const size_t rs = p->precision == PILA_F32 ? 4 : 8;
    return align256(rs * G) + align256(8 * G) + align256(sizeof(sat_stats));
}

int32_t check_params(const pila_geom* g, const pila_csr* c, const sat_params* p)
{
    PILA_TRY(check_geom(g));
    if (!c || !p) return fail(PILA_EINVAL, "csr or params is NULL");
    if (!c->row_ptr || !c->col || !c->len || !c->t_row_ptr || !c->t_col || !c->t_len || !c->support)
        return fail(PILA_EINVAL, "PILA arrays (pixel-major, ray-major and support) are required");
    if (c->n_support < 1) return fail(PILA_EINVAL, "empty support");
    if (p->m_cand < 1 || p->m_cand > kMaxCand) return fail(PILA_EINVAL, "m_cand must be in 1..64");
    if (p->n_steps < 0 || p->n_stages < 1) return fail(PILA_EINVAL, "bad n_steps / n_stages");
    if (p->precision != PILA_F64 && p->precision != PILA_F32)
        return fail(PILA_EINVAL, "precision must be PILA_F64 or PILA_F32");
    if (p->precision != g->len_dtype)
        return fail(PILA_EINVAL, "the residual precision must match the PILA length type");
    if (!(p->T0 > 0.0) && (p->q_auto < 1 || !(p->tn_ratio > 0.0)))
        return fail(PILA_EINVAL, "automatic T0 needs q_auto >= 1 and tn_ratio > 0");
    if (p->T0 > 0.0 && !(p->TN > 0.0 && std::isfinite(p->T0) && std::isfinite(p->TN)))
        return fail(PILA_EINVAL, "T0 and TN must be positive and finite");
    if (!(p->delta_max >= 0.0) || !std::isfinite(p->delta_max) || !(p->f_max >= p->f_min))
        return fail(PILA_EINVAL, "bad delta_max / value range");
    if (p->resync_every < 0) return fail(PILA_EINVAL, "resync_every < 0");
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
    J.r = ws;
    J.sq = (double*)(ws + align256(rs * G));
    J.stats = (sat_stats*)(ws + align256(rs * G) + align256(8 * G));
    J.tr_m = nullptr;
    J.tr_acc = nullptr;
    J.tr_dc = nullptr;
    return J;
}

int lds_budget(int n_waves)
{
    (void)n_waves;
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return 0;
    const int total = (int)prop.sharedMemPerBlock;
    const int reserve = (int)sizeof(ChainShared) + 1024;
    return total > reserve ? total - reserve : 0;
}

}  // namespace

}  // namespace pila

using namespace pila;

extern "C" int32_t sat_workspace_size(const pila_geom* geom, const sat_params* params, size_t* bytes)
{
    clear_error();
    PILA_TRY(check_geom(geom));
    if (!params || !bytes) return fail(PILA_EINVAL, "params or bytes is NULL");
    *bytes = chain_bytes(geom, params);
    return PILA_OK;
}

extern "C" int32_t sat_run(const pila_geom* geom, const pila_csr* csr, const double* d_sino,
                           const sat_params* params, double* d_image, void* d_ws, size_t ws_bytes,
                           sat_stats* h_stats, const sat_trace* trace, void* stream)
{
    clear_error();
    PILA_TRY(check_params(geom, csr, params));
    if (!d_sino || !d_image) return fail(PILA_EINVAL, "sinogram or image is NULL");
    const size_t need = chain_bytes(geom, params);
    if (!d_ws || ws_bytes < need)
        return fail(PILA_ENOMEM, "workspace of %zu bytes is below the %zu needed", ws_bytes, need);
    hipStream_t st = (hipStream_t)stream;
    ChainJob J = make_job(geom, csr, d_sino, params, d_image, (char*)d_ws);
    if (trace) {
        J.tr_m = trace->m_star;
        J.tr_acc = trace->accept;
        J.tr_dc = trace->dC;
    }
    int waves = params->m_cand < kMaxWaves ? params->m_cand : kMaxWaves;
    if (waves < 1) waves = 1;
    const int64_t G = (int64_t)geom->n_angles * geom->n_bins;
    const int64_t rbytes = G * (params->precision == PILA_F32 ? 4 : 8);
    const int budget = lds_budget(waves);
    const int lds = rbytes <= budget ? (int)rbytes : 0;
    PILA_HIP(hipFuncSetAttribute((const void*)sat_chain_kernel,
                                 hipFuncAttributeMaxDynamicSharedMemorySize, lds));
    sat_chain_kernel<<<1, waves * kWave, (size_t)lds, st>>>(J, lds);
    PILA_HIP(hipGetLastError());
    if (h_stats) {
        PILA_HIP(hipMemcpyAsync(h_stats, J.stats, sizeof(sat_stats), hipMemcpyDeviceToHost, st));
        PILA_HIP(hipStreamSynchronize(st));
    }
    return PILA_OK;
}

extern "C" int32_t sat_batch_workspace_size(int32_t n_jobs, const sat_job* jobs, size_t* bytes)
{
    clear_error();
    if (n_jobs < 0 || (n_jobs > 0 && !jobs) || !bytes) return fail(PILA_EINVAL, "bad batch arguments");
    size_t total = align256(sizeof(ChainJob) * (size_t)(n_jobs > 0 ? n_jobs : 1)) + 256;
    for (int32_t j = 0; j < n_jobs; ++j) {
        PILA_TRY(check_geom(jobs[j].geom));
        total += chain_bytes(jobs[j].geom, &jobs[j].params);
    }
    *bytes = total;
    return PILA_OK;
}

extern "C" int32_t sat_run_batch(int32_t n_jobs, const sat_job* jobs, const sat_launch* launch,
                                 void* d_ws, size_t ws_bytes, sat_stats* h_stats, void* stream)
{
    clear_error();
    size_t need = 0;
    PILA_TRY(sat_batch_workspace_size(n_jobs, jobs, &need));
    if (!d_ws || ws_bytes < need)
        return fail(PILA_ENOMEM, "workspace of %zu bytes is below the %zu needed", ws_bytes, need);
    if (n_jobs == 0) return PILA_OK;
    hipStream_t st = (hipStream_t)stream;
    char* ws = (char*)d_ws;
    ChainJob* d_jobs = (ChainJob*)ws;
    int* d_ticket = (int*)(ws + align256(sizeof(ChainJob) * (size_t)n_jobs));
    char* cur = ws + align256(sizeof(ChainJob) * (size_t)n_jobs) + 256;
    std::vector<ChainJob> host((size_t)n_jobs);
    for (int32_t j = 0; j < n_jobs; ++j) {
        const sat_job& jb = jobs[j];
        PILA_TRY(check_params(jb.geom, jb.csr, &jb.params));
        if (!jb.d_sino || !jb.d_image) return fail(PILA_EINVAL, "job %d: sinogram or image is NULL", j);
        host[j] = make_job(jb.geom, jb.csr, jb.d_sino, &jb.params, jb.d_image, cur);
        cur += chain_bytes(jb.geom, &jb.params);
    }
    int waves = 4, per_cu = 2, use_lds = 1;
    if (launch) {
        waves = launch->waves_per_chain;
        per_cu = launch->chains_per_cu;
        use_lds = launch->lds_residual;
    }
    if (waves != 1 && waves != 2 && waves != 4 && waves != 8 && waves != 16)
        return fail(PILA_EINVAL, "waves_per_chain must be 1, 2, 4, 8 or 16");
    if (per_cu < 1 || per_cu > 32) return fail(PILA_EINVAL, "chains_per_cu must be in 1..32");
    int dev = 0;
    hipDeviceProp_t prop;
    PILA_HIP(hipGetDevice(&dev));
    PILA_HIP(hipGetDeviceProperties(&prop, dev));
    int lds = 0;
    if (use_lds) {
        const int per_wg = (int)(prop.sharedMemPerBlock / (size_t)per_cu) - (int)sizeof(ChainShared) - 512;
        lds = per_wg > 0 ? (per_wg & ~255) : 0;
    }
    const int grid_max = prop.multiProcessorCount * per_cu;
    const int grid = n_jobs < grid_max ? n_jobs : grid_max;
    PILA_HIP(hipMemcpyAsync(d_jobs, host.data(), sizeof(ChainJob) * host.size(), hipMemcpyHostToDevice, st));
    PILA_HIP(hipFuncSetAttribute((const void*)sat_batch_kernel,
                                 hipFuncAttributeMaxDynamicSharedMemorySize, lds));
    zero_int_kernel<<<1, 1, 0, st>>>(d_ticket);
    sat_batch_kernel<<<grid, waves * kWave, (size_t)lds, st>>>(d_jobs, n_jobs, d_ticket, lds);
    PILA_HIP(hipGetLastError());
    if (h_stats) {
        for (int32_t j = 0; j < n_jobs; ++j)
            PILA_HIP(hipMemcpyAsync(&h_stats[j], host[j].stats, sizeof(sat_stats), hipMemcpyDeviceToHost, st));
    }
    // the descriptor upload reads host memory owned by this call
    PILA_HIP(hipStreamSynchronize(st));
    return PILA_OK;
}
