// Device side of the simulated annealing chains (section II-A Steps 1-4,
// section II-B Eq. 6-7, section III Eq. 8, section III-B BoME).
//
// One workgroup runs one chain; the host is not involved between steps.  Per
// step every estimate's change of the squared-residual sum,
// S_m = sum over its PILA row of l d (2 r + l d) (Eq. 7's inner sum), is
// reduced by the lanes that own it; after a barrier every wavefront takes the
// same first minimum over the M sums (BoME) and the same Metropolis decision
// on Delta C = sqrt(C^2 + S/KU) - C, written cancellation-free; the owner of
// an accepted estimate applies Eq. 6 to the residual (a row's rays are
// distinct, so no atomics) and a second barrier publishes it.
//
// Two bodies share this logic and give bit-identical results:
//  * run_chain_piped: the estimates do not depend on the chain state, so
//    Philox draws, support lookups and row offsets are computed a block of
//    steps at a time (one lane per step and estimate) and each estimate's row
//    is loaded into registers two steps ahead.  The image value and (when the
//    residual lives in global memory) the residual values are loaded one step
//    ahead and patched with the previous step's accepted change: the owner
//    publishes the new residual values of its row in a small LDS table keyed
//    by (angle, bin parity) and tagged with the step.  Rows must fit the
//    registers (max_row <= LPC * E).
//  * run_chain_simple: any row length and any M.
//
// Canonical sums: a row sum S is the sum of 64 partials (partial j takes the
// entries q = j mod 64 in ascending q, fused multiply-add) combined by an
// xor butterfly with distances 1, 2, 4, 8, 16, 32.  A workgroup of any shape
// with 16, 32 or 64 lanes per estimate forms exactly these operations (lanes
// keep 64 / LPC partials), so the result does not depend on the launch shape.
// Residual rebuilds sum each ray sequentially over its entries (one lane per
// ray), 64-ray tiles by the same butterfly, and tiles lane-strided, whether
// one workgroup or the whole GPU runs them.
//
// Visibility: within a workgroup (all waves on one CU, one vector L1) a
// store issued before s_barrier is seen by loads other waves issue after it,
// so barriers only drain LDS traffic and prefetched global loads stay in
// flight across them.
#pragma once

#include <cmath>
#include <type_traits>

#include "common.hpp"

namespace pila {

// Chain state carried between launches of a segmented chain.
struct ChainCarry {
    int64_t s_next, accepts, accepts_nz, since;
    int32_t resyncs, status, resync_due, done;
    double sse, T0, TN, drift_r, drift_sse;
};

struct ChainJob {
    int32_t N, U, K, P;
    int32_t precision, m_cand, n_stages, q_auto;
    int32_t max_row, schedule;   // schedule: PILA_SCHED_* cooling law
    int32_t k_lo, Kc, UL, proposal;  // LDS part of the residual: angles u < UL, bins k_lo ..
                                     // k_lo+Kc-1; proposal: PILA_PROP_* (clamp or redraw)
    uint32_t kdiv_m, kdiv_s;     // g / K = (g * kdiv_m) >> kdiv_s for g < 2^24 (kdiv_s = 0: divide)
    int32_t rkb, lenq;           // global residual layout: 8-bin blocks per angle group (rpos);
                                 // lenq: lengths are one byte each (LenQ)
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
    void* r;          // residual, U*K values of the chain's precision (global mode)
    double* tsum;     // per 64-ray tile: sum of squared residuals (ceil(U*K/64))
    double* tdrift;   // per tile: max |r_old - r64| at a rebuild
    ChainCarry* carry;
    sat_stats* stats;
    int32_t* tr_m;
    uint8_t* tr_acc;
    double* tr_dc;
    const int32_t* tcol;     // optional: per PILA entry, the slot word of ray_slot (else NULL)
    const uint64_t* cancel;  // served chains: host word that equals cancel_tag once cancelled
    uint64_t cancel_tag;
};

constexpr int kMaxCand = 64;
constexpr int kMaxWaves = 16;
// redraws of one estimate's change before it is given up (change 0)
constexpr uint64_t kRedrawMax = 256;

struct ChainShared {
    double S[kMaxCand];
    double fn[kMaxCand];
    double d[kMaxCand];
    int64_t rb[kMaxCand], re[kMaxCand];  // general body: each estimate's row
    int32_t p[kMaxCand];
    double red[kMaxWaves];
    double scalar[4];
    double fnstar;
    int32_t pstar;
    int32_t ticket;
    int32_t stop;
};

// A copy of a descriptor held in LDS whose every field the compiler knows to
// be the same in all lanes (so it lives in scalar registers, as a kernel
// argument would).
template <typename T>
__device__ __forceinline__ T lane0(T x)
{
    static_assert(sizeof(T) == 4 || sizeof(T) == 8, "32- or 64-bit fields");
    if constexpr (sizeof(T) == 4) {
        uint32_t u;
        __builtin_memcpy(&u, &x, 4);
        u = __builtin_amdgcn_readfirstlane(u);
        __builtin_memcpy(&x, &u, 4);
    } else {
        uint64_t u;
        __builtin_memcpy(&u, &x, 8);
        const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)u);
        const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(u >> 32));
        u = ((uint64_t)hi << 32) | lo;
        __builtin_memcpy(&x, &u, 8);
    }
    return x;
}

// uniform_job below copies every field by name: a field added to ChainJob
// must be added there too (this size check is the reminder)
static_assert(sizeof(ChainJob) == 320, "ChainJob changed: update uniform_job");

__device__ __forceinline__ ChainJob uniform_job(const ChainJob& d)
{
    ChainJob J;
#define PILA_F(f) J.f = lane0(d.f);
    PILA_F(N) PILA_F(U) PILA_F(K) PILA_F(P) PILA_F(precision) PILA_F(m_cand) PILA_F(n_stages)
    PILA_F(q_auto) PILA_F(max_row) PILA_F(schedule) PILA_F(k_lo) PILA_F(Kc) PILA_F(UL) PILA_F(proposal)
    PILA_F(kdiv_m) PILA_F(kdiv_s) PILA_F(rkb) PILA_F(lenq) PILA_F(n_steps) PILA_F(resync_every) PILA_F(seed) PILA_F(chain_id)
    PILA_F(T0) PILA_F(TN) PILA_F(tn_ratio) PILA_F(delta_max) PILA_F(f_min) PILA_F(f_max) PILA_F(ln09)
    PILA_F(row_ptr) PILA_F(col) PILA_F(len) PILA_F(t_row_ptr) PILA_F(t_col) PILA_F(t_len)
    PILA_F(support) PILA_F(sino) PILA_F(f) PILA_F(r) PILA_F(tsum) PILA_F(tdrift) PILA_F(carry)
    PILA_F(stats) PILA_F(tr_m) PILA_F(tr_acc) PILA_F(tr_dc) PILA_F(tcol) PILA_F(cancel) PILA_F(cancel_tag)
#undef PILA_F
    return J;
}

// Cancellation of a served chain: thread 0 reads the host word every
// kCancelEvery steps before a barrier, every thread reads its copy after a
// later barrier of the same step, so the whole workgroup leaves together.
// The read is a system-scope load of coherent host memory (it reaches host
// memory each time); it carries no ordering, so it invalidates no cache.
constexpr int64_t kCancelEvery = 1024;

__device__ __forceinline__ void cancel_probe(const ChainJob& J, ChainShared& sh, int64_t s)
{
    if (J.cancel && (s & (kCancelEvery - 1)) == 0 && threadIdx.x == 0)
        sh.stop = __hip_atomic_load(J.cancel, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM) == J.cancel_tag;
}
__device__ __forceinline__ bool cancel_seen(const ChainJob& J, const ChainShared& sh, int64_t s)
{
    return J.cancel && (s & (kCancelEvery - 1)) == 0 && sh.stop;
}

// pipelined workgroups hold at most 8 wavefronts (up to 256 registers per lane)
constexpr int kPipedThreads = 512;

// ---------------------------------------------------------------------------
// lane primitives
// ---------------------------------------------------------------------------
template <int CTRL>
__device__ __forceinline__ float dpp_mov(float x)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xF, 0xF, true));
}
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double x)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), CTRL, 0xF, 0xF, true);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float swz16(float x)
{
    return __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(x), 0x401F));
}
__device__ __forceinline__ double swz16(double x)
{
    const int lo = __builtin_amdgcn_ds_swizzle(__double2loint(x), 0x401F);
    const int hi = __builtin_amdgcn_ds_swizzle(__double2hiint(x), 0x401F);
    return __hiloint2double(hi, lo);
}

// value of lane ^ O (O = 1, 2, 4, 8, 16, 32).  For O = 4 and O = 8 the row
// mirrors are used, which equal the xor partner once every quad (O = 4) or
// half-row (O = 8) holds one value, as it does inside a butterfly.
template <int O, typename T>
__device__ __forceinline__ T xor_partner(T x)
{
    if constexpr (O == 1) return dpp_mov<0xB1>(x);
    else if constexpr (O == 2) return dpp_mov<0x4E>(x);
    else if constexpr (O == 4) return dpp_mov<0x141>(x);
    else if constexpr (O == 8) return dpp_mov<0x140>(x);
    else if constexpr (O == 16) return swz16(x);
    else return __shfl_xor(x, 32, kWave);
}

template <int O, int LPC, int K, typename T>
__device__ __forceinline__ void butterfly_level(T (&a)[K])
{
    if constexpr (O < LPC) {
#pragma unroll
        for (int k = 0; k < K; ++k) a[k] = a[k] + xor_partner<O>(a[k]);
    } else {
        constexpr int st = O / LPC;
#pragma unroll
        for (int k = 0; k < K; ++k)
            if (!(k & st)) {
                const T t = a[k] + a[k ^ st];
                a[k] = t;
                a[k ^ st] = t;
            }
    }
}

// Canonical 64-partial sum for groups of LPC lanes holding K = 64 / LPC
// partials each (partial j = lane-in-group + k * LPC); every lane of the
// group returns the total.
template <int LPC, typename T>
__device__ __forceinline__ T canon_sum(T (&a)[64 / LPC])
{
    constexpr int K = 64 / LPC;
    butterfly_level<1, LPC, K>(a);
    butterfly_level<2, LPC, K>(a);
    butterfly_level<4, LPC, K>(a);
    butterfly_level<8, LPC, K>(a);
    butterfly_level<16, LPC, K>(a);
    butterfly_level<32, LPC, K>(a);
    return a[0];
}

template <typename T>
__device__ __forceinline__ T wave_canon_sum(T x)
{
    T a[1] = {x};
    return canon_sum<64>(a);
}

__device__ __forceinline__ double wave_min(double x)
{
    x = fmin(x, xor_partner<1>(x));
    x = fmin(x, xor_partner<2>(x));
    x = fmin(x, xor_partner<4>(x));
    x = fmin(x, xor_partner<8>(x));
    x = fmin(x, xor_partner<16>(x));
    x = fmin(x, xor_partner<32>(x));
    return x;
}

__device__ __forceinline__ double readlane_f64(double v, int l)
{
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double uniform_f64(double v)
{
    const int lo = __builtin_amdgcn_readfirstlane(__double2loint(v));
    const int hi = __builtin_amdgcn_readfirstlane(__double2hiint(v));
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ int uniform_i32(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t uniform_i64(int64_t v)
{
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// ---------------------------------------------------------------------------
// Layout of a residual held in global memory: tiles of 4 angles x 8 bins
// (32 values: one 128-byte line in FP32), tile (u / 4, k / 8) at
// ((u / 4) rkb + k / 8) 32, value (u mod 4) 8 + k mod 8 inside it, with
// rkb = ceil(K / 8).  A pixel's ray moves by about (distance from the axis)
// x pi / U bins from one angle to the next, so consecutive entries of a
// PILA row (ascending angle) often share a tile and its cache line, where
// the row-major sinogram would give each entry a line of its own.  A
// residual held in LDS stays row-major (index g = u K + k).
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t rpos(const ChainJob& J, int u, int k)
{
    return ((uint32_t)((u >> 2) * J.rkb + (k >> 3)) << 5) | ((uint32_t)(u & 3) << 3) | (uint32_t)(k & 7);
}
__device__ __forceinline__ int angle_of(const ChainJob& J, int32_t g)
{
    return J.kdiv_s ? (int)(((uint64_t)(uint32_t)g * J.kdiv_m) >> J.kdiv_s) : (int)((uint32_t)g / (uint32_t)J.K);
}
__device__ __forceinline__ uint32_t rpos_g(const ChainJob& J, int32_t g)
{
    const int u = angle_of(J, g);
    return rpos(J, u, g - u * J.K);
}
// index of ray g in a residual array: tiled in global memory, row-major in LDS
template <bool GLOB>
__device__ __forceinline__ uint32_t ridx(const ChainJob& J, int32_t g)
{
    return GLOB ? rpos_g(J, g) : (uint32_t)g;
}

// ---------------------------------------------------------------------------
// cooling schedule: stage n = floor(s n_stages / n_steps), tracked
// incrementally without a 64-bit division per step; with N = n_stages,
//   Eq. 2 (linear):                        T_n = T0 - n (T0 - TN) / N
//   exponential (section III-C, 2nd Eq. 8): T_n = T0 (TN / T0)^(n / N)
//   cubic (Eq. 9):                          T_n = T0 - n^3 (T0 - TN) / N^3
// ---------------------------------------------------------------------------
struct Schedule {
    int64_t stage, next;  // current stage, first step of the following stage
    double T0, TN, dT, NN;
    int kind;
    double T, invT;  // temperature of the current stage and its reciprocal
    __device__ void start(int64_t s, int64_t n_steps, int32_t n_stages, double t0, double tn, int k)
    {
        T0 = t0;
        TN = tn;
        kind = k;
        NN = (double)n_stages;
        dT = (t0 - tn) / NN;
        stage = n_steps > 0 ? (s * (int64_t)n_stages) / n_steps : 0;
        next = first_of(stage + 1, n_steps, n_stages);
        set();
    }
    __device__ void set()
    {
        const double x = (double)stage;
        if (kind == PILA_SCHED_EXP)
            T = T0 * pow(TN / T0, x / NN);
        else if (kind == PILA_SCHED_CUBIC)
            T = T0 - (x * x * x) * ((T0 - TN) / (NN * NN * NN));
        else
            T = T0 - x * dT;
        invT = 1.0 / T;
    }
    __device__ static int64_t first_of(int64_t k, int64_t n_steps, int32_t n_stages)
    {
        return (k * n_steps + n_stages - 1) / n_stages;
    }
    __device__ double at(int64_t s, int64_t n_steps, int32_t n_stages)
    {
        if (s >= next) {
            while (s >= next) {
                ++stage;
                next = first_of(stage + 1, n_steps, n_stages);
            }
            set();
        }
        return T;
    }
};

// ---------------------------------------------------------------------------
// estimates, rebuilds and ordered sums
// ---------------------------------------------------------------------------

// Draw one estimate (Step 2, Eq. 3 with a clamp to [f_min, f_max]) and return
// its row sum (whole wavefront, canonical order) in every lane.
template <typename Real, bool GLOB, typename LenT = Real>
__device__ Real estimate_sum(const ChainJob& J, const Real* __restrict__ r, uint64_t c0, uint64_t c1,
                             uint64_t c2, int lane, int32_t* p_out, double* fn_out, double* d_out)
{
    const Words4 w = philox4x64(J.seed, J.chain_id, c0, c1, c2, 0);
    const int32_t p = J.support[__umul64hi(w.w0, (uint64_t)J.P)];
    double delta = J.delta_max * (2.0 * unit53(w.w1) - 1.0);
    const double fo = J.f[p];
    double fn = fo + delta;
    if (J.proposal == PILA_PROP_REDRAW) {
        // Eq. 3 as printed: the change is drawn again (counter word 3 = j)
        // for the same pixel until the new value is in range; the draws are
        // the same in every lane of the wavefront
        for (uint64_t j = 1; (fn < J.f_min || fn > J.f_max) && j <= kRedrawMax; ++j) {
            delta = J.delta_max * (2.0 * unit53(philox4x64(J.seed, J.chain_id, c0, c1, c2, j).w1) - 1.0);
            fn = fo + delta;
        }
        if (fn < J.f_min || fn > J.f_max) fn = fo;
    } else {
        if (fn < J.f_min) fn = J.f_min;
        if (fn > J.f_max) fn = J.f_max;
    }
    const double d = fn - fo;
    const LenT* len = (const LenT*)J.len;
    const int64_t b = J.row_ptr[p], e = J.row_ptr[p + 1];
    const Real dr = (Real)d;
    Real acc = 0;
    // U entries per lane in flight; each lane still adds its entries in
    // ascending order, so the sum is the canonical one
    constexpr int U = 8;
    for (int64_t q0 = b + lane; q0 < e; q0 += (int64_t)kWave * U) {
        int32_t cc[U];
        Real ll[U];
#pragma unroll
        for (int c = 0; c < U; ++c) {
            const int64_t q = q0 + (int64_t)c * kWave < e ? q0 + (int64_t)c * kWave : b;
            cc[c] = J.col[q];
            ll[c] = (Real)len[q];
        }
        Real rr[U];
#pragma unroll
        for (int c = 0; c < U; ++c) rr[c] = r[ridx<GLOB>(J, cc[c])];
#pragma unroll
        for (int c = 0; c < U; ++c) {
            if (q0 + (int64_t)c * kWave < e) {
                const Real t = dr * ll[c];
                acc = fma(t, (Real)2 * rr[c] + t, acc);
            }
        }
    }
    *p_out = p;
    *fn_out = fn;
    *d_out = d;
    return wave_canon_sum(acc);
}

// One 64-ray tile of a from-scratch FP64 residual r = A f - Pm (Eq. 1,
// Eq. 4), by one wavefront.  The four 16-lane quarters take the
// tile's rays four at a time (quarter q the rays q*16 + i, i = 0..15); the
// lanes of a quarter stride the ray's ray-major row by 16, so each load of
// a quarter reads 16 consecutive entries, and each lane keeps one FP64
// partial (its entries in ascending order, fused multiply-add).  An xor
// butterfly over the quarter adds the 16 partials.  Lane j then holds ray
// t*64 + j.  In-group and grid-wide rebuilds both run this function, so they
// give the same bits.
template <typename Real, bool GLOB, typename LenT = Real>
__device__ void rebuild_tile(const ChainJob& J, Real* __restrict__ r, int G, int t, bool measure,
                             int lane)
{
    constexpr int U4 = 4;  // entries per lane in flight
    const LenT* tl = (const LenT*)J.t_len;
    const int quarter = lane >> 4, ql = lane & 15;
    double mine = 0.0;
    for (int i = 0; i < 16; ++i) {
        const int gi = t * kWave + quarter * 16 + i;
        double acc = 0.0;
        if (gi < G) {
            const int64_t b = J.t_row_ptr[gi], e = J.t_row_ptr[gi + 1];
            for (int64_t q0 = b + ql; q0 < e; q0 += 16 * U4) {
                int32_t pc[U4];
                Real lc[U4];
#pragma unroll
                for (int c = 0; c < U4; ++c) {
                    const int64_t q = q0 + 16 * c < e ? q0 + 16 * c : b;
                    pc[c] = J.t_col[q];
                    lc[c] = (Real)tl[q];
                }
                double fv[U4];
#pragma unroll
                for (int c = 0; c < U4; ++c) fv[c] = J.f[pc[c]];
#pragma unroll
                for (int c = 0; c < U4; ++c)
                    if (q0 + 16 * c < e) acc = fma((double)lc[c], fv[c], acc);
            }
        }
        acc = acc + xor_partner<1>(acc);
        acc = acc + xor_partner<2>(acc);
        acc = acc + xor_partner<4>(acc);
        acc = acc + xor_partner<8>(acc);
        if (ql == i) mine = acc;
    }
    const int g = t * kWave + lane;
    const double acc = mine;
    double sq = 0.0, dr = 0.0;
    if (g < G) {
        const double r64 = acc - J.sino[g];
        const uint32_t at = ridx<GLOB>(J, g);
        if (measure) dr = fabs((double)r[at] - r64);
        r[at] = (Real)r64;
        sq = r64 * r64;
    }
    sq = wave_canon_sum(sq);
    if (measure) dr = -wave_min(-dr);  // max over the tile
    if (lane == 0) {
        J.tsum[t] = sq;
        if (measure) J.tdrift[t] = dr;
    }
}

// sum of the tile sums (lane-strided, then the butterfly) and max of the tile
// drifts, by one wavefront; every lane gets the results
__device__ inline void tile_totals(const ChainJob& J, int G, bool measure, int lane, double* sse,
                                   double* drift)
{
    const int T = (G + kWave - 1) / kWave;
    double a = 0.0, m = 0.0;
    for (int t = lane; t < T; t += kWave) {
        a += J.tsum[t];
        if (measure) m = fmax(m, J.tdrift[t]);
    }
    *sse = wave_canon_sum(a);
    *drift = measure ? -wave_min(-m) : 0.0;
}

// in-workgroup rebuild of the whole residual; returns (sse, drift) to all
template <typename Real, bool GLOB, typename LenT = Real>
__device__ void rebuild_in_group(const ChainJob& J, Real* r, ChainShared& sh, bool measure, int lane,
                                 int wave, int NW, double* sse, double* drift)
{
    const int G = J.U * J.K;
    const int T = (G + kWave - 1) / kWave;
    __syncthreads();
    for (int t = wave; t < T; t += NW) rebuild_tile<Real, GLOB, LenT>(J, r, G, t, measure, lane);
    __syncthreads();
    if (wave == 0) {
        double s, d;
        tile_totals(J, G, measure, lane, &s, &d);
        if (lane == 0) {
            sh.scalar[0] = s;
            sh.scalar[1] = d;
        }
    }
    __syncthreads();
    *sse = uniform_f64(sh.scalar[0]);
    *drift = uniform_f64(sh.scalar[1]);
    __syncthreads();
}

struct ChainState {
    double sse, T0, TN, drift_r, drift_sse;
    int64_t n_steps, accepts, accepts_nz, since, s_begin;
    int32_t status, resyncs;
};

// Eq. 8: T0 from q_auto uphill single-pixel estimates of the starting image
// (Philox counter (q, 0, 2, 0)), summed in q order.
template <typename Real, bool GLOB, typename LenT = Real>
__device__ void auto_temperature(const ChainJob& J, const Real* r, double sse, ChainShared& sh, int lane,
                                 int wave, int NW, double* T0, double* TN, int32_t* status)
{
    const double KU = (double)J.K * (double)J.U;
    const int64_t limit = 1000 * (int64_t)J.q_auto;
    int64_t found = 0;
    double sum = 0.0;
    for (int64_t q0 = 0; q0 < limit && found < J.q_auto; q0 += NW) {
        const int64_t q = q0 + wave;
        if (q < limit) {
            int32_t p;
            double fn, d;
            const double S = (double)estimate_sum<Real, GLOB, LenT>(J, r, (uint64_t)q, 0, 2, lane, &p, &fn, &d);
            const double cn = sqrt(fmax(sse + S, 0.0) / KU), co = sqrt(sse / KU);
            const double den = cn + co;
            if (lane == 0) sh.S[wave] = den == 0.0 ? 0.0 : (S / KU) / den;
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
            sh.scalar[2] = sum;
            sh.scalar[3] = (double)found;
        }
        __syncthreads();
        sum = uniform_f64(sh.scalar[2]);
        found = (int64_t)uniform_f64(sh.scalar[3]);
        __syncthreads();
    }
    if (found < J.q_auto) {
        *status = PILA_EINVAL;
        *T0 = *TN = 0.0;
    } else {
        *status = PILA_OK;
        *T0 = -sum / ((double)J.q_auto * J.ln09);
        *TN = *T0 / J.tn_ratio;
    }
}

// Step 1 and Eq. 8 inside the workgroup.
template <typename Real, bool GLOB, typename LenT = Real>
__device__ ChainState chain_setup(const ChainJob& J, Real* r, ChainShared& sh, int lane, int wave, int NW)
{
    ChainState cs;
    double drift;
    rebuild_in_group<Real, GLOB, LenT>(J, r, sh, false, lane, wave, NW, &cs.sse, &drift);
    cs.T0 = J.T0;
    cs.TN = J.TN;
    cs.status = PILA_OK;
    if (!(cs.T0 > 0.0))
        auto_temperature<Real, GLOB, LenT>(J, r, cs.sse, sh, lane, wave, NW, &cs.T0, &cs.TN, &cs.status);
    cs.n_steps = cs.status == PILA_OK ? J.n_steps : 0;
    cs.accepts = cs.accepts_nz = cs.since = cs.s_begin = 0;
    cs.resyncs = 0;
    cs.drift_r = cs.drift_sse = 0.0;
    return cs;
}

__device__ inline ChainState load_carry(const ChainJob& J)
{
    const ChainCarry& c = *J.carry;
    ChainState cs;
    cs.sse = c.sse;
    cs.T0 = c.T0;
    cs.TN = c.TN;
    cs.drift_r = c.drift_r;
    cs.drift_sse = c.drift_sse;
    cs.status = c.status;
    cs.n_steps = c.status == PILA_OK ? J.n_steps : 0;
    cs.accepts = c.accepts;
    cs.accepts_nz = c.accepts_nz;
    cs.since = c.since;
    cs.s_begin = c.s_next;
    cs.resyncs = c.resyncs;
    return cs;
}

__device__ inline void save_carry(const ChainJob& J, const ChainState& cs, int64_t s_next, bool resync_due)
{
    if (threadIdx.x != 0) return;
    ChainCarry& c = *J.carry;
    c.s_next = s_next;
    c.accepts = cs.accepts;
    c.accepts_nz = cs.accepts_nz;
    c.since = cs.since;
    c.resyncs = cs.resyncs;
    c.status = cs.status;
    c.resync_due = resync_due ? 1 : 0;
    c.done = s_next >= cs.n_steps ? 1 : 0;
    c.sse = cs.sse;
    c.T0 = cs.T0;
    c.TN = cs.TN;
    c.drift_r = cs.drift_r;
    c.drift_sse = cs.drift_sse;
}

__device__ inline void write_stats(const ChainJob& J, const ChainState& cs)
{
    if (threadIdx.x == 0 && J.stats) {
        const double KU = (double)J.K * (double)J.U;
        sat_stats st;
        st.steps = cs.n_steps;
        st.accepts = cs.accepts;
        st.accepts_nonzero = cs.accepts_nz;
        st.resyncs = cs.resyncs;
        st.status = cs.status;
        st.T0_used = cs.T0;
        st.TN_used = cs.TN;
        st.sse_final = cs.sse;
        st.cost_final = sqrt(fmax(cs.sse, 0.0) / KU);
        st.max_drift_r = cs.drift_r;
        st.max_drift_sse = cs.drift_sse;
        st.chain_launches = 0;
        st.body = 0;
        st.chain_kernel_ms = 0.0;
        st.t_begin = st.t_end = 0;
        *J.stats = st;
    }
    __syncthreads();
}

struct Decision {
    int ms;
    double S, dC;
    bool accept;
};

// BoME (first minimal S; a NaN never wins) and Step 4's acceptance.  Every
// wavefront computes the same answer; each lane forms the cost change of its
// own estimate so the cost arithmetic overlaps the minimum search.  The test
// N1 < exp(-dC / T) is settled by comparing -dC / T with ln N1 (computed
// ahead of time) whenever they differ by more than 1e-12 relative, far
// beyond the rounding of exp, the division and the logarithm; inside that
// band (and for N1 = 0) it is evaluated exactly as written.
__device__ __forceinline__ Decision decide(const double* S, int M, int lane, double sse, double co,
                                           double KU, double T, double invT, double N1, double lnN1)
{
    double v = lane < M ? S[lane] : INFINITY;
    if (v != v) v = INFINITY;
    const double cn = sqrt(fmax(sse + v, 0.0) / KU);
    const double den = cn + co;
    const double dC = den == 0.0 ? 0.0 : (v / KU) / den;
    const double vmin = wave_min(v);
    const unsigned long long mask = __ballot(v == vmin);
    Decision dn;
    dn.ms = mask ? uniform_i32(__ffsll((long long)mask) - 1) : 0;
    dn.S = readlane_f64(v, dn.ms);
    dn.dC = readlane_f64(dC, dn.ms);
    if (dn.dC <= 0.0) {
        dn.accept = true;
    } else {
        const double x = -dn.dC * invT;
        const double margin = 1e-12 * (fabs(lnN1) + fabs(x));
        if (N1 > 0.0 && x < lnN1 - margin)
            dn.accept = false;
        else if (N1 > 0.0 && x > lnN1 + margin)
            dn.accept = true;
        else
            dn.accept = N1 < exp(-dn.dC / T);
    }
    return dn;
}

// bookkeeping and trace after a decision; d_star is the winner's change
__device__ __forceinline__ void count_decision(const ChainJob& J, ChainState& cs, const Decision& dn,
                                               double d_star, int64_t s)
{
    if (dn.accept) {
        cs.sse += dn.S;
        ++cs.accepts;
        if (d_star != 0.0) {
            ++cs.accepts_nz;
            ++cs.since;
        }
    }
    if (threadIdx.x == 0) {
        if (J.tr_m) J.tr_m[s] = dn.ms;
        if (J.tr_acc) J.tr_acc[s] = dn.accept ? 1 : 0;
        if (J.tr_dc) J.tr_dc[s] = dn.dC;
    }
}

template <typename Real, bool GLOB, typename LenT = Real>
__device__ __forceinline__ void resync_in_group(const ChainJob& J, ChainState& cs, Real* r, ChainShared& sh,
                                                int lane, int wave, int NW)
{
    double sse64, drift;
    rebuild_in_group<Real, GLOB, LenT>(J, r, sh, true, lane, wave, NW, &sse64, &drift);
    cs.drift_r = fmax(cs.drift_r, drift);
    const double ds = sse64 > 0.0 ? fabs(cs.sse - sse64) / sse64 : fabs(cs.sse - sse64);
    cs.drift_sse = fmax(cs.drift_sse, ds);
    cs.sse = sse64;
    cs.since = 0;
    ++cs.resyncs;
}

// ---------------------------------------------------------------------------
// any row length, any M
// ---------------------------------------------------------------------------
template <typename Real, bool LDS, typename LenT = Real>
__device__ void run_chain_simple(const ChainJob& J, char* lds, ChainShared& sh, bool segmented = false)
{
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x >> 6, NW = blockDim.x >> 6;
    const double KU = (double)J.K * (double)J.U;
    const int M = J.m_cand;
    Real* r = LDS ? (Real*)lds : (Real*)J.r;
    // segmented (global residual only): the chain state comes from the carry
    // and the chain returns when a resync is due, which then runs grid-wide
    ChainState cs = segmented ? load_carry(J) : chain_setup<Real, !LDS, LenT>(J, r, sh, lane, wave, NW);
    Schedule sched;
    sched.start(cs.s_begin, cs.n_steps, J.n_stages, cs.T0, cs.TN, J.schedule);
    const bool f32 = sizeof(Real) == 4;
    const LenT* lenp = (const LenT*)J.len;

    // The wavefront's estimates are m = wave + k NW.  Those with k < KA have
    // their draws one step ahead: the support lookup is issued at the start
    // of the step before, the row offsets after that step's sums, so both
    // loads are in flight while the step runs.  Further estimates (M > KA NW)
    // are drawn at their step.  Estimates are scored two at a time, their
    // rows' loads interleaved; each lane still adds each row's entries in
    // ascending order, so the sums are the canonical ones.
    constexpr int KA = 2;
    constexpr int U = 8;  // entries per lane and row in flight
    const int KM = (M + NW - 1) / NW;
    int32_t dp[KA];
    int64_t db[KA], de[KA];
    double ddel[KA];
    auto draw = [&](int64_t st, int m, double* delta) -> int32_t {
        const Words4 w = philox4x64(J.seed, J.chain_id, (uint64_t)st, (uint64_t)m, 0, 0);
        *delta = J.delta_max * (2.0 * unit53(w.w1) - 1.0);
        return J.support[__umul64hi(w.w0, (uint64_t)J.P)];
    };
#pragma unroll
    for (int k = 0; k < KA; ++k) {
        const int m = wave + k * NW;
        dp[k] = 0;
        db[k] = de[k] = 0;
        ddel[k] = 0.0;
        if (m < M && cs.s_begin < cs.n_steps) {
            dp[k] = draw(cs.s_begin, m, &ddel[k]);
            db[k] = J.row_ptr[dp[k]];
            de[k] = J.row_ptr[dp[k] + 1];
        }
    }
    // the value an estimate proposes for pixel p: the change drawn for it,
    // clamped, or redrawn until in range (Eq. 3)
    auto propose = [&](int64_t st, int m, int32_t p, double delta, double* fn_out) -> double {
        const double fo = J.f[p];
        double fn = fo + delta;
        if (J.proposal == PILA_PROP_REDRAW) {
            for (uint64_t j = 1; (fn < J.f_min || fn > J.f_max) && j <= kRedrawMax; ++j) {
                delta = J.delta_max *
                        (2.0 * unit53(philox4x64(J.seed, J.chain_id, (uint64_t)st, (uint64_t)m, 0, j).w1) - 1.0);
                fn = fo + delta;
            }
            if (fn < J.f_min || fn > J.f_max) fn = fo;
        } else {
            if (fn < J.f_min) fn = J.f_min;
            if (fn > J.f_max) fn = J.f_max;
        }
        *fn_out = fn;
        return fn - fo;
    };

    for (int64_t s = cs.s_begin; s < cs.n_steps; ++s) {
        const double T = sched.at(s, cs.n_steps, J.n_stages);
        // next step's support lookups, in flight during this step
        int32_t np[KA];
        double ndel[KA];
#pragma unroll
        for (int k = 0; k < KA; ++k) {
            const int m = wave + k * NW;
            np[k] = 0;
            ndel[k] = 0.0;
            if (m < M && s + 1 < cs.n_steps) np[k] = draw(s + 1, m, &ndel[k]);
        }
        for (int k0 = 0; k0 < KM; k0 += 2) {
            int32_t pp[2];
            int64_t bb[2], ee[2];
            double fnn[2], dd[2];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int k = k0 + h, m = wave + k * NW;
                pp[h] = 0;
                bb[h] = ee[h] = 0;
                fnn[h] = dd[h] = 0.0;
                if (m < M) {
                    double delta;
                    if (k < KA) {
                        pp[h] = k == 0 ? dp[0] : dp[1];
                        bb[h] = k == 0 ? db[0] : db[1];
                        ee[h] = k == 0 ? de[0] : de[1];
                        delta = k == 0 ? ddel[0] : ddel[1];
                    } else {
                        pp[h] = draw(s, m, &delta);
                        bb[h] = J.row_ptr[pp[h]];
                        ee[h] = J.row_ptr[pp[h] + 1];
                    }
                    dd[h] = propose(s, m, pp[h], delta, &fnn[h]);
                }
            }
            const Real dra = (Real)dd[0], drb = (Real)dd[1];
            const int64_t la = ee[0] - bb[0], lb = ee[1] - bb[1];
            const int64_t lmax = la > lb ? la : lb;
            Real acca = 0, accb = 0;
            for (int64_t o = lane; o < lmax; o += (int64_t)kWave * U) {
                int32_t ca[U], cb[U];
                Real la_[U], lb_[U];
#pragma unroll
                for (int c = 0; c < U; ++c) {
                    const int64_t qa = bb[0] + (o + c * kWave < la ? o + c * kWave : 0);
                    const int64_t qb = bb[1] + (o + c * kWave < lb ? o + c * kWave : 0);
                    ca[c] = J.col[qa];
                    la_[c] = (Real)lenp[qa];
                    cb[c] = J.col[qb];
                    lb_[c] = (Real)lenp[qb];
                }
                Real ra[U], rb[U];
#pragma unroll
                for (int c = 0; c < U; ++c) {
                    ra[c] = r[ridx<!LDS>(J, ca[c])];
                    rb[c] = r[ridx<!LDS>(J, cb[c])];
                }
#pragma unroll
                for (int c = 0; c < U; ++c) {
                    if (o + c * kWave < la) {
                        const Real t = dra * la_[c];
                        acca = fma(t, (Real)2 * ra[c] + t, acca);
                    }
                }
#pragma unroll
                for (int c = 0; c < U; ++c) {
                    if (o + c * kWave < lb) {
                        const Real t = drb * lb_[c];
                        accb = fma(t, (Real)2 * rb[c] + t, accb);
                    }
                }
            }
            const Real Sa = wave_canon_sum(acca), Sb = wave_canon_sum(accb);
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int m = wave + (k0 + h) * NW;
                if (lane == 0 && m < M) {
                    sh.S[m] = (double)(h == 0 ? Sa : Sb);
                    sh.p[m] = pp[h];
                    sh.fn[m] = fnn[h];
                    sh.d[m] = dd[h];
                    sh.rb[m] = bb[h];
                    sh.re[m] = ee[h];
                }
            }
        }
        // next step's row offsets, in flight during the decision and scatter
#pragma unroll
        for (int k = 0; k < KA; ++k) {
            const int m = wave + k * NW;
            if (m < M && s + 1 < cs.n_steps) {
                dp[k] = np[k];
                ddel[k] = ndel[k];
                db[k] = J.row_ptr[np[k]];
                de[k] = J.row_ptr[np[k] + 1];
            }
        }
        const double co = sqrt(cs.sse / KU);
        const double N1 = unit53(philox4x64(J.seed, J.chain_id, (uint64_t)s, 0, 1, 0).w0);
        const double lnN1 = log(N1), invT = 1.0 / T;
        cancel_probe(J, sh, s);
        __syncthreads();
        const Decision dn = decide(sh.S, M, lane, cs.sse, co, KU, T, invT, N1, lnN1);
        const double d_star = uniform_f64(sh.d[dn.ms]);
        // Eq. 6 for the winner, by the whole workgroup (one entry per thread;
        // the row's rays are distinct, so no two threads touch one value); an
        // accepted zero change leaves image and residual as they are
        if (dn.accept && d_star != 0.0) {
            const int64_t b = sh.rb[dn.ms], e = sh.re[dn.ms];
            const Real dr = (Real)d_star;
            for (int64_t q = b + threadIdx.x; q < e; q += blockDim.x) {
                const uint32_t at = ridx<!LDS>(J, J.col[q]);
                r[at] = r[at] + dr * (Real)lenp[q];
            }
            if (threadIdx.x == 0) J.f[sh.p[dn.ms]] = sh.fn[dn.ms];
        }
        count_decision(J, cs, dn, d_star, s);
        if (f32 && J.resync_every > 0 && cs.since >= J.resync_every) {
            if (!LDS && segmented) {
                __syncthreads();
                save_carry(J, cs, s + 1, true);
                return;
            }
            resync_in_group<Real, !LDS, LenT>(J, cs, r, sh, lane, wave, NW);
        }
        __syncthreads();
        if (cancel_seen(J, sh, s)) {
            cs.status = PILA_ECANCELED;
            cs.n_steps = s + 1;
            break;
        }
    }
    if (segmented) {
        save_carry(J, cs, cs.n_steps, false);
        return;
    }
    write_stats(J, cs);
}

// ---------------------------------------------------------------------------
// split: one chain over G workgroups (one compute unit each).  With long rows
// and many estimates a step gathers tens of thousands of residual values,
// one address per lane, and one CU's texture path (one divergent address per
// clock) bounds it; G workgroups each score M / G of the estimates.
//
// Workgroup g scores the estimates m with m mod G == g against its own copy
// of the residual and of the image (group 0 holds the chain's own arrays)
// and publishes each sum; every workgroup then holds all M sums, takes the
// same BoME / Metropolis decision (the same arithmetic on the same values)
// and applies an accepted change to its own copies, so the copies stay equal
// bit for bit and no residual or image value crosses between compute units.
//
// A sum travels as two 64-bit words, each holding a step stamp in its upper
// half and one half of the sum's bits in its lower half, stored and polled
// with relaxed device-scope atomics: each word says by itself which step it
// belongs to, so the two words need no ordering between them.  The words
// are double-buffered by step parity; a workgroup is never more than one
// step ahead of another (it needs the other's sums of the step before), so
// the buffer it writes holds no sums another workgroup still waits for.
// Every wait is bounded by the wall clock: a workgroup that gives up ends the
// chain with PILA_ETIMEDOUT (the others then give up on it in turn).
//
// The estimates' pixels, changes and row offsets do not depend on the chain
// state: wavefront 0 draws all M of them one step ahead (one lane each), the
// image value with them, patched when the step in between changes that
// pixel, so the scoring wavefronts read them from LDS; each wavefront loads
// the first chunk of its next row (indices and lengths) after the decision,
// while the accepted change is applied.  Sums are the canonical ones (one
// wavefront per estimate, U entries per lane in flight).
// The chain state comes from the carry (segments end at FP32 resyncs, which
// run grid-wide on group 0's copy and are then copied to the others).
// ---------------------------------------------------------------------------
struct SplitX {
    unsigned long long* word;  // [2 parities][kMaxCand][2 halves]
    char* copies;              // groups 1 .. G-1: residual copy (r_bytes), then image copy (f_bytes)
    int64_t r_bytes, f_bytes;
    int64_t wait_ticks;        // wall-clock ticks (pila_device_info.wallclock_khz) a wait may last
    int32_t groups, pad;
};

struct SplitShared {
    ChainShared c;
    int64_t rb[2][kMaxCand], re[2][kMaxCand];
    double fn[2][kMaxCand], d[2][kMaxCand];
    int32_t p[2][kMaxCand];
    int32_t fail;
};

// stamp of step s in a word: 1 .. 2^31, never the 0 of a cleared word, and
// steps two apart (one parity buffer) always differ
__device__ __forceinline__ uint64_t split_stamp(int64_t s)
{
    return (uint64_t)((s & 0x7fffffff) + 1) << 32;
}

__device__ __forceinline__ unsigned long long* split_word(const SplitX& X, int64_t s, int m)
{
    return X.word + ((size_t)(s & 1) * kMaxCand + (size_t)m) * 2;
}

__device__ __forceinline__ void split_publish(const SplitX& X, int64_t s, int m, double S)
{
    const uint64_t bits = (uint64_t)__double_as_longlong(S), st = split_stamp(s);
    unsigned long long* w = split_word(X, s, m);
    __hip_atomic_store(w, st | (bits >> 32), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(w + 1, st | (bits & 0xffffffffull), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <typename Real, typename LenT = Real>
__device__ void run_chain_split(const ChainJob& J, const SplitX& X, int g, SplitShared& sp)
{
    ChainShared& sh = sp.c;
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x >> 6, NW = blockDim.x >> 6;
    const int G = X.groups;
    const double KU = (double)J.K * (double)J.U;
    const int M = J.m_cand;
    Real* r = (Real*)J.r;
    const LenT* lenp = (const LenT*)J.len;
    const bool f32 = sizeof(Real) == 4;
    ChainState cs = load_carry(J);
    Schedule sched;
    sched.start(cs.s_begin, cs.n_steps, J.n_stages, cs.T0, cs.TN, J.schedule);

    auto draw = [&](int64_t st, int m, double* delta) -> int32_t {
        const Words4 w = philox4x64(J.seed, J.chain_id, (uint64_t)st, (uint64_t)m, 0, 0);
        *delta = J.delta_max * (2.0 * unit53(w.w1) - 1.0);
        return J.support[__umul64hi(w.w0, (uint64_t)J.P)];
    };
    // the value estimate m proposes at step st for a pixel now holding fo:
    // the drawn change clamped, or redrawn until in range (Eq. 3)
    auto propose = [&](int64_t st, int m, double fo, double delta) -> double {
        double fn = fo + delta;
        if (J.proposal == PILA_PROP_REDRAW) {
            for (uint64_t j = 1; (fn < J.f_min || fn > J.f_max) && j <= kRedrawMax; ++j) {
                delta = J.delta_max *
                        (2.0 * unit53(philox4x64(J.seed, J.chain_id, (uint64_t)st, (uint64_t)m, 0, j).w1) - 1.0);
                fn = fo + delta;
            }
            if (fn < J.f_min || fn > J.f_max) fn = fo;
        } else {
            if (fn < J.f_min) fn = J.f_min;
            if (fn > J.f_max) fn = J.f_max;
        }
        return fn;
    };
    // wavefront 0, lane m: estimate m of step st into LDS buffer st mod 2
    const bool book = wave == 0 && lane < M;
    if (book && cs.s_begin < cs.n_steps) {
        const int64_t st = cs.s_begin;
        double delta;
        const int32_t p = draw(st, lane, &delta);
        const double fo = J.f[p];
        const double fn = propose(st, lane, fo, delta);
        const int b = (int)(st & 1);
        sp.p[b][lane] = p;
        sp.fn[b][lane] = fn;
        sp.d[b][lane] = fn - fo;
        sp.rb[b][lane] = J.row_ptr[p];
        sp.re[b][lane] = J.row_ptr[p + 1];
    }
    if (threadIdx.x == 0) sp.fail = 0;
    __syncthreads();

    // Each wavefront's first estimate of a step has the first U entries per
    // lane of its row (indices and lengths) loaded during the step before,
    // while that step's change is applied; further chunks and estimates are
    // read at the step.
    constexpr int U = 16;
    const int m1 = g + G * wave;  // the wavefront's first estimate
    auto row_chunk = [&](int64_t b, int64_t len, int32_t* cc, Real* ll) {
#pragma unroll
        for (int c = 0; c < U; ++c) {
            const int64_t q = lane + c * kWave < len ? b + lane + c * kWave : 0;
            cc[c] = J.col[q];
            ll[c] = (Real)lenp[q];
        }
    };
    int32_t pc[U];
    Real pl[U];
    if (m1 < M && cs.s_begin < cs.n_steps) {
        const int64_t rb = uniform_i64(sp.rb[cs.s_begin & 1][m1]);
        row_chunk(rb, uniform_i64(sp.re[cs.s_begin & 1][m1]) - rb, pc, pl);
    }
    for (int64_t s = cs.s_begin; s < cs.n_steps; ++s) {
        const int pb = (int)(s & 1);
        const double T = sched.at(s, cs.n_steps, J.n_stages);
        const bool more = s + 1 < cs.n_steps;
        // step s + 1's draws; the support lookups are in flight while this
        // step's rows are scored
        int32_t np = 0;
        double ndel = 0.0;
        if (book && more) np = draw(s + 1, lane, &ndel);
        // this workgroup's estimates: the wavefront's first one from the
        // prefetched chunk, then its other chunks and estimates
        auto score = [&](int m, bool first) {
            const int64_t b = uniform_i64(sp.rb[pb][m]), len = uniform_i64(sp.re[pb][m]) - b;
            const Real dr = (Real)uniform_f64(sp.d[pb][m]);
            Real acc = 0;
            int64_t o = 0;
            if (first) {
                Real rr[U];
#pragma unroll
                for (int c = 0; c < U; ++c) rr[c] = r[rpos_g(J, pc[c])];
#pragma unroll
                for (int c = 0; c < U; ++c) {
                    if (lane + c * kWave < len) {
                        const Real t = dr * pl[c];
                        acc = fma(t, (Real)2 * rr[c] + t, acc);
                    }
                }
                o = (int64_t)kWave * U;
            }
            for (; o < len; o += (int64_t)kWave * U) {
                int32_t cc[U];
                Real ll[U];
                row_chunk(b + o, len - o, cc, ll);
                Real rr[U];
#pragma unroll
                for (int c = 0; c < U; ++c) rr[c] = r[rpos_g(J, cc[c])];
#pragma unroll
                for (int c = 0; c < U; ++c) {
                    if (o + lane + c * kWave < len) {
                        const Real t = dr * ll[c];
                        acc = fma(t, (Real)2 * rr[c] + t, acc);
                    }
                }
            }
            const double S = (double)wave_canon_sum(acc);
            if (lane == 0) {
                sh.S[m] = S;
                split_publish(X, s, m, S);
            }
        };
        if (m1 < M) score(m1, true);
        for (int j = wave + NW;; j += NW) {
            const int m = g + G * j;
            if (m >= M) break;
            score(m, false);
        }
        // step s + 1's row offsets and image values, in flight during the
        // exchange; then the other workgroups' sums
        int64_t nb = 0, ne = 0;
        double nfo = 0.0;
        if (book && more) {
            nb = J.row_ptr[np];
            ne = J.row_ptr[np + 1];
            nfo = J.f[np];
        }
        const double co = sqrt(cs.sse / KU);
        const double N1 = unit53(philox4x64(J.seed, J.chain_id, (uint64_t)s, 0, 1, 0).w0);
        const double lnN1 = log(N1), invT = 1.0 / T;
        if (wave == 0) {
            bool need = lane < M && lane % G != g;
            const uint64_t want = split_stamp(s);
            const uint64_t t0 = wall_clock64();
            while (__ballot(need) != 0) {
                if (need) {
                    unsigned long long* w = split_word(X, s, lane);
                    const uint64_t hi = __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    const uint64_t lo = __hip_atomic_load(w + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    if ((hi & ~0xffffffffull) == want && (lo & ~0xffffffffull) == want) {
                        sh.S[lane] = __longlong_as_double((long long)((hi << 32) | (lo & 0xffffffffull)));
                        need = false;
                    }
                }
                if ((int64_t)(wall_clock64() - t0) > X.wait_ticks) {
                    if (lane == 0) sp.fail = 1;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
        }
        if (book && more) {
            sp.p[pb ^ 1][lane] = np;
            sp.rb[pb ^ 1][lane] = nb;
            sp.re[pb ^ 1][lane] = ne;
        }
        __syncthreads();
        if (sp.fail) {
            cs.status = PILA_ETIMEDOUT;
            cs.n_steps = 0;
            break;
        }
        // step s + 1's first chunk, in flight while this step's change is
        // applied
        int32_t qc[U];
        Real ql[U];
        if (m1 < M && more) {
            const int64_t rb = uniform_i64(sp.rb[pb ^ 1][m1]);
            row_chunk(rb, uniform_i64(sp.re[pb ^ 1][m1]) - rb, qc, ql);
        }
        const Decision dn = decide(sh.S, M, lane, cs.sse, co, KU, T, invT, N1, lnN1);
        const double d_star = uniform_f64(sp.d[pb][dn.ms]);
        const bool change = dn.accept && d_star != 0.0;
        int32_t pstar = 0;
        double fnstar = 0.0;
        // Eq. 6 on this workgroup's copies, up to kSc entries per thread at
        // once: all their loads, then all their stores (a row's rays are
        // distinct, so the entries do not alias)
        if (change) {
            const int64_t b = uniform_i64(sp.rb[pb][dn.ms]), e = uniform_i64(sp.re[pb][dn.ms]);
            const Real dr = (Real)d_star;
            constexpr int kSc = 8;
            const int64_t nt = blockDim.x;
            for (int64_t q0 = b + threadIdx.x; q0 < e; q0 += nt * kSc) {
                uint32_t at[kSc];
                Real lv[kSc], rv[kSc];
#pragma unroll
                for (int k = 0; k < kSc; ++k) {
                    const int64_t q = q0 + k * nt < e ? q0 + k * nt : q0;
                    at[k] = rpos_g(J, J.col[q]);
                    lv[k] = (Real)lenp[q];
                }
#pragma unroll
                for (int k = 0; k < kSc; ++k) rv[k] = r[at[k]];
#pragma unroll
                for (int k = 0; k < kSc; ++k)
                    if (q0 + k * nt < e) r[at[k]] = rv[k] + dr * lv[k];
            }
            pstar = uniform_i32(sp.p[pb][dn.ms]);
            fnstar = uniform_f64(sp.fn[pb][dn.ms]);
            if (threadIdx.x == 0) J.f[pstar] = fnstar;
        }
        count_decision(J, cs, dn, d_star, s);
        // step s + 1's estimates: the image value read before this step's
        // change, patched with it
        if (book && more) {
            const double fo = change && np == pstar ? fnstar : nfo;
            const double fn = propose(s + 1, lane, fo, ndel);
            sp.fn[pb ^ 1][lane] = fn;
            sp.d[pb ^ 1][lane] = fn - fo;
        }
#pragma unroll
        for (int c = 0; c < U; ++c) {
            pc[c] = qc[c];
            pl[c] = ql[c];
        }
        if (f32 && J.resync_every > 0 && cs.since >= J.resync_every) {
            __syncthreads();
            if (g == 0) save_carry(J, cs, s + 1, true);
            return;
        }
        __syncthreads();
    }
    if (g == 0) save_carry(J, cs, cs.n_steps, false);
}

// ---------------------------------------------------------------------------
// pipelined: rows in registers two steps ahead, operands one step ahead
// ---------------------------------------------------------------------------
// element i of a global array through a 32-bit byte offset from a uniform
// base (one address register per load); the host keeps every such array
// below 4 GiB
template <typename T>
__device__ __forceinline__ T ld32(const T* base, uint32_t i)
{
    return *(const T*)((const char*)base + i * (uint32_t)sizeof(T));
}
template <typename T>
__device__ __forceinline__ void st32(T* base, uint32_t i, T v)
{
    *(T*)((char*)base + i * (uint32_t)sizeof(T)) = v;
}

// A length loaded a step or two before it is used: FP32 lengths as they are;
// one-byte lengths as the raw byte in the register's bits, read back (q/180,
// an ALU operation on the loaded value, len_use) once the load has arrived,
// so that nothing waits for it when it is issued.
template <typename Real, typename LenT>
__device__ __forceinline__ Real len_hold(const LenT* lenp, uint32_t at)
{
    if constexpr (std::is_same<LenT, LenQ>::value && std::is_same<Real, float>::value)
        return __uint_as_float((uint32_t)ld32((const uint8_t*)lenp, at));
    else
        return (Real)ld32(lenp, at);
}
template <typename Real, typename LenT>
__device__ __forceinline__ Real len_use(Real v)
{
    if constexpr (std::is_same<LenT, LenQ>::value && std::is_same<Real, float>::value) {
        LenQ q;
        q.q = (uint8_t)__float_as_uint(v);
        return (Real)(float)q;
    } else {
        return v;
    }
}

// Where the residual value of ray g lives in the pipelined body's global
// mode: the LDS part (angles u < UL, bins k_lo .. k_lo + Kc - 1) as
// kRaySlotLds | index, else u << 22 | its position in the tiled global
// residual (rpos, below 2^22 for U <= 512 and K < 8192).  The patch-table
// slot of a global entry is 2 u + k mod 2, and k mod 2 is the position's
// lowest bit, so both come from the word with a few bit operations.
constexpr int kRaySlotLds = (int)0x80000000;
constexpr int kSlotPosBits = 22;
constexpr int32_t kSlotPosMask = (1 << kSlotPosBits) - 1;
constexpr int kSlotMaxAngles = 512;

__device__ __forceinline__ int32_t ray_slot(const ChainJob& J, int32_t g)
{
    const int u = (int)(((uint64_t)(uint32_t)g * J.kdiv_m) >> J.kdiv_s);  // g / K, g < 2^24
    const int k = g - u * J.K;
    const int kk = k - J.k_lo;
    if (u < J.UL && kk >= 0 && kk < J.Kc) return kRaySlotLds | (u * J.Kc + kk);
    return (u << kSlotPosBits) | (int32_t)rpos(J, u, k);
}

// patch-table slot (2 u + k mod 2) of a global entry's slot word
__device__ __forceinline__ int slot_patch(int32_t tk)
{
    return ((tk >> (kSlotPosBits - 1)) & ~1) | (tk & 1);
}

template <typename Real, int E>
struct RowSet {
    int32_t col[E];
    Real len[E];
    int32_t tk[E];  // where each ray's residual lives: LDS index (flagged) or patch slot
    Real rv[E];     // residual values of the row's rays
    double fo;      // image value of the pixel
    int32_t p, n;   // pixel, row length
    double delta;   // proposed change before the clamp
    double N1;      // acceptance uniform of the step
    double lnN1;
};

struct Draws {  // one block of steps: lane j <-> (step j / CPW, estimate slot j % CPW)
    int64_t base;
    uint32_t b;
    int32_t p, n;
    double delta, N1, lnN1;
};

// LDS part of the residual (global mode): angles u < UL, bins k_lo ..
// k_lo + Kc - 1, stored densely; the rest of the residual stays in global
// memory.  Loaded after every rebuild, written back before every rebuild
// and at the end so the global copy is complete whenever it is read whole.
template <typename Real>
__device__ void lds_residual_load(const ChainJob& J, const Real* r, Real* rl)
{
    const int n = J.UL * J.Kc;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const int u = i / J.Kc, k = J.k_lo + i % J.Kc;
        rl[i] = r[rpos(J, u, k)];
    }
}
template <typename Real>
__device__ void lds_residual_store(const ChainJob& J, Real* r, const Real* rl)
{
    const int n = J.UL * J.Kc;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const int u = i / J.Kc, k = J.k_lo + i % J.Kc;
        r[rpos(J, u, k)] = rl[i];
    }
}

// TK: the rows' slot words come precomputed from J.tcol (loaded instead of
// the ray indices, which are formed back from them where a global residual
// value is read or written)
// LATE: one-byte lengths are held raw and read back where used (lone
// chains: reading them back at the load made the step wait for it);
// otherwise at the load (batches, where the compiler places that better).
// Either way the same float results.
template <typename Real, bool RLDS, int CPW, int E, bool SERVED = false, bool TK = false, typename LenT = Real,
          bool LATE = false>
__device__ void run_chain_piped(const ChainJob& J, char* lds, ChainShared& sh, bool segmented)
{
    constexpr int LPC = kWave / CPW;  // lanes per estimate
    constexpr int BL = kWave / CPW;   // steps per block of draws
    constexpr int kLdsFlag = kRaySlotLds;
    constexpr bool kTK = TK && !RLDS;
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x >> 6, NW = blockDim.x >> 6;
    const int slot = lane / LPC, li = lane % LPC;
    const double KU = (double)J.K * (double)J.U;
    const int M = J.m_cand;
    const int m_mine = wave * CPW + slot;
    const bool active = m_mine < M;
    // RLDS: the whole residual lives in LDS.  Otherwise the residual is in
    // global memory except angles u < UL, which live in LDS (rl); rvB holds
    // the global values one step ahead and the table of the last accepted
    // row's new global values patches them.
    Real* r = RLDS ? (Real*)lds : (Real*)J.r;
    int64_t* pkey = (int64_t*)lds;
    Real* pval = (Real*)(lds + 16 * (size_t)J.U);
    Real* rl = (Real*)(lds + ((16 * (size_t)J.U + 2 * sizeof(Real) * (size_t)J.U + 15) & ~(size_t)15));
    const LenT* lenp = (const LenT*)J.len;

    ChainState cs = segmented ? load_carry(J) : chain_setup<Real, !RLDS, LenT>(J, r, sh, lane, wave, NW);
    const int64_t n_steps = cs.n_steps;
    const int64_t s_begin = cs.s_begin;
    if (!RLDS) {
        for (int q = threadIdx.x; q < 2 * J.U; q += blockDim.x) pkey[q] = -1;
        lds_residual_load<Real>(J, r, rl);
    }
    Schedule sched;
    sched.start(s_begin, n_steps, J.n_stages, cs.T0, cs.TN, J.schedule);

    Draws cur, nxt;
    auto fill = [&](Draws& D, int64_t base) {
        D.base = base;
        const int64_t s = base + lane / CPW;
        const int m = wave * CPW + lane % CPW;
        D.p = 0;
        D.n = 0;
        D.b = 0;
        D.delta = 0.0;
        D.N1 = 0.0;
        D.lnN1 = 0.0;
        // the key is made opaque here, so that the round keys are formed per
        // block instead of being held in scalar registers across the loop
        uint64_t k0 = lane0(J.seed), k1 = lane0(J.chain_id);
        asm volatile("" : "+s"(k0), "+s"(k1));
        if (s < n_steps) {
            if (m < M) {
                const Words4 w = philox4x64(k0, k1, (uint64_t)s, (uint64_t)m, 0, 0);
                D.p = J.support[__umul64hi(w.w0, (uint64_t)J.P)];
                D.delta = J.delta_max * (2.0 * unit53(w.w1) - 1.0);
                const int64_t b0 = J.row_ptr[D.p];
                D.b = (uint32_t)b0;
                D.n = (int32_t)(J.row_ptr[D.p + 1] - b0);
            }
            if (lane % CPW == 0) {
                D.N1 = unit53(philox4x64(k0, k1, (uint64_t)s, 0, 1, 0).w0);
                D.lnN1 = log(D.N1);
            }
        }
    };
    cur.base = nxt.base = -1;

    auto prefetch = [&](RowSet<Real, E>& S, int64_t t) {
        if (t >= n_steps) {
            S.p = 0;
            S.n = 0;
            S.delta = 0.0;
            S.N1 = 0.0;
            S.lnN1 = 0.0;
#pragma unroll
            for (int e = 0; e < E; ++e) {
                S.col[e] = 0;
                S.len[e] = (Real)0;
                S.tk[e] = 0;
            }
            return;
        }
        const int64_t base = t - t % BL;
        if (cur.base != base) {
            if (nxt.base == base)
                cur = nxt;
            else
                fill(cur, base);
        }
        const int j = (int)(t - base);
        if (j == BL / 2 && base + BL < n_steps) fill(nxt, base + BL);  // next block, early
        const int src = j * CPW + slot;
        S.p = __shfl(cur.p, src, kWave);
        S.n = __shfl(cur.n, src, kWave);
        const uint32_t b = (uint32_t)__shfl((int)cur.b, src, kWave);
        S.delta = __shfl(cur.delta, src, kWave);
        S.N1 = __shfl(cur.N1, j * CPW, kWave);
        S.lnN1 = __shfl(cur.lnN1, j * CPW, kWave);
        // loads are unconditional (entries past the row read entry 0) so that
        // nothing waits for them here; validity is tested where they are used
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int q = li + e * LPC;
            const uint32_t at = q < S.n ? b + (uint32_t)q : 0u;
            if (kTK)
                S.tk[e] = ld32(J.tcol, at);
            else
                S.col[e] = ld32(J.col, at);
            S.len[e] = LATE ? len_hold<Real, LenT>(lenp, at) : (Real)ld32(lenp, at);
        }
    };
    // where each ray of a row lives: LDS index (flagged) or patch-table slot
    auto table_slots = [&](RowSet<Real, E>& S) {
        if (RLDS || kTK) return;
#pragma unroll
        for (int e = 0; e < E; ++e) S.tk[e] = ray_slot(J, S.col[e]);
    };
    // position of entry e's ray in the residual: in LDS (RLDS) its index; in
    // the global residual (outside the LDS part) its tile position, from the
    // angle and bin of its slot word or from the ray index
    auto gcol = [&](const RowSet<Real, E>& S, int e) -> uint32_t {
        if (RLDS) return (uint32_t)S.col[e];
        return (uint32_t)(S.tk[e] & kSlotPosMask);
    };
    auto in_lds = [&](int tk) { return !RLDS && (tk & kLdsFlag) != 0; };
    // residual value at a position of the global residual, or of ray g in LDS
    auto rget = [&](uint32_t g) -> Real { return RLDS ? r[g] : ld32((const Real*)r, g); };
    auto lenv = [&](Real v) -> Real {
        if constexpr (LATE) return len_use<Real, LenT>(v);
        return v;
    };

    RowSet<Real, E> A, B, C;
    prefetch(A, s_begin);
    prefetch(B, s_begin + 1);
    __syncthreads();  // setup (residual, LDS part, temperatures, patch table) complete
    table_slots(A);
#pragma unroll
    for (int e = 0; e < E; ++e) A.rv[e] = in_lds(A.tk[e]) ? rl[A.tk[e] & ~kLdsFlag] : rget(gcol(A, e));
    A.fo = J.f[A.p];
    bool patch = false;     // apply the table of step s - 1 to X.rv
    int32_t lp = -1;        // last accepted pixel (step s - 1) and its value
    double lfn = 0.0;

    // One step with X the estimates of step s, Y those of s + 1 (their
    // global operands are loaded here) and Z those of s + 2 (rows loaded
    // here).  The loop below rotates the roles, so no registers are copied.
    // Returns true when the chain stops here: a segmented chain for a
    // resync, or a served chain that has been cancelled (then cancelled is set).
    bool cancelled = false;
    double co = sqrt(cs.sse / KU);  // C of Eq. 4 before the step
    auto step = [&](RowSet<Real, E>& X, RowSet<Real, E>& Y, RowSet<Real, E>& Z, int64_t s)
                    __attribute__((always_inline)) -> bool {
        const double T = sched.at(s, n_steps, J.n_stages);
        const double invT = sched.invT;
        // next step's global operands, issued before this step is scored so
        // that they have the whole step to arrive (the residual already holds
        // step s - 1's change; step s's is patched in at step s + 1); every
        // entry is written, so the set's values of two steps ago die here
        table_slots(Y);
        if (!RLDS) {
#pragma unroll
            for (int e = 0; e < E; ++e) {
                Y.rv[e] = (Real)0;
                if (!(Y.tk[e] & kLdsFlag)) Y.rv[e] = rget(gcol(Y, e));
            }
        }
        Y.fo = J.f[Y.p];
        if (!RLDS && patch) {  // the previous step's accepted change
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int tk = X.tk[e];
                if (!(tk & kLdsFlag)) {
                    const int ps = slot_patch(tk);
                    const int64_t key = pkey[ps];
                    if (key == (((int64_t)(s - 1)) << kSlotPosBits | (tk & kSlotPosMask))) X.rv[e] = pval[ps];
                }
            }
        }
        if (X.p == lp) X.fo = lfn;
        double fn = X.fo + X.delta;
        if (fn < J.f_min) fn = J.f_min;
        if (fn > J.f_max) fn = J.f_max;
        const double d = fn - X.fo;
        const Real dr = (Real)d;
        Real part[CPW];
#pragma unroll
        for (int k = 0; k < CPW; ++k) part[k] = (Real)0;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const Real t = (li + e * LPC < X.n) ? dr * lenv(X.len[e]) : (Real)0;
            part[e % CPW] = fma(t, (Real)2 * X.rv[e] + t, part[e % CPW]);
        }
        const Real S = canon_sum<LPC>(part);
        if (active && li == 0) {
            sh.S[m_mine] = (double)S;
            sh.d[m_mine] = d;
        }
        // the rows of step s + 2
        prefetch(Z, s + 2);
        if (SERVED) cancel_probe(J, sh, s);
        __syncthreads();
        const Decision dn = decide(sh.S, M, lane, cs.sse, co, KU, T, invT, X.N1, X.lnN1);
        const double d_star = uniform_f64(sh.d[dn.ms]);
        // an accepted zero change leaves image and residual as they are
        const bool changed = dn.accept && d_star != 0.0;
        if (changed && dn.ms == m_mine) {  // the owner of the winner applies Eq. 6
#pragma unroll
            for (int e = 0; e < E; ++e) {
                if (li + e * LPC < X.n) {
                    const Real rn = X.rv[e] + dr * lenv(X.len[e]);
                    if (RLDS) {
                        r[X.col[e]] = rn;
                    } else if (X.tk[e] & kLdsFlag) {
                        rl[X.tk[e] & ~kLdsFlag] = rn;
                    } else {
                        st32(r, gcol(X, e), rn);
                        const int ps = slot_patch(X.tk[e]);
                        pkey[ps] = ((int64_t)s << kSlotPosBits) | (X.tk[e] & kSlotPosMask);
                        pval[ps] = rn;
                    }
                }
            }
            if (li == 0) {
                J.f[X.p] = fn;
                sh.pstar = X.p;
                sh.fnstar = fn;
            }
        }
        count_decision(J, cs, dn, d_star, s);
        if (dn.accept && dn.S != 0.0) co = sqrt(cs.sse / KU);  // C of Eq. 4 only moves with the SSE
        if (sizeof(Real) == 4 && J.resync_every > 0 && cs.since >= J.resync_every) {
            if (!RLDS) {
                __syncthreads();
                lds_residual_store<Real>(J, r, rl);
            }
            if (segmented) {  // the FP64 rebuild runs grid-wide between launches
                save_carry(J, cs, s + 1, true);
                return true;
            }
            resync_in_group<Real, !RLDS, LenT>(J, cs, r, sh, lane, wave, NW);
            co = sqrt(cs.sse / KU);
            if (!RLDS) lds_residual_load<Real>(J, r, rl);
            // the next two sets are drawn again after the rebuild, so that no
            // row stays in registers across it
            prefetch(Y, s + 1);
            prefetch(Z, s + 2);
            table_slots(Y);
            __syncthreads();
#pragma unroll
            for (int e = 0; e < E; ++e) Y.rv[e] = in_lds(Y.tk[e]) ? rl[Y.tk[e] & ~kLdsFlag] : rget(gcol(Y, e));
            Y.fo = J.f[Y.p];
            lp = -1;
            patch = false;
            return false;
        }
        __syncthreads();
        if (changed) {
            lp = uniform_i32(sh.pstar);
            lfn = uniform_f64(sh.fnstar);
        } else {
            lp = -1;
        }
        patch = changed;
        // operands of step s + 1 that live in LDS
#pragma unroll
        for (int e = 0; e < E; ++e) {
            if (in_lds(Y.tk[e]))
                Y.rv[e] = rl[Y.tk[e] & ~kLdsFlag];
            else if (RLDS)
                Y.rv[e] = rget((uint32_t)Y.col[e]);
        }
        if (SERVED && cancel_seen(J, sh, s)) {
            cs.status = PILA_ECANCELED;
            cs.n_steps = s + 1;
            cancelled = true;
            return true;
        }
        return false;
    };

    for (int64_t s = s_begin; s < n_steps;) {
        if (step(A, B, C, s)) {
            if (SERVED && cancelled) break;
            return;
        }
        if (++s >= n_steps) break;
        if (step(B, C, A, s)) {
            if (SERVED && cancelled) break;
            return;
        }
        if (++s >= n_steps) break;
        if (step(C, A, B, s)) {
            if (SERVED && cancelled) break;
            return;
        }
        ++s;
    }
    if (!RLDS) {
        __syncthreads();
        lds_residual_store<Real>(J, r, rl);
    }
    if (segmented) {
        save_carry(J, cs, n_steps, false);
        return;
    }
    write_stats(J, cs);
}

// ---------------------------------------------------------------------------
// long rows: one estimate per wavefront, the first 64 E entries of a row in
// registers one step ahead (any further entries, as in the central pixels of
// an even bin count at 720 angles, are read in place during the step);
// residual values are read at the start of each step (after the previous
// step's scatter), so no patch table is needed.
// The residual lives in LDS for angles u < UL (over bins k_lo .. k_lo+Kc-1,
// at the start of the dynamic LDS) and in global memory otherwise, or wholly
// in LDS (RLDS).  Same canonical sums and decision as the other bodies.
// ---------------------------------------------------------------------------
template <typename Real, int E>
struct LongRow {
    int32_t col[E];
    Real len[E];
    int32_t p, n;
    uint32_t b;  // first entry of the row
    double delta, N1, lnN1;
};

template <typename Real, bool RLDS, int E, bool SERVED = false, typename LenT = Real, bool LATE = false>
__device__ void run_chain_long(const ChainJob& J, char* lds, ChainShared& sh, bool segmented)
{
    constexpr int BL = kWave;  // steps per block of draws: lane j <-> step base + j
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x >> 6, NW = blockDim.x >> 6;
    const double KU = (double)J.K * (double)J.U;
    const int M = J.m_cand;
    const bool active = wave < M;
    Real* r = RLDS ? (Real*)lds : (Real*)J.r;
    Real* rl = (Real*)lds;
    const LenT* lenp = (const LenT*)J.len;

    ChainState cs = segmented ? load_carry(J) : chain_setup<Real, !RLDS, LenT>(J, r, sh, lane, wave, NW);
    const int64_t n_steps = cs.n_steps;
    const int64_t s_begin = cs.s_begin;
    if (!RLDS) lds_residual_load<Real>(J, r, rl);
    Schedule sched;
    sched.start(s_begin, n_steps, J.n_stages, cs.T0, cs.TN, J.schedule);

    Draws cur, nxt;
    auto fill = [&](Draws& D, int64_t base) {
        D.base = base;
        const int64_t s = base + lane;
        D.p = 0;
        D.n = 0;
        D.b = 0;
        D.delta = 0.0;
        D.N1 = 0.0;
        D.lnN1 = 0.0;
        uint64_t k0 = lane0(J.seed), k1 = lane0(J.chain_id);
        asm volatile("" : "+s"(k0), "+s"(k1));
        if (s < n_steps) {
            if (active) {
                const Words4 w = philox4x64(k0, k1, (uint64_t)s, (uint64_t)wave, 0, 0);
                D.p = J.support[__umul64hi(w.w0, (uint64_t)J.P)];
                D.delta = J.delta_max * (2.0 * unit53(w.w1) - 1.0);
                const int64_t b0 = J.row_ptr[D.p];
                D.b = (uint32_t)b0;
                D.n = (int32_t)(J.row_ptr[D.p + 1] - b0);
            }
            D.N1 = unit53(philox4x64(k0, k1, (uint64_t)s, 0, 1, 0).w0);
            D.lnN1 = log(D.N1);
        }
    };
    cur.base = nxt.base = -1;
    auto prefetch = [&](LongRow<Real, E>& S, int64_t t) {
        if (t >= n_steps) {
            S.p = 0;
            S.n = 0;
            S.b = 0;
            S.delta = S.N1 = S.lnN1 = 0.0;
#pragma unroll
            for (int e = 0; e < E; ++e) {
                S.col[e] = 0;
                S.len[e] = (Real)0;
            }
            return;
        }
        const int64_t base = t - t % BL;
        if (cur.base != base) {
            if (nxt.base == base)
                cur = nxt;
            else
                fill(cur, base);
        }
        const int j = (int)(t - base);
        if (j == BL / 2 && base + BL < n_steps) fill(nxt, base + BL);
        S.p = __shfl(cur.p, j, kWave);
        S.n = __shfl(cur.n, j, kWave);
        const uint32_t b = (uint32_t)__shfl((int)cur.b, j, kWave);
        S.b = b;
        S.delta = __shfl(cur.delta, j, kWave);
        S.N1 = __shfl(cur.N1, j, kWave);
        S.lnN1 = __shfl(cur.lnN1, j, kWave);
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int q = lane + e * kWave;
            const uint32_t at = q < S.n ? b + (uint32_t)q : 0u;
            S.col[e] = ld32(J.col, at);
            S.len[e] = LATE ? len_hold<Real, LenT>(lenp, at) : (Real)ld32(lenp, at);
        }
    };
    // residual value of ray g: LDS part (angles u < UL: *lidx its index) or
    // global memory (*lidx = -1 - its position in the tiled layout)
    auto rget = [&](int32_t g, int* lidx) -> Real {
        if (RLDS) {
            *lidx = g;
            return r[g];
        }
        const int u = angle_of(J, g);
        if (u < J.UL) {
            *lidx = u * J.Kc + (g - u * J.K - J.k_lo);
            return rl[*lidx];
        }
        const uint32_t at = rpos(J, u, g - u * J.K);
        *lidx = -1 - (int)at;
        return ld32((const Real*)r, at);
    };

    LongRow<Real, E> A, B;
    prefetch(A, s_begin);
    __syncthreads();  // setup (residual, LDS part, temperatures) complete
    bool cancelled = false;
    // returns true when the chain stops here (segment end or cancellation)
    auto step = [&](LongRow<Real, E>& X, LongRow<Real, E>& Y, int64_t s)
                    __attribute__((always_inline)) -> bool {
        const double T = sched.at(s, n_steps, J.n_stages);
        const double invT = 1.0 / T;
        prefetch(Y, s + 1);
        Real rv[E];
        int li[E];
#pragma unroll
        for (int e = 0; e < E; ++e) rv[e] = rget(X.col[e], &li[e]);
        // (LATE) the lengths read back while the gathers are in flight
        Real ln[E];
#pragma unroll
        for (int e = 0; e < E; ++e) ln[e] = LATE ? len_use<Real, LenT>(X.len[e]) : X.len[e];
        const double fo = J.f[X.p];
        double fn = fo + X.delta;
        if (fn < J.f_min) fn = J.f_min;
        if (fn > J.f_max) fn = J.f_max;
        const double d = fn - fo;
        const Real dr = (Real)d;
        Real part[1] = {(Real)0};
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const Real t = (lane + e * kWave < X.n) ? dr * ln[e] : (Real)0;
            part[0] = fma(t, (Real)2 * rv[e] + t, part[0]);
        }
        // entries beyond the registers (rows longer than 64 E), read in
        // place, in the same per-lane order
        for (int q = kWave * E + lane; q < X.n; q += kWave) {
            int lo;
            const Real t = dr * (Real)ld32(lenp, X.b + (uint32_t)q);
            part[0] = fma(t, (Real)2 * rget(ld32(J.col, X.b + (uint32_t)q), &lo) + t, part[0]);
        }
        const Real S = canon_sum<kWave>(part);
        if (active && lane == 0) {
            sh.S[wave] = (double)S;
            sh.d[wave] = d;
        }
        const double co = sqrt(cs.sse / KU);
        if (SERVED) cancel_probe(J, sh, s);
        __syncthreads();
        const Decision dn = decide(sh.S, M, lane, cs.sse, co, KU, T, invT, X.N1, X.lnN1);
        const double d_star = uniform_f64(sh.d[dn.ms]);
        const bool changed = dn.accept && d_star != 0.0;
        if (changed && dn.ms == wave) {  // the owner of the winner applies Eq. 6
#pragma unroll
            for (int e = 0; e < E; ++e) {
                if (lane + e * kWave < X.n) {
                    const Real rn = rv[e] + dr * ln[e];
                    if (RLDS)
                        r[X.col[e]] = rn;
                    else if (li[e] >= 0)
                        rl[li[e]] = rn;
                    else
                        st32(r, (uint32_t)(-1 - li[e]), rn);
                }
            }
            // the entries beyond the registers: their rays differ from the
            // row's others, so their values are still the ones summed
            for (int q = kWave * E + lane; q < X.n; q += kWave) {
                const int32_t g = ld32(J.col, X.b + (uint32_t)q);
                int lo;
                const Real rn = rget(g, &lo) + dr * (Real)ld32(lenp, X.b + (uint32_t)q);
                if (RLDS)
                    r[g] = rn;
                else if (lo >= 0)
                    rl[lo] = rn;
                else
                    st32(r, (uint32_t)(-1 - lo), rn);
            }
            if (lane == 0) J.f[X.p] = fn;
        }
        count_decision(J, cs, dn, d_star, s);
        if (sizeof(Real) == 4 && J.resync_every > 0 && cs.since >= J.resync_every) {
            if (!RLDS) {
                __syncthreads();
                lds_residual_store<Real>(J, r, rl);
            }
            if (segmented) {
                save_carry(J, cs, s + 1, true);
                return true;
            }
            resync_in_group<Real, !RLDS, LenT>(J, cs, r, sh, lane, wave, NW);
            if (!RLDS) lds_residual_load<Real>(J, r, rl);
        }
        __syncthreads();
        if (SERVED && cancel_seen(J, sh, s)) {
            cs.status = PILA_ECANCELED;
            cs.n_steps = s + 1;
            cancelled = true;
            return true;
        }
        return false;
    };
    for (int64_t s = s_begin; s < n_steps;) {
        if (step(A, B, s)) {
            if (SERVED && cancelled) break;
            return;
        }
        if (++s >= n_steps) break;
        if (step(B, A, s)) {
            if (SERVED && cancelled) break;
            return;
        }
        ++s;
    }
    if (!RLDS) {
        __syncthreads();
        lds_residual_store<Real>(J, r, rl);
    }
    if (segmented) {
        save_carry(J, cs, n_steps, false);
        return;
    }
    write_stats(J, cs);
}

template <typename Real, typename LenT = Real>
__device__ void run_chain_simple_dispatch(const ChainJob& J, char* lds, int lds_bytes, ChainShared& sh)
{
    if ((int64_t)J.U * J.K * (int64_t)sizeof(Real) <= lds_bytes)
        run_chain_simple<Real, true, LenT>(J, lds, sh);
    else
        run_chain_simple<Real, false, LenT>(J, lds, sh);
}

}  // namespace pila
