/*
 * pila.h - C ABI of the MI355X (gfx950) library for simulated annealing
 * tomography (SAT) with a pre-calculated intersection lengths array (PILA).
 *
 * Method: N. T. Vo, M. B. H. Breese, H. O. Moser, "Feasibility of Simulated
 * Annealing Tomography" (arXiv 1411.4622).  Each entry point below names the
 * passage of the paper that defines the operation it performs.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Every function returns an int32 status (PILA_OK or a negative PILA_E*
 *   code).  Nothing aborts or exits; pila_last_error() returns a message for
 *   the last failure on the calling thread.
 * - Pointers prefixed d_ (and the device arrays inside pila_csr) are device
 *   memory on the current HIP device, allocated and owned by the caller.
 *   Pointers prefixed h_ and the arrays inside pila_geom are host memory,
 *   read or written only during the call.
 * - stream is a hipStream_t passed as void* (NULL = the null stream).
 *   Device work is enqueued on it asynchronously unless a function says
 *   it synchronises (it then waits for that stream only).
 * - Images are N x N row-major FP64, row 0 at the top: pixel (i, j) covers
 *   x in [j - N/2, j - N/2 + 1), y in [N/2 - 1 - i, N/2 - i), p = i*N + j.
 * - Sinograms are U x K row-major FP64, angle-major: ray g = u*K + k is the
 *   line x cos(a_u) + y sin(a_u) = k - (K-1)/2 (unit bin spacing, rays at
 *   bin centres).  Angles are given in degrees; multiples of 90 degrees use
 *   exact (cos, sin).
 * - A ray lying on a pixel edge (axis-parallel rays) belongs to the pixel
 *   whose half-open interval contains it; intersection lengths <= 1e-9
 *   (corner touches) are not stored.
 */
#ifndef PILA_H
#define PILA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define PILA_OK 0
#define PILA_EINVAL (-1)    /* bad argument (sizes, NULL pointers, non-finite input) */
#define PILA_ENOMEM (-2)    /* workspace or memory budget too small */
#define PILA_EHIP (-3)      /* HIP runtime error; the message carries its text */
#define PILA_ESIZE (-4)     /* buffer size does not match a previous phase */
#define PILA_ECANCELED (-5) /* request cancelled */
#define PILA_EBUSY (-6)     /* not admissible now; retry later */
#define PILA_ENOTFOUND (-7) /* unknown ticket */
#define PILA_ETIMEDOUT (-8) /* the workgroups of a split chain did not all run at once */

/* storage / arithmetic types */
#define PILA_F64 0
#define PILA_F32 1
#define PILA_U8 2  /* lengths only: one byte per length, round(180 l) (section II-B), read as
                      the float q / 180; chains take it with an FP32 or an FP64 residual */

/* cooling schedules (sat_params.schedule), section II-A and III-C */
#define PILA_SCHED_LINEAR 0 /* Eq. 2:  T_n = T0 - n (T0 - TN) / N */
#define PILA_SCHED_EXP 1    /* the faster drop of section III-C (its second Eq. 8):
                               T_n = T0 (TN / T0)^(n / N) */
#define PILA_SCHED_CUBIC 2  /* Eq. 9:  T_n = T0 - n^3 (T0 - TN) / N^3 */

/* what happens to a proposed value outside [f_min, f_max] (sat_params.proposal) */
#define PILA_PROP_CLAMP 0   /* clamped into the range */
#define PILA_PROP_REDRAW 1  /* the change is drawn again until the value is in range
                               (Step 2, Eq. 3 as printed) */

/* which chain body ran a chain (sat_stats.body): a kind plus flags, and for the
 * pipelined body its register shape: estimates per wavefront << 8 | row
 * entries per lane << 16; in a batch also its wavefronts per chain << 24 */
#define PILA_BODY_PIPED 1     /* rows in registers, estimates drawn ahead */
#define PILA_BODY_LONG 2      /* rows of more than 512 entries, one estimate per wavefront */
#define PILA_BODY_GENERAL 3   /* any row length and M, draws at the step (needed for redraw) */
#define PILA_BODY_SPLIT 4     /* one chain over several workgroups (their count in bits 8..15) */
#define PILA_BODY_GLOBAL_R 16 /* flag: the residual lives (partly) in global memory */
#define PILA_BODY_SEGMENTED 32 /* flag: FP32 resyncs ran grid-wide between launches */

/* ------------------------------------------------------------------------ */
/* Geometry and the PILA (section II-B, Eq. 5)                               */
/* ------------------------------------------------------------------------ */

typedef struct pila_geom {
    int32_t n;                /* image side N (N x N unit pixels), >= 1 */
    int32_t n_angles;         /* U, >= 1 */
    int32_t n_bins;           /* K, detector bins at unit spacing, >= 1 */
    int32_t len_dtype;        /* PILA_F64, PILA_F32 or PILA_U8: storage type of lengths */
    const double* angles_deg; /* host [U], finite */
    const uint8_t* mask;      /* host [N*N], nonzero = support pixel; NULL = all */
} pila_geom;

/*
 * A built PILA.  All arrays are caller-allocated device memory.
 *   row_ptr [N*N+1]  pixel-major CSR offsets (int64)
 *   col     [nnz]    ray index g = u*K + k, strictly ascending within a row
 *   len     [nnz]    intersection length (double, float or byte per len_dtype)
 *   support [n_support] support pixel indices, ascending
 *   trig    [2*U]    (cos, sin) of every angle, as used for the build
 *   t_row_ptr [U*K+1], t_col [nnz], t_len [nnz]: the same entries ray-major
 *                    (t_col = pixel index, ascending within a ray)
 * Rows of pixels outside the mask are empty.
 */
typedef struct pila_csr {
    int64_t nnz;       /* out of phase 1 */
    int32_t n_support; /* out of phase 1 */
    int32_t max_row;   /* out of phase 1: longest pixel-major row (entries) */
    int32_t k_lo, k_hi; /* out of phase 1: bins that support pixels can reach */
    int64_t* row_ptr;
    int32_t* col;
    void* len;
    int32_t* support;
    double* trig;
    int64_t* t_row_ptr;
    int32_t* t_col;
    void* t_len;
} pila_csr;

/*
 * pila_build_scratch_size - device scratch bytes pila_build needs for this
 * geometry (the mask and a few scalars): N*N + 256.
 */
int32_t pila_build_scratch_size(const pila_geom* geom, size_t* bytes);

/*
 * pila_build - intersection lengths of every support pixel with every ray
 * (section II-B: per pixel, the detector positions and lengths at each
 * angle, Eq. 5), stored pixel-major and ray-major.
 *
 * Two phases.  Phase 1 (csr->col == NULL): needs csr->row_ptr, csr->trig
 * and csr->t_row_ptr; fills them, sets csr->nnz, csr->n_support,
 * csr->max_row and csr->k_lo/k_hi, and synchronises the stream.  Phase 2
 * (csr->col != NULL): needs every array, sized from phase 1;
 * row_ptr/t_row_ptr must still hold phase 1's output.  Fills col, len,
 * support, t_col, t_len and synchronises.  d_scratch is caller device
 * memory of at least pila_build_scratch_size bytes, used during the call
 * only; the library allocates no device memory.
 * Errors: EINVAL for n, U or K < 1, a non-finite angle, a NULL array or
 * scratch, or len_dtype not PILA_F64/PILA_F32; ENOMEM when scratch_bytes
 * is too small; ESIZE when phase 2's row_ptr total does not equal
 * csr->nnz; EHIP on a runtime failure.
 */
int32_t pila_build(const pila_geom* geom, pila_csr* csr, void* d_scratch, size_t scratch_bytes,
                   void* stream);

/*
 * pila_forward - Eq. 1 for every ray: d_out[g] = sum over pixels of
 * l(p, g) * d_image[p], through the ray-major PILA (FP64 accumulation).
 * d_image [N*N] FP64, d_out [U*K] FP64.  Deterministic.  Asynchronous.
 */
int32_t pila_forward(const pila_geom* geom, const pila_csr* csr, const double* d_image,
                     double* d_out, void* stream);

/*
 * pila_backproject - transpose of Eq. 1: d_out[p] = sum over the rays
 * crossing p of l(p, g) * d_sino[g], through the pixel-major PILA (FP64
 * accumulation).  d_sino [U*K], d_out [N*N].  Deterministic.  Asynchronous.
 */
int32_t pila_backproject(const pila_geom* geom, const pila_csr* csr, const double* d_sino,
                         double* d_out, void* stream);

/* ------------------------------------------------------------------------ */
/* Simulated annealing (section II-A Steps 1-4, II-B Eq. 6-7, III Eq. 8,    */
/* III-B best of multiple estimates)                                          */
/* ------------------------------------------------------------------------ */

typedef struct sat_params {
    uint64_t seed;       /* Philox key word 0 */
    uint64_t chain_id;   /* Philox key word 1 */
    int64_t n_steps;     /* total steps (each: m_cand estimates, one update) */
    int32_t n_stages;    /* N of Eq. 2: temperature stages, >= 1 */
    int32_t m_cand;      /* N_e of the BoME strategy, 1..64 */
    double T0, TN;       /* Eq. 2 end points; T0 <= 0 selects Eq. 8 */
    int32_t q_auto;      /* Q of Eq. 8 (uphill estimates averaged), >= 1 */
    int32_t precision;   /* PILA_F64 or PILA_F32 residual sinogram */
    double tn_ratio;     /* T_N = T_0 / tn_ratio when Eq. 8 is used */
    double delta_max;    /* Eq. 3 step: change uniform in [-delta_max, delta_max) */
    double f_min, f_max; /* value range of a pixel */
    int64_t resync_every; /* FP32: FP64 recomputation of the residual after
                             this many accepted nonzero changes; 0 = never */
    int32_t schedule;     /* PILA_SCHED_LINEAR, _EXP or _CUBIC */
    int32_t proposal;     /* PILA_PROP_CLAMP or PILA_PROP_REDRAW (redraws use counter
                             (s, m, 0, j) for the j-th redraw, at most 256, after which
                             the value stays; chains that redraw run the general or
                             split body) */
} sat_params;

typedef struct sat_stats {
    int64_t steps, accepts, accepts_nonzero;
    int32_t resyncs;
    int32_t status;         /* PILA_OK, PILA_EINVAL when Eq. 8 failed, or
                               PILA_ETIMEDOUT (split chains, below) */
    double T0_used, TN_used;
    double sse_final;       /* running sum of squared residuals at the end */
    double cost_final;      /* Eq. 4 of the final image (running value) */
    double max_drift_r;     /* FP32: max |r32 - r64| seen at a resync */
    double max_drift_sse;   /* FP32: max relative |SSE_run - SSE64| at a resync */
    int32_t chain_launches; /* sat_run: launches of the chain kernel (one, or one
                               per resync segment); 0 from sat_run_batch */
    int32_t body;           /* PILA_BODY_* kind | flags of the body that ran the chain */
    double chain_kernel_ms; /* sat_run: summed duration of those launches, from
                               HIP events recorded around each of them */
    int64_t t_begin, t_end; /* sat_run_batch and the server: device wall clock
                               (pila_device_info.wallclock_khz) when the chain's
                               workgroup took it and when it finished; 0 from sat_run */
} sat_stats;

/* Optional per-step record, device arrays of n_steps elements (each may be
 * NULL): chosen estimate, acceptance, and the cost change Delta C. */
typedef struct sat_trace {
    int32_t* m_star;
    uint8_t* accept;
    double* dC;
} sat_trace;

/*
 * sat_workspace_size - device workspace bytes that sat_run needs: the chain
 * state, plus room for the slot words of the pipelined body or for the
 * copies of a split chain (below).  A workspace of at least the chain state
 * is accepted; the extra room only selects the faster bodies.
 */
int32_t sat_workspace_size(const pila_geom* geom, const sat_params* params, size_t* bytes);

/*
 * sat_workspace_min - the smallest workspace sat_run accepts: the chain
 * state alone (residual, per-tile sums, carry, statistics).  With it the
 * pipelined body forms slot words in place and chains that would be split
 * run on one workgroup (the general body); results are the same bits.
 */
int32_t sat_workspace_min(const pila_geom* geom, const sat_params* params, size_t* bytes);

/*
 * sat_run - one SAT chain.  From the starting image d_image (N*N, updated
 * in place) and the measured sinogram d_sino (Pm, U*K):
 *   r = A f - Pm and its sum of squares (Eq. 1, Eq. 4);
 *   T0/TN given, or from Eq. 8 (estimates from the starting image,
 *   Philox counter (q, 0, 2, 0));
 *   for step s: m_cand estimates (Philox4x64-10, key (seed, chain_id),
 *   counter (s, m, 0, 0)): pixel uniform over the support, change uniform
 *   in [-delta_max, delta_max), new value clamped to [f_min, f_max] or
 *   redrawn (params.proposal); each
 *   scored by the change of the squared-residual sum over its PILA row
 *   (Eq. 7); the first minimum is kept (BoME); accepted when its cost
 *   change Delta C <= 0 or N1 < exp(-Delta C / T) (Step 4; N1 from counter
 *   (s, 0, 1, 0)); T from Eq. 2 at stage floor(s * n_stages / n_steps);
 *   on acceptance the residual is updated over the row (Eq. 6).
 * precision PILA_F64 needs len_dtype PILA_F64 or PILA_U8; PILA_F32 needs
 * PILA_F32 or PILA_U8 (then the residual and the row sums are FP32, the cost
 * total FP64, and the residual is recomputed in FP64 every resync_every
 * nonzero accepts).  One-byte lengths enter every sum as q / 180.
 * h_stats (nullable) receives the chain's statistics: the call then
 * synchronises.  trace (nullable, host struct of device arrays) records
 * every step.  Errors: EINVAL (bad sizes/params, dtype mismatch, empty
 * support), ENOMEM (ws_bytes below sat_workspace_size), EHIP.
 * Split chains (PILA_BODY_SPLIT): when the residual does not fit in LDS,
 * m_cand >= 4 and m_cand * (nnz / n_support) >= 12288, and the workspace
 * has room for 15 copies of the residual and the image, the chain runs on
 * G = m_cand / 4 workgroups (at least 2, at most 16), each scoring its share of the
 * estimates on its own copies and exchanging the sums through the
 * workspace every step (same results as one workgroup).  The workgroups
 * must run at the same time: a workgroup that waits longer than 10 s for
 * the others (PILA_SPLIT_WAIT_MS in the environment, in ms, changes the
 * limit) ends the chain with stats.status = PILA_ETIMEDOUT, the image
 * holding the state it had reached.
 */
int32_t sat_run(const pila_geom* geom, const pila_csr* csr, const double* d_sino,
                const sat_params* params, double* d_image, void* d_ws, size_t ws_bytes,
                sat_stats* h_stats, const sat_trace* trace, void* stream);

/*
 * sat_run_static - sat_run without a caller workspace, for callers that
 * cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation).  The chain's workspace
 * is a static device array of PILA_STATIC_SCRATCH_BYTES that the library
 * holds on each GPU it runs on until the process ends; the call allocates
 * nothing.  Same arguments, semantics and results as sat_run (the slot
 * words, or a split chain's copies and exchange words, go into the array
 * when they fit after the chain state; the
 * statistics carry no kernel timing: chain_kernel_ms = 0).  Every call on a
 * GPU shares that GPU's array, so calls that overlap on one GPU (other
 * streams, other threads) race and give wrong results; each call writes
 * every workspace byte it reads, so nothing has to be cleared between
 * calls.  Errors: as sat_run, and ENOMEM when the chain state
 * (sat_workspace_size without the slot words: the residual, per-64-ray
 * sums, carry and stats, about U*K*(4 or 8) bytes) exceeds the array.
 */
#define PILA_STATIC_SCRATCH_BYTES ((size_t)64 << 20)
int32_t sat_run_static(const pila_geom* geom, const pila_csr* csr, const double* d_sino,
                       const sat_params* params, double* d_image, sat_stats* h_stats,
                       const sat_trace* trace, void* stream);

/* One independent chain of a batch. */
typedef struct sat_job {
    const pila_geom* geom;
    const pila_csr* csr;
    const double* d_sino;
    double* d_image;
    sat_params params;
    int32_t waves_per_chain; /* this chain's workgroup width (1, 2, 4, 8 or 16
                                wavefronts; 0 = the launch's), e.g. from a tuning
                                table per geometry */
    int32_t reserved;
} sat_job;

/* Launch shape of the batched kernel (nullable: library default). */
typedef struct sat_launch {
    int32_t waves_per_chain; /* 1, 2, 4, 8 or 16 wavefronts per chain */
    int32_t chains_per_cu;   /* resident chains per compute unit */
    int32_t lds_residual;    /* 1: keep a chain's residual in LDS when it fits */
    int32_t max_groups;      /* room in the three arrays below (0: not wanted) */
    /* out, per group of chains that one persistent kernel runs (unused
     * entries get desc 0): the kernel's duration from HIP events recorded
     * around it on its stream, its body (PILA_BODY_* kind | register shape:
     * estimates per wavefront << 8 | row entries per lane << 16 | wavefronts
     * per chain << 24) and its chain count.  Host arrays; filled when the
     * call returns. */
    float* h_group_ms;
    int32_t* h_group_desc;
    int32_t* h_group_chains;
} sat_launch;

/*
 * sat_batch_workspace_size / sat_run_batch - many independent chains (one
 * per slice) in persistent launches: one workgroup runs one chain at a
 * time and takes the next chain from a device ticket counter.  Chains are
 * grouped by body and register shape (each chain takes the pipelined body
 * at the smallest shape that holds its rows, else the long-row or general
 * body); each group is one persistent kernel, the groups run side by side
 * on streams forked from the caller's and joined back into it, and a
 * group hands out its longest chains first.  Each chain
 * computes exactly what sat_run computes for its job, independently of the
 * other jobs and of the launch shape's chain placement.  The call uploads
 * the chain descriptors from host memory it owns and synchronises the
 * stream before it returns, whether or not h_stats [n_jobs] (nullable)
 * asks for the statistics.
 */
int32_t sat_batch_workspace_size(int32_t n_jobs, const sat_job* jobs, size_t* bytes);
int32_t sat_run_batch(int32_t n_jobs, const sat_job* jobs, const sat_launch* launch, void* d_ws,
                      size_t ws_bytes, sat_stats* h_stats, void* stream);

/*
 * HIP graphs of chains (section II-A Steps 1-4 per chain, as sat_run and
 * sat_run_batch compute them).  A chain run alone enqueues one launch per
 * FP32 resync segment plus the grid-wide rebuilds between them (thousands of
 * launches for a long chain); a graph captures that sequence once and
 * replays it with one launch.
 *
 * sat_graph_create captures what sat_run would enqueue for these arguments
 * (no statistics, no kernel timing); sat_batch_graph_create what
 * sat_run_batch would enqueue for these jobs: the descriptors are uploaded
 * to d_ws once, synchronously, at creation, and the graph holds the ticket
 * reset, the slot words and every group's persistent kernel with the
 * fork/join dependencies between their streams.  Every pointer and size is
 * fixed at creation: each launch re-runs the chains from whatever the images
 * hold (callers copy the starting images in before a launch), with the
 * same buffers, and gives the bits sat_run / sat_run_batch would give.
 * sat_graph_launch enqueues one replay on a stream (asynchronous);
 * sat_graph_stats copies the statistics of the last replay (one per chain,
 * h_stats [chains]) and synchronises the stream; sat_graph_destroy frees
 * the graph (NULL accepted).  The library allocates no device memory for
 * a graph.  Errors: as sat_run / sat_run_batch, EHIP for capture failures.
 */
typedef struct sat_graph_s sat_graph;
int32_t sat_graph_create(const pila_geom* geom, const pila_csr* csr, const double* d_sino,
                         const sat_params* params, double* d_image, void* d_ws, size_t ws_bytes,
                         const sat_trace* trace, sat_graph** out);
int32_t sat_batch_graph_create(int32_t n_jobs, const sat_job* jobs, const sat_launch* launch, void* d_ws,
                               size_t ws_bytes, sat_graph** out);
int32_t sat_graph_launch(sat_graph* g, void* stream);
int32_t sat_graph_stats(sat_graph* g, sat_stats* h_stats, void* stream);
int32_t sat_graph_destroy(sat_graph* g);

/*
 * sat_drt_run - the comparison method of section III-A: the SAT chain of
 * sat_run (same estimates, temperatures, BoME choice and acceptance
 * uniforms, Philox counters (s, m, 0, 0) and (s, 0, 1, 0)) whose evaluation
 * step, instead of the PILA, projects each estimate's whole image by the
 * discrete Radon transform with bilinear interpolation (ray (u, k) sampled
 * at unit steps t = -T .. T, T = ceil(N / sqrt 2) + 1, at the points
 * (s_k cos - t sin, s_k sin + t cos), the image interpolated bilinearly
 * between pixel centres and zero outside) and takes its cost C' from Eq. 4;
 * Delta C = C' - C.  It needs no PILA and is here to measure what the PILA
 * saves (the paper reports over 300x on its CPU).  T0 and TN must be given.
 * d_image in: start, out: result.  h_cost_final (nullable) receives Eq. 4
 * of the final image; trace (nullable) records every step.  Synchronises
 * the stream.  Errors: EINVAL (sizes, T0/TN not given, params), ENOMEM
 * (workspace of sat_drt_workspace_size), EHIP.
 */
int32_t sat_drt_workspace_size(const pila_geom* geom, const sat_params* params, size_t* bytes);
int32_t sat_drt_run(const pila_geom* geom, const double* d_sino, const sat_params* params, double* d_image,
                    void* d_ws, size_t ws_bytes, double* h_cost_final, const sat_trace* trace, void* stream);

/* ------------------------------------------------------------------------ */
/* SIRT with exact lengths (section III-D, Eq. 10-11)                        */
/* ------------------------------------------------------------------------ */

typedef struct sirt_params {
    int32_t n_iter;
    int32_t flags;  /* 0, or PILA_SIRT_REUSE_LAYOUT */
    double lambda;  /* relaxation; 1 is the unrelaxed update */
} sirt_params;

/* sirt_params.flags: the workspace still holds the factor matrix and both
 * tile layouts that an earlier sirt_run on the same geometry and PILA built
 * in it (same workspace, unchanged since); the call skips building them */
#define PILA_SIRT_REUSE_LAYOUT 1

/* sirt_workspace_size - device workspace bytes that sirt_run needs: the
 * factor matrix, residuals and partial sums, the transposed image and the two
 * tile layouts sirt_run builds from the PILA (about 9 bytes per (pixel,
 * angle) of the support's 8 x 8 tiles and 9 bytes per (ray, image row or
 * column) in FP32; 15 GB at 1024 x 1024 and 720 angles). */
int32_t sirt_workspace_size(const pila_geom* geom, const sirt_params* params, size_t* bytes);

/*
 * sirt_run - simultaneous SIRT driven by the PILA: factor matrix
 * W_g = sum over support pixels of l(p, g)^2 (section III-D); each
 * iteration res = Pm - A f (ray-major PILA), then every support pixel moves
 * by (lambda / U) * sum over its row of l * res_g / W_g (Eq. 10-11 summed
 * over all rays crossing the pixel).  d_image (N*N) in: start, out: result.
 * h_cost (nullable, n_iter doubles) receives Eq. 4 of the image entering
 * each iteration; the call then synchronises.  Both projections run on
 * tile layouts built at the start of the call (with W), unless
 * params->flags holds PILA_SIRT_REUSE_LAYOUT: then the workspace must hold
 * them from an earlier call on the same geometry and PILA, and a call of
 * n_iter iterations continues exactly where the earlier one stopped (the
 * layouts sit at offsets that do not depend on n_iter).  EINVAL for other
 * flags.  A tile whose entries do not
 * have the two-neighbour shape is summed from the CSR rows instead (the
 * environment variable PILA_SIRT_CSR=1 forces that for every tile, for
 * tests).  Sums are deterministic; their order differs from a row walk, so
 * results match the plain definition to rounding (1e-10 relative in tests).
 */
int32_t sirt_run(const pila_geom* geom, const pila_csr* csr, const double* d_sino,
                 const sirt_params* params, double* d_image, void* d_ws, size_t ws_bytes,
                 double* h_cost, void* stream);

/*
 * sirt_seq_run - SIRT with exact lengths pixel by pixel, as section III-D
 * describes it: the factor matrix W and the calculated projections Pc = A f
 * are computed once; then n_iter times, m_per times, a support pixel p is
 * chosen (Philox4x64-10, key (seed, 0), counter (n * m_per + m, 0, 3, 0),
 * uniform over the support), moves by (lambda / U) * sum over its PILA row
 * of l * (Pm_g - Pc_g) / W_g (Eq. 10-11 summed over all rays that cross the
 * pixel, rays with W_g = 0 adding nothing), and its rays get Pc_g += change
 * * l (Eq. 6).  d_image (N*N) in: start, out: result.  h_cost (nullable,
 * n_iter doubles) receives Eq. 4 of the running projections after each
 * iteration; the call then synchronises.  One wavefront runs the sequence
 * (each update reads the projections the previous one wrote).  Row sums
 * are added in a fixed order that differs from a row walk: results match
 * the plain definition to rounding.  Errors: EINVAL (sizes, NULL arrays,
 * non-finite lambda, empty support), ENOMEM (workspace), EHIP.
 */
typedef struct sirt_seq_params {
    int32_t n_iter;    /* N: iterations */
    int32_t reserved;
    int64_t m_per;     /* M: pixel updates per iteration */
    double lambda;     /* relaxation; 1 is the formula as printed */
    uint64_t seed;     /* Philox key word 0 of the pixel choice */
} sirt_seq_params;

int32_t sirt_seq_workspace_size(const pila_geom* geom, const sirt_seq_params* params, size_t* bytes);
int32_t sirt_seq_run(const pila_geom* geom, const pila_csr* csr, const double* d_sino,
                     const sirt_seq_params* params, double* d_image, void* d_ws, size_t ws_bytes,
                     double* h_cost, void* stream);

/* ------------------------------------------------------------------------ */
/* Serving: many independent chains (one slice each, section II-A Steps 1-4  */
/* per slice) admitted against a memory budget and run by resident          */
/* workgroups that take new requests as earlier ones finish                  */
/* ------------------------------------------------------------------------ */

typedef struct srv_s srv_t; /* opaque server handle */

typedef struct srv_config {
    size_t mem_budget;       /* device bytes the server allocates at creation and never
                                exceeds: PILA cache, chain states, build scratch */
    int32_t max_slots;       /* chains resident at once, one workgroup each (a whole compute
                                unit), >= 3; 0 = three quarters of the compute units: the
                                rest stay free for other kernels (the caller's copies, PILA
                                builds), whose workgroups would otherwise wait for ours */
    int32_t waves_per_chain; /* 4 or 8 (0 = 8) */
    int32_t ring_size;       /* tickets submitted and not yet reaped; power of two, 0 = 1024 */
    int32_t idle_us;         /* a queue's resident workgroups all exit together when none
                                of its chains runs and no request came for this long; the
                                server relaunches them on the next submission (0 = 20000) */
    int32_t general_slots;   /* of max_slots, those that run the general body (chains no
                                other body takes: FP64, large M); 0 = max_slots / 16 */
    int32_t long_slots;      /* of max_slots, those that run FP32 chains whose rows are too
                                long for the pipelined body's registers (up to 1536
                                entries); 0 = max_slots / 4.  The rest run the pipelined
                                body */
} srv_config;

typedef struct srv_request {
    const pila_geom* geom;   /* host; len_dtype must equal params.precision.  The server
                                builds the PILA on first use and caches it */
    const double* d_sino;    /* device [U*K], caller-owned, unchanged until reaped */
    double* d_image;         /* device [N*N]: f0 in, the chain's final image out;
                                caller-owned, untouched by others until reaped */
    sat_params params;       /* as for sat_run */
} srv_request;

typedef struct srv_status {
    int64_t submitted;       /* tickets issued */
    int64_t reaped;          /* tickets whose results were returned by srv_poll */
    int64_t in_flight;       /* issued, not yet reaped */
    int64_t launches;        /* launches of the resident kernel so far */
    size_t bytes_used;       /* of mem_budget */
    size_t bytes_budget;
    int32_t pila_cached;     /* geometries whose PILA is resident */
    int32_t kernel_running;  /* the resident kernel has not exited yet */
} srv_status;

/*
 * srv_create - allocate the server on the current device: mem_budget bytes
 * of device memory, a ring of ring_size request descriptors in pinned host
 * memory, and three non-blocking streams, one per resident kernel (PILA
 * builds run on the null stream).  No device memory is allocated after this
 * call (PILA builds use the budget too).  The resident kernels run while
 * requests are in flight and for idle_us after: a device-wide
 * synchronisation (hipDeviceSynchronize) waits for them, so callers
 * synchronise their own streams instead.  HIP maps streams onto a few
 * hardware queues (GPU_MAX_HW_QUEUES, 4 by default), each run in order: work
 * on any stream that shares a hardware queue with a resident kernel waits
 * until that kernel ends.  The three streams have hardware queues of their
 * own when the process holds no more streams than hardware queues, counting
 * the null stream: e.g. a caller that works on the null stream and creates
 * the server before other streams; otherwise raise GPU_MAX_HW_QUEUES.
 * Errors: EINVAL (NULL arguments, bad sizes), ENOMEM (budget too small for
 * the server's own bookkeeping), EHIP.
 */
int32_t srv_create(const srv_config* cfg, srv_t** out);

/*
 * srv_prepare - build and cache the PILA of a geometry now (Eq. 5), so that
 * later submissions of that geometry do not build.  Synchronises the
 * server's build stream.  ENOMEM when it cannot fit even after evicting
 * every unused cached PILA.
 */
int32_t srv_prepare(srv_t* s, const pila_geom* geom);

/*
 * srv_submit - admit one chain.  Its sinogram and starting image must be
 * complete in device memory when this is called (the work that wrote them
 * has finished).  Admission needs the geometry's PILA (built
 * if absent, evicting least recently used PILAs that no admitted request
 * uses) and chain state of sat_workspace_size bytes inside the budget, and
 * a free ring slot.  On success *ticket names the request; its chain is
 * taken by the next free resident workgroup in ticket order.
 * Errors: EBUSY when not admissible now (retry after reaping others),
 * EINVAL (as sat_run), ENOMEM when the request could never fit the budget.
 */
int32_t srv_submit(srv_t* s, const srv_request* req, uint64_t* ticket);

/*
 * srv_poll - *done = 1 and *stats (nullable) filled when the ticket's chain
 * has finished; its image is then final in d_image and the ticket is reaped
 * (its memory returns to the budget).  *done = 0 otherwise.  Also relaunches
 * the resident kernel when it has exited with requests still waiting.
 * ENOTFOUND for unknown or already reaped tickets.
 */
int32_t srv_poll(srv_t* s, uint64_t ticket, int32_t* done, sat_stats* stats);

/*
 * srv_cancel - ask the ticket's chain to stop: a waiting chain never starts,
 * a running one stops within 1024 steps.  Either way srv_poll then reports
 * it done with stats.status = PILA_ECANCELED (the image holds the state
 * reached).  ENOTFOUND for unknown or reaped tickets.
 */
int32_t srv_cancel(srv_t* s, uint64_t ticket);

int32_t srv_get_status(srv_t* s, srv_status* st);

/*
 * srv_destroy - cancel what still runs, wait for the resident kernel to
 * exit, and free everything.  NULL is accepted.
 */
int32_t srv_destroy(srv_t* s);

/* ------------------------------------------------------------------------ */
/* Device information and errors                                             */
/* ------------------------------------------------------------------------ */

typedef struct pila_device_info {
    int32_t cu_count;
    int32_t lds_per_block;   /* bytes */
    int32_t clock_khz;
    int32_t warp_size;
    size_t hbm_bytes;
    char name[64];
    int32_t wallclock_khz;   /* rate of the device wall clock of sat_stats.t_begin/t_end */
    int32_t pad;
} pila_device_info;

int32_t pila_get_device_info(pila_device_info* info);

/* Message of the last failure on the calling thread ("" if none). */
const char* pila_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PILA_H */
