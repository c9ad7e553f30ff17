/*
 * Plain FP64 CPU oracle for simulated annealing tomography with a
 * pre-calculated intersection lengths array (PILA).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no source with the HIP library.
 *
 * Everything here is written for obviousness, not speed: scalar loops in
 * the order the paper states the method, FP64 throughout (FP32 only where a
 * chain is explicitly run with an FP32 residual), built with
 * -ffp-contract=off so every a*b+c rounds twice.
 *
 * Passages followed (Vo, Breese, Moser, "Feasibility of Simulated Annealing
 * Tomography"):
 *   Eq. 1            projection = sum over crossed pixels of value x length
 *   Sec. II-A        Steps 1-4 of SAT, Eq. 2 (linear cooling), Eq. 3
 *                    (random change of one pixel), Eq. 4 (RMS cost),
 *                    acceptance rule of Step 4
 *   Sec. II-B        PILA: per pixel, the (detector position, length) pairs
 *                    of every angle, from a Siddon ray trace; Eq. 6
 *                    (sinogram update) and Eq. 7 (cost update)
 *   Sec. II-B        one-byte lengths: round(180 l)
 *   Sec. III         Eq. 8 (initial temperature from Q uphill estimates),
 *                    T_N = T_0 / 10^3
 *   Sec. III-A       the comparison method: SAT whose evaluation step
 *                    projects the whole image by bilinear interpolation
 *   Sec. III-B       best of multiple estimates (BoME)
 *   Sec. III-C       the exponential schedule (the second Eq. 8) and the
 *                    cubic one (Eq. 9)
 *   Sec. III-D       Eq. 10-11 SIRT with exact lengths and the factor matrix,
 *                    simultaneous and pixel by pixel
 *
 * Readings where the paper is silent (geometry, RNG, clamped proposals,
 * simultaneous SIRT, stage indexing) are stated next to the code that
 * applies them.
 *
 * Parity status: every exported function is pinned by the CPU test suite
 * (Philox against numpy's Philox4x64-10; PILA against brute-force clipping
 * and hand-derived lengths; projection against closed-form chords; Eq. 7
 * against full recomputation of Eq. 4; the chain against an independent
 * replay with dense projection; SIRT against dense Landweber; the
 * sequential SIRT against a one-pixel closed form, its weighted-residual
 * descent and its fixed point; the bilinear DRT against scipy's bilinear
 * sampling and closed forms; the one-byte lengths against the rounding
 * bound).  The FP32 residual mode is pinned by rounding-error bounds: each
 * FP32 row sum against the exact sum of the same float operands, and the
 * running residual against a from-scratch dense residual (exact to one
 * float rounding right after a resync, within the accumulated rounding
 * bound otherwise).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_TAU 1e-9 /* lengths at or below this are grazes and are dropped */

/* ------------------------------------------------------------------------ */
/* Philox4x64-10 counter-based generator (Salmon, Moraes, Dror, Shaw, SC'11) */
/* ------------------------------------------------------------------------ */

static const uint64_t PH_M0 = 0xD2E7470EE14C6C93ULL;
static const uint64_t PH_M1 = 0xCA5A826395121157ULL;
static const uint64_t PH_W0 = 0x9E3779B97F4A7C15ULL; /* golden ratio */
static const uint64_t PH_W1 = 0xBB67AE8584CAA73BULL; /* sqrt(3) - 1 */

void or_philox(const uint64_t key[2], const uint64_t ctr[4], uint64_t out[4])
{
    uint64_t k0 = key[0], k1 = key[1];
    uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += PH_W0;
            k1 += PH_W1;
        }
        unsigned __int128 p0 = (unsigned __int128)PH_M0 * x0;
        unsigned __int128 p1 = (unsigned __int128)PH_M1 * x2;
        uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        uint64_t y0 = hi1 ^ x1 ^ k0;
        uint64_t y2 = hi0 ^ x3 ^ k1;
        x0 = y0;
        x1 = lo1;
        x2 = y2;
        x3 = lo0;
    }
    out[0] = x0;
    out[1] = x1;
    out[2] = x2;
    out[3] = x3;
}

/* 53-bit uniform double in [0, 1) from a 64-bit word */
static double u01(uint64_t w) { return (double)(w >> 11) * (1.0 / 9007199254740992.0); }

/* uniform index in [0, n): high word of the 128-bit product w * n */
static uint64_t uindex(uint64_t w, uint64_t n)
{
    return (uint64_t)(((unsigned __int128)w * n) >> 64);
}

/* ------------------------------------------------------------------------ */
/* Geometry (reading of Eq. 1 and Fig. 1: unit pixels, rays at bin centres) */
/* ------------------------------------------------------------------------ */

/* (cos, sin) of an angle in degrees; exact at multiples of 90 degrees so
 * that axis-parallel rays are recognised as such. */
void or_trig(int32_t U, const double* deg, double* cs)
{
    for (int u = 0; u < U; ++u) {
        double d = deg[u];
        double c, s;
        if (fmod(d, 90.0) == 0.0) {
            long q = (long)(d / 90.0) % 4;
            if (q < 0) q += 4;
            static const double tc[4] = {1.0, 0.0, -1.0, 0.0};
            static const double ts[4] = {0.0, 1.0, 0.0, -1.0};
            c = tc[q];
            s = ts[q];
        } else {
            double a = d * (M_PI / 180.0);
            c = cos(a);
            s = sin(a);
        }
        cs[2 * u] = c;
        cs[2 * u + 1] = s;
    }
}

/* Column of an image x coordinate, row of an image y coordinate (pixel
 * (i, j) covers x in [j - N/2, j - N/2 + 1) and y in [N/2-1-i, N/2-i)). */
static long col_of(long double x, long double h) { return (long)floorl(x + h); }
static long row_of(long double y, long double h) { return -(long)floorl(y - h + 1.0L); }

static int cmp_ld(const void* a, const void* b)
{
    long double x = *(const long double*)a, y = *(const long double*)b;
    return (x > y) - (x < y);
}

/*
 * Siddon ray trace of one ray  x cos + y sin = s  through the N x N grid:
 * the ray's parameter values where it crosses the grid lines are merged in
 * order, and each piece between consecutive crossings is charged to the
 * pixel that contains its midpoint.  A ray lying exactly on a grid line
 * (only possible when it is axis-parallel) belongs to the pixel whose
 * half-open interval contains it.  Pieces of the same pixel are summed and
 * lengths <= OR_TAU dropped (corner grazes).  Returns the pixel count.
 *
 * The trace runs in x87 extended precision: a piece cut from a pixel corner
 * by a ray at a small angle alpha to a grid line has a length that moves by
 * about 1 / (|cos alpha| |sin alpha|) per unit shift of the ray, so FP64
 * crossing parameters of size ~N would leave errors above 1e-12 in the
 * lengths of large grids.  Results are rounded to double at the end.
 * ts must hold at least 2N + 4 entries.
 */
static int siddon_ray(int N, double c_, double sn_, double s_, const uint8_t* mask, int32_t* pix,
                      double* len, long double* ts, long double* acc)
{
    const long double h = N / 2.0L, c = c_, sn = sn_, s = s_;
    int n = 0;
    if (sn == 0.0L) { /* vertical ray x = s * c */
        long j = col_of(s * c, h);
        if (j < 0 || j >= N) return 0;
        for (int i = 0; i < N; ++i) {
            int p = i * N + (int)j;
            if (mask && !mask[p]) continue;
            pix[n] = p;
            len[n] = 1.0;
            ++n;
        }
        return n;
    }
    if (c == 0.0L) { /* horizontal ray y = s * sn */
        long i = row_of(s * sn, h);
        if (i < 0 || i >= N) return 0;
        for (int j = 0; j < N; ++j) {
            int p = (int)i * N + j;
            if (mask && !mask[p]) continue;
            pix[n] = p;
            len[n] = 1.0;
            ++n;
        }
        return n;
    }
    /* The ray is the line x c + y sn = s for the given (c, sn), whose norm
     * rho differs from 1 by rounding: its foot point is s (c, sn) / rho^2,
     * and (-sn, c) has length rho, so parameter differences scale by rho. */
    const long double rho2 = c * c + sn * sn, rho = sqrtl(rho2);
    const long double x0 = s * c / rho2, y0 = s * sn / rho2;
    long double tx1 = (x0 + h) / sn, tx2 = (x0 - h) / sn;
    long double ty1 = (-h - y0) / c, ty2 = (h - y0) / c;
    long double tlo = fmaxl(fminl(tx1, tx2), fminl(ty1, ty2));
    long double thi = fminl(fmaxl(tx1, tx2), fmaxl(ty1, ty2));
    if (!(thi > tlo)) return 0;
    int nt = 0;
    ts[nt++] = tlo;
    ts[nt++] = thi;
    for (int j = 0; j <= N; ++j) {
        long double t = (x0 - (-h + j)) / sn;
        if (t > tlo && t < thi) ts[nt++] = t;
    }
    for (int i = 0; i <= N; ++i) {
        long double t = ((-h + i) - y0) / c;
        if (t > tlo && t < thi) ts[nt++] = t;
    }
    qsort(ts, (size_t)nt, sizeof(long double), cmp_ld);
    int last = -1;
    for (int q = 0; q + 1 < nt; ++q) {
        long double d = (ts[q + 1] - ts[q]) * rho;
        if (!(d > 0.0L)) continue;
        long double tm = 0.5L * (ts[q] + ts[q + 1]);
        long j = col_of(x0 - tm * sn, h);
        long i = row_of(y0 + tm * c, h);
        if (j < 0) j = 0;
        if (j >= N) j = N - 1;
        if (i < 0) i = 0;
        if (i >= N) i = N - 1;
        int p = (int)i * N + (int)j;
        if (p == last) {
            acc[n - 1] += d;
        } else {
            pix[n] = p;
            acc[n] = d;
            ++n;
            last = p;
        }
    }
    /* drop grazes and masked pixels, keep trace order */
    int m = 0;
    for (int q = 0; q < n; ++q) {
        double l = (double)acc[q];
        if (l > OR_TAU && (!mask || mask[pix[q]])) {
            pix[m] = pix[q];
            len[m] = l;
            ++m;
        }
    }
    return m;
}

/*
 * Ray-major listing of the whole system: for every ray g = u*K + k the
 * pixels it crosses and the lengths.  Two-phase: with pix == NULL only the
 * per-ray counts (cnt[G]) are produced and the total returned; otherwise
 * off[G+1] must hold the prefix of those counts and pix/len are filled.
 */
int64_t or_rays(int32_t N, int32_t U, int32_t K, const double* deg, const uint8_t* mask,
                int32_t* cnt, const int64_t* off, int32_t* pix, double* len)
{
    double* cs = (double*)malloc(sizeof(double) * 2 * (size_t)U);
    long double* ts = (long double*)malloc(sizeof(long double) * (2 * (size_t)N + 8));
    long double* acc = (long double*)malloc(sizeof(long double) * (2 * (size_t)N + 8));
    int32_t* bp = (int32_t*)malloc(sizeof(int32_t) * (2 * (size_t)N + 8));
    double* bl = (double*)malloc(sizeof(double) * (2 * (size_t)N + 8));
    or_trig(U, deg, cs);
    int64_t total = 0;
    for (int u = 0; u < U; ++u) {
        for (int k = 0; k < K; ++k) {
            double s = k - (K - 1) / 2.0;
            int n = siddon_ray(N, cs[2 * u], cs[2 * u + 1], s, mask, bp, bl, ts, acc);
            int64_t g = (int64_t)u * K + k;
            if (pix) {
                memcpy(pix + off[g], bp, sizeof(int32_t) * (size_t)n);
                memcpy(len + off[g], bl, sizeof(double) * (size_t)n);
            } else if (cnt) {
                cnt[g] = n;
            }
            total += n;
        }
    }
    free(cs);
    free(ts);
    free(acc);
    free(bp);
    free(bl);
    return total;
}

/* One ray g = u*K + k traced on its own: its pixels (trace order) and
 * lengths.  pix/len need room for 2N entries.  Returns the count. */
int32_t or_trace_ray(int32_t N, int32_t K, double deg, int32_t k, const uint8_t* mask,
                     int32_t* pix, double* len)
{
    double cs[2];
    or_trig(1, &deg, cs);
    long double* ts = (long double*)malloc(sizeof(long double) * (2 * (size_t)N + 8));
    long double* acc = (long double*)malloc(sizeof(long double) * (2 * (size_t)N + 8));
    int n = siddon_ray(N, cs[0], cs[1], k - (K - 1) / 2.0, mask, pix, len, ts, acc);
    free(ts);
    free(acc);
    return n;
}

/*
 * PILA row of one pixel (Eq. 5) without building the whole array: every ray
 * that could reach the pixel (bins within one unit of the projection of the
 * pixel centre, a superset of its shadow) is traced in full and the pixel's
 * piece kept.  Entries come out in ascending g.  g/len need room for 4U.
 */
int32_t or_pixel_row(int32_t N, int32_t U, int32_t K, const double* deg, const uint8_t* mask,
                     int32_t p, int32_t* g_out, double* len_out)
{
    if (mask && !mask[p]) return 0;
    double* cs = (double*)malloc(sizeof(double) * 2 * (size_t)U);
    long double* ts = (long double*)malloc(sizeof(long double) * (2 * (size_t)N + 8));
    long double* acc = (long double*)malloc(sizeof(long double) * (2 * (size_t)N + 8));
    int32_t* bp = (int32_t*)malloc(sizeof(int32_t) * (2 * (size_t)N + 8));
    double* bl = (double*)malloc(sizeof(double) * (2 * (size_t)N + 8));
    or_trig(U, deg, cs);
    const double h = N / 2.0;
    const double xc = (p % N) - h + 0.5, yc = h - 0.5 - (p / N);
    int32_t n = 0;
    for (int u = 0; u < U; ++u) {
        double t0 = xc * cs[2 * u] + yc * cs[2 * u + 1];
        long k0 = (long)floor(t0 + (K - 1) / 2.0 - 1.0);
        for (long k = k0; k <= k0 + 3; ++k) {
            if (k < 0 || k >= K) continue;
            double s = k - (K - 1) / 2.0;
            if (fabs(s - t0) > 1.0) continue;
            int m = siddon_ray(N, cs[2 * u], cs[2 * u + 1], s, mask, bp, bl, ts, acc);
            for (int q = 0; q < m; ++q)
                if (bp[q] == p) {
                    g_out[n] = (int32_t)(u * K + k);
                    len_out[n] = bl[q];
                    ++n;
                }
        }
    }
    free(cs);
    free(ts);
    free(acc);
    free(bp);
    free(bl);
    return n;
}

/*
 * PILA (Eq. 5): the ray-major listing regrouped by pixel.  Row p lists the
 * rays g = u*K + k that cross pixel p, in ascending g, with their lengths.
 * Inputs are the ray-major arrays from or_rays.  row_ptr has N*N+1 entries.
 */
void or_pila_from_rays(int32_t N, int32_t U, int32_t K, const int64_t* off, const int32_t* pix,
                       const double* len, int64_t* row_ptr, int32_t* col, double* plen)
{
    const int64_t NP = (int64_t)N * N, G = (int64_t)U * K;
    memset(row_ptr, 0, sizeof(int64_t) * (size_t)(NP + 1));
    for (int64_t e = 0; e < off[G]; ++e) row_ptr[pix[e] + 1] += 1;
    for (int64_t p = 0; p < NP; ++p) row_ptr[p + 1] += row_ptr[p];
    int64_t* cur = (int64_t*)malloc(sizeof(int64_t) * (size_t)NP);
    memcpy(cur, row_ptr, sizeof(int64_t) * (size_t)NP);
    for (int64_t g = 0; g < G; ++g) {
        for (int64_t e = off[g]; e < off[g + 1]; ++e) {
            int64_t q = cur[pix[e]]++;
            col[q] = (int32_t)g;
            plen[q] = len[e];
        }
    }
    free(cur);
}

/* Eq. 1 for every ray: out[g] = sum over the pixels crossed by ray g of
 * f[p] * l(p, g), visiting the PILA pixel by pixel. */
void or_forward(int32_t N, int32_t U, int32_t K, const int64_t* row_ptr, const int32_t* col,
                const double* len, const double* f, double* out)
{
    const int64_t NP = (int64_t)N * N, G = (int64_t)U * K;
    for (int64_t g = 0; g < G; ++g) out[g] = 0.0;
    for (int64_t p = 0; p < NP; ++p)
        for (int64_t e = row_ptr[p]; e < row_ptr[p + 1]; ++e) out[col[e]] += f[p] * len[e];
}

/* Transpose of Eq. 1: out[p] = sum over the rays crossing p of l * y[g]. */
void or_backward(int32_t N, const int64_t* row_ptr, const int32_t* col, const double* len,
                 const double* y, double* out)
{
    const int64_t NP = (int64_t)N * N;
    for (int64_t p = 0; p < NP; ++p) {
        double a = 0.0;
        for (int64_t e = row_ptr[p]; e < row_ptr[p + 1]; ++e) a += len[e] * y[col[e]];
        out[p] = a;
    }
}

/* ------------------------------------------------------------------------ */
/* Simulated annealing (Sec. II-A, II-B, III, III-B)                         */
/* ------------------------------------------------------------------------ */

typedef struct {
    uint64_t seed, chain_id;
    int64_t n_steps;
    int32_t n_stages;   /* N of Eq. 2 */
    int32_t m_cand;     /* N_e of the BoME strategy */
    double T0, TN;      /* T0 <= 0: Eq. 8 from q_auto uphill estimates */
    int32_t q_auto;
    int32_t precision;  /* 0 = FP64 residual, 1 = FP32 residual */
    double tn_ratio;    /* T_N = T_0 / tn_ratio when T0 is automatic */
    double delta_max, f_min, f_max;
    int64_t resync_every; /* FP32: full FP64 recomputation every so many nonzero accepts */
    int32_t schedule;     /* 0: Eq. 2 (linear), 1: Sec. III-C's second Eq. 8 (exponential),
                             2: Eq. 9 (cubic) */
    int32_t proposal;     /* 0: new value clamped to [f_min, f_max]; 1: redrawn until it
                             falls inside (Eq. 3 as printed) */
} or_sat_params;

typedef struct {
    int64_t steps, accepts, accepts_nonzero;
    int32_t resyncs, pad;
    double T0_used, TN_used, sse_final, cost_final, max_drift_r, max_drift_sse;
} or_sat_stats;

/* Temperature of step s.  The n_steps steps are split into n_stages stages
 * of equal length (M repetitions per stage, Sec. II-A); stage
 * n = floor(s * n_stages / n_steps), n = 0 .. n_stages-1, and with N the
 * number of stages:
 *   schedule 0, Eq. 2:                  T_n = T0 - n (T0 - TN) / N
 *   schedule 1, Sec. III-C (second (8)): T_n = T0 (TN / T0)^(n / N)
 *   schedule 2, Eq. 9:                  T_n = T0 - n^3 (T0 - TN) / N^3   */
double or_temperature(int64_t s, int64_t n_steps, int32_t n_stages, double T0, double TN,
                      int32_t schedule)
{
    int64_t n = (s * (int64_t)n_stages) / n_steps;
    double x = (double)n, Nn = (double)n_stages;
    if (schedule == 1) return T0 * pow(TN / T0, x / Nn);
    if (schedule == 2) return T0 - (x * x * x) * ((T0 - TN) / (Nn * Nn * Nn));
    return T0 - x * ((T0 - TN) / Nn);
}

/* Change of the RMS cost C (Eq. 4) when the sum of squared residuals moves
 * from sse to sse + dS, in a form free of cancellation:
 * C' - C = (dS / KU) / (C' + C). */
static double cost_change(double sse, double dS, double KU)
{
    double cn = sqrt(fmax(sse + dS, 0.0) / KU);
    double co = sqrt(sse / KU);
    double den = cn + co;
    if (den == 0.0) return 0.0;
    return (dS / KU) / den;
}

/* A random single-pixel estimate (Step 2, Eq. 3).  Philox counter
 * (c0, c1, purpose, 0) gives the pixel (uniform over the support, word 0)
 * and the change (uniform in [-dmax, dmax), word 1).  A new value outside
 * [f_min, f_max] is clamped into it (proposal 0), or the change is drawn
 * again from counter (c0, c1, purpose, j), j = 1, 2, ..., for the same
 * pixel until the new value falls inside (proposal 1, Eq. 3 as printed);
 * after OR_REDRAW_MAX draws without success the value stays (change 0). */
#define OR_REDRAW_MAX 256
static void draw_estimate(const uint64_t key[2], uint64_t c0, uint64_t c1, uint64_t purpose,
                          int64_t P, const int32_t* support, const double* f,
                          const or_sat_params* prm, int32_t* p_out, double* fn_out, double* d_out)
{
    uint64_t ctr[4] = {c0, c1, purpose, 0}, w[4];
    or_philox(key, ctr, w);
    int32_t p = support[uindex(w[0], (uint64_t)P)];
    double fo = f[p];
    double delta = prm->delta_max * (2.0 * u01(w[1]) - 1.0);
    double fn = fo + delta;
    if (prm->proposal == 1) {
        int j = 0;
        while ((fn < prm->f_min || fn > prm->f_max) && j < OR_REDRAW_MAX) {
            ++j;
            ctr[3] = (uint64_t)j;
            or_philox(key, ctr, w);
            delta = prm->delta_max * (2.0 * u01(w[1]) - 1.0);
            fn = fo + delta;
        }
        if (fn < prm->f_min || fn > prm->f_max) fn = fo;
    } else {
        if (fn < prm->f_min) fn = prm->f_min;
        if (fn > prm->f_max) fn = prm->f_max;
    }
    *p_out = p;
    *fn_out = fn;
    *d_out = fn - fo;
}

/* Eq. 7's inner sum for one estimate: change of the sum of squared
 * residuals when pixel p changes by d, over the pixel's PILA row. */
double or_delta_sse64(const int64_t* row_ptr, const int32_t* col, const double* len,
                          const double* r, int32_t p, double d, double* sabs)
{
    double S = 0.0, A = 0.0;
    for (int64_t e = row_ptr[p]; e < row_ptr[p + 1]; ++e) {
        double t = d * len[e];
        double term = t * (2.0 * r[col[e]] + t);
        S += term;
        A += fabs(term);
    }
    if (sabs) *sabs = A;
    return S;
}

float or_delta_sse32(const int64_t* row_ptr, const int32_t* col, const double* len,
                         const float* r, int32_t p, double d)
{
    float S = 0.0f;
    float df = (float)d;
    for (int64_t e = row_ptr[p]; e < row_ptr[p + 1]; ++e) {
        float t = df * (float)len[e];
        S += t * (2.0f * r[col[e]] + t);
    }
    return S;
}

/* From-scratch residual r = A f - Pm in FP64 (Eq. 1 and Eq. 4). */
static double full_residual(int32_t N, int32_t U, int32_t K, const int64_t* row_ptr,
                            const int32_t* col, const double* len, int lenf32, const double* f,
                            const double* sino, double* r64)
{
    const int64_t NP = (int64_t)N * N, G = (int64_t)U * K;
    for (int64_t g = 0; g < G; ++g) r64[g] = 0.0;
    for (int64_t p = 0; p < NP; ++p)
        for (int64_t e = row_ptr[p]; e < row_ptr[p + 1]; ++e) {
            double l = lenf32 ? (double)(float)len[e] : len[e];
            r64[col[e]] += f[p] * l;
        }
    double sse = 0.0;
    for (int64_t g = 0; g < G; ++g) {
        r64[g] -= sino[g];
        sse += r64[g] * r64[g];
    }
    return sse;
}

/*
 * Eq. 8: starting from the initial image, draw single-pixel estimates until
 * q_auto of them raise the cost, and set T0 = -mean(C' - C) / ln 0.9 over
 * those (90 % acceptance of an average uphill move).  Estimates use Philox
 * counter (q, 0, 2, 0).  Returns -1 if fewer than q_auto uphill estimates
 * appear within 1000 * q_auto draws.
 */
static int auto_t0(const or_sat_params* prm, int64_t P, const int32_t* support,
                   const int64_t* row_ptr, const int32_t* col, const double* len, const double* f,
                   const double* r64, const float* r32, double sse, double KU, double* T0)
{
    uint64_t key[2] = {prm->seed, prm->chain_id};
    double sum = 0.0;
    int64_t found = 0;
    int64_t limit = 1000 * (int64_t)prm->q_auto;
    for (int64_t q = 0; q < limit && found < prm->q_auto; ++q) {
        int32_t p;
        double fn, d;
        draw_estimate(key, (uint64_t)q, 0, 2, P, support, f, prm, &p, &fn, &d);
        double S = prm->precision ? (double)or_delta_sse32(row_ptr, col, len, r32, p, d)
                                  : or_delta_sse64(row_ptr, col, len, r64, p, d, NULL);
        double dC = cost_change(sse, S, KU);
        if (dC > 0.0) {
            sum += dC;
            ++found;
        }
    }
    if (found < prm->q_auto) return -1;
    *T0 = -sum / ((double)prm->q_auto * log(0.9));
    return 0;
}

/*
 * One SAT chain (Steps 1-4 with PILA, Eq. 6-7, BoME, Eq. 2 cooling).
 *
 * Step s, estimate m < m_cand: Philox counter (s, m, 0, 0) draws the
 * estimate; its change of the squared-residual sum S_m comes from Eq. 7's
 * inner sum over the pixel's PILA row.  The best estimate is the first
 * minimal S_m (minimal C' is minimal S, C' being increasing in S).  The cost
 * change Delta C = C' - C decides acceptance (Step 4): accept when
 * Delta C <= 0, else when N1 < exp(-Delta C / T) with N1 uniform in [0, 1)
 * from Philox counter (s, 0, 1, 0).  On acceptance the pixel takes its new
 * value, the residual sinogram gets Eq. 6 on the pixel's row, and the
 * running sum of squares gets S.
 *
 * f is the N*N image (in: starting image, out: result).  sino is Pm (U*K).
 * Trace arrays (n_steps each, nullable): chosen estimate, acceptance,
 * Delta C, and the scale sum|terms| / KU / (C' + C) that bounds the
 * rounding of Delta C.  r_out (nullable, U*K) receives the final running
 * residual (the FP32 one widened, in FP32 mode).  Returns 0, or -1 on bad input, -2 when Eq. 8 finds
 * too few uphill estimates.
 */
int or_sat_run(int32_t N, int32_t U, int32_t K, const uint8_t* mask, const int64_t* row_ptr,
               const int32_t* col, const double* len, const double* sino,
               const or_sat_params* prm, double* f, or_sat_stats* st, int32_t* tr_m,
               uint8_t* tr_acc, double* tr_dc, double* tr_scale, double* r_out)
{
    const int64_t NP = (int64_t)N * N, G = (int64_t)U * K;
    const double KU = (double)K * (double)U;
    if (prm->m_cand < 1 || prm->n_steps < 0 || prm->n_stages < 1) return -1;
    int64_t P = 0;
    for (int64_t p = 0; p < NP; ++p) P += (!mask || mask[p]) ? 1 : 0;
    if (P == 0) return -1;
    int32_t* support = (int32_t*)malloc(sizeof(int32_t) * (size_t)P);
    P = 0;
    for (int64_t p = 0; p < NP; ++p)
        if (!mask || mask[p]) support[P++] = (int32_t)p;

    const int f32 = prm->precision != 0;
    double* r64 = (double*)malloc(sizeof(double) * (size_t)G);
    float* r32 = f32 ? (float*)malloc(sizeof(float) * (size_t)G) : NULL;
    double sse = full_residual(N, U, K, row_ptr, col, len, f32, f, sino, r64);
    if (f32)
        for (int64_t g = 0; g < G; ++g) r32[g] = (float)r64[g];

    double T0 = prm->T0, TN = prm->TN;
    if (!(T0 > 0.0)) {
        if (auto_t0(prm, P, support, row_ptr, col, len, f, r64, r32, sse, KU, &T0) != 0) {
            free(support);
            free(r64);
            free(r32);
            return -2;
        }
        TN = T0 / prm->tn_ratio;
    }

    uint64_t key[2] = {prm->seed, prm->chain_id};
    int64_t accepts = 0, accepts_nz = 0, since_sync = 0;
    int32_t resyncs = 0;
    double drift_r = 0.0, drift_sse = 0.0;

    for (int64_t s = 0; s < prm->n_steps; ++s) {
        double T = or_temperature(s, prm->n_steps, prm->n_stages, T0, TN, prm->schedule);
        int32_t best_m = -1, best_p = 0;
        double best_S = INFINITY, best_fn = 0.0, best_d = 0.0, best_abs = 0.0;
        for (int32_t m = 0; m < prm->m_cand; ++m) {
            int32_t p;
            double fn, d, sabs = 0.0;
            draw_estimate(key, (uint64_t)s, (uint64_t)m, 0, P, support, f, prm, &p, &fn, &d);
            double S = f32 ? (double)or_delta_sse32(row_ptr, col, len, r32, p, d)
                           : or_delta_sse64(row_ptr, col, len, r64, p, d, &sabs);
            if (S < best_S || best_m < 0) {
                best_S = S;
                best_m = m;
                best_p = p;
                best_fn = fn;
                best_d = d;
                best_abs = sabs;
            }
        }
        double dC = cost_change(sse, best_S, KU);
        uint64_t actr[4] = {(uint64_t)s, 0, 1, 0}, aw[4];
        or_philox(key, actr, aw);
        double N1 = u01(aw[0]);
        int accept = (dC <= 0.0) || (N1 < exp(-dC / T));
        if (tr_m) tr_m[s] = best_m;
        if (tr_acc) tr_acc[s] = (uint8_t)accept;
        if (tr_dc) tr_dc[s] = dC;
        if (tr_scale) {
            double den = sqrt(fmax(sse + best_S, 0.0) / KU) + sqrt(sse / KU);
            tr_scale[s] = den > 0.0 ? (best_abs / KU) / den : 0.0;
        }
        if (accept) {
            f[best_p] = best_fn;
            for (int64_t e = row_ptr[best_p]; e < row_ptr[best_p + 1]; ++e) {
                if (f32)
                    r32[col[e]] += (float)best_d * (float)len[e];
                else
                    r64[col[e]] += best_d * len[e];
            }
            sse += best_S;
            ++accepts;
            if (best_d != 0.0) {
                ++accepts_nz;
                ++since_sync;
            }
            if (f32 && prm->resync_every > 0 && since_sync >= prm->resync_every) {
                double sse64 = full_residual(N, U, K, row_ptr, col, len, 1, f, sino, r64);
                for (int64_t g = 0; g < G; ++g) {
                    double dr = fabs((double)r32[g] - r64[g]);
                    if (dr > drift_r) drift_r = dr;
                    r32[g] = (float)r64[g];
                }
                double ds = sse64 > 0.0 ? fabs(sse - sse64) / sse64 : fabs(sse - sse64);
                if (ds > drift_sse) drift_sse = ds;
                sse = sse64;
                since_sync = 0;
                ++resyncs;
            }
        }
    }
    if (st) {
        st->steps = prm->n_steps;
        st->accepts = accepts;
        st->accepts_nonzero = accepts_nz;
        st->resyncs = resyncs;
        st->pad = 0;
        st->T0_used = T0;
        st->TN_used = TN;
        st->sse_final = sse;
        st->cost_final = sqrt(fmax(sse, 0.0) / KU);
        st->max_drift_r = drift_r;
        st->max_drift_sse = drift_sse;
    }
    if (r_out)
        for (int64_t g = 0; g < G; ++g) r_out[g] = f32 ? (double)r32[g] : r64[g];
    free(support);
    free(r64);
    free(r32);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* SIRT with exact lengths (Sec. III-D, Eq. 10-11), simultaneous form       */
/* ------------------------------------------------------------------------ */

/*
 * Factor matrix (Sec. III-D): W_g = sum over support pixels of l(p, g)^2.
 * Iteration: res = Pm - A f over all rays at once; every pixel then moves by
 * (lambda / U) * sum over its PILA row of l * res_g / W_g (Eq. 10 with the
 * per-angle change of Eq. 11, summed over all rays that cross the pixel,
 * scaled by a relaxation lambda; lambda = 1 is the unrelaxed formula).
 * cost[it] (nullable) receives Eq. 4 of the image entering iteration it.
 */
int or_sirt_run(int32_t N, int32_t U, int32_t K, const int64_t* row_ptr, const int32_t* col,
                const double* len, const double* sino, int32_t n_iter, double lambda, double* f,
                double* cost)
{
    const int64_t NP = (int64_t)N * N, G = (int64_t)U * K;
    const double KU = (double)K * (double)U;
    double* W = (double*)calloc((size_t)G, sizeof(double));
    double* res = (double*)malloc(sizeof(double) * (size_t)G);
    for (int64_t p = 0; p < NP; ++p)
        for (int64_t e = row_ptr[p]; e < row_ptr[p + 1]; ++e) W[col[e]] += len[e] * len[e];
    for (int32_t it = 0; it < n_iter; ++it) {
        or_forward(N, U, K, row_ptr, col, len, f, res);
        double sse = 0.0;
        for (int64_t g = 0; g < G; ++g) {
            res[g] = sino[g] - res[g];
            sse += res[g] * res[g];
        }
        if (cost) cost[it] = sqrt(sse / KU);
        for (int64_t p = 0; p < NP; ++p) {
            if (row_ptr[p] == row_ptr[p + 1]) continue;
            double a = 0.0;
            for (int64_t e = row_ptr[p]; e < row_ptr[p + 1]; ++e) a += len[e] * res[col[e]] / W[col[e]];
            f[p] = f[p] + (lambda / (double)U) * a;
        }
    }
    free(W);
    free(res);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* SIRT with exact lengths, pixel by pixel (Sec. III-D as described)        */
/* ------------------------------------------------------------------------ */

/*
 * Sequential form of Eq. 10-11: the factor matrix W_g = sum over support
 * pixels of l(p, g)^2 is computed once and the calculated projections
 * Pc = A f once; then n_iter times, m_per times: a support pixel p is chosen
 * (Philox key (seed, 0), counter (n * m_per + m, 0, 3, 0), uniform over the
 * support as the annealing chain chooses pixels), it moves by
 * (lambda / U) * sum over its PILA row of l * (Pm_g - Pc_g) / W_g (rays with
 * W_g = 0 add nothing; lambda = 1 is the formula as printed), and its rays'
 * calculated projections get Eq. 6 with that change.  cost[n] (nullable)
 * receives Eq. 4 of the running projections after iteration n.  f is the
 * N*N image (in: start, out: result); support holds the P support pixels.
 */
int or_sirt_seq_run(int32_t N, int32_t U, int32_t K, const int64_t* row_ptr, const int32_t* col,
                    const double* len, const double* sino, int64_t P, const int32_t* support,
                    int32_t n_iter, int64_t m_per, double lambda, uint64_t seed, double* f,
                    double* cost)
{
    const int64_t NP = (int64_t)N * N, G = (int64_t)U * K;
    const double KU = (double)K * (double)U;
    if (P < 1 || n_iter < 0 || m_per < 0) return -1;
    double* W = (double*)calloc((size_t)G, sizeof(double));
    double* Pc = (double*)malloc(sizeof(double) * (size_t)G);
    for (int64_t p = 0; p < NP; ++p)
        for (int64_t e = row_ptr[p]; e < row_ptr[p + 1]; ++e) W[col[e]] += len[e] * len[e];
    or_forward(N, U, K, row_ptr, col, len, f, Pc);
    const uint64_t key[2] = {seed, 0};
    for (int32_t n = 0; n < n_iter; ++n) {
        for (int64_t m = 0; m < m_per; ++m) {
            uint64_t ctr[4] = {(uint64_t)n * (uint64_t)m_per + (uint64_t)m, 0, 3, 0}, w[4];
            or_philox(key, ctr, w);
            int32_t p = support[uindex(w[0], (uint64_t)P)];
            double a = 0.0;
            for (int64_t e = row_ptr[p]; e < row_ptr[p + 1]; ++e)
                if (W[col[e]] > 0.0) a += len[e] * (sino[col[e]] - Pc[col[e]]) / W[col[e]];
            double df = (lambda / (double)U) * a;
            f[p] = f[p] + df;
            for (int64_t e = row_ptr[p]; e < row_ptr[p + 1]; ++e) Pc[col[e]] += df * len[e];
        }
        if (cost) {
            double sse = 0.0;
            for (int64_t g = 0; g < G; ++g) sse += (Pc[g] - sino[g]) * (Pc[g] - sino[g]);
            cost[n] = sqrt(sse / KU);
        }
    }
    free(W);
    free(Pc);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* The projector the PILA replaces: DRT by bilinear interpolation (Sec.     */
/* III-A's comparison method), and annealing with it                        */
/* ------------------------------------------------------------------------ */

/* Bilinear interpolation of the image at (x, y): pixel (i, j) holds its
 * value at its centre (j - N/2 + 1/2, N/2 - 1/2 - i); outside the grid the
 * image is zero.  With ov_p >= 0 pixel ov_p reads ov_v instead. */
static double bilinear(int32_t N, const double* f, double x, double y, int64_t ov_p, double ov_v)
{
    const double h = N / 2.0;
    double cx = x + h - 0.5, cy = h - 0.5 - y; /* column and row coordinates */
    double j0 = floor(cx), i0 = floor(cy);
    double ax = cx - j0, ay = cy - i0;
    double v = 0.0;
    for (int di = 0; di < 2; ++di)
        for (int dj = 0; dj < 2; ++dj) {
            double i = i0 + di, j = j0 + dj;
            if (i < 0 || j < 0 || i >= N || j >= N) continue;
            int64_t p = (int64_t)i * N + (int64_t)j;
            double fv = (p == ov_p) ? ov_v : f[p];
            double wgt = (di ? ay : 1.0 - ay) * (dj ? ax : 1.0 - ax);
            v += wgt * fv;
        }
    return v;
}

/* Samples per ray of the DRT: unit spacing t = -T .. T along the ray with
 * T = ceil(N / sqrt 2) + 1, which covers every point where the bilinear
 * image can be nonzero. */
int32_t or_drt_half_span(int32_t N) { return (int32_t)ceil(N / sqrt(2.0)) + 1; }

/* DRT of one ray (u, k): the sum of bilinear samples at unit steps along
 * x cos + y sin = s_k, i.e. the points (s c - t sn, s sn + t c). */
static double drt_ray(int32_t N, int32_t K, const double* cs, int32_t u, int32_t k, const double* f,
                      int64_t ov_p, double ov_v)
{
    const double c = cs[2 * u], sn = cs[2 * u + 1];
    const double s = k - (K - 1) / 2.0;
    const int32_t T = or_drt_half_span(N);
    double acc = 0.0;
    for (int32_t t = -T; t <= T; ++t) acc += bilinear(N, f, s * c - t * sn, s * sn + t * c, ov_p, ov_v);
    return acc;
}

/* Eq. 1 computed the conventional way: out[u*K + k] is the DRT of ray
 * (u, k) of image f by bilinear interpolation. */
void or_drt(int32_t N, int32_t U, int32_t K, const double* deg, const double* f, double* out)
{
    double* cs = (double*)malloc(sizeof(double) * 2 * (size_t)U);
    or_trig(U, deg, cs);
    for (int32_t u = 0; u < U; ++u)
        for (int32_t k = 0; k < K; ++k) out[(int64_t)u * K + k] = drt_ray(N, K, cs, u, k, f, -1, 0.0);
    free(cs);
}

/*
 * SAT with the DRT in the evaluation step (Steps 1-4 of Sec. II-A without
 * the PILA): every estimate's image is projected in full by the bilinear
 * DRT and its cost C' taken from Eq. 4 directly; the first estimate of
 * least C' is kept (BoME); Delta C = C' - C decides acceptance as in
 * or_sat_run, with the same estimates, temperatures and acceptance
 * uniforms (Philox counters (s, m, 0, 0) and (s, 0, 1, 0)).  T0 and TN are
 * given.  Trace arrays (nullable, n_steps each): chosen estimate,
 * acceptance, Delta C.  Returns 0, or -1 on bad input.
 */
int or_satdrt_run(int32_t N, int32_t U, int32_t K, const double* deg, const uint8_t* mask,
                  const double* sino, const or_sat_params* prm, double* f, int32_t* tr_m,
                  uint8_t* tr_acc, double* tr_dc, double* cost_final)
{
    const int64_t NP = (int64_t)N * N;
    const double KU = (double)K * (double)U;
    if (prm->m_cand < 1 || prm->n_steps < 0 || prm->n_stages < 1 || !(prm->T0 > 0.0)) return -1;
    int64_t P = 0;
    for (int64_t p = 0; p < NP; ++p) P += (!mask || mask[p]) ? 1 : 0;
    if (P == 0) return -1;
    int32_t* support = (int32_t*)malloc(sizeof(int32_t) * (size_t)P);
    P = 0;
    for (int64_t p = 0; p < NP; ++p)
        if (!mask || mask[p]) support[P++] = (int32_t)p;
    double* cs = (double*)malloc(sizeof(double) * 2 * (size_t)U);
    or_trig(U, deg, cs);
    /* Eq. 4 of an image (with one pixel overridden) through the full DRT */
#define OR_DRT_COST(OVP, OVV, OUT)                                                  \
    do {                                                                            \
        double sse_ = 0.0;                                                          \
        for (int32_t u_ = 0; u_ < U; ++u_)                                          \
            for (int32_t k_ = 0; k_ < K; ++k_) {                                    \
                double d_ = drt_ray(N, K, cs, u_, k_, f, (OVP), (OVV)) -            \
                            sino[(int64_t)u_ * K + k_];                             \
                sse_ += d_ * d_;                                                    \
            }                                                                       \
        (OUT) = sqrt(sse_ / KU);                                                    \
    } while (0)
    double C;
    OR_DRT_COST(-1, 0.0, C);
    const uint64_t key[2] = {prm->seed, prm->chain_id};
    for (int64_t s = 0; s < prm->n_steps; ++s) {
        double T = or_temperature(s, prm->n_steps, prm->n_stages, prm->T0, prm->TN, prm->schedule);
        int32_t best_m = -1, best_p = 0;
        double best_C = INFINITY, best_fn = 0.0;
        for (int32_t m = 0; m < prm->m_cand; ++m) {
            int32_t p;
            double fn, d, Cm;
            draw_estimate(key, (uint64_t)s, (uint64_t)m, 0, P, support, f, prm, &p, &fn, &d);
            OR_DRT_COST(p, fn, Cm);
            if (Cm < best_C || best_m < 0) {
                best_C = Cm;
                best_m = m;
                best_p = p;
                best_fn = fn;
            }
        }
        double dC = best_C - C;
        uint64_t actr[4] = {(uint64_t)s, 0, 1, 0}, aw[4];
        or_philox(key, actr, aw);
        double N1 = u01(aw[0]);
        int accept = (dC <= 0.0) || (N1 < exp(-dC / T));
        if (tr_m) tr_m[s] = best_m;
        if (tr_acc) tr_acc[s] = (uint8_t)accept;
        if (tr_dc) tr_dc[s] = dC;
        if (accept) {
            f[best_p] = best_fn;
            C = best_C;
        }
    }
#undef OR_DRT_COST
    if (cost_final) *cost_final = C;
    free(support);
    free(cs);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* One-byte lengths (Sec. II-B: length x 180, rounded)                       */
/* ------------------------------------------------------------------------ */

/* q = round(180 l) (halves away from zero) for each of n lengths; every
 * length lies in [0, sqrt 2], so q fits one byte (at most 255). */
void or_quantize_u8(int64_t n, const double* len, uint8_t* q)
{
    for (int64_t i = 0; i < n; ++i) q[i] = (uint8_t)lround(180.0 * len[i]);
}

/* The length a one-byte entry stands for, q / 180, as a float (the type the
 * residual arithmetic of an FP32 chain uses), widened to double. */
void or_dequantize_u8(int64_t n, const uint8_t* q, double* len)
{
    for (int64_t i = 0; i < n; ++i) len[i] = (double)((float)q[i] / 180.0f);
}
