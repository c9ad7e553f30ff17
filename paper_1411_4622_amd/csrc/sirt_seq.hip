// SIRT with exact lengths, pixel by pixel (section III-D as the paper
// describes it: a pixel is chosen, Eq. 11 gives its change from its PILA row
// and the factor matrix, Eq. 10 applies it, and the pixel's rays get the new
// calculated projections through the PILA before the next pixel is chosen).
//
// The updates form one sequence, each reading the projections the previous
// one wrote, so one wavefront runs it: per update, the lanes take the
// pixel's row entries, the row sum is added in the canonical 64-partial
// order, lane 0 updates the pixel, the lanes scatter the change to the
// row's rays (distinct rays: no atomics).  The calculated projections live
// in LDS when they fit, else in global memory.  Pixels are drawn by the same
// Philox4x64-10 as the annealing chain (key (seed, 0), counter (update, 0,
// 3, 0)), uniform over the support.
#include <algorithm>
#include <cmath>
#include <vector>

#include "sat_chain.hpp"
#include "sat_host.hpp"

namespace pila {
namespace {

struct SeqArgs {
    int32_t U, K, P, n_iter;
    int64_t m_per;
    double lambda;
    uint64_t seed;
    const int64_t* row_ptr;
    const int32_t* col;
    const void* len;
    const int32_t* support;
    const double* sino;
    double* W;     // factor matrix (U*K)
    double* pc;    // calculated projections (U*K)
    double* f;     // image (N*N)
    double* cost;  // Eq. 4 after each iteration (n_iter)
};

// Factor matrix W_g = sum of l^2 over the ray's support pixels and the
// projections Pc_g = sum of f_p l, each ray summed in ascending pixel order
// (one thread per ray; products and sums rounded separately).
template <typename LenT>
__global__ __launch_bounds__(256) void seq_setup_kernel(int64_t G, const int64_t* __restrict__ rp,
                                                        const int32_t* __restrict__ ci,
                                                        const LenT* __restrict__ ln, const double* __restrict__ f,
                                                        double* __restrict__ W, double* __restrict__ pc)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < G; g += stride) {
        double w = 0.0, s = 0.0;
        for (int64_t q = rp[g]; q < rp[g + 1]; ++q) {
            const double l = (double)ln[q];
            w = w + l * l;
            s = s + f[ci[q]] * l;
        }
        W[g] = w;
        pc[g] = s;
    }
}

template <typename LenT, bool PCLDS>
__global__ __launch_bounds__(64) void sirt_seq_kernel(SeqArgs A)
{
    extern __shared__ __align__(16) char lds[];
    const int lane = threadIdx.x;
    const int64_t G = (int64_t)A.U * A.K;
    double* pc = PCLDS ? (double*)lds : A.pc;
    if (PCLDS) {
        for (int64_t g = lane; g < G; g += kWave) pc[g] = A.pc[g];
        __syncthreads();
    }
    const LenT* len = (const LenT*)A.len;
    const double scale = A.lambda / (double)A.U;
    for (int32_t n = 0; n < A.n_iter; ++n) {
        for (int64_t m = 0; m < A.m_per; ++m) {
            const uint64_t t = (uint64_t)n * (uint64_t)A.m_per + (uint64_t)m;
            const Words4 w = philox4x64(A.seed, 0, t, 0, 3, 0);
            const int32_t p = A.support[__umul64hi(w.w0, (uint64_t)A.P)];
            const int64_t b = A.row_ptr[p], e = A.row_ptr[p + 1];
            double part = 0.0;
            for (int64_t q = b + lane; q < e; q += kWave) {
                const int32_t g = A.col[q];
                const double wg = A.W[g];
                if (wg > 0.0) part = part + ((double)len[q] * (A.sino[g] - pc[g])) / wg;
            }
            const double df = scale * wave_canon_sum(part);
            if (lane == 0) A.f[p] = A.f[p] + df;
            for (int64_t q = b + lane; q < e; q += kWave) {
                const int32_t g = A.col[q];
                pc[g] = pc[g] + df * (double)len[q];
            }
            __syncthreads();  // this update's projections before the next reads them
        }
        if (A.cost) {
            double sq = 0.0;
            for (int64_t g = lane; g < G; g += kWave) {
                const double d = pc[g] - A.sino[g];
                sq = sq + d * d;
            }
            sq = wave_canon_sum(sq);
            if (lane == 0) A.cost[n] = sqrt(sq / ((double)A.K * (double)A.U));
        }
    }
}

size_t seq_bytes(const pila_geom* g, int32_t n_iter)
{
    const size_t G = (size_t)g->n_angles * g->n_bins;
    return 2 * align256(8 * G) + align256(8 * (size_t)(n_iter > 0 ? n_iter : 1));
}

template <typename LenT>
int32_t seq_impl(const pila_geom* geom, const pila_csr* csr, const double* d_sino, const sirt_seq_params* prm,
                 double* d_image, char* ws, double* h_cost, hipStream_t st)
{
    const int64_t G = (int64_t)geom->n_angles * geom->n_bins;
    SeqArgs A;
    A.U = geom->n_angles;
    A.K = geom->n_bins;
    A.P = csr->n_support;
    A.n_iter = prm->n_iter;
    A.m_per = prm->m_per;
    A.lambda = prm->lambda;
    A.seed = prm->seed;
    A.row_ptr = csr->row_ptr;
    A.col = csr->col;
    A.len = csr->len;
    A.support = csr->support;
    A.sino = d_sino;
    A.W = (double*)ws;
    A.pc = (double*)(ws + align256(8 * (size_t)G));
    A.f = d_image;
    A.cost = (double*)(ws + 2 * align256(8 * (size_t)G));
    if (G > 0)
        seq_setup_kernel<LenT><<<(unsigned)std::min<int64_t>((G + 255) / 256, 4096), 256, 0, st>>>(
            G, csr->t_row_ptr, csr->t_col, (const LenT*)csr->t_len, d_image, A.W, A.pc);
    PILA_HIP(hipGetLastError());
    hipDeviceProp_t prop;
    PILA_TRY(device_props(&prop));
    const int64_t budget = (int64_t)prop.sharedMemPerBlock - 1024;
    if (prm->n_iter > 0 && A.P > 0) {
        if (G * 8 <= budget) {
            const void* k = (const void*)sirt_seq_kernel<LenT, true>;
            PILA_TRY(set_lds(k, (int)(G * 8)));
            void* args[] = {&A};
            PILA_HIP(hipLaunchKernel(k, dim3(1), dim3(kWave), args, (size_t)(G * 8), st));
        } else {
            sirt_seq_kernel<LenT, false><<<1, kWave, 0, st>>>(A);
        }
    }
    PILA_HIP(hipGetLastError());
    if (h_cost && prm->n_iter > 0) {
        PILA_HIP(hipMemcpyAsync(h_cost, A.cost, sizeof(double) * (size_t)prm->n_iter, hipMemcpyDeviceToHost, st));
        PILA_HIP(hipStreamSynchronize(st));
    }
    return PILA_OK;
}

}  // namespace
}  // namespace pila

using namespace pila;

extern "C" int32_t sirt_seq_workspace_size(const pila_geom* geom, const sirt_seq_params* params, size_t* bytes)
{
    clear_error();
    PILA_TRY(check_geom(geom));
    if (!params || !bytes) return fail(PILA_EINVAL, "params or bytes is NULL");
    if (params->n_iter < 0 || params->m_per < 0) return fail(PILA_EINVAL, "n_iter and m_per must be >= 0");
    *bytes = seq_bytes(geom, params->n_iter);
    return PILA_OK;
}

extern "C" int32_t sirt_seq_run(const pila_geom* geom, const pila_csr* csr, const double* d_sino,
                                const sirt_seq_params* params, double* d_image, void* d_ws, size_t ws_bytes,
                                double* h_cost, void* stream)
{
    clear_error();
    PILA_TRY(check_geom(geom));
    if (!csr || !params || !d_sino || !d_image) return fail(PILA_EINVAL, "csr, params, sinogram or image is NULL");
    if (!csr->row_ptr || !csr->col || !csr->len || !csr->support || !csr->t_row_ptr || !csr->t_col || !csr->t_len)
        return fail(PILA_EINVAL, "PILA arrays (pixel-major, ray-major and support) are required");
    if (params->n_iter < 0 || params->m_per < 0) return fail(PILA_EINVAL, "n_iter and m_per must be >= 0");
    if (!std::isfinite(params->lambda)) return fail(PILA_EINVAL, "lambda is not finite");
    if (params->m_per > 0 && csr->n_support < 1) return fail(PILA_EINVAL, "empty support");
    const size_t need = seq_bytes(geom, params->n_iter);
    if (!d_ws || ws_bytes < need)
        return fail(PILA_ENOMEM, "workspace of %zu bytes is below the %zu needed", ws_bytes, need);
    hipStream_t st = (hipStream_t)stream;
    if (geom->len_dtype == PILA_F64)
        return seq_impl<double>(geom, csr, d_sino, params, d_image, (char*)d_ws, h_cost, st);
    if (geom->len_dtype == PILA_F32)
        return seq_impl<float>(geom, csr, d_sino, params, d_image, (char*)d_ws, h_cost, st);
    return seq_impl<LenQ>(geom, csr, d_sino, params, d_image, (char*)d_ws, h_cost, st);
}
