// Background tail fit and extrapolated false-alarm rate (Sec. IV, Eqs. (6)-(7)).
//
// The cumulative background count n_b(x) falls linearly on a log scale for large network SNR, so
// above x_fit the counted background of Eq. (6) is replaced by the least-squares line of Eq. (7),
// log n_b = alpha + beta x, fitted to the counts on a grid of edges (the counts come from
// hs_timeslide_coinc).  The fit is a few dozen host operations.  On the device, one pass over the
// records settles the background records and the zero-lag ones inside the fit range and lists
// the other zero-lag ones; then each workgroup stages a chunk of records in LDS and counts, for
// every listed one, the background records of its chunk at or above its statistic (the records
// are read once, whatever the number of zero-lag coincidences); a last pass forms Eq. (6).
#include <cmath>

#include "hs_internal.h"

namespace hs {

static constexpr int FAR_CHUNK = 1024;  // records staged per workgroup of far_count

// Background records get -1, zero-lag ones at or above x_fit the fitted rate; the other zero-lag
// records are listed (in any order: each one's result depends on it alone) with their statistic.
__global__ __launch_bounds__(256) void far_mark(const hs_coinc *__restrict__ c, int64_t n_c, double t_b, double alpha,
                                                double beta, double x_fit, double *__restrict__ far_out,
                                                uint32_t *__restrict__ n_list, uint32_t *__restrict__ list,
                                                float *__restrict__ list_stat, unsigned long long *__restrict__ cnt) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n_c) return;
    const hs_coinc x = c[i];
    if (x.slide != 0) {
        far_out[i] = -1.0;
        return;
    }
    const double rho = sqrt((double)x.stat);
    if (rho >= x_fit) {
        far_out[i] = exp(alpha + beta * rho) / t_b;
        return;
    }
    const uint32_t k = atomicAdd(n_list, 1u);
    list[k] = (uint32_t)i;
    list_stat[k] = x.stat;
    cnt[k] = 0ull;
}

// cnt[k] += #{background records of this workgroup's chunk with stat >= list_stat[k]}: the chunk's
// statistics are staged in LDS, and each thread takes listed records in turn and compares them
// with the whole chunk (every lane reads the same LDS words: broadcasts, no bank conflicts).
__global__ __launch_bounds__(256) void far_count(const hs_coinc *__restrict__ c, int64_t n_c,
                                                 const uint32_t *__restrict__ n_list,
                                                 const float *__restrict__ list_stat,
                                                 unsigned long long *__restrict__ cnt) {
    __shared__ float4 st4[FAR_CHUNK / 4];
    float *st = reinterpret_cast<float *>(st4);
    const int64_t c0 = (int64_t)blockIdx.x * FAR_CHUNK;
    const int tid = threadIdx.x;
    for (int j = tid; j < FAR_CHUNK; j += 256) {
        const int64_t r = c0 + j;
        // -inf never reaches a statistic: padding and zero-lag records count for nothing
        st[j] = (r < n_c && c[r].slide != 0) ? c[r].stat : -INFINITY;
    }
    __syncthreads();
    const uint32_t nl = *n_list;
    for (uint32_t k = tid; k < nl; k += 256) {
        const float s = list_stat[k];
        uint32_t m = 0;
#pragma unroll 8
        for (int j = 0; j < FAR_CHUNK / 4; ++j) {
            const float4 q = st4[j];
            m += (q.x >= s ? 1u : 0u) + (q.y >= s ? 1u : 0u) + (q.z >= s ? 1u : 0u) + (q.w >= s ? 1u : 0u);
        }
        if (m) atomicAdd(&cnt[k], (unsigned long long)m);
    }
}

__global__ __launch_bounds__(256) void far_finish(const uint32_t *__restrict__ n_list,
                                                  const uint32_t *__restrict__ list,
                                                  const unsigned long long *__restrict__ cnt, double t_b,
                                                  double *__restrict__ far_out) {
    const uint32_t nl = *n_list;
    for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < nl; k += gridDim.x * blockDim.x)
        far_out[list[k]] = (1.0 + (double)cnt[k]) / t_b;
}

}  // namespace hs

using namespace hs;

extern "C" int hs_far_fit(const float *edges, const int64_t *counts, int32_t n_edges, float x_min, double *alpha,
                          double *beta, int32_t *n_used) {
    HS_REQUIRE(alpha && beta && n_used, "hs_far_fit: null output");
    HS_REQUIRE(n_edges >= 0 && (n_edges == 0 || (edges && counts)), "hs_far_fit: bad edges");
    double sx = 0.0, sy = 0.0;
    int m = 0;
    for (int e = 0; e < n_edges; ++e)
        if (edges[e] >= x_min && counts[e] > 0) {
            sx += (double)edges[e];
            sy += std::log((double)counts[e]);
            ++m;
        }
    *n_used = m;
    HS_REQUIRE(m >= 2, "hs_far_fit: the fit needs two edges >= x_min with non-zero counts (got %d)", m);
    const double xm = sx / m, ym = sy / m;
    double sxy = 0.0, sxx = 0.0;
    for (int e = 0; e < n_edges; ++e)
        if (edges[e] >= x_min && counts[e] > 0) {
            const double dx = (double)edges[e] - xm;
            sxy += dx * (std::log((double)counts[e]) - ym);
            sxx += dx * dx;
        }
    HS_REQUIRE(sxx > 0.0, "hs_far_fit: the fit needs two distinct edges");
    *beta = sxy / sxx;
    *alpha = ym - *beta * xm;
    return HS_OK;
}

extern "C" int hs_far(hs_ctx *ctx, const hs_coinc *c, int64_t n_c, double t_b, double alpha, double beta,
                      float x_fit, double *far_out) {
    HS_REQUIRE(ctx && n_c >= 0, "hs_far: bad argument");
    HS_REQUIRE(t_b > 0.0, "hs_far: background time must be positive");
    if (n_c == 0) return HS_OK;
    HS_REQUIRE(c && far_out, "hs_far: null argument");
    HS_REQUIRE(n_c < (int64_t(1) << 31), "hs_far: too many coincidences");
    HS_HIP(hipSetDevice(ctx->device));
    uint32_t *n_list, *list;
    float *list_stat;
    unsigned long long *cnt;
    Carver cv;
    cv.add(&n_list, 1);
    cv.add(&list, n_c);
    cv.add(&list_stat, n_c);
    cv.add(&cnt, n_c);
    HS_TRY(cv.commit(ctx));
    HS_TRY(fill_u32(ctx, n_list, 1, 0));
    const unsigned g = (unsigned)cdiv(n_c, 256);
    hipLaunchKernelGGL(far_mark, dim3(g), dim3(256), 0, ctx->stream, c, n_c, t_b, alpha, beta, (double)x_fit, far_out,
                       n_list, list, list_stat, cnt);
    hipLaunchKernelGGL(far_count, dim3((unsigned)cdiv(n_c, FAR_CHUNK)), dim3(256), 0, ctx->stream, c, n_c, n_list,
                       list_stat, cnt);
    hipLaunchKernelGGL(far_finish, dim3(g < 1024 ? g : 1024), dim3(256), 0, ctx->stream, n_list, list, cnt, t_b,
                       far_out);
    HS_HIP(hipGetLastError());
    return HS_OK;
}

extern "C" double hs_far_threshold(double alpha, double beta, double t_b, double ifar) {
    return (std::log(t_b / ifar) - alpha) / beta;
}
