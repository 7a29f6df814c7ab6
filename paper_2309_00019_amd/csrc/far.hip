// Background tail fit and extrapolated false-alarm rate (Sec. IV, Eqs. (6)-(7)).
//
// The cumulative background count n_b(x) falls linearly on a log scale for large network SNR, so
// above x_fit the counted background of Eq. (6) is replaced by the least-squares line of Eq. (7),
// log n_b = alpha + beta x, fitted to the counts on a grid of edges (the counts come from
// hs_timeslide_coinc).  The fit is a few dozen host operations; the per-foreground counting of
// background survivors runs on the device (one workgroup per coincidence of the sorted output,
// background records scanned with a workgroup reduction).
#include <cmath>

#include "hs_internal.h"

namespace hs {

__global__ __launch_bounds__(256) void far_kernel(const hs_coinc *__restrict__ c, int64_t n_c, double t_b,
                                                  double alpha, double beta, double x_fit,
                                                  double *__restrict__ far_out) {
    __shared__ unsigned long long red[256];
    const int64_t i = blockIdx.x;
    const hs_coinc x = c[i];
    if (x.slide != 0) {
        if (threadIdx.x == 0) far_out[i] = -1.0;
        return;
    }
    const double rho = sqrt((double)x.stat);
    if (rho >= x_fit) {
        if (threadIdx.x == 0) far_out[i] = exp(alpha + beta * rho) / t_b;
        return;
    }
    unsigned long long cnt = 0;
    for (int64_t j = threadIdx.x; j < n_c; j += 256) {
        const hs_coinc y = c[j];
        cnt += (y.slide != 0 && y.stat >= x.stat) ? 1ull : 0ull;
    }
    red[threadIdx.x] = cnt;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) far_out[i] = (1.0 + (double)red[0]) / t_b;
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
    hipLaunchKernelGGL(far_kernel, dim3((unsigned)n_c), dim3(256), 0, ctx->stream, c, n_c, t_b, alpha, beta,
                       (double)x_fit, far_out);
    HS_HIP(hipGetLastError());
    return HS_OK;
}

extern "C" double hs_far_threshold(double alpha, double beta, double t_b, double ifar) {
    return (std::log(t_b / ifar) - alpha) / beta;
}
