// Bank preparation: template sigma and pre-whitened, sigma-normalised spectra.
//
// sigma^2 = (h, h) = 4 df sum_{k_lo..k_hi} |h~_k|^2 / S_k (Sec. II, Eq. (2) with x = y = h),
// accumulated in float64.  The stored spectrum w~_k = scale * 4 df h~_k / (sqrt(S_k) sigma) folds
// the PSD weight, the 4 df of Eq. (2) and the template normalisation into the template, so the
// per-template hot loop is a bare conjugate multiply with the whitened data followed by an
// inverse FFT (the SNR of Eq. (1) in the quadrature form of Appendix A).
#include <cmath>

#include "hs_internal.h"
#include "storage.h"

namespace hs {

template <typename ST>
__global__ __launch_bounds__(256) void prepare_bank_kernel(
    int64_t n, double df, int32_t kf, const double *__restrict__ psd, const float2 *__restrict__ raw,
    const int64_t *__restrict__ offset, const int32_t *__restrict__ k0, const int32_t *__restrict__ kstart,
    const int32_t *__restrict__ k1, typename ST::elem *__restrict__ out, int32_t *__restrict__ klo_out,
    int32_t *__restrict__ khi_out, float *__restrict__ r2s_out, double *__restrict__ sigma_out,
    int32_t *__restrict__ bad, bool low_precision) {
    __shared__ double s_sum[256];
    __shared__ double s_max[256];
    const int t = blockIdx.x;
    const int tid = threadIdx.x;
    const int64_t off = offset[t];
    const int32_t a0 = k0[t], a1 = k1[t];
    const int32_t lo = max(max(kf, kstart[t]), 1);
    const int32_t hi = min(a1, (int32_t)(n / 2 - 1));
    if (a1 < a0 || hi < lo || lo < a0) {
        if (tid == 0) {
            atomicOr(bad, 1);
            klo_out[t] = lo;
            khi_out[t] = lo - 1;
            r2s_out[t] = 0.0f;
            sigma_out[t] = 0.0;
        }
        for (int64_t k = a0 + tid; k <= a1; k += 256) out[off + (k - a0)] = ST::pack(0.0f, 0.0f);
        return;
    }
    double sum = 0.0, mx = 0.0;
    bool psd_ok = true;
    for (int64_t k = lo + tid; k <= hi; k += 256) {
        const float2 h = raw[off + (k - a0)];
        psd_ok = psd_ok && psd[k] > 0.0 && psd[k] < INFINITY;
        const double a2 = ((double)h.x * (double)h.x + (double)h.y * (double)h.y) / psd[k];
        sum += a2;
        mx = fmax(mx, a2);
    }
    if (!psd_ok) atomicOr(bad, 2);
    s_sum[tid] = sum;
    s_max[tid] = mx;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (tid < o) {
            s_sum[tid] += s_sum[tid + o];
            s_max[tid] = fmax(s_max[tid], s_max[tid + o]);
        }
        __syncthreads();
    }
    // a template with no power in its band (or a non-finite one) has no normalisation
    if (!(s_sum[0] > 0.0 && s_sum[0] < INFINITY)) {
        if (tid == 0) {
            atomicOr(bad, 4);
            klo_out[t] = lo;
            khi_out[t] = hi;
            r2s_out[t] = 0.0f;
            sigma_out[t] = 0.0;
        }
        for (int64_t k = a0 + tid; k <= a1; k += 256) out[off + (k - a0)] = ST::pack(0.0f, 0.0f);
        return;
    }
    const double sigma = sqrt(4.0 * df * s_sum[0]);
    const double norm = 4.0 * df / sigma;
    double scale = 1.0;
    if (low_precision) {
        // keep the largest stored magnitude in [2^13, 2^14)
        const double mval = sqrt(s_max[0]) * norm;
        int e = 0;
        (void)frexp(mval, &e);
        scale = ldexp(1.0, 14 - e);
    }
    for (int64_t k = a0 + tid; k <= a1; k += 256) {
        float re = 0.0f, im = 0.0f;
        if (k >= lo && k <= hi) {
            const float2 h = raw[off + (k - a0)];
            const double g = norm * scale / sqrt(psd[k]);
            re = (float)((double)h.x * g);
            im = (float)((double)h.y * g);
        }
        out[off + (k - a0)] = ST::pack(re, im);
    }
    if (tid == 0) {
        klo_out[t] = lo;
        khi_out[t] = hi;
        r2s_out[t] = (float)(1.0 / (scale * scale));
        sigma_out[t] = sigma;
    }
}

// Edges of p contiguous bins of equal template power pw_k = |h~_k|^2 / S_k over [lo, hi]:
// edge l (0 < l < p) is the first bin whose cumulative power reaches l/p of the total.
// Each thread sums a contiguous chunk, a block scan gives chunk prefixes, and the thread
// whose prefix interval [P_t, P_t + s_t) contains the threshold walks its chunk to find the
// crossing (if rounding leaves it past the chunk, the edge is the next chunk's first bin),
// so every threshold is placed exactly once and deterministically.
__global__ __launch_bounds__(256) void chisq_edges_kernel(int64_t n, int32_t kf, const double *__restrict__ psd,
                                                          const float2 *__restrict__ raw,
                                                          const int64_t *__restrict__ offset,
                                                          const int32_t *__restrict__ k0,
                                                          const int32_t *__restrict__ kstart,
                                                          const int32_t *__restrict__ k1, int p,
                                                          int32_t *__restrict__ edges) {
    __shared__ double sc[256];
    const int t = blockIdx.x;
    const int tid = threadIdx.x;
    const int64_t off = offset[t];
    const int32_t a0 = k0[t], a1 = k1[t];
    const int32_t lo = max(max(kf, kstart[t]), 1);
    const int32_t hi = min(a1, (int32_t)(n / 2 - 1));
    if (a1 < a0 || hi < lo || lo < a0) return;  // flagged by the preparation kernel
    const int64_t K = (int64_t)hi - lo + 1;
    const int64_t chunk = (K + 255) / 256;
    const int64_t c0 = lo + tid * chunk;
    const int64_t c1 = min((int64_t)hi, c0 + chunk - 1);
    auto pw = [&](int64_t k) {
        const float2 h = raw[off + (k - a0)];
        return ((double)h.x * (double)h.x + (double)h.y * (double)h.y) / psd[k];
    };
    double s = 0.0;
    for (int64_t k = c0; k <= c1; ++k) s += pw(k);
    sc[tid] = s;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
        const double add = tid >= o ? sc[tid - o] : 0.0;
        __syncthreads();
        sc[tid] += add;
        __syncthreads();
    }
    const double next = sc[tid];
    const double prev = tid > 0 ? sc[tid - 1] : 0.0;
    const double total = sc[255];
    int32_t *e = edges + (int64_t)t * (p + 1);
    if (!(total > 0.0 && total < INFINITY)) {  // flagged by the preparation kernel; edges stay defined
        if (tid == 0)
            for (int l = 0; l <= p; ++l) e[l] = (int32_t)(lo + (K * l) / p);
        return;
    }
    for (int l = 1; l < p; ++l) {
        const double T = (double)l * total / (double)p;
        if (!(prev <= T && T < next)) continue;
        double cum = prev;
        int64_t where = c1 + 1;
        for (int64_t k = c0; k <= c1; ++k) {
            cum += pw(k);
            if (cum >= T) {
                where = k;
                break;
            }
        }
        e[l] = (int32_t)where;
    }
    if (tid == 0) {
        e[0] = lo;
        e[p] = hi + 1;
    }
}

}  // namespace hs

using namespace hs;

extern "C" int hs_prepare_bank(hs_ctx *ctx, int64_t n, double fs, double f_low, const double *psd,
                               int32_t n_tmpl, const void *raw, const int64_t *offset, const int32_t *k0,
                               const int32_t *kstart, const int32_t *k1, int32_t dtype, void *spectra_out,
                               int32_t *k_lo_out, int32_t *k_hi_out, float *rho2_scale_out,
                               double *sigma_out, int32_t chisq_bins, int32_t *chisq_edges_out) {
    HS_REQUIRE(ctx && psd && raw && offset && k0 && kstart && k1 && spectra_out && k_lo_out && k_hi_out &&
                   rho2_scale_out && sigma_out,
               "hs_prepare_bank: null argument");
    HS_REQUIRE(n_tmpl >= 0, "hs_prepare_bank: negative n_tmpl");
    HS_REQUIRE(is_pow2(n) && n >= 16 && n <= (int64_t(1) << 24), "hs_prepare_bank: n must be a power of two");
    HS_REQUIRE(fs > 0 && f_low >= 0, "hs_prepare_bank: bad fs/f_low");
    HS_REQUIRE(dtype == HS_F32 || dtype == HS_BF16 || dtype == HS_F16, "hs_prepare_bank: bad dtype %d", dtype);
    HS_REQUIRE(chisq_bins == 0 || (chisq_bins >= 2 && chisq_bins <= 16 && chisq_edges_out),
               "hs_prepare_bank: chisq_bins must be 0 or in [2, 16] with an edge buffer");
    if (n_tmpl == 0) return HS_OK;
    HS_HIP(hipSetDevice(ctx->device));
    int64_t kf = (int64_t)std::ceil(f_low * (double)n / fs);
    if (kf < 1) kf = 1;
    HS_REQUIRE(kf < n / 2, "hs_prepare_bank: f_low at or above Nyquist");
    int32_t *bad;
    Carver cv;
    cv.add(&bad, 1);
    HS_TRY(cv.commit(ctx));
    HS_TRY(fill_u32(ctx, reinterpret_cast<uint32_t *>(bad), 1, 0));
    const double df = fs / (double)n;
    const float2 *r = static_cast<const float2 *>(raw);
    if (dtype == HS_F32)
        hipLaunchKernelGGL(prepare_bank_kernel<StoreF32>, dim3(n_tmpl), dim3(256), 0, ctx->stream, n, df, (int32_t)kf,
                           psd, r, offset, k0, kstart, k1, static_cast<float2 *>(spectra_out), k_lo_out, k_hi_out,
                           rho2_scale_out, sigma_out, bad, false);
    else if (dtype == HS_BF16)
        hipLaunchKernelGGL(prepare_bank_kernel<StoreBF16>, dim3(n_tmpl), dim3(256), 0, ctx->stream, n, df,
                           (int32_t)kf, psd, r, offset, k0, kstart, k1, static_cast<uint32_t *>(spectra_out), k_lo_out,
                           k_hi_out, rho2_scale_out, sigma_out, bad, true);
    else
        hipLaunchKernelGGL(prepare_bank_kernel<StoreF16>, dim3(n_tmpl), dim3(256), 0, ctx->stream, n, df,
                           (int32_t)kf, psd, r, offset, k0, kstart, k1, static_cast<uint32_t *>(spectra_out), k_lo_out,
                           k_hi_out, rho2_scale_out, sigma_out, bad, true);
    HS_HIP(hipGetLastError());
    if (chisq_bins >= 2) {
        hipLaunchKernelGGL(chisq_edges_kernel, dim3(n_tmpl), dim3(256), 0, ctx->stream, n, (int32_t)kf, psd, r, offset,
                           k0, kstart, k1, (int)chisq_bins, chisq_edges_out);
        HS_HIP(hipGetLastError());
    }
    int32_t hbad = 0;
    HS_TRY(read_back(ctx, bad, &hbad, sizeof(hbad)));
    HS_REQUIRE((hbad & 1) == 0, "hs_prepare_bank: a template has an empty band or k1 < k0 / k_lo < k0");
    HS_REQUIRE((hbad & 2) == 0, "hs_prepare_bank: the PSD is not positive and finite inside a template band");
    HS_REQUIRE((hbad & 4) == 0, "hs_prepare_bank: a template has no (or non-finite) power inside its band");
    return HS_OK;
}
