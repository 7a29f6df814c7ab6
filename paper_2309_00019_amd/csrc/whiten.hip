// PSD estimation (Welch, float64) and whitened data spectrum (float32 transform).
//
// The paper weights its inner product (Sec. II, Eq. (2)) by the one-sided PSD S_n(f) but does
// not say how S_n is obtained; this file takes Welch's method (periodic Hann window, 50 %
// overlap, mean of periodograms, no detrending, one-sided density) interpolated linearly onto
// the segment's frequency grid.  Both steps run once per segment, off the per-template loop.
#include <cmath>

#include "dft.h"
#include "hs_internal.h"

namespace hs {

// Windowed Welch segments as complex float64: seg[j][i] = strain[j*step + i] * w[i],
// w[i] = 1/2 - 1/2 cos(2 pi i / L) taken from the float64 twiddle table of length L.
__global__ __launch_bounds__(256) void welch_segments(const float *__restrict__ strain, int64_t L,
                                                      int64_t step, int64_t n_seg,
                                                      const double2 *__restrict__ tw,
                                                      double2 *__restrict__ seg) {
    const int64_t gid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (gid >= L * n_seg) return;
    const int64_t j = gid / L;
    const int64_t i = gid - j * L;
    const double w = 0.5 - 0.5 * tw[i].x;
    seg[gid] = double2{(double)strain[j * step + i] * w, 0.0};
}

// Mean periodogram with density scaling and one-sided doubling, bins 0..L/2.
__global__ __launch_bounds__(256) void welch_average(const double2 *__restrict__ X, int64_t L,
                                                     int64_t n_seg, double fs, double wss,
                                                     double *__restrict__ pw) {
    const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (q > L / 2) return;
    double acc = 0.0;
    for (int64_t j = 0; j < n_seg; ++j) {
        const double2 v = X[j * L + q];
        acc += v.x * v.x + v.y * v.y;
    }
    double p = acc / (double)n_seg / (fs * wss);
    if (q > 0 && q < L / 2) p *= 2.0;
    pw[q] = p;
}

// Linear interpolation from the Welch grid (j fs / L) onto k fs / n, k = 0..n/2:
// p = slope * (f_k - f_j) + p_j with slope = (p_{j+1} - p_j) / (f_{j+1} - f_j), rounded
// operation by operation (no contraction) so it matches a plain evaluation of the formula.
__global__ __launch_bounds__(256) void welch_interp(const double *__restrict__ pw, int64_t L, int64_t n,
                                                    double fs, double *__restrict__ psd) {
    const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k > n / 2) return;
    const int64_t ratio = n / L;  // n and L are powers of two, L <= n
    const int64_t j = k / ratio;
    if (j >= L / 2) {
        psd[k] = pw[L / 2];
        return;
    }
    const double fk = __dmul_rn((double)k, fs / (double)n);
    const double fj = __dmul_rn((double)j, fs / (double)L);
    const double fj1 = __dmul_rn((double)(j + 1), fs / (double)L);
    const double slope = __ddiv_rn(__dsub_rn(pw[j + 1], pw[j]), __dsub_rn(fj1, fj));
    psd[k] = __dadd_rn(__dmul_rn(slope, __dsub_rn(fk, fj)), pw[j]);
}

// The real series as n/2 complex samples z[j] = s[2j] + i s[2j+1] (the transform of a real
// series of length n from one of length n/2).
__global__ __launch_bounds__(256) void pack_pairs(const float *__restrict__ s, int64_t h, float2 *__restrict__ z) {
    const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (j < h) z[j] = float2{s[2 * j], s[2 * j + 1]};
}

// With Z the n/2-point transform of z, the even and odd samples' transforms are
// E_k = (Z_k + conj Z_{n/2-k}) / 2 and O_k = (Z_k - conj Z_{n/2-k}) / (2i) (Z_{n/2} = Z_0), and
// the series' transform is X_k = E_k + exp(-2 pi i k / n) O_k.  Then d~[k] = dt X[k] / sqrt(S[k])
// for k_lo <= k < n/2, 0 below k_lo; the recombination runs in float64 (exact sincospi of k / n).
__global__ __launch_bounds__(256) void whiten_r2c(const float2 *__restrict__ Z, int64_t n, int64_t k_lo,
                                                  double dt, const double *__restrict__ psd,
                                                  float2 *__restrict__ out) {
    const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t h = n / 2;
    if (k >= h) return;
    if (k < k_lo) {
        out[k] = float2{0.0f, 0.0f};
        return;
    }
    const float2 a = Z[k], b = Z[(h - k) & (h - 1)];
    const double er = 0.5 * ((double)a.x + (double)b.x), ei = 0.5 * ((double)a.y - (double)b.y);
    const double orr = 0.5 * ((double)a.y + (double)b.y), oi = -0.5 * ((double)a.x - (double)b.x);
    double sn, cs;
    sincospi(2.0 * (double)k / (double)n, &sn, &cs);  // exp(-2 pi i k / n) = cs - i sn
    const double xr = er + (cs * orr + sn * oi), xi = ei + (cs * oi - sn * orr);
    const double g = dt / sqrt(psd[k]);
    out[k] = float2{(float)(xr * g), (float)(xi * g)};
}

}  // namespace hs

using namespace hs;

extern "C" {

int hs_welch_psd(hs_ctx *ctx, const float *strain, int64_t n, double fs, int64_t seg_len, double *psd_out) {
    HS_REQUIRE(ctx && strain && psd_out, "hs_welch_psd: null argument");
    HS_REQUIRE(is_pow2(n) && is_pow2(seg_len) && seg_len >= 16 && seg_len <= n && seg_len <= 65536,
               "hs_welch_psd: need powers of two with 16 <= seg_len <= min(n, 65536) (n=%lld seg_len=%lld)",
               (long long)n, (long long)seg_len);
    HS_REQUIRE(n <= (int64_t(1) << 26), "hs_welch_psd: n too large");
    HS_REQUIRE(fs > 0, "hs_welch_psd: fs must be positive");
    HS_HIP(hipSetDevice(ctx->device));
    const int64_t L = seg_len, step = L / 2;
    const int64_t n_seg = (n - L) / step + 1;
    const int lg = ilog2(L);
    const double2 *tw;
    HS_TRY(twiddles_f64(ctx, lg, &tw));
    // sum of squared window values, from the same float64 values the kernel reads
    const double wss = hann_sumsq(ctx, lg);
    double2 *a, *b;
    double *pw;
    Carver cv;
    cv.add(&a, L * n_seg);
    cv.add(&b, L * n_seg);
    cv.add(&pw, L / 2 + 1);
    HS_TRY(cv.commit(ctx));
    hipLaunchKernelGGL(welch_segments, dim3((unsigned)cdiv(L * n_seg, 256)), dim3(256), 0, ctx->stream,
                       strain, L, step, n_seg, tw, a);
    HS_HIP(hipGetLastError());
    double2 *X;
    HS_TRY(fft_c2c_f64(ctx, a, b, lg, n_seg, -1, &X));
    hipLaunchKernelGGL(welch_average, dim3((unsigned)cdiv(L / 2 + 1, 256)), dim3(256), 0, ctx->stream, X, L,
                       n_seg, fs, wss, pw);
    hipLaunchKernelGGL(welch_interp, dim3((unsigned)cdiv(n / 2 + 1, 256)), dim3(256), 0, ctx->stream, pw, L, n,
                       fs, psd_out);
    HS_HIP(hipGetLastError());
    return HS_OK;
}

int hs_whiten(hs_ctx *ctx, const float *strain, int64_t n, double fs, double f_low, const double *psd,
              void *spec_out) {
    HS_REQUIRE(ctx && strain && psd && spec_out, "hs_whiten: null argument");
    HS_REQUIRE(is_pow2(n) && n >= 1024 && n <= (int64_t(1) << 22), "hs_whiten: n must be a power of two in [2^10, 2^22]");
    HS_REQUIRE(fs > 0 && f_low >= 0, "hs_whiten: bad fs/f_low");
    HS_HIP(hipSetDevice(ctx->device));
    int64_t k_lo = (int64_t)std::ceil(f_low * (double)n / fs);
    if (k_lo < 1) k_lo = 1;
    // real-input transform: an n/2-point complex transform of the sample pairs, recombined
    const int64_t h = n / 2;
    float2 *a, *b;
    Carver cv;
    cv.add(&a, h);
    cv.add(&b, h);
    HS_TRY(cv.commit(ctx));
    hipLaunchKernelGGL(pack_pairs, dim3((unsigned)cdiv(h, 256)), dim3(256), 0, ctx->stream, strain, h, a);
    HS_HIP(hipGetLastError());
    float2 *Z;
    HS_TRY(fft_c2c_f32(ctx, a, b, ilog2(h), 1, -1, &Z));
    hipLaunchKernelGGL(whiten_r2c, dim3((unsigned)cdiv(h, 256)), dim3(256), 0, ctx->stream, Z, n, k_lo,
                       1.0 / fs, psd, static_cast<float2 *>(spec_out));
    HS_HIP(hipGetLastError());
    return HS_OK;
}

}  // extern "C"
