// Power-consistency chi-square at trigger samples and the re-weighted SNR of Eq. (4).
//
// Sec. II down-weights triggers with the chi-square test it cites; the test splits the template
// band into p bins of equal template power and compares each bin's share of the complex SNR with
// 1/p of the total.  Only triggers (a few per template) are tested, so each trigger gets one
// workgroup that evaluates the p band-limited SNRs z_l at its sample by direct sums over the band:
// q_k = d~_k conj(w~_k) times the phasor W_N^{(k m) mod N} from the two-level twiddle table,
// accumulated in float64 per bin, reduced across the workgroup with wavefront shuffles.
#include <cmath>

#include "dft.h"
#include "hs_internal.h"
#include "storage.h"

namespace hs {

template <typename ST, int P>
__global__ __launch_bounds__(256) void chisq_kernel(const float2 *__restrict__ dspec, int64_t n,
                                                    const typename ST::elem *__restrict__ spectra,
                                                    const int64_t *__restrict__ offset, const int32_t *__restrict__ k0,
                                                    const int32_t *__restrict__ klo, const int32_t *__restrict__ khi,
                                                    const float *__restrict__ r2s, const int32_t *__restrict__ edges,
                                                    const hs_trigger *trig, int32_t n_tmpl, int64_t seg_t0,
                                                    int64_t tps, float rho_min, const float2 *__restrict__ twlo,
                                                    const float2 *__restrict__ twhi, float *__restrict__ chisq_out,
                                                    hs_trigger *trig_out, float *__restrict__ bins_out,
                                                    int32_t *__restrict__ bad) {
    __shared__ double red[4][2 * P];
    const int64_t i = blockIdx.x;
    const hs_trigger tr = trig[i];
    const int tid = threadIdx.x;
    bool skip = !(tr.snr >= rho_min);
    int64_t m = 0;
    if (!skip) {
        const int64_t dt = tr.tick - seg_t0;
        if (tr.tmpl < 0 || tr.tmpl >= n_tmpl) {
            if (tid == 0) atomicOr(bad, 1);
            skip = true;
        } else if (dt < 0 || dt % tps != 0 || dt / tps >= n) {
            if (tid == 0) atomicOr(bad, 2);
            skip = true;
        } else {
            m = dt / tps;
        }
    }
    if (skip) {
        if (tid == 0) {
            chisq_out[i] = 0.0f;
            trig_out[i] = tr;
        }
        if (bins_out && tid < P) bins_out[i * P + tid] = 0.0f;
        return;
    }
    const int t = tr.tmpl;
    const int32_t *e = edges + (int64_t)t * (P + 1);
    const int64_t base = offset[t] - k0[t];
    const uint64_t mask = (uint64_t)n - 1;
    // every bin is clamped to the template's band, which lies inside [1, n/2 - 1]
    const int64_t band_lo = klo[t] > 1 ? klo[t] : 1;
    const int64_t band_hi = khi[t] < n / 2 - 1 ? khi[t] : n / 2 - 1;
#pragma unroll
    for (int l = 0; l < P; ++l) {
        double ar = 0.0, ai = 0.0;
        const int64_t b0 = e[l] > band_lo ? e[l] : band_lo;
        const int64_t b1 = e[l + 1] < band_hi + 1 ? e[l + 1] : band_hi + 1;
        for (int64_t k = b0 + tid; k < b1; k += 256) {
            const float2 q = cmulc(dspec[k], ST::load(spectra, base + k));
            const uint64_t idx = ((uint64_t)k * (uint64_t)m) & mask;
            const float2 w = cmul(twhi[idx >> 10], twlo[idx & 1023]);
            const float2 v = cmul(q, w);
            ar += (double)v.x;
            ai += (double)v.y;
        }
        for (int o = 32; o > 0; o >>= 1) {
            ar += __shfl_down(ar, o);
            ai += __shfl_down(ai, o);
        }
        if ((tid & 63) == 0) {
            red[tid >> 6][2 * l] = ar;
            red[tid >> 6][2 * l + 1] = ai;
        }
    }
    __syncthreads();
    if (tid == 0) {
        const double s = sqrt((double)r2s[t]);  // undoes the storage scale of the template
        double zr[P], zi[P], Zr = 0.0, Zi = 0.0;
#pragma unroll
        for (int l = 0; l < P; ++l) {
            zr[l] = (red[0][2 * l] + red[1][2 * l] + red[2][2 * l] + red[3][2 * l]) * s;
            zi[l] = (red[0][2 * l + 1] + red[1][2 * l + 1] + red[2][2 * l + 1] + red[3][2 * l + 1]) * s;
            Zr += zr[l];
            Zi += zi[l];
        }
        double chi2 = 0.0;
#pragma unroll
        for (int l = 0; l < P; ++l) {
            const double dr = zr[l] - Zr / P, di = zi[l] - Zi / P;
            chi2 += dr * dr + di * di;
            if (bins_out) bins_out[i * P + l] = (float)(P * (dr * dr + di * di));
        }
        const double c = chi2 * P / (2.0 * P - 2.0);
        double rw = (double)tr.snr;
        if (c >= 1.0) rw = rw / pow((1.0 + c * c * c) / 2.0, 1.0 / 6.0);
        chisq_out[i] = (float)c;
        hs_trigger o = tr;
        o.snr = (float)rw;
        trig_out[i] = o;
    }
}

template <typename ST>
static int launch_chisq(hs_ctx *ctx, int p, int64_t n_trig, const float2 *d, int64_t n, const hs_bank *bank,
                        const hs_trigger *trig, int64_t seg_t0, int64_t tps, float rho_min, const float2 *twlo,
                        const float2 *twhi, float *chisq_out, hs_trigger *trig_out, float *bins_out,
                        int32_t *bad) {
    const auto *sp = static_cast<const typename ST::elem *>(bank->spectra);
#define HS_CQ(PP)                                                                                                  \
    case PP:                                                                                                       \
        hipLaunchKernelGGL((chisq_kernel<ST, PP>), dim3((unsigned)n_trig), dim3(256), 0, ctx->stream, d, n, sp,     \
                           bank->offset, bank->k0, bank->k_lo, bank->k_hi, bank->rho2_scale, bank->chisq_edges,    \
                           trig, bank->n_tmpl, seg_t0,                                                           \
                           tps, rho_min, twlo, twhi, chisq_out, trig_out, bins_out, bad);                         \
        break;
    switch (p) {
        HS_CQ(2) HS_CQ(4) HS_CQ(8) HS_CQ(16)
    default: return set_error(HS_EINVAL, "hs_chisq: chisq_bins must be 2, 4, 8 or 16 (got %d)", p);
    }
#undef HS_CQ
    HS_HIP(hipGetLastError());
    return HS_OK;
}

}  // namespace hs

using namespace hs;

extern "C" int hs_chisq(hs_ctx *ctx, const void *spec, int64_t n, double fs, const hs_bank *bank,
                        const hs_trigger *trig, int64_t n_trig, int64_t seg_t0, int64_t ticks_per_sample,
                        float rho_min, float *chisq_out, hs_trigger *trig_out, float *bins_out) {
    HS_REQUIRE(ctx && bank, "hs_chisq: null argument");
    HS_REQUIRE(n_trig >= 0 && n_trig < (int64_t(1) << 31), "hs_chisq: bad trigger count");
    if (n_trig == 0) return HS_OK;
    HS_REQUIRE(spec && trig && chisq_out && trig_out, "hs_chisq: null argument");
    HS_REQUIRE(is_pow2(n) && n >= 8192 && n <= (int64_t(1) << 22), "hs_chisq: n must be a power of two in [2^13, 2^22]");
    HS_REQUIRE(bank->n == n && bank->fs == fs, "hs_chisq: bank prepared for another n or fs");
    HS_REQUIRE(bank->chisq_bins >= 2 && bank->chisq_edges, "hs_chisq: bank has no chi-square bins");
    HS_REQUIRE(ticks_per_sample > 0, "hs_chisq: ticks_per_sample must be positive");
    HS_HIP(hipSetDevice(ctx->device));
    const int log2N = ilog2(n);
    const float2 *twlo, *twhi;
    HS_TRY(twiddles_f32(ctx, log2N, &twlo));
    HS_TRY(twiddles_f32(ctx, log2N - 10, &twhi));
    int32_t *bad;
    Carver cv;
    cv.add(&bad, 1);
    HS_TRY(cv.commit(ctx));
    HS_TRY(fill_u32(ctx, reinterpret_cast<uint32_t *>(bad), 1, 0));
    const float2 *d = static_cast<const float2 *>(spec);
    switch (bank->dtype) {
    case HS_F32:
        HS_TRY(launch_chisq<StoreF32>(ctx, bank->chisq_bins, n_trig, d, n, bank, trig, seg_t0, ticks_per_sample,
                                      rho_min, twlo, twhi, chisq_out, trig_out, bins_out, bad));
        break;
    case HS_BF16:
        HS_TRY(launch_chisq<StoreBF16>(ctx, bank->chisq_bins, n_trig, d, n, bank, trig, seg_t0, ticks_per_sample,
                                       rho_min, twlo, twhi, chisq_out, trig_out, bins_out, bad));
        break;
    case HS_F16:
        HS_TRY(launch_chisq<StoreF16>(ctx, bank->chisq_bins, n_trig, d, n, bank, trig, seg_t0, ticks_per_sample,
                                      rho_min, twlo, twhi, chisq_out, trig_out, bins_out, bad));
        break;
    default: return set_error(HS_EINVAL, "hs_chisq: bad bank dtype");
    }
    int32_t hbad = 0;
    HS_TRY(read_back(ctx, bad, &hbad, sizeof(hbad)));
    HS_REQUIRE(hbad == 0, "hs_chisq: trigger template outside the bank or tick outside this segment (code %d)", hbad);
    return HS_OK;
}
