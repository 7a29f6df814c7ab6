// Power-consistency chi-square at trigger samples and the re-weighted SNR of Eq. (4).
//
// Sec. II down-weights triggers with the chi-square test it cites; the test splits the template
// band into p bins of equal template power and compares each bin's share of the complex SNR with
// 1/p of the total.  Only triggers at or above rho_min are tested: they are compacted first, then
// one workgroup per (trigger, bin) evaluates the band-limited SNR z_l at the trigger's sample by
// a direct sum over the bin (float64 phasor recurrence and accumulation), and a last kernel forms
// chi2, the per-bin terms and the re-weighted SNR.  Splitting by bin gives p workgroups per
// trigger, enough to fill the GPU when only a few hundred triggers need the test.
#include <cmath>

#include "dft.h"
#include "hs_internal.h"
#include "storage.h"

namespace hs {

static constexpr int CQ_THREADS = 256;

// Triggers below rho_min (and invalid ones) are copied through here; the others are flagged
// for the band-limited sums.
__global__ void chisq_select(const hs_trigger *trig, int64_t n_trig, int32_t n_tmpl, int64_t seg_t0, int64_t tps,
                             int64_t n, float rho_min, int p, uint32_t *__restrict__ flag,
                             float *__restrict__ chisq_out, hs_trigger *trig_out, float *__restrict__ bins_out,
                             int32_t *__restrict__ bad) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n_trig) return;
    const hs_trigger tr = trig[i];
    bool active = tr.snr >= rho_min;
    if (active) {
        const int64_t dt = tr.tick - seg_t0;
        if (tr.tmpl < 0 || tr.tmpl >= n_tmpl) {
            atomicOr(bad, 1);
            active = false;
        } else if (dt < 0 || dt % tps != 0 || dt / tps >= n) {
            atomicOr(bad, 2);
            active = false;
        }
    }
    flag[i] = active ? 1u : 0u;
    if (!active) {
        chisq_out[i] = 0.0f;
        trig_out[i] = tr;
        if (bins_out)
            for (int l = 0; l < p; ++l) bins_out[i * p + l] = 0.0f;
    }
}

__global__ void chisq_compact(const uint32_t *__restrict__ flag, const uint64_t *__restrict__ off, int64_t n,
                              uint32_t *__restrict__ act) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n && flag[i]) act[off[i]] = (uint32_t)i;
}

// Groups of at most CQ_GROUP consecutive active triggers of one template share each pass over
// the template's band (active triggers are in trigger order, so a template's are contiguous).
static constexpr int CQ_GROUP = 8;
static constexpr int CQ_UNROLL = 2;

// A new group starts at the first trigger of each run of one template and every CQ_GROUP
// triggers within the run.  O(n_act): run starts are flagged, numbered by a prefix sum, and each
// trigger's offset in its run is taken from its run's first index.
__global__ void chisq_run_starts(const hs_trigger *trig, const uint32_t *__restrict__ act, int64_t n_act,
                                 uint32_t *__restrict__ rs) {
    const int64_t a = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (a >= n_act) return;
    rs[a] = (a == 0 || trig[act[a - 1]].tmpl != trig[act[a]].tmpl) ? 1u : 0u;
}

__global__ void chisq_run_first(const uint32_t *__restrict__ rs, const uint64_t *__restrict__ roff, int64_t n_act,
                                uint32_t *__restrict__ rfirst) {
    const int64_t a = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (a < n_act && rs[a]) rfirst[roff[a]] = (uint32_t)a;
}

// In place: start[a] (holding the run-start flag on entry) becomes the group-start flag.
__global__ void chisq_group_starts(const uint64_t *__restrict__ roff, const uint32_t *__restrict__ rfirst,
                                   int64_t n_act, uint32_t *__restrict__ start) {
    const int64_t a = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (a >= n_act) return;
    const uint64_t run = roff[a] + start[a] - 1;  // inclusive count of run starts, minus one
    start[a] = ((a - (int64_t)rfirst[run]) % CQ_GROUP == 0) ? 1u : 0u;
}

__global__ void chisq_group_list(const uint32_t *__restrict__ start, const uint64_t *__restrict__ off, int64_t n_act,
                                 uint32_t *__restrict__ gfirst) {
    const int64_t a = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (a < n_act && start[a]) gfirst[off[a]] = (uint32_t)a;
}

// Bit pattern of lane 0's value in scalar registers (for values every lane computes alike).
__device__ __forceinline__ double uniform_f64(double x) {
    const uint64_t u = (uint64_t)__double_as_longlong(x);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)u);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(u >> 32));
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// P_j(w_j) = sum_{i < nb} q_i w_j^i for NG triggers at once by Horner's rule from the top term
// down, q_i = d~ conj(w~) at bin k_f + 256 i.  CQ_UNROLL terms per trip, their loads issued
// before the arithmetic; the trip count is rounded up at the top, where the extra terms are zeros
// entering a zero polynomial (their loads are clamped to the last bin and discarded).
template <typename ST, int NG>
__device__ __forceinline__ void horner(const float2 *__restrict__ dspec, const typename ST::elem *__restrict__ spectra,
                                       int64_t base, int64_t k_f, int64_t nb, const double *sr, const double *si,
                                       double *hr, double *hi) {
    const int64_t top = (nb + CQ_UNROLL - 1) / CQ_UNROLL * CQ_UNROLL;
    for (int64_t jj = top - 1; jj >= 0; jj -= CQ_UNROLL) {
        float2 q[CQ_UNROLL];
#pragma unroll
        for (int u = 0; u < CQ_UNROLL; ++u) {
            const int64_t i = jj - u < nb ? jj - u : nb - 1;
            const int64_t k = k_f + i * CQ_THREADS;
            q[u] = cmulc(dspec[k], ST::load(spectra, base + k));
        }
#pragma unroll
        for (int u = 0; u < CQ_UNROLL; ++u) {
            const bool live = jj - u < nb;
            const double qr = live ? (double)q[u].x : 0.0, qi = live ? (double)q[u].y : 0.0;
#pragma unroll
            for (int j = 0; j < NG; ++j) {
                const double nr = fma(hr[j], sr[j], fma(-hi[j], si[j], qr));
                hi[j] = fma(hr[j], si[j], fma(hi[j], sr[j], qi));
                hr[j] = nr;
            }
        }
    }
}

// z_l for one (bin l, group of active triggers of one template): sum over the bins of l of
// q_k exp(+2 pi i k m / N), q_k = d~_k conj(w~_k) formed once per bin in float32 and shared by the
// group's triggers; everything after it in float64.  With v = exp(2 pi i m / N) and b0 the first
// bin, thread tid owns the bins b0 + tid + 256 i (i < nb) and
//     z_l = v^b0 sum_tid v^tid P_tid(v^256),   P_tid(w) = sum_i q_i w^i.
// Each thread evaluates its P by Horner's rule (one complex multiply-add per bin and trigger);
// the sum over threads is a tree whose level s joins blocks of 2^s threads with the factor
// v^(2^s) (shuffles inside a wavefront, then the four wavefronts through LDS), and v^b0 is applied
// last.  Every power of v used is an exact float64 sincospi of (E m mod N) / N, computed once per
// workgroup (one per lane), so no twiddle table is read; v^256 is the same in every lane and
// lives in scalar registers.
// The widest of a template's p bins (the lowest index among equals).  The bins partition the
// band over which the filter forms z, so sum_l z_l = z; for triggers that carry the filter's own
// rho and arg z, the widest bin's sum is formed as z minus the others instead of being read.
__device__ __forceinline__ int widest_bin(const int32_t *e, int p) {
    int w = 0;
    int32_t best = e[1] - e[0];
    for (int l = 1; l < p; ++l)
        if (e[l + 1] - e[l] > best) {
            best = e[l + 1] - e[l];
            w = l;
        }
    return w;
}

static constexpr int CQ_PH = 10;  // v^1, v^2, ..., v^128, v^256, v^b0

template <typename ST>
__global__ __launch_bounds__(CQ_THREADS) void chisq_bin_sums(
    const float2 *__restrict__ dspec, int64_t n, const typename ST::elem *__restrict__ spectra,
    const int64_t *__restrict__ offset, const int32_t *__restrict__ k0, const int32_t *__restrict__ klo,
    const int32_t *__restrict__ khi, const int32_t *__restrict__ edges, int p, const hs_trigger *trig,
    const uint32_t *__restrict__ act, int64_t n_act, const uint32_t *__restrict__ gfirst, int64_t seg_t0,
    int64_t tps, bool skip_widest, double2 *__restrict__ zl) {
    static_assert(CQ_THREADS == 256, "the tree below joins four wavefronts of 64 with v^64 and v^128");
    constexpr int G = CQ_GROUP;
    __shared__ double2 ph[G][CQ_PH];
    __shared__ double2 red[CQ_THREADS / 64][G];
    const int64_t a0 = gfirst[blockIdx.x];
    // the last equal-power bin is the widest by far (up to ~80 % of a long template's band), so
    // its workgroups are dispatched first and the short ones fill the end of the grid
    const int l = p - 1 - (int)blockIdx.y;
    const int tid = threadIdx.x;
    const int t = trig[act[a0]].tmpl;
    int g = 1;
    while (g < G && a0 + g < n_act && trig[act[a0 + g]].tmpl == t) ++g;
    const int32_t *e = edges + (int64_t)t * (p + 1);
    if (skip_widest && l == widest_bin(e, p)) return;  // formed from the peak in chisq_finish
    const int64_t base = offset[t] - k0[t];
    // every bin is clamped to the template's band, which lies inside [1, n/2 - 1]
    const int64_t band_lo = klo[t] > 1 ? klo[t] : 1;
    const int64_t band_hi = khi[t] < n / 2 - 1 ? khi[t] : n / 2 - 1;
    const int64_t b0 = e[l] > band_lo ? e[l] : band_lo;
    const int64_t b1 = e[l + 1] < band_hi + 1 ? e[l + 1] : band_hi + 1;
    if (tid < g * CQ_PH) {
        const int j = tid / CQ_PH, s = tid - j * CQ_PH;
        const uint64_t m = (uint64_t)((trig[act[a0 + j]].tick - seg_t0) / tps);
        const uint64_t ex = s < 9 ? (uint64_t(1) << s) : (uint64_t)b0;
        double sn, cs;
        sincospi((double)((ex * m) & ((uint64_t)n - 1)) * (2.0 / (double)n), &sn, &cs);
        ph[j][s] = double2{cs, sn};
    }
    __syncthreads();
    const int64_t k_f = b0 + tid;
    const int64_t nb = k_f < b1 ? (b1 - 1 - k_f) / CQ_THREADS + 1 : 0;
    double hr[G], hi[G], sr[G], si[G];
#pragma unroll
    for (int j = 0; j < G; ++j) {
        hr[j] = hi[j] = sr[j] = si[j] = 0.0;
        if (j < g) {
            sr[j] = uniform_f64(ph[j][8].x);
            si[j] = uniform_f64(ph[j][8].y);
        }
    }
    switch (g) {  // a loop without per-trigger predicates for each group size
    case 1: horner<ST, 1>(dspec, spectra, base, k_f, nb, sr, si, hr, hi); break;
    case 2: horner<ST, 2>(dspec, spectra, base, k_f, nb, sr, si, hr, hi); break;
    case 3: horner<ST, 3>(dspec, spectra, base, k_f, nb, sr, si, hr, hi); break;
    case 4: horner<ST, 4>(dspec, spectra, base, k_f, nb, sr, si, hr, hi); break;
    case 5: horner<ST, 5>(dspec, spectra, base, k_f, nb, sr, si, hr, hi); break;
    case 6: horner<ST, 6>(dspec, spectra, base, k_f, nb, sr, si, hr, hi); break;
    case 7: horner<ST, 7>(dspec, spectra, base, k_f, nb, sr, si, hr, hi); break;
    default: horner<ST, 8>(dspec, spectra, base, k_f, nb, sr, si, hr, hi); break;
    }
    // tree inside the wavefront: after level s, lane L with L mod 2^(s+1) = 0 holds
    // sum_{u < 2^(s+1)} v^u P_{L+u}; its partner block starts at L + 2^s
#pragma unroll
    for (int j = 0; j < G; ++j) {
        if (j < g) {
            double x = hr[j], y = hi[j];
#pragma unroll
            for (int s = 0; s < 6; ++s) {
                const double xd = __shfl_down(x, 1 << s), yd = __shfl_down(y, 1 << s);
                const double2 v = ph[j][s];
                x += v.x * xd - v.y * yd;
                y += v.x * yd + v.y * xd;
            }
            if ((tid & 63) == 0) red[tid >> 6][j] = double2{x, y};
        }
    }
    __syncthreads();
    if (tid < g) {
        const double2 v64 = ph[tid][6], v128 = ph[tid][7], vb = ph[tid][9];
        const double2 r0 = red[0][tid], r1 = red[1][tid], r2 = red[2][tid], r3 = red[3][tid];
        const double ax = r0.x + (v64.x * r1.x - v64.y * r1.y), ay = r0.y + (v64.x * r1.y + v64.y * r1.x);
        const double bx = r2.x + (v64.x * r3.x - v64.y * r3.y), by = r2.y + (v64.x * r3.y + v64.y * r3.x);
        const double cx = ax + (v128.x * bx - v128.y * by), cy = ay + (v128.x * by + v128.y * bx);
        zl[(a0 + tid) * p + l] = double2{vb.x * cx - vb.y * cy, vb.x * cy + vb.y * cx};
    }
}

// chi2 = p sum_l |z_l - z/p|^2, chi2_r = chi2 / (2p - 2), Eq. (4) re-weighting; one thread per
// active trigger.  With from_peak the trigger's rho and arg z give z, and the widest bin's z_l is
// z minus the other bins' sums.
__global__ void chisq_finish(const double2 *__restrict__ zl, const uint32_t *__restrict__ act, int64_t n_act, int p,
                             const hs_trigger *trig, const float *__restrict__ r2s,
                             const int32_t *__restrict__ edges, bool from_peak, float *__restrict__ chisq_out,
                             hs_trigger *trig_out, float *__restrict__ bins_out) {
    const int64_t a = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (a >= n_act) return;
    const uint32_t i = act[a];
    const hs_trigger tr = trig[i];
    const double s = sqrt((double)r2s[tr.tmpl]);  // undoes the storage scale of the template
    const int w = from_peak ? widest_bin(edges + (int64_t)tr.tmpl * (p + 1), p) : -1;
    double Zr = 0.0, Zi = 0.0;
    if (from_peak) {
        Zr = (double)tr.snr * cos((double)tr.phase);
        Zi = (double)tr.snr * sin((double)tr.phase);
    } else {
        for (int l = 0; l < p; ++l) {
            Zr += zl[a * p + l].x * s;
            Zi += zl[a * p + l].y * s;
        }
    }
    double wr = Zr, wi = Zi;  // the widest bin: z minus the others
    if (from_peak)
        for (int l = 0; l < p; ++l)
            if (l != w) {
                wr -= zl[a * p + l].x * s;
                wi -= zl[a * p + l].y * s;
            }
    double chi2 = 0.0;
    for (int l = 0; l < p; ++l) {
        const double zr = l == w ? wr : zl[a * p + l].x * s, zi = l == w ? wi : zl[a * p + l].y * s;
        const double dr = zr - Zr / p, di = zi - Zi / p;
        chi2 += dr * dr + di * di;
        if (bins_out) bins_out[(int64_t)i * p + l] = (float)(p * (dr * dr + di * di));
    }
    const double c = chi2 * p / (2.0 * p - 2.0);
    double rw = (double)tr.snr;
    if (c >= 1.0) rw = rw / pow((1.0 + c * c * c) / 2.0, 1.0 / 6.0);
    chisq_out[i] = (float)c;
    hs_trigger o = tr;
    o.snr = (float)rw;
    trig_out[i] = o;
}

template <typename ST>
static int launch_bin_sums(hs_ctx *ctx, dim3 gs, const float2 *d, int64_t n, const hs_bank *bank, int p,
                           const hs_trigger *trig, const uint32_t *act, int64_t n_act, const uint32_t *gfirst,
                           int64_t seg_t0, int64_t tps, bool skip_widest, double2 *zl) {
    hipLaunchKernelGGL(chisq_bin_sums<ST>, gs, dim3(CQ_THREADS), 0, ctx->stream, d, n,
                       static_cast<const typename ST::elem *>(bank->spectra), bank->offset, bank->k0, bank->k_lo,
                       bank->k_hi, bank->chisq_edges, p, trig, act, n_act, gfirst, seg_t0, tps, skip_widest, zl);
    HS_HIP(hipGetLastError());
    return HS_OK;
}

}  // namespace hs

using namespace hs;

static int chisq_impl(hs_ctx *ctx, const void *spec, int64_t n, double fs, const hs_bank *bank,
                      const hs_trigger *trig, int64_t n_trig, int64_t seg_t0, int64_t ticks_per_sample,
                      float rho_min, float *chisq_out, hs_trigger *trig_out, float *bins_out, bool from_peak) {
    HS_REQUIRE(ctx && bank, "hs_chisq: null argument");
    HS_REQUIRE(n_trig >= 0 && n_trig < (int64_t(1) << 31), "hs_chisq: bad trigger count");
    if (n_trig == 0) return HS_OK;
    HS_REQUIRE(spec && trig && chisq_out && trig_out, "hs_chisq: null argument");
    HS_REQUIRE(is_pow2(n) && n >= 8192 && n <= (int64_t(1) << 22), "hs_chisq: n must be a power of two in [2^13, 2^22]");
    HS_REQUIRE(bank->n == n && bank->fs == fs, "hs_chisq: bank prepared for another n or fs");
    HS_REQUIRE(bank->chisq_bins >= 2 && bank->chisq_bins <= 16 && bank->chisq_edges,
               "hs_chisq: bank has no chi-square bins (2..16)");
    HS_REQUIRE(ticks_per_sample > 0, "hs_chisq: ticks_per_sample must be positive");
    HS_REQUIRE(bank->dtype == HS_F32 || bank->dtype == HS_BF16 || bank->dtype == HS_F16, "hs_chisq: bad bank dtype");
    HS_HIP(hipSetDevice(ctx->device));
    const int p = bank->chisq_bins;
    uint32_t *flag, *act;
    uint64_t *off, *tmp;
    int32_t *bad;
    Carver cv;
    cv.add(&flag, n_trig);
    cv.add(&off, n_trig + 1);
    cv.add(&act, n_trig);
    cv.add(&tmp, scan_tmp_elems(n_trig));
    cv.add(&bad, 1);
    HS_TRY(cv.commit(ctx));
    HS_TRY(fill_u32(ctx, reinterpret_cast<uint32_t *>(bad), 1, 0));
    const unsigned g = (unsigned)cdiv(n_trig, 256);
    hipLaunchKernelGGL(chisq_select, dim3(g), dim3(256), 0, ctx->stream, trig, n_trig, bank->n_tmpl, seg_t0,
                       ticks_per_sample, n, rho_min, p, flag, chisq_out, trig_out, bins_out, bad);
    HS_HIP(hipGetLastError());
    HS_TRY(exclusive_scan_u32(ctx, flag, n_trig, off, tmp));
    hipLaunchKernelGGL(chisq_compact, dim3(g), dim3(256), 0, ctx->stream, flag, off, n_trig, act);
    HS_HIP(hipGetLastError());
    uint64_t n_act = 0;
    int32_t hbad = 0;
    HS_TRY(read_back2(ctx, off + n_trig, &n_act, sizeof(n_act), bad, &hbad, sizeof(hbad)));
    HS_REQUIRE(hbad == 0, "hs_chisq: trigger template outside the bank or tick outside this segment (code %d)", hbad);
    if (n_act == 0) return HS_OK;
    double2 *zl;
    uint32_t *gstart, *gfirst, *rfirst;
    uint64_t *goff;
    Carver cv2;  // re-carves the same buffers first, then the groups and the bin sums
    cv2.add(&flag, n_trig);
    cv2.add(&off, n_trig + 1);
    cv2.add(&act, n_trig);
    cv2.add(&tmp, scan_tmp_elems(n_trig));
    cv2.add(&bad, 1);
    cv2.add(&zl, (size_t)n_act * p);
    cv2.add(&gstart, (size_t)n_act);
    cv2.add(&goff, (size_t)n_act + 1);
    cv2.add(&gfirst, (size_t)n_act);
    cv2.add(&rfirst, (size_t)n_act);
    HS_TRY(cv2.commit(ctx));
    const unsigned ga = (unsigned)cdiv((int64_t)n_act, 256);
    hipLaunchKernelGGL(chisq_run_starts, dim3(ga), dim3(256), 0, ctx->stream, trig, act, (int64_t)n_act, gstart);
    HS_HIP(hipGetLastError());
    HS_TRY(exclusive_scan_u32(ctx, gstart, (int64_t)n_act, goff, tmp));
    hipLaunchKernelGGL(chisq_run_first, dim3(ga), dim3(256), 0, ctx->stream, gstart, goff, (int64_t)n_act, rfirst);
    HS_HIP(hipGetLastError());
    hipLaunchKernelGGL(chisq_group_starts, dim3(ga), dim3(256), 0, ctx->stream, goff, rfirst, (int64_t)n_act,
                       gstart);
    HS_HIP(hipGetLastError());
    HS_TRY(exclusive_scan_u32(ctx, gstart, (int64_t)n_act, goff, tmp));
    hipLaunchKernelGGL(chisq_group_list, dim3(ga), dim3(256), 0, ctx->stream, gstart, goff, (int64_t)n_act, gfirst);
    HS_HIP(hipGetLastError());
    uint64_t n_groups = 0;
    HS_TRY(read_back(ctx, goff + n_act, &n_groups, sizeof(n_groups)));
    const dim3 gs((unsigned)n_groups, (unsigned)p);  // (group of triggers, bin): x holds the large count
    const float2 *d = static_cast<const float2 *>(spec);
    switch (bank->dtype) {
    case HS_F32:
        HS_TRY((launch_bin_sums<StoreF32>(ctx, gs, d, n, bank, p, trig, act, (int64_t)n_act, gfirst, seg_t0,
                                          ticks_per_sample, from_peak, zl)));
        break;
    case HS_BF16:
        HS_TRY((launch_bin_sums<StoreBF16>(ctx, gs, d, n, bank, p, trig, act, (int64_t)n_act, gfirst, seg_t0,
                                           ticks_per_sample, from_peak, zl)));
        break;
    default:
        HS_TRY((launch_bin_sums<StoreF16>(ctx, gs, d, n, bank, p, trig, act, (int64_t)n_act, gfirst, seg_t0,
                                          ticks_per_sample, from_peak, zl)));
        break;
    }
    hipLaunchKernelGGL(chisq_finish, dim3((unsigned)cdiv((int64_t)n_act, 256)), dim3(256), 0, ctx->stream, zl, act,
                       (int64_t)n_act, p, trig, bank->rho2_scale, bank->chisq_edges, from_peak, chisq_out, trig_out,
                       bins_out);
    HS_HIP(hipGetLastError());
    return HS_OK;
}

extern "C" int hs_chisq(hs_ctx *ctx, const void *spec, int64_t n, double fs, const hs_bank *bank,
                        const hs_trigger *trig, int64_t n_trig, int64_t seg_t0, int64_t ticks_per_sample,
                        float rho_min, float *chisq_out, hs_trigger *trig_out, float *bins_out) {
    return chisq_impl(ctx, spec, n, fs, bank, trig, n_trig, seg_t0, ticks_per_sample, rho_min, chisq_out, trig_out,
                      bins_out, false);
}

extern "C" int hs_chisq_at_peaks(hs_ctx *ctx, const void *spec, int64_t n, double fs, const hs_bank *bank,
                                 const hs_trigger *trig, int64_t n_trig, int64_t seg_t0, int64_t ticks_per_sample,
                                 float rho_min, float *chisq_out, hs_trigger *trig_out, float *bins_out) {
    return chisq_impl(ctx, spec, n, fs, bank, trig, n_trig, seg_t0, ticks_per_sample, rho_min, chisq_out, trig_out,
                      bins_out, true);
}
