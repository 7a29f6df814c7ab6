/*
 * hs.h -- C ABI of libhs, the MI355X (gfx950) hierarchical matched-filter search.
 *
 * The library computes, on one GPU, the frequency-domain matched filter of a
 * compact-binary template bank against whitened detector strain and the
 * post-filter steps of the two-stage hierarchical search of
 * "Obtaining Statistical Significance of Gravitational Wave Signals in
 * Hierarchical Search" (Soni, Dhurandhar, Mitra):
 *
 *   hs_welch_psd        one-sided PSD S_n(f) of Eq. (2), estimated from the data
 *   hs_whiten           data Fourier transform divided by sqrt(S_n) on the band
 *   hs_prepare_bank     template sigma (Eq. (2) with x = y = h) and pre-whitened,
 *                       sigma-normalised template spectra
 *   hs_matched_filter   complex SNR series of Eq. (1)/(2), threshold (Sec. II)
 *   hs_snr_series       the same SNR series written out in full (diagnostics)
 *   hs_cluster_triggers peak clustering of above-threshold samples into triggers
 *   hs_chisq            power-consistency chi-square and re-weighted SNR (Eq. (4));
 *                       hs_chisq_at_peaks for triggers carrying the filter's own z
 *   hs_timeslide_coinc  two-detector coincidence over time slides, per-slide
 *                       clustering, background counts for Eq. (6) (Secs. I-II)
 *   hs_followup         stage-1 selection and union of fine-bank neighbourhoods
 *                       (Sec. III)
 *
 * Conventions shared by every call
 *  - Pointers marked "device" are HIP device pointers owned by the caller; the
 *    library never frees caller memory.  Pointers marked "host" are ordinary
 *    host memory.  The context owns its own scratch (grown on demand).
 *  - All device work is enqueued on the stream given to hs_create, in order.
 *    Calls that return a count through a host pointer synchronise that stream
 *    before returning; the others return without synchronising.
 *  - Every call returns an hs_status.  On failure the call leaves its outputs
 *    unspecified (except HS_EOVERFLOW, below) and hs_last_error() describes
 *    the failure.  Nothing is thrown across the ABI.
 *  - HS_EOVERFLOW: a capacity-bounded output (cap records) was too small.  The
 *    required record count is stored in the count output so the caller can
 *    grow the buffer and call again; the records written are unspecified.
 *  - Frequencies: df = fs / n, bin k is f_k = k df.  Complex spectra are
 *    interleaved (re, im) float pairs ("complex64").  Data transform convention
 *    x~[k] = dt sum_j x[j] exp(-2 pi i k j / n).
 *  - Time is int64 "ticks" chosen by the caller; a sample of a segment at fs
 *    spans ticks_per_sample ticks.
 */
#ifndef HS_H
#define HS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hs_ctx hs_ctx;

typedef enum {
    HS_OK = 0,
    HS_EINVAL = -1,     /* invalid argument (shape, size, pointer, range) */
    HS_ENOMEM = -2,     /* device or host allocation failed */
    HS_EOVERFLOW = -3,  /* output capacity too small; required count returned */
    HS_EDEVICE = -4     /* HIP runtime error */
} hs_status;

typedef enum { HS_F32 = 0, HS_BF16 = 1, HS_F16 = 2 } hs_dtype;

/* One above-threshold sample of one template's SNR series.
 * tpos = position of the template in the tmpl_ids list of the filter call,
 * m = sample index (coalescence sample, 0..n-1), rho2 = rho^2, phase = arg z. */
typedef struct { int32_t tpos; int32_t m; float rho2; float phase; } hs_candidate;      /* 16 B */

/* A clustered single-detector trigger (Sec. II: a stored SNR peak). */
typedef struct { int32_t seg; int32_t tmpl; int64_t tick; float snr; float phase; } hs_trigger; /* 24 B */

/* A surviving coincidence of slide `slide` (0 = zero lag).  tick_l is the
 * unshifted L tick.  stat = rho_H^2 + rho_L^2 (the value every decision uses),
 * snr_c = sqrt(stat). */
typedef struct {
    int32_t slide; int32_t tmpl; int64_t tick_h; int64_t tick_l;
    float snr_h; float snr_l; float stat; float snr_c;
} hs_coinc;                                                                             /* 40 B */

/* A prepared bank (all pointers device, owned by the caller; filled by
 * hs_prepare_bank).  Template t's prepared spectrum for bin k lives at
 * spectra[offset[t] + k - k0[t]] (element of `dtype`: complex64, or a pair of
 * bf16/f16), non-zero only on the integration band [k_lo[t], k_hi[t]]. */
typedef struct {
    int32_t n_tmpl;
    int32_t dtype;            /* hs_dtype */
    int64_t n;                /* FFT length the bank was prepared for */
    double fs;                /* sample rate the bank was prepared for */
    const int64_t *offset;    /* [n_tmpl] */
    const int32_t *k0;        /* [n_tmpl] first stored bin */
    const int32_t *k_lo;      /* [n_tmpl] first band bin */
    const int32_t *k_hi;      /* [n_tmpl] last band bin (inclusive) */
    const void *spectra;
    const float *rho2_scale;  /* [n_tmpl] factor applied to |z|^2 (undoes storage scaling) */
    int32_t chisq_bins;       /* p of the power-consistency test (0 = no edges) */
    const int32_t *chisq_edges; /* [n_tmpl][p + 1] bin edges (NULL when chisq_bins == 0) */
} hs_bank;

/* Context: binds a device and a HIP stream (hipStream_t; NULL = default stream). */
int hs_create(hs_ctx **ctx, int device, void *hip_stream);
int hs_destroy(hs_ctx *ctx);
/* Message of the last failure on this thread ("" if none). */
const char *hs_last_error(void);
/* ABI version; changes whenever a struct or signature changes. */
int hs_abi_version(void);

/* Matched-filter schedule: bytes of the pass-A -> pass-B intermediate per batch
 * (batch = bytes / (8 n) templates, at least 1).  Default 128 MiB, or the
 * HS_MF_BATCH_MB environment variable at hs_create (MiB, used only when in
 * [1, 65536]); set by the autotuner.
 * HS_EINVAL if bytes < 1 MiB or > 64 GiB.  hs_get_mf_batch_bytes returns the
 * current value (0 for a NULL context). */
int hs_set_mf_batch_bytes(hs_ctx *ctx, int64_t bytes);
int64_t hs_get_mf_batch_bytes(const hs_ctx *ctx);

/* Matched-filter tile: threads per pass-B workgroup, 64, 128 (default) or 256;
 * a workgroup transforms threads / (N1/16) rows of N1 = n/512 points (widened
 * to one row when N1/16 exceeds it).  Results do not depend on it; set by the
 * autotuner.  HS_EINVAL for other values.  hs_get_mf_tile returns the current
 * value (0 for a NULL context). */
int hs_set_mf_tile(hs_ctx *ctx, int32_t pass_b_threads);
int32_t hs_get_mf_tile(const hs_ctx *ctx);

/* Matched-filter tile of the first pass: columns k1 per pass-A workgroup, 16, 32
 * or 64 (default); a workgroup of 16 x cols threads transforms cols columns of
 * 512 points and writes each row of the intermediate in pieces of 8 cols bytes
 * (capped at N1 = n/512 columns).  Results do not depend on it; set by the
 * autotuner.  HS_EINVAL for other values.  hs_get_mf_pa_cols returns the
 * current value (0 for a NULL context). */
int hs_set_mf_pa_cols(hs_ctx *ctx, int32_t cols);
int32_t hs_get_mf_pa_cols(const hs_ctx *ctx);

/*
 * One-sided Welch PSD (the weight S_n of Eq. (2); the paper does not say how
 * it is estimated).  Segments of seg_len samples every seg_len/2 samples,
 * periodic Hann window w[i] = 1/2 - 1/2 cos(2 pi i / seg_len), periodograms
 * scaled by 1/(fs sum w^2), doubled for 0 < j < seg_len/2, averaged, then
 * linearly interpolated onto f_k = k fs/n, k = 0..n/2.  Arithmetic in float64.
 *   strain  device float  [n]
 *   psd_out device double [n/2 + 1]
 * Requires n, seg_len powers of two, 16 <= seg_len <= n, seg_len <= 2^16.
 */
int hs_welch_psd(hs_ctx *ctx, const float *strain, int64_t n, double fs, int64_t seg_len,
                 double *psd_out);

/*
 * Whitened data spectrum d~[k] = x~[k] / sqrt(S[k]) for k_lo <= k <= n/2 - 1,
 * zero for k < k_lo; k_lo = max(1, ceil(f_low n / fs)) (lower limit of Eq. (2)).
 * The transform is real-input: an n/2-point complex transform in float32 of the
 * sample pairs, recombined and divided in float64.
 *   strain   device float  [n]          n a power of two, 2^10 <= n <= 2^22
 *   psd      device double [n/2 + 1]    positive and finite on the band (not
 *            checked here: the call does not synchronise; hs_prepare_bank checks it)
 *   spec_out device complex64 [n/2]     bins 0..n/2-1
 * The leading m/2 bins of spec_out are also the whitened spectrum of the same
 * data ideally decimated to m samples (same df), which is how a lower-rate
 * stage reuses it.
 */
int hs_whiten(hs_ctx *ctx, const float *strain, int64_t n, double fs, double f_low,
              const double *psd, void *spec_out);

/*
 * Bank preparation.  For each template t (raw spectrum h~ stored band-packed
 * at raw[offset[t] + k - k0[t]] for k0[t] <= k <= k1[t], complex64):
 *   k_lo = max(1, ceil(f_low n / fs), kstart[t]),  k_hi = min(k1[t], n/2 - 1)
 *   sigma^2 = 4 df sum_{k_lo..k_hi} |h~_k|^2 / S_k            (float64)
 *   w~_k = scale_t * 4 df h~_k / (sqrt(S_k) sigma) on the band, 0 elsewhere
 * stored as `dtype` in spectra_out with the SAME layout as raw (offsets,
 * k0..k1).  scale_t is 1 for HS_F32 and a power of two keeping the largest
 * element near 2^14 for HS_BF16/HS_F16; rho2_scale_out[t] = 1/scale_t^2.
 * With this, sum_k d~_k conj(w~_k) e^{2 pi i k m / n} / scale_t is the complex
 * SNR z[m] of Eq. (1)/(2) (quadrature form of Appendix A).
 * With chisq_bins = p >= 2 it also writes the edges of the p contiguous bins of
 * equal template power |h~_k|^2 / S_k used by hs_chisq (the power-consistency
 * test Sec. II cites): chisq_edges_out[t][0] = k_lo, [t][p] = k_hi + 1, and
 * edge l (0 < l < p) = the first bin whose cumulative power from k_lo reaches
 * l/p of the template's total (float64 sums).
 *   psd device double [n/2 + 1]; raw, offset, k0, kstart, k1 device;
 *   spectra_out device (element size 8 for F32, 4 otherwise);
 *   k_lo_out, k_hi_out, rho2_scale_out, sigma_out device [n_tmpl];
 *   chisq_edges_out device int32 [n_tmpl][p + 1] (NULL when chisq_bins == 0).
 * HS_EINVAL if a band is empty or k1 >= k0 is violated, chisq_bins is 1 or > 16,
 * the PSD is not positive and finite inside a band, or a template has no
 * (or non-finite) power inside its band.
 */
int hs_prepare_bank(hs_ctx *ctx, int64_t n, double fs, double f_low, const double *psd,
                    int32_t n_tmpl, const void *raw, const int64_t *offset, const int32_t *k0,
                    const int32_t *kstart, const int32_t *k1, int32_t dtype, void *spectra_out,
                    int32_t *k_lo_out, int32_t *k_hi_out, float *rho2_scale_out,
                    double *sigma_out, int32_t chisq_bins, int32_t *chisq_edges_out);

/*
 * Matched filter + threshold (Sec. II: a sample is kept when rho >= thr,
 * compared as rho^2 >= thr^2 in float32).  For each template tmpl_ids[p]:
 *   z[m] = sum_{k in band} spec[k] conj(w~[k]) e^{+2 pi i k m / n} / scale,  m = 0..n-1
 * and every m with |z[m]|^2 >= thr^2 is appended to cand as {p, m, |z|^2, arg z}.
 * Candidate order is unspecified (hs_cluster_triggers imposes one).
 *   spec     device complex64, bins 0..n/2-1 (from hs_whiten at this n, or the
 *            leading bins of a longer segment's spectrum with the same df)
 *   bank     prepared at this n and fs
 *   tmpl_ids device int32 [n_ids], each in [0, bank->n_tmpl)
 *   cand     device hs_candidate [cap];  n_cand host: number found
 * n must be a power of two with 2^13 <= n <= 2^20.
 */
int hs_matched_filter(hs_ctx *ctx, const void *spec, int64_t n, double fs, const hs_bank *bank,
                      const int32_t *tmpl_ids, int32_t n_ids, float thr, hs_candidate *cand,
                      int64_t cap, int64_t *n_cand);

/*
 * hs_matched_filter without any allocation, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc.  Same arguments, results and errors as
 * hs_matched_filter (same kernels; its twiddle tables are computed on the
 * device in float64 and rounded once, so an SNR may differ from
 * hs_matched_filter's by an ulp-level amount).  Its scratch (the pass-A ->
 * pass-B intermediate, candidate lists, counters, per-template records and
 * twiddles) lives in a fixed device array of HS_MF_NOALLOC_SCRATCH_BYTES per
 * GPU, held until the process ends and located by hs_create; the call makes
 * no hipMalloc, hipFree or pinned-host allocation, and copies its counts
 * straight into the caller's host memory.  Templates are filtered in batches
 * that fit the array beside the candidate lists (2 cap + 64 records of 16 B),
 * n_ids records of 32 B and 36 KB of twiddles; HS_EINVAL when these leave no
 * room for one template's 8 n-byte intermediate (at n = 2^19 with 1,000
 * templates cap may reach about 1.96 M), or when the context's device is
 * beyond 63.  Like hs_matched_filter it synchronises its stream to return
 * n_cand, so the call itself cannot be recorded into a graph: it serves code
 * around a capture, not inside one.
 * Every allocation-free call on one GPU shares that GPU's array and leaves
 * its contents behind (counters are cleared at the start of each call):
 * calls that overlap on one GPU (other streams, threads or contexts) race and
 * must be serialised by the caller.
 */
#define HS_MF_NOALLOC_SCRATCH_BYTES (64ll << 20)
int hs_matched_filter_noalloc(hs_ctx *ctx, const void *spec, int64_t n, double fs, const hs_bank *bank,
                              const int32_t *tmpl_ids, int32_t n_ids, float thr, hs_candidate *cand,
                              int64_t cap, int64_t *n_cand);

/* The complex SNR series z[m] of hs_matched_filter written out in full:
 * z_out device complex64 [n_ids][n]. */
int hs_snr_series(hs_ctx *ctx, const void *spec, int64_t n, double fs, const hs_bank *bank,
                  const int32_t *tmpl_ids, int32_t n_ids, void *z_out);

/*
 * Peak clustering (Sec. II: a trigger is the peak of the SNR; rule not given,
 * reading): among the candidates of the valid region m_lo <= m < m_hi,
 * candidate m of template position p survives iff every other such candidate
 * m' of p with |m' - m| <= window has rho2' < rho2, or rho2' == rho2 and
 * m' > m.  Candidates outside the valid region are ignored (a segment that
 * overlaps its neighbours keeps only the samples its circular transform gets
 * right, Sec. V; m_lo = 0, m_hi = n keeps all).  Survivors are written as
 * triggers {seg, tmpl_ids[p], seg_t0 + m * ticks_per_sample, sqrt(rho2), phase}
 * sorted by (p, m); seg_t0 may be negative (only valid samples are emitted).
 * Candidates must have distinct (tpos, m), 0 <= m < n, 0 <= tpos < n_ids;
 * HS_EINVAL unless 0 <= m_lo <= m_hi <= n.
 *   cand device [n_cand]; tmpl_ids device [n_ids]; out device [cap]; n_out host.
 */
int hs_cluster_triggers(hs_ctx *ctx, const hs_candidate *cand, int64_t n_cand, int64_t n,
                        const int32_t *tmpl_ids, int32_t n_ids, int64_t window, int64_t m_lo,
                        int64_t m_hi, int32_t seg, int64_t seg_t0, int64_t ticks_per_sample,
                        hs_trigger *out, int64_t cap, int64_t *n_out);

/*
 * Power-consistency chi-square and re-weighted SNR of Sec. II, Eq. (4).  For every
 * trigger with snr >= rho_min (others are copied unchanged with chi2_r = 0), at
 * its sample m = (tick - seg_t0) / ticks_per_sample of this segment:
 *   z_l = sum_{k in bin l} spec[k] conj(w~[k]) e^{2 pi i k m / n} / scale   (p bins)
 *   chi2 = p sum_l |z_l - z/p|^2,  z = sum_l z_l,  chi2_r = chi2 / (2p - 2)
 *   rho~ = snr / [(1 + chi2_r^3)/2]^(1/6) if chi2_r >= 1, else snr     (Eq. (4))
 * Bin sums accumulate in float64.  trig_out receives the triggers with snr
 * replaced by rho~ (the statistic hs_timeslide_coinc then combines).
 *   spec, bank as for hs_matched_filter (bank prepared with chisq_bins >= 2);
 *   trig device hs_trigger [n_trig] of this segment (tmpl in [0, n_tmpl));
 *   chisq_out device float [n_trig]; trig_out device hs_trigger [n_trig]
 *   (may alias trig); bins_out device float [n_trig][p] or NULL: the per-bin
 *   terms X_l = p |z_l - z/p|^2 (sum over l = chi2; zero for copied triggers).
 * HS_EINVAL if a trigger's tmpl or tick does not belong to this bank/segment.
 */
int hs_chisq(hs_ctx *ctx, const void *spec, int64_t n, double fs, const hs_bank *bank,
             const hs_trigger *trig, int64_t n_trig, int64_t seg_t0, int64_t ticks_per_sample,
             float rho_min, float *chisq_out, hs_trigger *trig_out, float *bins_out);

/*
 * hs_chisq for triggers at the filter's peaks: as hs_chisq, but every trigger
 * with snr >= rho_min must carry the filter's own rho and arg z at its sample
 * (snr and phase as hs_cluster_triggers writes them from hs_matched_filter's
 * candidates for the same spec and bank).  The p bins partition the band over
 * which the filter forms z, so sum_l z_l = z exactly; the widest bin's z_l is
 * formed as z - sum of the other bins and its template elements are not read
 * (for a long template that bin holds most of the band).  Results agree with
 * hs_chisq to the filter's float32 error in z.  Same arguments and errors.
 * The input must be the filter's own (unweighted) triggers: when trig_out
 * aliases trig the buffer afterwards holds re-weighted SNRs, and passing it
 * to hs_chisq_at_peaks again would take those for |z| (nothing detects this).
 */
int hs_chisq_at_peaks(hs_ctx *ctx, const void *spec, int64_t n, double fs, const hs_bank *bank,
                      const hs_trigger *trig, int64_t n_trig, int64_t seg_t0, int64_t ticks_per_sample,
                      float rho_min, float *chisq_out, hs_trigger *trig_out, float *bins_out);

/*
 * Two-detector coincidence over time slides (Sec. I; Sec. II, Eq. (6)).
 * A pair (H trigger i, L trigger j) with the same tmpl is coincident at slide
 * k in [0, n_slides] iff |((t_i - t_j - k step + T/2) mod T) - T/2| <= window,
 * T = wrap.  stat = (float)((double)snr_i^2 + (double)snr_j^2) (network SNR
 * squared, Appendix A).  Per slide, a coincidence survives iff no other of
 * the same slide within circular |tick_h' - tick_h| <= cluster_w has a larger
 * stat, or an equal stat and a smaller (tmpl, tick_h, tick_l).  Survivors of
 * every slide are written to out sorted by (slide, tick_h).  bg_counts[e] =
 * number of survivors with slide >= 1 and (double)stat >= (double)edges[e]^2.
 * Statistic floor: with min_snr_c > 0, pairs with (double)stat <
 * (double)min_snr_c^2 are not formed at all.  Since a coincidence can only be
 * removed by a better one, the survivors at or above the floor and every
 * count at an edge >= min_snr_c are exactly those of the full definition;
 * coincidences below the floor are absent from out (min_snr_c <= 0: none is
 * dropped).  This bounds the work of long rings and many slides by the pairs
 * above the floor.
 *   h, l device hs_trigger [nh], [nl]; ticks in [0, wrap); tmpl in [0, n_tmpl)
 *   edges host float [n_edges]; bg_counts host int64 [n_edges]
 *   out device hs_coinc [cap]; n_out host
 * Requires 0 <= 2 window < wrap, step > 0, 0 < cluster_w < 2^31,
 * ceil(wrap / cluster_w) <= 2^26, 1 <= n_tmpl <= 2^24, n_slides >= 0,
 * n_slides * step + 3 wrap < 2^50, fewer than 2^32 coincident pairs (above the
 * floor), 0 <= n_edges <= 4096, no NaN edge, a finite min_snr_c and no edge
 * below a positive min_snr_c (HS_EINVAL otherwise).
 * Background time is n_slides * wrap ticks (Eq. (6) T_b).
 */
int hs_timeslide_coinc(hs_ctx *ctx, const hs_trigger *h, int64_t nh, const hs_trigger *l,
                       int64_t nl, int32_t n_tmpl, int64_t n_slides, int64_t step,
                       int64_t window, int64_t wrap, int64_t cluster_w, float min_snr_c,
                       const float *edges, int32_t n_edges, int64_t *bg_counts, hs_coinc *out,
                       int64_t cap, int64_t *n_out);

/*
 * Stage-1 follow-up (Sec. III): coincidences with (double)stat >= rho_min^2
 * are followed; the neighbourhood of coarse template c is every fine template
 * f with |mchirp_f - mchirp_c| <= frac * mchirp_c (float64, inclusive); a
 * followed coincidence adds its neighbourhood to segment tick_h / seg_ticks
 * and to segment tick_l / seg_ticks.  Row s of fine_ids (device int32
 * [n_seg][n_fine]) receives the sorted unique fine ids of segment s, and
 * n_ids[s] (host) their count.
 *   c device [n_c]; coarse_mchirp device double [n_coarse];
 *   fine_mchirp device double [n_fine]
 */
int hs_followup(hs_ctx *ctx, const hs_coinc *c, int64_t n_c, float rho_min,
                const double *coarse_mchirp, int32_t n_coarse, const double *fine_mchirp,
                int32_t n_fine, double frac, int64_t seg_ticks, int32_t n_seg, int32_t *fine_ids,
                int32_t *n_ids);

/*
 * Background tail fit of Sec. IV, Eq. (7): ordinary least squares of
 * log counts[e] = alpha + beta edges[e] over the edges with edges[e] >= x_min
 * and counts[e] > 0 (counts = the cumulative background counts n_b(edges[e])
 * of hs_timeslide_coinc; natural logarithm, equal weights, float64).  Host
 * pointers; no device work.  HS_EINVAL if fewer than two edges qualify.
 */
int hs_far_fit(const float *edges, const int64_t *counts, int32_t n_edges, float x_min, double *alpha,
               double *beta, int32_t *n_used);

/*
 * Hybrid false-alarm rate (Eq. (6) below the fit range, Eq. (7) above) of every
 * zero-lag coincidence of c (an hs_timeslide_coinc output: slide 0 = foreground,
 * slides >= 1 = background survivors).  With rho = sqrt((double)stat):
 *   rho <  x_fit: far = (1 + #{background records with stat >= this stat}) / t_b
 *   rho >= x_fit: far = exp(alpha + beta rho) / t_b
 * (per second when t_b is in seconds); background records get -1.
 *   c device [n_c]; far_out device double [n_c].
 */
int hs_far(hs_ctx *ctx, const hs_coinc *c, int64_t n_c, double t_b, double alpha, double beta, float x_fit,
           double *far_out);

/* Statistic at which the fitted FAR exp(alpha + beta x) / t_b equals 1 / ifar
 * (t_b and ifar in the same unit): (log(t_b / ifar) - alpha) / beta. */
double hs_far_threshold(double alpha, double beta, double t_b, double ifar);

/* ---------------------------------------------------------------------------
 * Learned follow-up proposer (an addition on top of Sec. III's neighbourhood
 * rule).  The neighbourhood of a followed coarse template c (every fine f with
 * |mchirp_f - mchirp_c| <= frac mchirp_c) is split into 64 cells:
 *   u = (mchirp_f - mchirp_c) / (frac mchirp_c)          (float64, this order)
 *   cell = 4 min(15, max(0, floor((u + 1) * 8))) + #{q_edges[e] <= q_f}
 * and an MLP scores the cells from 16 features of the stage-1 coincidence;
 * only the smallest set of most probable cells whose softmax probabilities
 * sum to at least p_cum is re-filtered.  All 64 cells = the plain rule.
 *
 * Model: device float [HS_MLP_MODEL] =
 *   [mu (16), inv_std (16), W1 16x128, b1, W2 128x128, b2, W3 128x128, b3,
 *    W4 128x64, b4], each W row-major [input][output]; the HS_MLP_PARAMS values
 * after the first 32 are trained.  h0 = (x - mu) inv_std, h_i = relu(h_{i-1}
 * W_i + b_i) (i = 1..3), logits = h3 W4 + b4.  FP32 throughout.
 * ------------------------------------------------------------------------- */
#define HS_MLP_FEATURES 16
#define HS_MLP_CELLS 64
#define HS_MLP_PARAMS 43456
#define HS_MLP_MODEL (32 + HS_MLP_PARAMS)

/*
 * Features of coincidences (float32 [n_c][16], computed in float64):
 *   0 snr_h, 1 snr_l, 2 snr_c (of the coincidence record),
 *   3 (chi2_r,H + chi2_r,L) / 2,
 *   4..11 (X_H,l + X_L,l) / (2 (2p - 2) / p)   (hs_chisq bins_out, p = 8),
 *   12 coarse_mchirp[tmpl], 13 coarse_q[tmpl],
 *   14 ((tick_h - tick_l - slide step + wrap/2) mod wrap - wrap/2) / ticks_per_second,
 *   15 phase_H - phase_L wrapped into (-pi, pi] (IEEE remainder by 2 pi).
 * The H (L) trigger of a coincidence is the record of trig_h (trig_l) with
 * the coincidence's tmpl and tick_h (tick_l); trigger arrays must be sorted
 * by (seg, tmpl, tick) with seg = floor(tick / seg_ticks), as produced by
 * hs_cluster_triggers per segment (increasing template ids) concatenated in
 * segment order.  chisq_* [n] and bins_* [n][8] are hs_chisq's outputs for
 * those triggers.  All arrays device; HS_EINVAL if chisq_bins != 8, a
 * template id is outside [0, n_coarse) or a trigger is missing.
 */
int hs_proposer_features(hs_ctx *ctx, const hs_coinc *c, int64_t n_c, const hs_trigger *trig_h,
                         int64_t n_h, const float *chisq_h, const float *bins_h,
                         const hs_trigger *trig_l, int64_t n_l, const float *chisq_l,
                         const float *bins_l, int32_t chisq_bins, int64_t seg_ticks,
                         const double *coarse_mchirp, const double *coarse_q, int32_t n_coarse,
                         int64_t step, int64_t wrap, int64_t ticks_per_second, float *feat_out);

/* MLP logits: model device [HS_MLP_MODEL], x device float [n][16],
 * logits_out device float [n][64]. */
int hs_mlp_forward(hs_ctx *ctx, const float *model, const float *x, int64_t n, float *logits_out);

/*
 * One training step on a batch: loss = mean over the batch of the softmax
 * cross-entropy of the logits against labels (cells in [0, 64)); gradient by
 * backpropagation (sums in a fixed order: deterministic); then Adam
 * (Kingma & Ba 2015, Algorithm 1; beta1 0.9, beta2 0.999, eps 1e-8) at step
 * t >= 1 with learning rate lr on the trained values model[32..].
 *   model, adam_m, adam_v device float ([HS_MLP_MODEL], [HS_MLP_PARAMS] x 2;
 *   the moments start at zero); x device [n][16]; labels device int32 [n];
 *   grad_out device float [HS_MLP_PARAMS] or NULL (receives the gradient);
 *   loss_out host float (loss before the update).
 * HS_EINVAL on a label outside [0, 64), t < 1 or n < 1.
 */
int hs_mlp_train_step(hs_ctx *ctx, float *model, float *adam_m, float *adam_v, int64_t t, float lr,
                      const float *x, const int32_t *labels, int64_t n, float *grad_out,
                      float *loss_out);

/*
 * Cell selection: per row, softmax of the logits (float32), cells taken in
 * decreasing probability (equal probabilities: lower cell first) until the
 * running sum reaches P (all 64 if it never does), where P = p_cum for rows
 * with x[2] (the network SNR feature) >= rho_split and p_cum_low otherwise
 * (two tiers; rho_split = -inf gives one).  mask_out device uint64 [n], bit
 * c = cell c selected.
 */
int hs_mlp_propose(hs_ctx *ctx, const float *model, const float *x, int64_t n, float p_cum,
                   float rho_split, float p_cum_low, uint64_t *mask_out);

/*
 * Follow-up restricted to cells: as hs_followup, but a followed coincidence i
 * adds only the fine templates of its neighbourhood whose cell bit is set in
 * cell_mask[i] (cells as above).  fine_q device double [n_fine] (m1/m2);
 * q_edges host double [3]; cell_mask device uint64 [n_c].
 */
int hs_followup_cells(hs_ctx *ctx, const hs_coinc *c, int64_t n_c, float rho_min,
                      const double *coarse_mchirp, int32_t n_coarse, const double *fine_mchirp,
                      const double *fine_q, int32_t n_fine, double frac, const double *q_edges,
                      const uint64_t *cell_mask, int64_t seg_ticks, int32_t n_seg,
                      int32_t *fine_ids, int32_t *n_ids);

#ifdef __cplusplus
}
#endif

#endif /* HS_H */
