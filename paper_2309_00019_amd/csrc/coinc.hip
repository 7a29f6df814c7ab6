// Two-detector coincidence over time slides with per-slide clustering and background counts
// (Sec. I and Sec. II: time-shifted background, Eq. (6) false-alarm rate; Appendix A: network
// SNR as the coincident statistic).
//
// For a pair (H trigger i, L trigger j) of the same template, d = (t_i - t_j) mod T fixes every
// slide k at which they coincide: k step must lie within +-window of d + jT for some integer j,
// so the admissible slides are read off directly -- the work is O(same-template pairs), not
// O(slides x triggers), and all time arithmetic is exact int64.  With a statistic floor, pairs
// whose statistic lies below it are not formed at all; L triggers are grouped by template and,
// within a template, into buckets of SNR^2 (highest first), so an H trigger stops scanning at the
// first bucket that cannot reach the floor.
//
// Per-slide clustering (rule: a coincidence survives iff no other of the same slide within
// circular |tick_h' - tick_h| <= W_c is better, "better" = larger stat, then smaller
// (tmpl, tick_h, tick_l)) reuses the tile idea of trigger clustering: bins are (slide, tile of
// W_c ticks of tick_h); a bin's best member is found by three atomic passes -- atomicMax on
// (stat bits, ~tmpl), then atomicMin on the tick_h offset in the tile among the members equal
// so far, then atomicMin on tick_l -- and only that champion can survive; since the three values
// describe it completely, every coincidence checks the champions of the neighbouring tiles of its
// slide itself and marks those it beats within reach (no per-bin lists).
// When the (slide, tile) bins exceed CO_BATCH_BINS the pairs are written in slide order (per-slide
// counts from the counting pass, per-slide cursors in the writing pass) and the bins of a batch of
// consecutive slides are processed at a time, so the slide range and the ring length are bounded
// only by the pair count; survivors are compacted in bin order, i.e. sorted by (slide, tick_h).
#include <algorithm>
#include <cmath>
#include <vector>

#include "hs_internal.h"

namespace hs {

static constexpr int CO_MAX_EDGES = 4096;
static constexpr int64_t CO_BATCH_BINS = int64_t(1) << 26;  // (slide, tile) bins per batch of slides
static constexpr int64_t CO_MAX_GROUPS = int64_t(1) << 25;  // (template, SNR band, time block) groups of L

// SNR^2 bands of the L triggers of a template under a statistic floor, highest first: band p
// holds CO_BAND_LO[p] <= snr^2 < CO_BAND_LO[p - 1] (band 0 has no upper bound).
static constexpr int CO_BANDS = 8;
__constant__ double CO_BAND_LO[CO_BANDS] = {100.0, 64.0, 49.0, 36.0, 30.0, 25.0, 20.0, -1.0};

__device__ __forceinline__ int co_band(float snr, int n_bands) {
    if (n_bands == 1) return 0;
    const double s2 = (double)snr * (double)snr;
    int p = 0;
    while (p < CO_BANDS - 1 && !(s2 >= CO_BAND_LO[p])) ++p;
    return p;
}

// Grouping of the L triggers: group ((tmpl * n_bands) + band) * n_blocks + tick / block_len.
struct LGroups {
    int32_t n_bands;
    int64_t n_blocks, block_len;
};

__device__ __forceinline__ int64_t co_group(const hs_trigger &t, const LGroups &lg) {
    return ((int64_t)t.tmpl * lg.n_bands + co_band(t.snr, lg.n_bands)) * lg.n_blocks + t.tick / lg.block_len;
}

struct RawCoinc {
    uint32_t i, j, k;
    float stat;
};

__device__ __forceinline__ int64_t pos_mod(int64_t a, int64_t T) {
    int64_t r = a % T;
    return r < 0 ? r + T : r;
}

struct SlideGeom {
    int64_t K, step, window, wrap, jmax;
    double inv_step;  // 1 / step, rounded
};

// floor(a / b) for b > 0 and |a| < 2^50: a float64 estimate (within one of the quotient) corrected
// to the exact integer; int64 division is a long instruction sequence on the GPU.
__device__ __forceinline__ int64_t floor_div_r(int64_t a, int64_t b, double inv_b) {
    int64_t q = (int64_t)floor((double)a * inv_b);
    if (q * b > a) --q;
    else if ((q + 1) * b <= a) ++q;
    return q;
}

// Calls f(k) for every slide k in [0, K] with |circ(d - k step)| <= window, d in [0, T).  The
// circular distance is |d + jw T - k step| for some integer jw; a jw whose interval
// [d + jw T - window, d + jw T + window] misses [0, K step] admits no slide and is skipped before
// any division (at most one jw remains when K step + 2 window < T).
template <typename F>
__device__ __forceinline__ void for_each_slide(int64_t d, const SlideGeom &g, F f) {
    for (int64_t jw = -1; jw <= g.jmax; ++jw) {
        const int64_t e = d + jw * g.wrap;
        if (e + g.window < 0 || e - g.window > g.K * g.step) continue;
        int64_t lo = -floor_div_r(g.window - d - jw * g.wrap, g.step, g.inv_step);  // ceil
        int64_t hi = floor_div_r(d + g.window + jw * g.wrap, g.step, g.inv_step);
        if (lo < 0) lo = 0;
        if (hi > g.K) hi = g.K;
        for (int64_t k = lo; k <= hi; ++k) f(k);
    }
}

__device__ __forceinline__ bool trig_ok(const hs_trigger &t, int32_t n_tmpl, int64_t wrap) {
    return t.tmpl >= 0 && t.tmpl < n_tmpl && t.tick >= 0 && t.tick < wrap;
}

// L triggers grouped by (template, SNR^2 band, time block), highest band first.
__global__ void co_group_count(const hs_trigger *__restrict__ l, int64_t nl, int32_t n_tmpl, int64_t wrap, LGroups lg,
                               uint32_t *__restrict__ cnt, int32_t *__restrict__ bad) {
    const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (j >= nl) return;
    const hs_trigger t = l[j];
    if (!trig_ok(t, n_tmpl, wrap)) {
        atomicOr(bad, 1);
        return;
    }
    atomicAdd(&cnt[co_group(t, lg)], 1u);
}

__global__ void co_group_scatter(const hs_trigger *__restrict__ l, int64_t nl, int32_t n_tmpl, int64_t wrap, LGroups lg,
                                 const uint64_t *__restrict__ start, uint32_t *__restrict__ cursor,
                                 uint32_t *__restrict__ lidx) {
    const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (j >= nl) return;
    const hs_trigger t = l[j];
    if (!trig_ok(t, n_tmpl, wrap)) return;
    const int64_t g = co_group(t, lg);
    lidx[start[g] + atomicAdd(&cursor[g], 1u)] = (uint32_t)j;
}

// Calls f(index into l, trigger, stat) for every L trigger of H trigger a's template that can
// coincide with a at some slide and whose statistic with a is at or above the floor
// (stat2_min = floor^2 in float64; 0 = no floor).  A coincidence needs t_L in
// [t_H - K step - window, t_H + window] (mod T), so only the time blocks meeting that interval
// are read (each at most once); under a floor the template's SNR^2 bands are taken from the
// highest and the scan stops at the first band that cannot reach the floor (a margin of 2^-20
// relative covers the float32 rounding of stat).  for_each_slide then decides exactly.
template <typename F>
__device__ __forceinline__ void for_each_partner(const hs_trigger &a, const hs_trigger *__restrict__ l,
                                                 const uint64_t *__restrict__ lstart,
                                                 const uint32_t *__restrict__ lidx, const LGroups &lg,
                                                 const SlideGeom &g, double stat2_min, F f) {
    const double sa = (double)a.snr * (double)a.snr;
    const int64_t reach = g.K * g.step + 2 * g.window;  // length of the t_L interval
    int64_t b0 = 0, nb = lg.n_blocks;  // blocks b0, b0 + 1, ... (mod n_blocks), nb of them
    if (reach < g.wrap) {
        const int64_t lo = pos_mod(a.tick - g.K * g.step - g.window, g.wrap);
        const int64_t hi = lo + reach;  // < 2 wrap
        b0 = lo / lg.block_len;
        const int64_t cnt = hi < g.wrap ? hi / lg.block_len - b0 + 1
                                        : (lg.n_blocks - b0) + (hi - g.wrap) / lg.block_len + 1;
        nb = cnt < lg.n_blocks ? cnt : lg.n_blocks;
    }
    for (int p = 0; p < lg.n_bands; ++p) {
        if (stat2_min > 0.0 && p > 0 && sa + CO_BAND_LO[p - 1] < stat2_min * (1.0 - 0x1p-20)) break;
        const int64_t gb = ((int64_t)a.tmpl * lg.n_bands + p) * lg.n_blocks;
        for (int64_t u = 0; u < nb; ++u) {
            int64_t blk = b0 + u;
            if (blk >= lg.n_blocks) blk -= lg.n_blocks;
            for (uint64_t q = lstart[gb + blk]; q < lstart[gb + blk + 1]; ++q) {
                const uint32_t jl = lidx[q];
                const hs_trigger b = l[jl];
                const float stat = (float)(sa + (double)b.snr * (double)b.snr);
                if ((double)stat < stat2_min) continue;
                f(jl, b, stat);
            }
        }
    }
}

// Pairs per H trigger and, when the bins need several batches of slides (scnt non-null), per
// slide as well.
__global__ void co_pair_count(const hs_trigger *__restrict__ h, int64_t nh, const hs_trigger *__restrict__ l,
                              int32_t n_tmpl, SlideGeom g, LGroups lg, double stat2_min,
                              const uint64_t *__restrict__ lstart,
                              const uint32_t *__restrict__ lidx, uint32_t *__restrict__ pc,
                              uint32_t *__restrict__ scnt, int32_t *__restrict__ bad) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= nh) return;
    const hs_trigger a = h[i];
    uint32_t c = 0;
    if (!trig_ok(a, n_tmpl, g.wrap)) {
        atomicOr(bad, 1);
    } else {
        for_each_partner(a, l, lstart, lidx, lg, g, stat2_min, [&](uint32_t, const hs_trigger &b, float) {
            int64_t d = a.tick - b.tick;  // both ticks in [0, wrap)
            if (d < 0) d += g.wrap;
            for_each_slide(d, g, [&](int64_t k) {
                ++c;
                if (scnt) atomicAdd(&scnt[k], 1u);
            });
        });
    }
    pc[i] = c;
}

// The pairs, written at per-H-trigger offsets (one batch of slides) or straight into slide order
// through per-slide cursors (several batches; the order within a slide is unspecified and nothing
// downstream depends on it).
template <bool BY_SLIDE>
__global__ void co_pair_write(const hs_trigger *__restrict__ h, int64_t nh, const hs_trigger *__restrict__ l,
                              int32_t n_tmpl, SlideGeom g, LGroups lg, double stat2_min,
                              const uint64_t *__restrict__ lstart, const uint32_t *__restrict__ lidx,
                              const uint64_t *__restrict__ poff, const uint64_t *__restrict__ soff,
                              uint32_t *__restrict__ scur, RawCoinc *__restrict__ raw) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= nh) return;
    const hs_trigger a = h[i];
    if (!trig_ok(a, n_tmpl, g.wrap)) return;
    uint64_t w = BY_SLIDE ? 0 : poff[i];
    for_each_partner(a, l, lstart, lidx, lg, g, stat2_min, [&](uint32_t jl, const hs_trigger &b, float stat) {
        int64_t d = a.tick - b.tick;  // both ticks in [0, wrap)
        if (d < 0) d += g.wrap;
        for_each_slide(d, g, [&](int64_t k) {
            const RawCoinc r{(uint32_t)i, jl, (uint32_t)k, stat};
            if (BY_SLIDE) raw[soff[k] + atomicAdd(&scur[k], 1u)] = r;
            else raw[w++] = r;
        });
    });
}

// Champion of a bin, first pass: the statistic, then the smaller template.  Never 0 for a real
// coincidence (the low word is at least 2^31), so 0 marks an empty bin.
__device__ __forceinline__ uint64_t coinc_key(float stat, int32_t tmpl) {
    return ((uint64_t)__float_as_uint(stat) << 32) | (uint64_t)(0xFFFFFFFFu - (uint32_t)tmpl);
}

struct BinGeom {
    int64_t cw, n_tiles, k0;  // k0: first slide of the batch
    double inv_cw;            // 1 / cw, rounded
};

__device__ __forceinline__ int64_t coinc_bin(const RawCoinc &r, int64_t tick_h, const BinGeom &bg, int64_t *tile) {
    *tile = floor_div_r(tick_h, bg.cw, bg.inv_cw);
    return ((int64_t)r.k - bg.k0) * bg.n_tiles + *tile;
}

// Bin champions (a read first skips the atomic when the bin already holds a larger key; values
// only grow, so a stale read can only let a useless atomic through).
__global__ void co_bin(const RawCoinc *__restrict__ raw, int64_t P, const hs_trigger *__restrict__ h,
                       BinGeom bg, unsigned long long *__restrict__ best) {
    const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (q >= P) return;
    const RawCoinc r = raw[q];
    const hs_trigger a = h[r.i];
    int64_t tile;
    const int64_t b = coinc_bin(r, a.tick, bg, &tile);
    const unsigned long long key = coinc_key(r.stat, a.tmpl);
    if (__hip_atomic_load(&best[b], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < key) atomicMax(&best[b], key);
}

// Second pass: the earliest tick_h among the members with the champion's (stat, tmpl).
__global__ void co_bin_th(const RawCoinc *__restrict__ raw, int64_t P, const hs_trigger *__restrict__ h,
                          BinGeom bg, const unsigned long long *__restrict__ best, uint32_t *__restrict__ best_th) {
    const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (q >= P) return;
    const RawCoinc r = raw[q];
    const hs_trigger a = h[r.i];
    int64_t tile;
    const int64_t b = coinc_bin(r, a.tick, bg, &tile);
    if (coinc_key(r.stat, a.tmpl) == best[b]) atomicMin(&best_th[b], (uint32_t)(a.tick - tile * bg.cw));
}

// Third pass: the earliest tick_l among the members equal so far.
__global__ void co_bin_tie(const RawCoinc *__restrict__ raw, int64_t P, const hs_trigger *__restrict__ h,
                           const hs_trigger *__restrict__ l, BinGeom bg, const unsigned long long *__restrict__ best,
                           const uint32_t *__restrict__ best_th, unsigned long long *__restrict__ best_tl) {
    const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (q >= P) return;
    const RawCoinc r = raw[q];
    const hs_trigger a = h[r.i];
    int64_t tile;
    const int64_t b = coinc_bin(r, a.tick, bg, &tile);
    if (coinc_key(r.stat, a.tmpl) == best[b] && (uint32_t)(a.tick - tile * bg.cw) == best_th[b])
        atomicMin(&best_tl[b], (unsigned long long)l[r.j].tick);
}

// true iff coincidence (s2, tm2, th2, tl2) is better than (s1, tm1, th1, tl1)
__device__ __forceinline__ bool coinc_better(float s2, int32_t tm2, int64_t th2, int64_t tl2, float s1, int32_t tm1,
                                             int64_t th1, int64_t tl1) {
    if (s2 != s1) return s2 > s1;
    if (tm2 != tm1) return tm2 < tm1;
    if (th2 != th1) return th2 < th1;
    return tl2 < tl1;
}

// Only the champion of a bin can survive (its members lie within W_c of each other), and a
// bin's champion is fully described by its key and tie value.  Per coincidence: the bin's
// champion records its index; every coincidence compares itself with the champions of the
// neighbouring tiles of its slide (circular offsets -2..2, distinct, excluding its own tile: the
// last tile may be partial, so a reach of W_c can span two tiles across the wrap) and marks those
// it beats within reach.
__global__ __launch_bounds__(256) void co_veto(const RawCoinc *__restrict__ raw, int64_t P,
                                               const hs_trigger *__restrict__ h, const hs_trigger *__restrict__ l,
                                               BinGeom bg, int64_t wrap, const unsigned long long *__restrict__ best,
                                               const uint32_t *__restrict__ best_th,
                                               const unsigned long long *__restrict__ best_tl,
                                               uint32_t *__restrict__ slot, uint32_t *__restrict__ veto) {
    const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (q >= P) return;
    const RawCoinc r = raw[q];
    const hs_trigger a = h[r.i];
    const int64_t tl = l[r.j].tick;
    int64_t tile;
    const int64_t b = coinc_bin(r, a.tick, bg, &tile);
    if (coinc_key(r.stat, a.tmpl) == best[b] && (uint32_t)(a.tick - tile * bg.cw) == best_th[b] &&
        (unsigned long long)tl == best_tl[b])
        slot[b] = (uint32_t)q;
    const int64_t nt = bg.n_tiles;
    const int64_t slide0 = ((int64_t)r.k - bg.k0) * nt;
    int64_t seen[4];
    int ns = 0;
    for (int dd = -2; dd <= 2; ++dd) {
        if (dd == 0) continue;
        const int64_t t2 = pos_mod(tile + dd, nt);
        if (t2 == tile) continue;
        bool dup = false;
        for (int u = 0; u < ns; ++u) dup |= (seen[u] == t2);
        if (dup) continue;
        seen[ns++] = t2;
        const int64_t nb = slide0 + t2;
        const unsigned long long kb = best[nb];
        if (kb == 0) continue;  // empty bin
        const float s2 = __uint_as_float((uint32_t)(kb >> 32));
        const int32_t tm2 = (int32_t)(0xFFFFFFFFu - (uint32_t)(kb & 0xFFFFFFFFull));
        const int64_t th2 = t2 * bg.cw + (int64_t)best_th[nb];
        if (!coinc_better(r.stat, a.tmpl, a.tick, tl, s2, tm2, th2, (int64_t)best_tl[nb])) continue;
        int64_t d2 = pos_mod(th2 - a.tick + wrap / 2, wrap) - wrap / 2;
        if (d2 < 0) d2 = -d2;
        if (d2 <= bg.cw) veto[nb] = 1u;
    }
}

__global__ __launch_bounds__(256) void co_flag(const unsigned long long *__restrict__ best,
                                               const uint32_t *__restrict__ veto, int64_t bins,
                                               uint32_t *__restrict__ flag) {
    const int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (b < bins) flag[b] = (best[b] != 0 && veto[b] == 0) ? 1u : 0u;
}

__global__ void co_emit(const RawCoinc *__restrict__ raw, const hs_trigger *__restrict__ h,
                        const hs_trigger *__restrict__ l, int64_t bins, const uint32_t *__restrict__ flag,
                        const uint32_t *__restrict__ slot, const uint64_t *__restrict__ off, int64_t base,
                        hs_coinc *__restrict__ out, int64_t cap) {
    const int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (b >= bins || !flag[b]) return;
    const uint64_t pos = (uint64_t)base + off[b];
    if (pos >= (uint64_t)cap) return;
    const RawCoinc r = raw[slot[b]];
    const hs_trigger a = h[r.i], c = l[r.j];
    hs_coinc o;
    o.slide = (int32_t)r.k;
    o.tmpl = a.tmpl;
    o.tick_h = a.tick;
    o.tick_l = c.tick;
    o.snr_h = a.snr;
    o.snr_l = c.snr;
    o.stat = r.stat;
    o.snr_c = sqrtf(r.stat);
    out[pos] = o;
}

// hist[c] += number of surviving coincidences in bins [first, bins) (first skips the zero-lag
// slide when the batch holds it) with exactly c of the ascending thresholds e2s[0..n_e) at or
// below (double)stat (a binary search per survivor; workgroup histograms in LDS).  The count at
// threshold i is then the sum of hist[c] over c > i.
__global__ __launch_bounds__(256) void co_background(const RawCoinc *__restrict__ raw, int64_t first, int64_t bins,
                                                     const uint32_t *__restrict__ flag,
                                                     const uint32_t *__restrict__ slot, const double *__restrict__ e2s,
                                                     int n_e, unsigned long long *__restrict__ hist) {
    __shared__ uint32_t sh[CO_MAX_EDGES + 1];
    for (int i = threadIdx.x; i <= n_e; i += 256) sh[i] = 0u;
    __syncthreads();
    for (int64_t b = first + blockIdx.x * (int64_t)256 + threadIdx.x; b < bins; b += (int64_t)gridDim.x * 256) {
        if (!flag[b]) continue;
        const double x = (double)raw[slot[b]].stat;
        int lo = 0, hi = n_e;  // e2s[< lo] <= x < e2s[>= hi]
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (e2s[mid] <= x) lo = mid + 1;
            else hi = mid;
        }
        atomicAdd(&sh[lo], 1u);
    }
    __syncthreads();
    for (int i = threadIdx.x; i <= n_e; i += 256)
        if (sh[i]) atomicAdd(&hist[i], (unsigned long long)sh[i]);
}

}  // namespace hs

using namespace hs;

extern "C" int hs_timeslide_coinc(hs_ctx *ctx, const hs_trigger *h, int64_t nh, const hs_trigger *l, int64_t nl,
                                  int32_t n_tmpl, int64_t n_slides, int64_t step, int64_t window, int64_t wrap,
                                  int64_t cluster_w, float min_snr_c, const float *edges, int32_t n_edges,
                                  int64_t *bg_counts, hs_coinc *out, int64_t cap, int64_t *n_out) {
    HS_REQUIRE(ctx && n_out, "hs_timeslide_coinc: null argument");
    HS_REQUIRE(nh >= 0 && nl >= 0 && n_slides >= 0 && step > 0 && window >= 0 && wrap > 0 && 2 * window < wrap &&
                   cluster_w > 0 && cluster_w < (int64_t(1) << 31) && n_edges >= 0 && cap >= 0,
               "hs_timeslide_coinc: bad geometry (slides=%lld step=%lld window=%lld wrap=%lld cluster_w=%lld)",
               (long long)n_slides, (long long)step, (long long)window, (long long)wrap, (long long)cluster_w);
    HS_REQUIRE(n_tmpl > 0 && n_tmpl <= (1 << 24), "hs_timeslide_coinc: n_tmpl must be in [1, 2^24]");
    HS_REQUIRE(nh < (int64_t(1) << 31) && nl < (int64_t(1) << 31) && n_slides < (int64_t(1) << 31),
               "hs_timeslide_coinc: input too large");
    HS_REQUIRE(!std::isnan(min_snr_c) && min_snr_c < INFINITY, "hs_timeslide_coinc: min_snr_c must be finite");
    HS_REQUIRE(n_edges == 0 || (edges && bg_counts), "hs_timeslide_coinc: null edges/bg_counts");
    HS_REQUIRE(n_edges <= CO_MAX_EDGES, "hs_timeslide_coinc: at most %d edges (got %d)", CO_MAX_EDGES, (int)n_edges);
    const double floor2 = min_snr_c > 0.0f ? (double)min_snr_c * (double)min_snr_c : 0.0;
    for (int e = 0; e < n_edges; ++e) {
        HS_REQUIRE(!std::isnan(edges[e]), "hs_timeslide_coinc: edges[%d] is NaN", e);
        HS_REQUIRE(floor2 == 0.0 || (double)edges[e] * (double)edges[e] >= floor2,
                   "hs_timeslide_coinc: edges[%d] = %g lies below min_snr_c = %g (its count would be incomplete)", e,
                   (double)edges[e], (double)min_snr_c);
    }
    *n_out = 0;
    for (int e = 0; e < n_edges; ++e) bg_counts[e] = 0;
    if (nh == 0 || nl == 0) return HS_OK;
    HS_REQUIRE(h && l && (out || cap == 0), "hs_timeslide_coinc: null argument");
    HS_HIP(hipSetDevice(ctx->device));
    const int64_t n_tiles = cdiv(wrap, cluster_w);
    HS_REQUIRE(n_tiles <= CO_BATCH_BINS, "hs_timeslide_coinc: %lld tiles of the cluster window per slide exceed %lld",
               (long long)n_tiles, (long long)CO_BATCH_BINS);
    HS_REQUIRE(n_slides <= (int64_t(1) << 50) / step && n_slides * step + 3 * wrap < (int64_t(1) << 50),
               "hs_timeslide_coinc: n_slides * step + 3 wrap must stay below 2^50 ticks");
    SlideGeom g{n_slides, step, window, wrap, (n_slides * step + window) / wrap + 1, 1.0 / (double)step};
    const int64_t n_sl = n_slides + 1;
    // L groups: SNR^2 bands only under a floor; time blocks about a quarter of the t_L interval
    // an H trigger can meet (one block when that interval covers the ring), within CO_MAX_GROUPS
    LGroups lg;
    lg.n_bands = floor2 > 0.0 ? CO_BANDS : 1;
    {
        const int64_t reach = n_slides * step + 2 * window;
        int64_t nbk = reach >= wrap ? 1 : cdiv(4 * wrap, reach > 0 ? reach : 1);
        const int64_t cap_b = CO_MAX_GROUPS / ((int64_t)n_tmpl * lg.n_bands);
        if (nbk > cap_b) nbk = cap_b;
        if (nbk < 1) nbk = 1;
        lg.block_len = cdiv(wrap, nbk);
        lg.n_blocks = cdiv(wrap, lg.block_len);
    }
    const int64_t n_groups = (int64_t)n_tmpl * lg.n_bands * lg.n_blocks;

    // (slide, tile) bins are processed in batches of whole slides; with several batches the pairs
    // are written in slide order
    const int64_t per_batch = CO_BATCH_BINS / n_tiles;  // slides per batch (>= 1)
    const int64_t bb = std::min<int64_t>(per_batch, n_sl) * n_tiles;  // bins of the largest batch
    const int64_t n_batches = cdiv(n_sl, per_batch);
    const bool by_slide = n_batches > 1;

    // --- phase 1: group L by (template, SNR^2 band, time block), count pairs per H trigger ----
    uint32_t *lcnt, *lcur, *lidx, *pc, *scnt, *scur;
    uint64_t *lstart, *poff, *soff, *tmp1;
    int32_t *bad;
    const int64_t n_scan1 = std::max<int64_t>(std::max<int64_t>(nh, n_groups), by_slide ? n_sl : 1);
    auto carve1 = [&](Carver &cv) {
        cv.add(&lcnt, n_groups);
        cv.add(&lcur, n_groups);
        cv.add(&lstart, n_groups + 1);
        cv.add(&lidx, nl);
        cv.add(&pc, nh);
        cv.add(&poff, nh + 1);
        cv.add(&scnt, by_slide ? n_sl : 1);
        cv.add(&scur, by_slide ? n_sl : 1);
        cv.add(&soff, by_slide ? n_sl + 1 : 1);
        cv.add(&tmp1, scan_tmp_elems(n_scan1));
        cv.add(&bad, 1);
    };
    {
        Carver cv;
        carve1(cv);
        HS_TRY(cv.commit(ctx));
    }
    HS_TRY(fill_u32(ctx, lcnt, n_groups, 0));
    HS_TRY(fill_u32(ctx, lcur, n_groups, 0));
    HS_TRY(fill_u32(ctx, reinterpret_cast<uint32_t *>(bad), 1, 0));
    if (by_slide) {
        HS_TRY(fill_u32(ctx, scnt, n_sl, 0));
        HS_TRY(fill_u32(ctx, scur, n_sl, 0));
    }
    hipLaunchKernelGGL(co_group_count, dim3((unsigned)cdiv(nl, 256)), dim3(256), 0, ctx->stream, l, nl, n_tmpl, wrap,
                       lg, lcnt, bad);
    HS_HIP(hipGetLastError());
    HS_TRY(exclusive_scan_u32(ctx, lcnt, n_groups, lstart, tmp1));
    hipLaunchKernelGGL(co_group_scatter, dim3((unsigned)cdiv(nl, 256)), dim3(256), 0, ctx->stream, l, nl, n_tmpl,
                       wrap, lg, lstart, lcur, lidx);
    hipLaunchKernelGGL(co_pair_count, dim3((unsigned)cdiv(nh, 256)), dim3(256), 0, ctx->stream, h, nh, l, n_tmpl, g,
                       lg, floor2, lstart, lidx, pc, by_slide ? scnt : nullptr, bad);
    HS_HIP(hipGetLastError());
    HS_TRY(exclusive_scan_u32(ctx, pc, nh, poff, tmp1));
    uint64_t P = 0;
    int32_t hbad = 0;
    HS_TRY(read_back2(ctx, poff + nh, &P, sizeof(P), bad, &hbad, sizeof(hbad)));
    HS_REQUIRE(hbad == 0, "hs_timeslide_coinc: trigger with tmpl outside [0, n_tmpl) or tick outside [0, wrap)");
    if (P == 0) return HS_OK;
    HS_REQUIRE(P < (uint64_t(1) << 32), "hs_timeslide_coinc: %llu coincident pairs exceed 2^32",
               (unsigned long long)P);

    // --- phase 2: materialise the pairs (in slide order when there are several batches) ------
    // Phase-1 buffers are re-carved first, in the same order, so they keep their contents
    // (arena growth preserves what was written).
    RawCoinc *raw;
    uint32_t *veto, *flag, *slot, *best_th;
    unsigned long long *best, *best_tl, *bgc;
    uint64_t *boff, *tmp2;
    double *e2;
    {
        Carver cv;
        carve1(cv);
        cv.add(&raw, P);
        cv.add(&veto, bb);
        cv.add(&flag, bb);
        cv.add(&slot, bb);
        cv.add(&best_th, bb);
        cv.add(&best, bb);
        cv.add(&best_tl, bb);
        cv.add(&boff, bb + 1);
        cv.add(&tmp2, scan_tmp_elems(bb));
        cv.add(&e2, n_edges > 0 ? n_edges : 1);
        cv.add(&bgc, n_edges + 1);
        HS_TRY(cv.commit(ctx));
    }
    std::vector<uint64_t> hsoff;
    if (by_slide) {
        HS_TRY(exclusive_scan_u32(ctx, scnt, n_sl, soff, tmp1));
        hsoff.resize(n_sl + 1);
        HS_TRY(read_back(ctx, soff, hsoff.data(), (n_sl + 1) * sizeof(uint64_t)));
        HS_REQUIRE(hsoff[n_sl] == P, "hs_timeslide_coinc: internal pair count mismatch");
        hipLaunchKernelGGL(co_pair_write<true>, dim3((unsigned)cdiv(nh, 256)), dim3(256), 0, ctx->stream, h, nh, l,
                           n_tmpl, g, lg, floor2, lstart, lidx, poff, soff, scur, raw);
    } else {
        hipLaunchKernelGGL(co_pair_write<false>, dim3((unsigned)cdiv(nh, 256)), dim3(256), 0, ctx->stream, h, nh, l,
                           n_tmpl, g, lg, floor2, lstart, lidx, poff, soff, scur, raw);
    }
    HS_HIP(hipGetLastError());

    // thresholds in ascending order (ties keep their order), counted over the batches' bins
    std::vector<double> hs2(n_edges);
    std::vector<int> order(n_edges);
    if (n_edges > 0) {
        std::vector<double> he2(n_edges);
        for (int e = 0; e < n_edges; ++e) {
            he2[e] = (double)edges[e] * (double)edges[e];
            order[e] = e;
        }
        std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return he2[x] < he2[y]; });
        for (int i = 0; i < n_edges; ++i) hs2[i] = he2[order[i]];
        HS_HIP(hipMemcpyAsync(e2, hs2.data(), n_edges * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
        HS_TRY(fill_u64(ctx, reinterpret_cast<uint64_t *>(bgc), n_edges + 1, 0));
    }

    // --- phase 3: per batch of slides, bin by (slide, tile), champions, vetoes, emit, count ----
    uint64_t total = 0;
    for (int64_t k0 = 0; k0 < n_sl; k0 += per_batch) {
        const int64_t k1 = std::min(n_sl, k0 + per_batch);
        const uint64_t q0 = by_slide ? hsoff[k0] : 0, q1 = by_slide ? hsoff[k1] : P;
        if (q1 == q0) continue;
        const int64_t nb = (k1 - k0) * n_tiles;
        const int64_t Pb = (int64_t)(q1 - q0);
        const RawCoinc *rb = raw + q0;
        BinGeom bgm{cluster_w, n_tiles, k0, 1.0 / (double)cluster_w};
        const unsigned gq = (unsigned)cdiv(Pb, 256);
        HS_TRY(fill_u32(ctx, veto, nb, 0));
        HS_TRY(fill_u32(ctx, best_th, nb, 0xFFFFFFFFu));
        HS_TRY(fill_u64(ctx, reinterpret_cast<uint64_t *>(best), nb, 0));
        HS_TRY(fill_u64(ctx, reinterpret_cast<uint64_t *>(best_tl), nb, ~uint64_t(0)));
        hipLaunchKernelGGL(co_bin, dim3(gq), dim3(256), 0, ctx->stream, rb, Pb, h, bgm, best);
        hipLaunchKernelGGL(co_bin_th, dim3(gq), dim3(256), 0, ctx->stream, rb, Pb, h, bgm, best, best_th);
        hipLaunchKernelGGL(co_bin_tie, dim3(gq), dim3(256), 0, ctx->stream, rb, Pb, h, l, bgm, best, best_th, best_tl);
        hipLaunchKernelGGL(co_veto, dim3(gq), dim3(256), 0, ctx->stream, rb, Pb, h, l, bgm, wrap, best, best_th,
                           best_tl, slot, veto);
        hipLaunchKernelGGL(co_flag, dim3((unsigned)cdiv(nb, 256)), dim3(256), 0, ctx->stream, best, veto, nb, flag);
        HS_HIP(hipGetLastError());
        HS_TRY(exclusive_scan_u32(ctx, flag, nb, boff, tmp2));
        hipLaunchKernelGGL(co_emit, dim3((unsigned)cdiv(nb, 256)), dim3(256), 0, ctx->stream, rb, h, l, nb, flag, slot,
                           boff, (int64_t)total, out, cap);
        HS_HIP(hipGetLastError());
        if (n_edges > 0) {
            const int64_t first = k0 == 0 ? n_tiles : 0;
            const int64_t span = nb - first;
            if (span > 0) {
                const unsigned gb = (unsigned)(cdiv(span, 256) < 1024 ? cdiv(span, 256) : 1024);
                hipLaunchKernelGGL(co_background, dim3(gb), dim3(256), 0, ctx->stream, rb, first, nb, flag, slot, e2,
                                   (int)n_edges, bgc);
                HS_HIP(hipGetLastError());
            }
        }
        uint64_t kept = 0;
        HS_TRY(read_back(ctx, boff + nb, &kept, sizeof(kept)));
        total += kept;
    }
    if (n_edges > 0) {
        std::vector<unsigned long long> hh(n_edges + 1);
        HS_TRY(read_back(ctx, bgc, hh.data(), (n_edges + 1) * sizeof(unsigned long long)));
        unsigned long long above = 0;
        for (int i = n_edges - 1; i >= 0; --i) {
            above += hh[i + 1];
            bg_counts[order[i]] = (int64_t)above;
        }
    }
    *n_out = (int64_t)total;
    if ((int64_t)total > cap)
        return set_error(HS_EOVERFLOW, "hs_timeslide_coinc: %llu coincidences exceed capacity %lld",
                         (unsigned long long)total, (long long)cap);
    return HS_OK;
}
