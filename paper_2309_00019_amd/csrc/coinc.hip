// Two-detector coincidence over time slides with per-slide clustering and background counts
// (Sec. I and Sec. II: time-shifted background, Eq. (6) false-alarm rate; Appendix A: network
// SNR as the coincident statistic).
//
// For a pair (H trigger i, L trigger j) of the same template, d = (t_i - t_j) mod T fixes every
// slide k at which they coincide: k step must lie within +-window of d + jT for some integer j,
// so the admissible slides are read off directly -- the work is O(same-template pairs), not
// O(slides x triggers), and all time arithmetic is exact int64.
//
// Per-slide clustering (rule: a coincidence survives iff no other of the same slide within
// circular |tick_h' - tick_h| <= W_c is better, "better" = larger stat, then smaller
// (tmpl, tick_h, tick_l)) reuses the tile idea of trigger clustering: bins are (slide, tile of
// W_c ticks of tick_h); a bin's best member is found with a 64-bit atomicMax on
// (stat bits, 0xFFFF - tmpl, 0xFFFF - tick_h offset in the tile) plus an atomicMin on tick_l for
// exact ties; only that champion can survive, and since the key and the tie value describe it
// completely, every coincidence checks the champions of the neighbouring tiles of its slide
// itself and marks those it beats within reach (no per-bin lists).
// Survivors are compacted in bin order, i.e. sorted by (slide, tick_h).
#include <algorithm>
#include <cmath>
#include <vector>

#include "hs_internal.h"

namespace hs {

static constexpr int CO_MAX_EDGES = 4096;

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

__global__ void co_group_count(const hs_trigger *__restrict__ l, int64_t nl, int32_t n_tmpl, int64_t wrap,
                               uint32_t *__restrict__ cnt, int32_t *__restrict__ bad) {
    const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (j >= nl) return;
    const hs_trigger t = l[j];
    if (!trig_ok(t, n_tmpl, wrap)) {
        atomicOr(bad, 1);
        return;
    }
    atomicAdd(&cnt[t.tmpl], 1u);
}

__global__ void co_group_scatter(const hs_trigger *__restrict__ l, int64_t nl, int32_t n_tmpl, int64_t wrap,
                                 const uint64_t *__restrict__ start, uint32_t *__restrict__ cursor,
                                 uint32_t *__restrict__ lidx) {
    const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (j >= nl) return;
    const hs_trigger t = l[j];
    if (!trig_ok(t, n_tmpl, wrap)) return;
    lidx[start[t.tmpl] + atomicAdd(&cursor[t.tmpl], 1u)] = (uint32_t)j;
}

__global__ void co_pair_count(const hs_trigger *__restrict__ h, int64_t nh, const hs_trigger *__restrict__ l,
                              int32_t n_tmpl, SlideGeom g, const uint64_t *__restrict__ lstart,
                              const uint32_t *__restrict__ lidx, uint32_t *__restrict__ pc,
                              int32_t *__restrict__ bad) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= nh) return;
    const hs_trigger a = h[i];
    uint32_t c = 0;
    if (!trig_ok(a, n_tmpl, g.wrap)) {
        atomicOr(bad, 1);
    } else {
        for (uint64_t p = lstart[a.tmpl]; p < lstart[a.tmpl + 1]; ++p) {
            const hs_trigger b = l[lidx[p]];
            int64_t d = a.tick - b.tick;  // both ticks in [0, wrap)
            if (d < 0) d += g.wrap;
            for_each_slide(d, g, [&](int64_t) { ++c; });
        }
    }
    pc[i] = c;
}

__global__ void co_pair_write(const hs_trigger *__restrict__ h, int64_t nh, const hs_trigger *__restrict__ l,
                              int32_t n_tmpl, SlideGeom g, const uint64_t *__restrict__ lstart,
                              const uint32_t *__restrict__ lidx, const uint64_t *__restrict__ poff,
                              RawCoinc *__restrict__ raw) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= nh) return;
    const hs_trigger a = h[i];
    if (!trig_ok(a, n_tmpl, g.wrap)) return;
    uint64_t w = poff[i];
    const double sa = (double)a.snr * (double)a.snr;
    for (uint64_t p = lstart[a.tmpl]; p < lstart[a.tmpl + 1]; ++p) {
        const uint32_t jl = lidx[p];
        const hs_trigger b = l[jl];
        int64_t d = a.tick - b.tick;  // both ticks in [0, wrap)
        if (d < 0) d += g.wrap;
        const float stat = (float)(sa + (double)b.snr * (double)b.snr);
        for_each_slide(d, g, [&](int64_t k) {
            raw[w++] = RawCoinc{(uint32_t)i, jl, (uint32_t)k, stat};
        });
    }
}

__device__ __forceinline__ uint64_t coinc_key(float stat, int32_t tmpl, int64_t off_in_tile) {
    return ((uint64_t)__float_as_uint(stat) << 32) | ((uint64_t)(0xFFFF - tmpl) << 16) |
           (uint64_t)(0xFFFF - off_in_tile);
}

struct BinGeom {
    int64_t cw, n_tiles;
    double inv_cw;  // 1 / cw, rounded
};

__device__ __forceinline__ int64_t coinc_bin(const RawCoinc &r, int64_t tick_h, const BinGeom &bg, int64_t *tile) {
    *tile = floor_div_r(tick_h, bg.cw, bg.inv_cw);
    return (int64_t)r.k * bg.n_tiles + *tile;
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
    const unsigned long long key = coinc_key(r.stat, a.tmpl, a.tick - tile * bg.cw);
    if (__hip_atomic_load(&best[b], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < key) atomicMax(&best[b], key);
}

__global__ void co_bin_tie(const RawCoinc *__restrict__ raw, int64_t P, const hs_trigger *__restrict__ h,
                           const hs_trigger *__restrict__ l, BinGeom bg, const unsigned long long *__restrict__ best,
                           unsigned long long *__restrict__ best_tl) {
    const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (q >= P) return;
    const RawCoinc r = raw[q];
    const hs_trigger a = h[r.i];
    int64_t tile;
    const int64_t b = coinc_bin(r, a.tick, bg, &tile);
    if (coinc_key(r.stat, a.tmpl, a.tick - tile * bg.cw) == best[b])
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
                                               const unsigned long long *__restrict__ best_tl,
                                               uint32_t *__restrict__ slot, uint32_t *__restrict__ veto) {
    const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (q >= P) return;
    const RawCoinc r = raw[q];
    const hs_trigger a = h[r.i];
    const int64_t tl = l[r.j].tick;
    int64_t tile;
    const int64_t b = coinc_bin(r, a.tick, bg, &tile);
    if (coinc_key(r.stat, a.tmpl, a.tick - tile * bg.cw) == best[b] && (unsigned long long)tl == best_tl[b])
        slot[b] = (uint32_t)q;
    const int64_t nt = bg.n_tiles;
    const int64_t slide0 = (int64_t)r.k * nt;
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
        if (kb == 0) continue;  // empty bin (a key's low 16 bits are never 0)
        const float s2 = __uint_as_float((uint32_t)(kb >> 32));
        const int32_t tm2 = 0xFFFF - (int32_t)((kb >> 16) & 0xFFFF);
        const int64_t th2 = t2 * bg.cw + (0xFFFF - (int64_t)(kb & 0xFFFF));
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
                        const uint32_t *__restrict__ slot, const uint64_t *__restrict__ off,
                        hs_coinc *__restrict__ out, int64_t cap) {
    const int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (b >= bins || !flag[b]) return;
    const uint64_t pos = off[b];
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

// hist[c] += number of surviving coincidences with slide >= 1 and exactly c of the ascending
// thresholds e2s[0..n_e) at or below (double)stat (a binary search per survivor; workgroup
// histograms in LDS).  The count at threshold i is then the sum of hist[c] over c > i.
__global__ __launch_bounds__(256) void co_background(const RawCoinc *__restrict__ raw, int64_t n_tiles, int64_t bins,
                                                     const uint32_t *__restrict__ flag,
                                                     const uint32_t *__restrict__ slot, const double *__restrict__ e2s,
                                                     int n_e, unsigned long long *__restrict__ hist) {
    __shared__ uint32_t sh[CO_MAX_EDGES + 1];
    for (int i = threadIdx.x; i <= n_e; i += 256) sh[i] = 0u;
    __syncthreads();
    for (int64_t b = n_tiles + blockIdx.x * (int64_t)256 + threadIdx.x; b < bins; b += (int64_t)gridDim.x * 256) {
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
                                  int64_t cluster_w, const float *edges, int32_t n_edges, int64_t *bg_counts,
                                  hs_coinc *out, int64_t cap, int64_t *n_out) {
    HS_REQUIRE(ctx && n_out, "hs_timeslide_coinc: null argument");
    HS_REQUIRE(nh >= 0 && nl >= 0 && n_slides >= 0 && step > 0 && window >= 0 && wrap > 0 && 2 * window < wrap &&
                   cluster_w > 0 && cluster_w < 65536 && n_edges >= 0 && cap >= 0,
               "hs_timeslide_coinc: bad geometry (slides=%lld step=%lld window=%lld wrap=%lld cluster_w=%lld)",
               (long long)n_slides, (long long)step, (long long)window, (long long)wrap, (long long)cluster_w);
    HS_REQUIRE(n_tmpl > 0 && n_tmpl <= 65536, "hs_timeslide_coinc: n_tmpl must be in [1, 65536]");
    HS_REQUIRE(nh < (int64_t(1) << 31) && nl < (int64_t(1) << 31) && n_slides < (int64_t(1) << 31),
               "hs_timeslide_coinc: input too large");
    HS_REQUIRE(n_edges == 0 || (edges && bg_counts), "hs_timeslide_coinc: null edges/bg_counts");
    HS_REQUIRE(n_edges <= CO_MAX_EDGES, "hs_timeslide_coinc: at most %d edges (got %d)", CO_MAX_EDGES, (int)n_edges);
    for (int e = 0; e < n_edges; ++e)
        HS_REQUIRE(!std::isnan(edges[e]), "hs_timeslide_coinc: edges[%d] is NaN", e);
    *n_out = 0;
    for (int e = 0; e < n_edges; ++e) bg_counts[e] = 0;
    if (nh == 0 || nl == 0) return HS_OK;
    HS_REQUIRE(h && l && (out || cap == 0), "hs_timeslide_coinc: null argument");
    HS_HIP(hipSetDevice(ctx->device));
    const int64_t n_tiles = cdiv(wrap, cluster_w);
    const int64_t bins = (n_slides + 1) * n_tiles;
    HS_REQUIRE(bins <= (int64_t(1) << 28), "hs_timeslide_coinc: %lld (slide, tile) bins exceed 2^28",
               (long long)bins);
    HS_REQUIRE(n_slides <= (int64_t(1) << 50) / step && n_slides * step + 3 * wrap < (int64_t(1) << 50),
               "hs_timeslide_coinc: n_slides * step + 3 wrap must stay below 2^50 ticks");
    SlideGeom g{n_slides, step, window, wrap, (n_slides * step + window) / wrap + 1, 1.0 / (double)step};
    BinGeom bgm{cluster_w, n_tiles, 1.0 / (double)cluster_w};

    // --- phase 1: group L by template, count pairs per H trigger -------------------------------
    uint32_t *lcnt, *lcur, *lidx, *pc;
    uint64_t *lstart, *poff, *tmp1;
    int32_t *bad;
    {
        Carver cv;
        cv.add(&lcnt, n_tmpl);
        cv.add(&lcur, n_tmpl);
        cv.add(&lstart, n_tmpl + 1);
        cv.add(&lidx, nl);
        cv.add(&pc, nh);
        cv.add(&poff, nh + 1);
        cv.add(&tmp1, scan_tmp_elems(nh > n_tmpl ? nh : n_tmpl));
        cv.add(&bad, 1);
        HS_TRY(cv.commit(ctx));
    }
    HS_TRY(fill_u32(ctx, lcnt, n_tmpl, 0));
    HS_TRY(fill_u32(ctx, lcur, n_tmpl, 0));
    HS_TRY(fill_u32(ctx, reinterpret_cast<uint32_t *>(bad), 1, 0));
    hipLaunchKernelGGL(co_group_count, dim3((unsigned)cdiv(nl, 256)), dim3(256), 0, ctx->stream, l, nl, n_tmpl, wrap,
                       lcnt, bad);
    HS_HIP(hipGetLastError());
    HS_TRY(exclusive_scan_u32(ctx, lcnt, n_tmpl, lstart, tmp1));
    hipLaunchKernelGGL(co_group_scatter, dim3((unsigned)cdiv(nl, 256)), dim3(256), 0, ctx->stream, l, nl, n_tmpl,
                       wrap, lstart, lcur, lidx);
    hipLaunchKernelGGL(co_pair_count, dim3((unsigned)cdiv(nh, 256)), dim3(256), 0, ctx->stream, h, nh, l, n_tmpl, g,
                       lstart, lidx, pc, bad);
    HS_HIP(hipGetLastError());
    HS_TRY(exclusive_scan_u32(ctx, pc, nh, poff, tmp1));
    uint64_t P = 0;
    int32_t hbad = 0;
    HS_TRY(read_back2(ctx, poff + nh, &P, sizeof(P), bad, &hbad, sizeof(hbad)));
    HS_REQUIRE(hbad == 0, "hs_timeslide_coinc: trigger with tmpl outside [0, n_tmpl) or tick outside [0, wrap)");
    if (P == 0) return HS_OK;
    HS_REQUIRE(P < (uint64_t(1) << 32), "hs_timeslide_coinc: %llu coincident pairs exceed 2^32",
               (unsigned long long)P);

    // --- phase 2: materialise pairs, bin by (slide, tile), find champions ----------------------
    // Phase-1 buffers are re-carved first, in the same order, so they keep their contents
    // (arena growth preserves what was written).
    RawCoinc *raw;
    uint32_t *veto, *flag, *slot;
    unsigned long long *best, *best_tl, *bgc;
    uint64_t *boff, *tmp2;
    double *e2;
    {
        Carver cv;
        cv.add(&lcnt, n_tmpl);
        cv.add(&lcur, n_tmpl);
        cv.add(&lstart, n_tmpl + 1);
        cv.add(&lidx, nl);
        cv.add(&pc, nh);
        cv.add(&poff, nh + 1);
        cv.add(&tmp1, scan_tmp_elems(nh > n_tmpl ? nh : n_tmpl));
        cv.add(&bad, 1);
        cv.add(&raw, P);
        cv.add(&veto, bins);
        cv.add(&flag, bins);
        cv.add(&slot, bins);
        cv.add(&best, bins);
        cv.add(&best_tl, bins);
        cv.add(&boff, bins + 1);
        cv.add(&tmp2, scan_tmp_elems(bins));
        cv.add(&e2, n_edges > 0 ? n_edges : 1);
        cv.add(&bgc, n_edges + 1);
        HS_TRY(cv.commit(ctx));
    }
    hipLaunchKernelGGL(co_pair_write, dim3((unsigned)cdiv(nh, 256)), dim3(256), 0, ctx->stream, h, nh, l, n_tmpl, g,
                       lstart, lidx, poff, raw);
    HS_HIP(hipGetLastError());
    HS_TRY(fill_u32(ctx, veto, bins, 0));
    HS_TRY(fill_u64(ctx, reinterpret_cast<uint64_t *>(best), bins, 0));
    HS_TRY(fill_u64(ctx, reinterpret_cast<uint64_t *>(best_tl), bins, ~uint64_t(0)));
    const unsigned gp = (unsigned)cdiv((int64_t)P, 256);
    hipLaunchKernelGGL(co_bin, dim3(gp), dim3(256), 0, ctx->stream, raw, (int64_t)P, h, bgm, best);
    hipLaunchKernelGGL(co_bin_tie, dim3(gp), dim3(256), 0, ctx->stream, raw, (int64_t)P, h, l, bgm, best, best_tl);
    hipLaunchKernelGGL(co_veto, dim3(gp), dim3(256), 0, ctx->stream, raw, (int64_t)P, h, l, bgm, wrap, best, best_tl,
                       slot, veto);
    hipLaunchKernelGGL(co_flag, dim3((unsigned)cdiv(bins, 256)), dim3(256), 0, ctx->stream, best, veto, bins, flag);
    HS_HIP(hipGetLastError());
    HS_TRY(exclusive_scan_u32(ctx, flag, bins, boff, tmp2));
    hipLaunchKernelGGL(co_emit, dim3((unsigned)cdiv(bins, 256)), dim3(256), 0, ctx->stream, raw, h, l, bins, flag, slot,
                       boff, out, cap);
    HS_HIP(hipGetLastError());
    uint64_t total = 0;
    if (n_edges > 0) {
        // thresholds in ascending order (ties keep their order), counted in one pass over the bins
        std::vector<double> he2(n_edges);
        std::vector<int> order(n_edges);
        for (int e = 0; e < n_edges; ++e) {
            he2[e] = (double)edges[e] * (double)edges[e];
            order[e] = e;
        }
        std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return he2[x] < he2[y]; });
        std::vector<double> hs2(n_edges);
        for (int i = 0; i < n_edges; ++i) hs2[i] = he2[order[i]];
        HS_HIP(hipMemcpyAsync(e2, hs2.data(), n_edges * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
        HS_TRY(fill_u64(ctx, reinterpret_cast<uint64_t *>(bgc), n_edges + 1, 0));
        const int64_t span = bins - n_tiles;
        const unsigned gb = (unsigned)(span <= 0 ? 1 : (cdiv(span, 256) < 1024 ? cdiv(span, 256) : 1024));
        hipLaunchKernelGGL(co_background, dim3(gb), dim3(256), 0, ctx->stream, raw, n_tiles, bins, flag, slot, e2,
                           (int)n_edges, bgc);
        HS_HIP(hipGetLastError());
        std::vector<unsigned long long> hh(n_edges + 1);
        HS_TRY(read_back2(ctx, bgc, hh.data(), (n_edges + 1) * sizeof(unsigned long long), boff + bins, &total,
                          sizeof(total)));
        unsigned long long above = 0;
        for (int i = n_edges - 1; i >= 0; --i) {
            above += hh[i + 1];
            bg_counts[order[i]] = (int64_t)above;
        }
    } else {
        HS_TRY(read_back(ctx, boff + bins, &total, sizeof(total)));
    }
    *n_out = (int64_t)total;
    if ((int64_t)total > cap)
        return set_error(HS_EOVERFLOW, "hs_timeslide_coinc: %llu coincidences exceed capacity %lld",
                         (unsigned long long)total, (long long)cap);
    return HS_OK;
}
