// Peak clustering of above-threshold samples into triggers.
//
// The paper stores a trigger at the peak of the SNR (Sec. II) without giving the rule; the rule
// taken: candidate m of one template survives iff every other candidate m' of that template with
// |m' - m| <= W has rho2' < rho2, or rho2' == rho2 and m' > m.  Ranking uses the 64-bit key
// (float bits of rho2) << 32 | (2^32 - 1 - m), whose order is exactly that rule (rho2 >= 0).
//
// Work is O(candidates) and needs no sort: time is cut into tiles of exactly W samples.  Two
// candidates in one tile are within W of each other, so only a tile's key maximum (its champion,
// found with one atomicMax per candidate) can survive; the window of a champion in tile b lies
// inside tiles b-1, b, b+1, so the champion only scans the candidates binned to its two
// neighbour tiles.  Survivors occupy at most one slot per (template, tile); compacting the slots
// in bin order yields triggers sorted by (template position, m) with no sort.
#include "hs_internal.h"

namespace hs {

__device__ __forceinline__ uint64_t cand_key(float rho2, int32_t m) {
    return ((uint64_t)__float_as_uint(rho2) << 32) | (uint64_t)(0xFFFFFFFFu - (uint32_t)m);
}

__global__ void clu_bin(const hs_candidate *__restrict__ cand, int64_t n_cand, int32_t n_ids, int64_t n,
                        int64_t W, int64_t n_tiles, uint32_t *__restrict__ cnt, unsigned long long *__restrict__ best,
                        int32_t *__restrict__ bad) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n_cand) return;
    const hs_candidate c = cand[i];
    if (c.tpos < 0 || c.tpos >= n_ids || c.m < 0 || (int64_t)c.m >= n) {
        atomicOr(bad, 1);
        return;
    }
    const int64_t b = (int64_t)c.tpos * n_tiles + (uint32_t)c.m / (uint32_t)W;
    atomicAdd(&cnt[b], 1u);
    atomicMax(&best[b], (unsigned long long)cand_key(c.rho2, c.m));
}

__global__ void clu_scatter(const hs_candidate *__restrict__ cand, int64_t n_cand, int32_t n_ids, int64_t n,
                            int64_t W, int64_t n_tiles, const uint64_t *__restrict__ start,
                            uint32_t *__restrict__ cursor, uint32_t *__restrict__ lists) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n_cand) return;
    const hs_candidate c = cand[i];
    if (c.tpos < 0 || c.tpos >= n_ids || c.m < 0 || (int64_t)c.m >= n) return;
    const int64_t b = (int64_t)c.tpos * n_tiles + (uint32_t)c.m / (uint32_t)W;
    const uint32_t p = atomicAdd(&cursor[b], 1u);
    lists[start[b] + p] = (uint32_t)i;
}

__global__ void clu_champion(const hs_candidate *__restrict__ cand, int64_t n_cand, int32_t n_ids, int64_t n,
                             int64_t W, int64_t n_tiles, const uint64_t *__restrict__ start,
                             const uint32_t *__restrict__ lists, const unsigned long long *__restrict__ best,
                             uint32_t *__restrict__ flag, uint32_t *__restrict__ slot) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n_cand) return;
    const hs_candidate c = cand[i];
    if (c.tpos < 0 || c.tpos >= n_ids || c.m < 0 || (int64_t)c.m >= n) return;
    const int64_t tile = (uint32_t)c.m / (uint32_t)W;
    const int64_t b = (int64_t)c.tpos * n_tiles + tile;
    const uint64_t key = cand_key(c.rho2, c.m);
    if (key != best[b]) return;
    for (int d = -1; d <= 1; d += 2) {
        const int64_t nt = tile + d;
        if (nt < 0 || nt >= n_tiles) continue;
        const int64_t nb = b + d;
        for (uint64_t p = start[nb]; p < start[nb + 1]; ++p) {
            const hs_candidate o = cand[lists[p]];
            const int64_t dm = (int64_t)o.m - (int64_t)c.m;
            if ((dm <= W && dm >= -W) && cand_key(o.rho2, o.m) > key) return;
        }
    }
    flag[b] = 1u;
    slot[b] = (uint32_t)i;
}

__global__ void clu_emit(const hs_candidate *__restrict__ cand, int64_t bins, const uint32_t *__restrict__ flag,
                         const uint32_t *__restrict__ slot, const uint64_t *__restrict__ off,
                         const int32_t *__restrict__ tmpl_ids, int32_t seg, int64_t seg_t0, int64_t tps,
                         hs_trigger *__restrict__ out, int64_t cap) {
    const int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (b >= bins || !flag[b]) return;
    const uint64_t pos = off[b];
    if (pos >= (uint64_t)cap) return;
    const hs_candidate c = cand[slot[b]];
    hs_trigger t;
    t.seg = seg;
    t.tmpl = tmpl_ids[c.tpos];
    t.tick = seg_t0 + (int64_t)c.m * tps;
    t.snr = sqrtf(c.rho2);
    t.phase = c.phase;
    out[pos] = t;
}

}  // namespace hs

using namespace hs;

extern "C" int hs_cluster_triggers(hs_ctx *ctx, const hs_candidate *cand, int64_t n_cand, int64_t n,
                                   const int32_t *tmpl_ids, int32_t n_ids, int64_t window, int32_t seg,
                                   int64_t seg_t0, int64_t ticks_per_sample, hs_trigger *out, int64_t cap,
                                   int64_t *n_out) {
    HS_REQUIRE(ctx && n_out, "hs_cluster_triggers: null argument");
    HS_REQUIRE(n_cand >= 0 && n > 0 && n_ids >= 0 && window >= 1 && cap >= 0,
               "hs_cluster_triggers: bad sizes (n_cand=%lld n=%lld n_ids=%d window=%lld)", (long long)n_cand,
               (long long)n, n_ids, (long long)window);
    HS_REQUIRE(n_cand < (int64_t(1) << 32) && n <= (int64_t(1) << 30), "hs_cluster_triggers: input too large");
    *n_out = 0;
    if (n_cand == 0 || n_ids == 0) return HS_OK;
    HS_REQUIRE(cand && tmpl_ids && (out || cap == 0), "hs_cluster_triggers: null argument");
    HS_HIP(hipSetDevice(ctx->device));
    // a window of n or more samples joins every candidate of a template (one tile): the same
    // clustering as a window of n, which keeps the tile index a 32-bit quotient in the kernels
    if (window > n) window = n;
    const int64_t n_tiles = cdiv(n, window);
    const int64_t bins = (int64_t)n_ids * n_tiles;
    HS_REQUIRE(bins <= (int64_t(1) << 28), "hs_cluster_triggers: %lld (template, tile) bins exceed 2^28; "
               "use a wider window", (long long)bins);
    uint32_t *cnt, *cursor, *lists, *flag, *slot;
    unsigned long long *best;
    uint64_t *start, *off, *tmp;
    int32_t *bad;
    Carver cv;
    cv.add(&cnt, bins);
    cv.add(&cursor, bins);
    cv.add(&flag, bins);
    cv.add(&slot, bins);
    cv.add(&best, bins);
    cv.add(&start, bins + 1);
    cv.add(&off, bins + 1);
    cv.add(&tmp, scan_tmp_elems(bins));
    cv.add(&lists, n_cand);
    cv.add(&bad, 1);
    HS_TRY(cv.commit(ctx));
    HS_TRY(fill_u32(ctx, cnt, bins, 0));
    HS_TRY(fill_u32(ctx, cursor, bins, 0));
    HS_TRY(fill_u32(ctx, flag, bins, 0));
    HS_TRY(fill_u64(ctx, reinterpret_cast<uint64_t *>(best), bins, 0));
    HS_TRY(fill_u32(ctx, reinterpret_cast<uint32_t *>(bad), 1, 0));
    const unsigned gc = (unsigned)cdiv(n_cand, 256);
    hipLaunchKernelGGL(clu_bin, dim3(gc), dim3(256), 0, ctx->stream, cand, n_cand, n_ids, n, window, n_tiles, cnt,
                       best, bad);
    HS_HIP(hipGetLastError());
    HS_TRY(exclusive_scan_u32(ctx, cnt, bins, start, tmp));
    hipLaunchKernelGGL(clu_scatter, dim3(gc), dim3(256), 0, ctx->stream, cand, n_cand, n_ids, n, window, n_tiles,
                       start, cursor, lists);
    hipLaunchKernelGGL(clu_champion, dim3(gc), dim3(256), 0, ctx->stream, cand, n_cand, n_ids, n, window, n_tiles,
                       start, lists, best, flag, slot);
    HS_HIP(hipGetLastError());
    HS_TRY(exclusive_scan_u32(ctx, flag, bins, off, tmp));
    hipLaunchKernelGGL(clu_emit, dim3((unsigned)cdiv(bins, 256)), dim3(256), 0, ctx->stream, cand, bins, flag, slot,
                       off, tmpl_ids, seg, seg_t0, ticks_per_sample, out, cap);
    HS_HIP(hipGetLastError());
    uint64_t total = 0;
    int32_t hbad = 0;
    HS_TRY(read_back2(ctx, off + bins, &total, sizeof(total), bad, &hbad, sizeof(hbad)));
    HS_REQUIRE(hbad == 0, "hs_cluster_triggers: candidate with tpos outside [0, n_ids) or m outside [0, n)");
    *n_out = (int64_t)total;
    if ((int64_t)total > cap)
        return set_error(HS_EOVERFLOW, "hs_cluster_triggers: %llu triggers exceed capacity %lld",
                         (unsigned long long)total, (long long)cap);
    return HS_OK;
}
