// Peak clustering of above-threshold samples into triggers.
//
// The paper stores a trigger at the peak of the SNR (Sec. II) without giving the rule; the rule
// taken: candidate m of one template survives iff every other candidate m' of that template with
// |m' - m| <= W has rho2' < rho2, or rho2' == rho2 and m' > m.  Ranking uses the 64-bit key
// (float bits of rho2) << 32 | (2^32 - 1 - m), whose order is exactly that rule (rho2 >= 0).
//
// Work is O(candidates) and needs no sort and no per-tile lists: time is cut into tiles of
// exactly W samples.  Two candidates in one tile are within W of each other, so only a tile's key
// maximum (its champion, found with a 64-bit atomicMax) can survive, and a champion's window lies
// inside its own tile and the two neighbouring ones.  The champion of tile b therefore survives
// iff no candidate of tile b - 1 or b + 1 within W of it has a larger key, and every candidate can
// check that itself against the champions of its two neighbour tiles (the champion's m is the low
// half of its key), marking the ones it beats.  Survivors occupy at most one slot per
// (template, tile); compacting the slots in bin order yields triggers sorted by (template
// position, m) with no sort.  Only candidates of the valid region [m_lo, m_hi) take part (a
// segment that overlaps its neighbours keeps the samples its circular transform gets right).
#include "hs_internal.h"

namespace hs {

__device__ __forceinline__ uint64_t cand_key(float rho2, int32_t m) {
    return ((uint64_t)__float_as_uint(rho2) << 32) | (uint64_t)(0xFFFFFFFFu - (uint32_t)m);
}

__device__ __forceinline__ int64_t key_m(uint64_t key) { return (int64_t)(0xFFFFFFFFu - (uint32_t)key); }

__device__ __forceinline__ bool cand_ok(const hs_candidate &c, int32_t n_ids, int64_t n) {
    return c.tpos >= 0 && c.tpos < n_ids && c.m >= 0 && (int64_t)c.m < n;
}

// Tile champions.  Candidates arrive in runs that share a bin (the filter writes each row's
// candidates in sample order), so a wavefront first takes the maximum over each run of equal bins
// (a segmented scan with shuffles; the bins are below 2^28) and only a run's last lane issues the
// atomic, and only when the bin's current value does not already beat it (values only grow, so a
// stale read, atomic like the updates, can only let a useless atomic through).
__global__ __launch_bounds__(256) void clu_best(const hs_candidate *__restrict__ cand, int64_t n_cand,
                                                int32_t n_ids, int64_t n, int64_t W, int64_t n_tiles, int64_t m_lo,
                                                int64_t m_hi, unsigned long long *__restrict__ best,
                                                int32_t *__restrict__ bad) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    int32_t b = -1;
    unsigned long long k = 0;
    if (i < n_cand) {
        const hs_candidate c = cand[i];
        if (!cand_ok(c, n_ids, n)) {
            atomicOr(bad, 1);
        } else if ((int64_t)c.m >= m_lo && (int64_t)c.m < m_hi) {
            b = (int32_t)((int64_t)c.tpos * n_tiles + (uint32_t)c.m / (uint32_t)W);
            k = cand_key(c.rho2, c.m);
        }
    }
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int s = 1; s < 64; s <<= 1) {
        const int32_t bu = __shfl_up(b, s);
        const unsigned long long ku = __shfl_up(k, s);
        if (lane >= s && bu == b && ku > k) k = ku;
    }
    const int32_t bn = __shfl_down(b, 1);
    const bool tail = lane == 63 || bn != b;
    if (tail && b >= 0 && __hip_atomic_load(&best[b], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < k)
        atomicMax(&best[b], k);
}

// Champion slots and vetoes: the candidate holding its bin's maximum records its index; every
// candidate marks the champion of a neighbour tile that lies within W and has a smaller key.
__global__ __launch_bounds__(256) void clu_veto(const hs_candidate *__restrict__ cand, int64_t n_cand,
                                                int32_t n_ids, int64_t n, int64_t W, int64_t n_tiles, int64_t m_lo,
                                                int64_t m_hi, const unsigned long long *__restrict__ best,
                                                uint32_t *__restrict__ slot, uint32_t *__restrict__ veto) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n_cand) return;
    const hs_candidate c = cand[i];
    if (!cand_ok(c, n_ids, n) || (int64_t)c.m < m_lo || (int64_t)c.m >= m_hi) return;
    const int64_t tile = (uint32_t)c.m / (uint32_t)W;
    const int64_t b = (int64_t)c.tpos * n_tiles + tile;
    const uint64_t key = cand_key(c.rho2, c.m);
    if (key == best[b]) slot[b] = (uint32_t)i;
    for (int d = -1; d <= 1; d += 2) {
        const int64_t nt = tile + d;
        if (nt < 0 || nt >= n_tiles) continue;
        const uint64_t kb = best[b + d];
        if (kb == 0 || kb >= key) continue;  // empty tile (keys are never 0) or a better champion
        const int64_t dm = key_m(kb) - (int64_t)c.m;
        if (dm <= W && dm >= -W) veto[b + d] = 1u;
    }
}

__global__ __launch_bounds__(256) void clu_flag(const unsigned long long *__restrict__ best,
                                                const uint32_t *__restrict__ veto, int64_t bins,
                                                uint32_t *__restrict__ flag) {
    const int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (b < bins) flag[b] = (best[b] != 0 && veto[b] == 0) ? 1u : 0u;
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
                                   const int32_t *tmpl_ids, int32_t n_ids, int64_t window, int64_t m_lo,
                                   int64_t m_hi, int32_t seg, int64_t seg_t0, int64_t ticks_per_sample,
                                   hs_trigger *out, int64_t cap, int64_t *n_out) {
    HS_REQUIRE(ctx && n_out, "hs_cluster_triggers: null argument");
    HS_REQUIRE(n_cand >= 0 && n > 0 && n_ids >= 0 && window >= 1 && cap >= 0,
               "hs_cluster_triggers: bad sizes (n_cand=%lld n=%lld n_ids=%d window=%lld)", (long long)n_cand,
               (long long)n, n_ids, (long long)window);
    HS_REQUIRE(m_lo >= 0 && m_lo <= m_hi && m_hi <= n, "hs_cluster_triggers: valid region [%lld, %lld) outside [0, %lld]",
               (long long)m_lo, (long long)m_hi, (long long)n);
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
    uint32_t *veto, *flag, *slot;
    unsigned long long *best;
    uint64_t *off, *tmp;
    int32_t *bad;
    Carver cv;
    cv.add(&veto, bins);
    cv.add(&flag, bins);
    cv.add(&slot, bins);
    cv.add(&best, bins);
    cv.add(&off, bins + 1);
    cv.add(&tmp, scan_tmp_elems(bins));
    cv.add(&bad, 1);
    HS_TRY(cv.commit(ctx));
    HS_TRY(fill_u32(ctx, veto, bins, 0));
    HS_TRY(fill_u64(ctx, reinterpret_cast<uint64_t *>(best), bins, 0));
    HS_TRY(fill_u32(ctx, reinterpret_cast<uint32_t *>(bad), 1, 0));
    const unsigned gc = (unsigned)cdiv(n_cand, 256);
    const unsigned gb = (unsigned)cdiv(bins, 256);
    hipLaunchKernelGGL(clu_best, dim3(gc), dim3(256), 0, ctx->stream, cand, n_cand, n_ids, n, window, n_tiles, m_lo,
                       m_hi, best, bad);
    hipLaunchKernelGGL(clu_veto, dim3(gc), dim3(256), 0, ctx->stream, cand, n_cand, n_ids, n, window, n_tiles, m_lo,
                       m_hi, best, slot, veto);
    hipLaunchKernelGGL(clu_flag, dim3(gb), dim3(256), 0, ctx->stream, best, veto, bins, flag);
    HS_HIP(hipGetLastError());
    HS_TRY(exclusive_scan_u32(ctx, flag, bins, off, tmp));
    hipLaunchKernelGGL(clu_emit, dim3(gb), dim3(256), 0, ctx->stream, cand, bins, flag, slot, off, tmpl_ids, seg,
                       seg_t0, ticks_per_sample, out, cap);
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
