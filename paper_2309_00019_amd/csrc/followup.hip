// Stage-1 follow-up (Sec. III): coincidences with Lambda_1 >= threshold (here the network SNR,
// decided as (double)stat >= rho_min^2) select fine-bank neighbourhoods -- every fine template
// within a relative chirp-mass distance `frac` of the coarse template -- and the union of the
// selected neighbourhoods is formed per segment (the segment of the H trigger and the segment of
// the unshifted L trigger), as sorted unique fine ids.
#include "hs_internal.h"

namespace hs {

__device__ __forceinline__ int64_t seg_of(int64_t tick, int64_t seg_ticks) {
    int64_t q = tick / seg_ticks;
    if ((tick % seg_ticks != 0) && tick < 0) --q;
    return q;
}

__global__ void fu_select(const hs_coinc *__restrict__ c, int64_t n_c, double r2min, int32_t n_coarse,
                          uint32_t *__restrict__ flag, int32_t *__restrict__ bad) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n_c) return;
    const hs_coinc x = c[i];
    uint32_t f = 0;
    if ((double)x.stat >= r2min) {
        if (x.tmpl < 0 || x.tmpl >= n_coarse) atomicOr(bad, 1);
        else f = 1;
    }
    flag[i] = f;
}

__global__ void fu_compact(const uint32_t *__restrict__ flag, const uint64_t *__restrict__ off, int64_t n_c,
                           uint32_t *__restrict__ sel) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n_c && flag[i]) sel[off[i]] = (uint32_t)i;
}

// Cell of fine template f inside the neighbourhood of a coarse template of chirp mass mc:
// 16 bins of u = (mc_f - mc) / (frac mc) in [-1, 1] times 4 mass-ratio bins.  Every operation is
// a separately rounded float64 operation (no contraction) so the bin decision is reproducible.
__device__ __forceinline__ int fu_cell(double mc_f, double mc, double frac, double q_f, double qe0, double qe1,
                                      double qe2) {
    const double u = __ddiv_rn(__dsub_rn(mc_f, mc), __dmul_rn(frac, mc));
    int ib = (int)floor(__dmul_rn(__dadd_rn(u, 1.0), 8.0));
    ib = ib < 0 ? 0 : (ib > 15 ? 15 : ib);
    return 4 * ib + (q_f >= qe0) + (q_f >= qe1) + (q_f >= qe2);
}

__global__ void fu_mark(const hs_coinc *__restrict__ c, const uint32_t *__restrict__ sel, int64_t n_sel,
                        const double *__restrict__ coarse_mc, const double *__restrict__ fine_mc, int32_t n_fine,
                        double frac, int64_t seg_ticks, int32_t n_seg, const uint64_t *__restrict__ cell_mask,
                        const double *__restrict__ fine_q, double qe0, double qe1, double qe2,
                        uint32_t *__restrict__ mark) {
    const int64_t total = n_sel * (int64_t)n_fine;
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < total;
         q += (int64_t)gridDim.x * blockDim.x) {
        const int64_t s = q / n_fine;
        const int32_t f = (int32_t)(q - s * n_fine);
        const uint32_t ci = sel[s];
        const hs_coinc x = c[ci];
        const double mc = coarse_mc[x.tmpl];
        if (fabs(fine_mc[f] - mc) <= frac * mc) {
            if (cell_mask) {
                const int cell = fu_cell(fine_mc[f], mc, frac, fine_q[f], qe0, qe1, qe2);
                if (!((cell_mask[ci] >> cell) & 1ull)) continue;
            }
            const int64_t sh = seg_of(x.tick_h, seg_ticks);
            const int64_t sl = seg_of(x.tick_l, seg_ticks);
            if (sh >= 0 && sh < n_seg) mark[sh * n_fine + f] = 1u;
            if (sl >= 0 && sl < n_seg) mark[sl * n_fine + f] = 1u;
        }
    }
}

__global__ void fu_emit(const uint32_t *__restrict__ mark, const uint64_t *__restrict__ off, int32_t n_fine,
                        int32_t n_seg, int32_t *__restrict__ ids) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= (int64_t)n_seg * n_fine || !mark[i]) return;
    const int64_t s = i / n_fine;
    const int32_t f = (int32_t)(i - s * n_fine);
    ids[s * n_fine + (int64_t)(off[i] - off[s * n_fine])] = f;
}

__global__ void fu_row_counts(const uint64_t *__restrict__ off, int32_t n_fine, int32_t n_seg,
                              uint64_t *__restrict__ counts) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < n_seg) counts[s] = off[(int64_t)(s + 1) * n_fine] - off[(int64_t)s * n_fine];
}

}  // namespace hs

using namespace hs;

static int followup_impl(hs_ctx *ctx, const hs_coinc *c, int64_t n_c, float rho_min, const double *coarse_mchirp,
                         int32_t n_coarse, const double *fine_mchirp, const double *fine_q, int32_t n_fine, double frac,
                         const double *q_edges, const uint64_t *cell_mask, int64_t seg_ticks, int32_t n_seg,
                         int32_t *fine_ids, int32_t *n_ids) {
    HS_REQUIRE(ctx && n_ids, "hs_followup: null argument");
    HS_REQUIRE(n_c >= 0 && n_coarse >= 0 && n_fine >= 0 && n_seg >= 0 && seg_ticks > 0 && frac >= 0,
               "hs_followup: bad sizes");
    HS_REQUIRE(n_c < (int64_t(1) << 32) && (int64_t)n_seg * n_fine < (int64_t(1) << 32) &&
                   (double)n_c * (double)n_fine < 9.0e18,
               "hs_followup: input too large");
    for (int s = 0; s < n_seg; ++s) n_ids[s] = 0;
    if (n_seg == 0 || n_fine == 0 || n_c == 0) return HS_OK;
    HS_REQUIRE(c && coarse_mchirp && fine_mchirp && fine_ids, "hs_followup: null argument");
    HS_REQUIRE(!cell_mask || (fine_q && q_edges), "hs_followup_cells: null argument");
    HS_HIP(hipSetDevice(ctx->device));
    const int64_t cells = (int64_t)n_seg * n_fine;
    uint32_t *flag, *sel, *mark;
    uint64_t *soff, *moff, *tmp, *counts;
    int32_t *bad;
    Carver cv;
    cv.add(&flag, n_c);
    cv.add(&soff, n_c + 1);
    cv.add(&sel, n_c);
    cv.add(&mark, cells);
    cv.add(&moff, cells + 1);
    cv.add(&tmp, scan_tmp_elems(cells > n_c ? cells : n_c));
    cv.add(&counts, n_seg);
    cv.add(&bad, 1);
    HS_TRY(cv.commit(ctx));
    HS_TRY(fill_u32(ctx, mark, cells, 0));
    HS_TRY(fill_u32(ctx, reinterpret_cast<uint32_t *>(bad), 1, 0));
    const double r2min = (double)rho_min * (double)rho_min;
    hipLaunchKernelGGL(fu_select, dim3((unsigned)cdiv(n_c, 256)), dim3(256), 0, ctx->stream, c, n_c, r2min, n_coarse,
                       flag, bad);
    HS_HIP(hipGetLastError());
    HS_TRY(exclusive_scan_u32(ctx, flag, n_c, soff, tmp));
    hipLaunchKernelGGL(fu_compact, dim3((unsigned)cdiv(n_c, 256)), dim3(256), 0, ctx->stream, flag, soff, n_c, sel);
    HS_HIP(hipGetLastError());
    uint64_t n_sel = 0;
    int32_t hbad = 0;
    HS_TRY(read_back2(ctx, soff + n_c, &n_sel, sizeof(n_sel), bad, &hbad, sizeof(hbad)));
    HS_REQUIRE(hbad == 0, "hs_followup: followed coincidence with tmpl outside [0, n_coarse)");
    if (n_sel > 0) {
        const int64_t work = (int64_t)n_sel * n_fine;
        int64_t g = cdiv(work, 256);
        if (g > 65536) g = 65536;
        const double qe0 = cell_mask ? q_edges[0] : 0.0, qe1 = cell_mask ? q_edges[1] : 0.0,
                     qe2 = cell_mask ? q_edges[2] : 0.0;
        hipLaunchKernelGGL(fu_mark, dim3((unsigned)g), dim3(256), 0, ctx->stream, c, sel, (int64_t)n_sel, coarse_mchirp,
                           fine_mchirp, n_fine, frac, seg_ticks, n_seg, cell_mask, fine_q, qe0, qe1, qe2, mark);
        HS_HIP(hipGetLastError());
    }
    HS_TRY(exclusive_scan_u32(ctx, mark, cells, moff, tmp));
    hipLaunchKernelGGL(fu_emit, dim3((unsigned)cdiv(cells, 256)), dim3(256), 0, ctx->stream, mark, moff, n_fine, n_seg,
                       fine_ids);
    hipLaunchKernelGGL(fu_row_counts, dim3((unsigned)cdiv(n_seg, 256)), dim3(256), 0, ctx->stream, moff, n_fine, n_seg,
                       counts);
    HS_HIP(hipGetLastError());
    std::vector<uint64_t> hc(n_seg);
    HS_TRY(read_back(ctx, counts, hc.data(), n_seg * sizeof(uint64_t)));
    for (int s = 0; s < n_seg; ++s) n_ids[s] = (int32_t)hc[s];
    return HS_OK;
}

extern "C" int hs_followup(hs_ctx *ctx, const hs_coinc *c, int64_t n_c, float rho_min, const double *coarse_mchirp,
                           int32_t n_coarse, const double *fine_mchirp, int32_t n_fine, double frac,
                           int64_t seg_ticks, int32_t n_seg, int32_t *fine_ids, int32_t *n_ids) {
    return followup_impl(ctx, c, n_c, rho_min, coarse_mchirp, n_coarse, fine_mchirp, nullptr, n_fine, frac, nullptr,
                         nullptr, seg_ticks, n_seg, fine_ids, n_ids);
}

// Learned-proposer variant: each followed coincidence contributes only the cells of its
// neighbourhood selected in cell_mask (an addition on top of Sec. III's rule).
extern "C" int hs_followup_cells(hs_ctx *ctx, const hs_coinc *c, int64_t n_c, float rho_min,
                                 const double *coarse_mchirp, int32_t n_coarse, const double *fine_mchirp,
                                 const double *fine_q, int32_t n_fine, double frac, const double *q_edges,
                                 const uint64_t *cell_mask, int64_t seg_ticks, int32_t n_seg, int32_t *fine_ids,
                                 int32_t *n_ids) {
    HS_REQUIRE(ctx && n_ids, "hs_followup_cells: null argument");
    if (n_c > 0 && n_fine > 0 && n_seg > 0)
        HS_REQUIRE(cell_mask && fine_q && q_edges, "hs_followup_cells: null argument");
    return followup_impl(ctx, c, n_c, rho_min, coarse_mchirp, n_coarse, fine_mchirp, fine_q, n_fine, frac, q_edges,
                         cell_mask, seg_ticks, n_seg, fine_ids, n_ids);
}
