// Power-consistency chi-square at trigger samples and the re-weighted SNR of Eq. (4).
//
// Sec. II down-weights triggers with the chi-square test it cites; the test splits the template
// band into p bins of equal template power and compares each bin's share of the complex SNR with
// 1/p of the total.  Only triggers at or above rho_min are tested: they are compacted first and
// gathered into groups of up to CQ_GROUP triggers of one template; the band-limited SNRs z_l at
// the triggers' samples are direct sums over each bin (Horner's rule in float64, one pass over the
// bin's template elements per group; see chisq_bin_sums), and a last kernel forms chi2, the
// per-bin terms and the re-weighted SNR.  Splitting by bin gives p workgroups per four groups,
// enough to fill the GPU when only a few hundred triggers need the test.
#include <cmath>

#include "dft.h"
#include "hs_internal.h"
#include "storage.h"

namespace hs {

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

// Per group b: its first active index gfirst[b] (gfirst[n_groups] = n_act closes the last
// group) and its template gtmpl[b]; per active trigger a: its sample in the segment, msamp[a].
// The bin-sum workgroups then find everything they need with two rounds of independent loads.
__global__ void chisq_group_list(const uint32_t *__restrict__ start, const uint64_t *__restrict__ off, int64_t n_act,
                                 const hs_trigger *trig, const uint32_t *__restrict__ act, int64_t seg_t0, int64_t tps,
                                 uint32_t *__restrict__ gfirst, int32_t *__restrict__ gtmpl,
                                 uint32_t *__restrict__ msamp) {
    const int64_t a = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (a >= n_act) return;
    const hs_trigger tr = trig[act[a]];
    msamp[a] = (uint32_t)((tr.tick - seg_t0) / tps);
    if (start[a]) {
        gfirst[off[a]] = (uint32_t)a;
        gtmpl[off[a]] = tr.tmpl;
    }
    if (a == n_act - 1) gfirst[off[a] + start[a]] = (uint32_t)n_act;
}

// Bit pattern of lane 0's value in scalar registers (for values every lane computes alike).
__device__ __forceinline__ double uniform_f64(double x) {
    const uint64_t u = (uint64_t)__double_as_longlong(x);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)u);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(u >> 32));
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

__device__ __forceinline__ int64_t uniform_i64(int64_t x) {
    const uint64_t u = (uint64_t)x;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)u);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(u >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// One Horner step h_j <- h_j w_j + q for NG triggers (float64).
template <int NG>
__device__ __forceinline__ void horner_step(float2 q, const double *sr, const double *si, double *hr, double *hi) {
    const double qr = (double)q.x, qi = (double)q.y;
#pragma unroll
    for (int j = 0; j < NG; ++j) {
        const double nr = fma(hr[j], sr[j], fma(-hi[j], si[j], qr));
        hi[j] = fma(hr[j], si[j], fma(hi[j], sr[j], qi));
        hr[j] = nr;
    }
}

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

static constexpr int CQ_WAVES = 4;  // groups per workgroup, one wavefront each
static constexpr int CQ_ROWS = 4;   // rows of 64 bins per staged data window

// template elements are read once: stream them past the caches
template <typename E>
__device__ __forceinline__ E stream_load(const E *p) {
    if constexpr (sizeof(E) == 8) {
        const uint64_t u = __builtin_nontemporal_load(reinterpret_cast<const uint64_t *>(p));
        E e;
        __builtin_memcpy(&e, &u, 8);
        return e;
    } else {
        static_assert(sizeof(E) == 4, "8- or 4-byte template elements");
        const uint32_t u = __builtin_nontemporal_load(reinterpret_cast<const uint32_t *>(p));
        E e;
        __builtin_memcpy(&e, &u, 4);
        return e;
    }
}

// State of one wavefront over the windows of its workgroup.
struct WinCtx {
    const float2 *dspec;
    int64_t n, kb, n_win, b0, b1, w_lo, w_hi;  // [w_lo, w_hi]: the windows that meet [b0, b1)
    int wv, lane;
};

// The windows from the top down for a wavefront whose group has NG triggers (0: the wavefront
// only stages data).  Every wavefront of the workgroup runs n_win + 1 barriers here, whatever NG.
// The next window's loads (data rows to stage, this wavefront's template elements) are issued
// before the current window's Horner steps, unconditionally (a template load outside [b0, b1)
// reads a bin of the template's own range and its value is replaced by zero when stepped), so
// their count is fixed and the steps never wait for them.  The steps cover the windows that meet
// the wavefront's bin, every row of them: rows outside the bin hold zeros, which above it leave
// the zero polynomial zero and below it are powers of w down to the lowest window's first row.
template <typename ST, int NG>
__device__ __forceinline__ void run_windows(const WinCtx &c, float2 (*win)[CQ_ROWS][64],
                                            const typename ST::elem *__restrict__ tmpl, const double *sr,
                                            const double *si, double *hr, double *hi) {
    constexpr int R = CQ_ROWS, NW = CQ_WAVES;
    constexpr int SR = (R + NW - 1) / NW;  // rows each wavefront stages: wv, wv + NW, ... (below R)
    float2 dn[SR];
    typename ST::elem tc[R], tn[R];
    // Bins fit in 32 bits (n <= 2^22): offsets from scalar bases.  A wavefront whose row is past
    // the window loads the window's last row and does not store it, so every wavefront issues the
    // same loads on every trip.
    const int32_t kmax = (int32_t)(c.n / 2 - 1);
    auto stage = [&](int64_t wi) {
        const int32_t k0 = (int32_t)(c.kb + 64 * wi * R);
#pragma unroll
        for (int u = 0; u < SR; ++u) {
            const int row = c.wv + u * NW < R ? c.wv + u * NW : R - 1;
            const int32_t k = k0 + 64 * row + c.lane;
            dn[u] = c.dspec[(uint32_t)(k < kmax ? k : kmax)];  // beyond the union's top: any bin of the band
        }
    };
    auto put = [&](float2(*w)[64]) {
#pragma unroll
        for (int u = 0; u < SR; ++u)
            if (c.wv + u * NW < R) w[c.wv + u * NW][c.lane] = dn[u];
    };
    // the raw elements and a mask of those inside [b0, b1): the mask is applied when the window is
    // stepped, so nothing waits for the loads while they are in flight
    const typename ST::elem *t0 = tmpl + c.b0;
    const int32_t len = (int32_t)(c.b1 - c.b0);
    auto fetch = [&](int64_t wi, typename ST::elem *te) {
        const int32_t r0 = (int32_t)(c.kb + 64 * wi * R - c.b0);  // bin - b0 of the window's first bin
        uint32_t in = 0;
#pragma unroll
        for (int u = 0; u < R; ++u) {
            const int32_t r = r0 + 64 * u + c.lane;
            in |= (uint32_t)r < (uint32_t)len ? (1u << u) : 0u;
            const int32_t rc = r < 0 ? 0 : (r < len ? r : len - 1);
            te[u] = stream_load(t0 + (uint32_t)rc);
        }
        return in;
    };
    int buf = 0;
    uint32_t mc = 0, mn = 0;
    if (c.n_win > 0) {
        stage(c.n_win - 1);
        put(win[0]);
        if constexpr (NG > 0) mc = fetch(c.n_win - 1, tc);
    }
    __syncthreads();
    for (int64_t wi = c.n_win - 1; wi >= 0; --wi) {
        // issued on every trip (the last one refetches its own window), so that the number of
        // loads in flight is the same on every path and the steps below never wait for them
        const int64_t wn = wi > 0 ? wi - 1 : 0;
        stage(wn);
        if constexpr (NG > 0) mn = fetch(wn, tn);
        if constexpr (NG > 0) {
            if (wi >= c.w_lo && wi <= c.w_hi) {
#pragma unroll
                for (int u = R - 1; u >= 0; --u) {
                    const float2 t = (mc >> u) & 1u ? ST::unpack(tc[u]) : float2{0.0f, 0.0f};
                    horner_step<NG>(cmulc(win[buf][u][c.lane], t), sr, si, hr, hi);
                }
                // keeps the steps here, ahead of the wait for the next window (the compiler
                // would otherwise sink them below it)
#pragma unroll
                for (int j = 0; j < NG; ++j) asm volatile("" : "+v"(hr[j]), "+v"(hi[j]));
            }
        }
        put(win[buf ^ 1]);
        if constexpr (NG > 0) {
#pragma unroll
            for (int u = 0; u < R; ++u) tc[u] = tn[u];
            mc = mn;
        }
        __syncthreads();
        buf ^= 1;
    }
}

// z_l for one (bin l, group of active triggers of one template): sum over the bins of l of
// q_k exp(+2 pi i k m / N), q_k = d~_k conj(w~_k) formed once per bin in float32 and shared by the
// group's triggers; everything after it in float64.
//
// A workgroup takes bin l of CQ_WAVES consecutive groups, one wavefront each.  The bank is sorted
// by chirp mass, so their bins cover nearly the same bins k, and the data spectrum is staged once
// for all of them: the union of their ranges is cut into rows of 64 bins from its lowest bin kb,
// lane L of every wavefront owns the bins kb + L + 64 r, and windows of CQ_ROWS rows are staged
// in LDS (double-buffered) from the top down.  Each wavefront reads only its own template from
// HBM.  With v = exp(2 pi i m / N), q = 0 outside the bin and kw = kb + 64 r0 the first bin of
// the lowest window that meets the bin (row r0),
//     z_l = v^kw sum_L v^L P_L(v^64),   P_L(w) = sum_{r >= r0} q(kb + L + 64 r) w^(r - r0).
// Each lane evaluates its P by Horner's rule over the rows (one complex multiply-add per bin and
// trigger), the sum over lanes is a tree whose level s joins blocks of 2^s lanes with the factor
// v^(2^s), and v^kw is applied last.  Every power of v used is an exact float64 sincospi of
// (E m mod N) / N, computed once per wavefront (one per lane), so no twiddle table is read; v^64
// is the same in every lane and lives in scalar registers.  Any bank order gives the same sums;
// the sorted order only keeps the unions, and so the staged rows, short.
template <typename ST>
__global__ __launch_bounds__(64 * CQ_WAVES) void chisq_bin_sums(
    const float2 *__restrict__ dspec, int64_t n, const typename ST::elem *__restrict__ spectra,
    const int64_t *__restrict__ offset, const int32_t *__restrict__ k0, const int32_t *__restrict__ klo,
    const int32_t *__restrict__ khi, const int32_t *__restrict__ edges, int p, int64_t n_groups,
    const uint32_t *__restrict__ gfirst, const int32_t *__restrict__ gtmpl, const uint32_t *__restrict__ msamp,
    bool skip_widest, double2 *__restrict__ zl) {
    constexpr int G = CQ_GROUP, NW = CQ_WAVES, R = CQ_ROWS;
    __shared__ double2 ph[NW][G][8];  // per trigger: v^1, ..., v^32 (tree), v^64 (Horner), v^kw
    __shared__ float2 win[2][R][64];
    __shared__ int64_t span[NW][2];
    // the wavefront index and everything derived from it are the same in every lane: scalar
    const int tid = threadIdx.x, wv = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
    // the last equal-power bin is the widest by far (up to ~80 % of a long template's band), so
    // its workgroups are dispatched first and the short ones fill the end of the grid
    const int l = p - 1 - (int)blockIdx.y;
    const int64_t gb = (int64_t)blockIdx.x * NW + wv;
    int g = 0;
    int64_t a0 = 0, base = 0, b0 = 0, b1 = 0;
    bool write = false;  // this wavefront's group takes bin l (the widest may be formed from the peak)
    if (gb < n_groups) {
        a0 = gfirst[gb];
        g = (int)(gfirst[gb + 1] - a0);  // 1..CQ_GROUP
        const int t = gtmpl[gb];
        const int32_t *e = edges + (int64_t)t * (p + 1);
        if (!(skip_widest && l == widest_bin(e, p))) {
            write = true;
            base = offset[t] - k0[t];
            // every bin is clamped to the template's band, which lies inside [1, n/2 - 1]
            const int64_t band_lo = klo[t] > 1 ? klo[t] : 1;
            const int64_t band_hi = khi[t] < n / 2 - 1 ? khi[t] : n / 2 - 1;
            b0 = e[l] > band_lo ? e[l] : band_lo;
            b1 = e[l + 1] < band_hi + 1 ? e[l + 1] : band_hi + 1;
        }
    }
    const bool reads = write && b1 > b0;
    if (lane == 0) {
        span[wv][0] = reads ? b0 : INT64_MAX;
        span[wv][1] = reads ? b1 : INT64_MIN;
    }
    __syncthreads();
    int64_t kb = INT64_MAX, top = INT64_MIN;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        const int64_t lo = uniform_i64(span[w][0]), hi = uniform_i64(span[w][1]);
        kb = lo < kb ? lo : kb;
        top = hi > top ? hi : top;
    }
    const int64_t n_win = top > kb ? (top - 1 - kb) / (64 * R) + 1 : 0;  // the same in every wavefront
    // the windows this wavefront steps; its polynomial starts at the first row of w_lo
    const int64_t w_lo = reads ? (b0 - kb) / (64 * R) : 1, w_hi = reads ? (b1 - 1 - kb) / (64 * R) : 0;
    const int64_t kw = reads ? kb + 64 * R * w_lo : 0;  // kb is INT64_MAX when no wavefront reads
    if (reads && lane < 8 * g) {
        const int j = lane >> 3, s = lane & 7;
        const uint64_t m = msamp[a0 + j];
        const uint64_t ex = s < 7 ? (uint64_t(1) << s) : (uint64_t)kw;
        double sn, cs;
        sincospi((double)((ex * m) & ((uint64_t)n - 1)) * (2.0 / (double)n), &sn, &cs);
        ph[wv][j][s] = double2{cs, sn};
    }
    __syncthreads();  // the phases
    double hr[G], hi[G], sr[G], si[G];
#pragma unroll
    for (int j = 0; j < G; ++j) {
        hr[j] = hi[j] = sr[j] = si[j] = 0.0;
        if (reads && j < g) {
            sr[j] = uniform_f64(ph[wv][j][6].x);
            si[j] = uniform_f64(ph[wv][j][6].y);
        }
    }
    const WinCtx c{dspec, n, kb, n_win, b0, b1, w_lo, w_hi, wv, lane};
    const typename ST::elem *tmpl = spectra + base;
    const int gs = reads ? g : 0;
    switch (gs) {  // a loop without per-trigger predicates for each group size
    case 0: run_windows<ST, 0>(c, win, tmpl, sr, si, hr, hi); break;
    case 1: run_windows<ST, 1>(c, win, tmpl, sr, si, hr, hi); break;
    case 2: run_windows<ST, 2>(c, win, tmpl, sr, si, hr, hi); break;
    case 3: run_windows<ST, 3>(c, win, tmpl, sr, si, hr, hi); break;
    case 4: run_windows<ST, 4>(c, win, tmpl, sr, si, hr, hi); break;
    case 5: run_windows<ST, 5>(c, win, tmpl, sr, si, hr, hi); break;
    case 6: run_windows<ST, 6>(c, win, tmpl, sr, si, hr, hi); break;
    case 7: run_windows<ST, 7>(c, win, tmpl, sr, si, hr, hi); break;
    default: run_windows<ST, 8>(c, win, tmpl, sr, si, hr, hi); break;
    }
    if (!write) return;
    // tree inside the wavefront: after level s, lane L with L mod 2^(s+1) = 0 holds
    // sum_{u < 2^(s+1)} v^u P_{L+u}; its partner block starts at L + 2^s
#pragma unroll
    for (int j = 0; j < G; ++j) {
        if (j < gs) {
            double x = hr[j], y = hi[j];
#pragma unroll
            for (int s = 0; s < 6; ++s) {
                const double xd = __shfl_down(x, 1 << s), yd = __shfl_down(y, 1 << s);
                const double2 v = ph[wv][j][s];
                x += v.x * xd - v.y * yd;
                y += v.x * yd + v.y * xd;
            }
            if (lane == 0) {
                const double2 vb = ph[wv][j][7];
                zl[(a0 + j) * p + l] = double2{vb.x * x - vb.y * y, vb.x * y + vb.y * x};
            }
        } else if (j < g && lane == 0) {
            zl[(a0 + j) * p + l] = double2{0.0, 0.0};  // an empty bin
        }
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
static int launch_bin_sums(hs_ctx *ctx, int64_t n_groups, const float2 *d, int64_t n, const hs_bank *bank, int p,
                           const uint32_t *gfirst, const int32_t *gtmpl, const uint32_t *msamp, bool skip_widest,
                           double2 *zl) {
    // (CQ_WAVES groups, bin): x holds the large count
    const dim3 gs((unsigned)cdiv(n_groups, CQ_WAVES), (unsigned)p);
    hipLaunchKernelGGL(chisq_bin_sums<ST>, gs, dim3(64 * CQ_WAVES), 0, ctx->stream, d, n,
                       static_cast<const typename ST::elem *>(bank->spectra), bank->offset, bank->k0, bank->k_lo,
                       bank->k_hi, bank->chisq_edges, p, n_groups, gfirst, gtmpl, msamp, skip_widest, zl);
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
    uint32_t *gstart, *gfirst, *rfirst, *msamp;
    int32_t *gtmpl;
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
    cv2.add(&gfirst, (size_t)n_act + 1);
    cv2.add(&rfirst, (size_t)n_act);
    cv2.add(&gtmpl, (size_t)n_act);
    cv2.add(&msamp, (size_t)n_act);
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
    hipLaunchKernelGGL(chisq_group_list, dim3(ga), dim3(256), 0, ctx->stream, gstart, goff, (int64_t)n_act, trig, act,
                       seg_t0, ticks_per_sample, gfirst, gtmpl, msamp);
    HS_HIP(hipGetLastError());
    uint64_t n_groups = 0;
    HS_TRY(read_back(ctx, goff + n_act, &n_groups, sizeof(n_groups)));
    const float2 *d = static_cast<const float2 *>(spec);
    switch (bank->dtype) {
    case HS_F32:
        HS_TRY((launch_bin_sums<StoreF32>(ctx, (int64_t)n_groups, d, n, bank, p, gfirst, gtmpl, msamp, from_peak, zl)));
        break;
    case HS_BF16:
        HS_TRY((launch_bin_sums<StoreBF16>(ctx, (int64_t)n_groups, d, n, bank, p, gfirst, gtmpl, msamp, from_peak, zl)));
        break;
    default:
        HS_TRY((launch_bin_sums<StoreF16>(ctx, (int64_t)n_groups, d, n, bank, p, gfirst, gtmpl, msamp, from_peak, zl)));
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
