// Matched filter (Sec. II, Eqs. (1)-(2); quadrature form of Appendix A): for every template,
//   z[m] = sum_{k in band} d~[k] conj(w~[k]) exp(+2 pi i k m / N),   m = 0..N-1,
// with d~ the whitened data and w~ the prepared (whitened, sigma-normalised) template, then
// rho^2 = |z|^2 compared against thr^2 (Sec. II: the threshold is inclusive, rho >= thr).
//
// The N-point inverse transform is split four-step with N = 512 * N1:
//   k = k1 + N1 k2  (k1 < N1, k2 < 512),   m = m2 + 512 m1  (m2 < 512, m1 < N1)
//   pass A:  Y[m2][k1] = W_N^{k1 m2} sum_{k2} q[k1 + N1 k2] W_512^{k2 m2},   q = d~ conj(w~)
//   pass B:  z[m2 + 512 m1] = sum_{k1} Y[m2][k1] W_N1^{k1 m1}
// (W_L = exp(+2 pi i / L)).  The data and templates only occupy k < N/2, i.e. k2 < 256, so the
// 512-point transform of pass A is pruned to two 256-point transforms (of x[k2] and of
// x[k2] W_512^{k2}, giving the even and odd outputs).  The product d~ conj(w~) is formed while
// loading (only bins inside the template's band are read), and pass B ends with the threshold
// and a wavefront-ballot compaction: one atomic per wavefront that holds candidates.
//
// Pass A: a workgroup of 16 x COLS threads owns COLS consecutive columns k1 of one template
// (COLS = 16, 32 or 64, at most N1); thread (c = tid % COLS, l = tid / COLS) loads x[l + 16 j],
// j < 16, of column c (COLS lanes read 8 COLS contiguous bytes of spectrum per row), does a
// radix-16 DFT over j in registers, exchanges through LDS, and a second radix-16 DFT finishes
// each 256-point transform; every row of the intermediate is written in pieces of 8 COLS bytes.
// Pass B: each lane holds 16 points of a row; N1/16 lanes share a row; radix-16 passes with
// LDS exchanges (Stockham indexing), the last pass ending in registers for the epilogue.
// A few workgroups fit a CU (LDS-limited), so memory latency is hidden only if every global load
// of a workgroup is issued before its first LDS barrier: the band loads,
// one per-call record with the template's band and scale (instead of a chain ids -> offset ->
// band), and in pass B one twiddle per radix group, whose powers are then formed by at most 14
// products (relative error ~1e-6, far below the SNR tolerance) instead of table loads that would
// wait behind each barrier.  So arranged, pass A streams at the HBM rate a device copy reaches
// and pass B is bound by its VALU work.
#include <cmath>
#include <mutex>

#include "dft.h"
#include "hs_internal.h"
#include "storage.h"

namespace hs {

// Pass-A columns per workgroup (the context's pass-A tile, at most N1): each row of the
// intermediate is written in pieces of 8 COLS bytes (at N = 2^19 64 columns, 512-byte pieces, ran
// 4-5 % faster per template than 16 and 8 columns 43 % slower).  The exchange buffer holds 16
// l-blocks of 16 x COLS values, padded.
template <int COLS> constexpr int pa_lds_stride() { return COLS * 16 + COLS; }
static constexpr int MF_STRIPES = 64;                 // candidate lists (power of two)

// Candidate lists: MF_STRIPES lists of stripe_cap records followed by one spill list of
// spill_cap records; count[0..MF_STRIPES-1] are the per-list reservation counters (they may run
// past stripe_cap -- the excess went to the spill list) and count[MF_STRIPES] the spill counter.
// mf_compact concatenates the lists (stripe order, then the spill list) into the caller's buffer.
__global__ __launch_bounds__(256) void mf_compact(const hs_candidate *__restrict__ buf,
                                                  const unsigned long long *__restrict__ count, int64_t stripe_cap,
                                                  int64_t spill_cap, hs_candidate *__restrict__ out, int64_t cap) {
    const int s = blockIdx.y;  // 0..MF_STRIPES (the last one is the spill list)
    unsigned long long off = 0;
    for (int q = 0; q < s; ++q) off += count[q] < (unsigned long long)stripe_cap ? count[q] : stripe_cap;
    const unsigned long long lim = s < MF_STRIPES ? (unsigned long long)stripe_cap : (unsigned long long)spill_cap;
    const unsigned long long n = count[s] < lim ? count[s] : lim;
    const hs_candidate *src = buf + (size_t)s * stripe_cap;
    for (unsigned long long i = blockIdx.x * 256ull + threadIdx.x; i < n; i += (unsigned long long)gridDim.x * 256ull)
        if (off + i < (unsigned long long)cap) out[off + i] = src[i];
}

// Stores record o at reservation index idx of stripe list `stripe`, spilling past its capacity.
__device__ __forceinline__ void mf_store_one(hs_candidate *lists, unsigned long long *count, int stripe,
                                             int64_t stripe_cap, int64_t spill_cap, unsigned long long idx,
                                             const hs_candidate &o) {
    if (idx < (unsigned long long)stripe_cap) {
        lists[(size_t)stripe * stripe_cap + idx] = o;
    } else {
        const unsigned long long j = atomicAdd(&count[MF_STRIPES], 1ull);
        if (j < (unsigned long long)spill_cap) lists[(size_t)MF_STRIPES * stripe_cap + j] = o;
    }
}

// Per-call work list: one record per position of tmpl_ids, so each workgroup of pass A / pass B
// finds its template's band and scale with a single scalar load.  An id outside the bank or a
// band outside [1, n/2 - 1] sets *bad and gets an empty band and a zero scale (the passes then
// read nothing from the bank; the call reports the error).
struct alignas(32) MfItem {
    int64_t base;  // element index of bin 0 in the spectra (offset - k0)
    int32_t lo, hi;
    float sc;      // rho^2 scale of the template's storage
    int32_t pad[3];
};

__global__ void mf_items(const int32_t *__restrict__ ids, int32_t n_ids, int32_t n_tmpl,
                         const int64_t *__restrict__ offset, const int32_t *__restrict__ k0,
                         const int32_t *__restrict__ klo, const int32_t *__restrict__ khi,
                         const float *__restrict__ r2scale, int64_t half, MfItem *__restrict__ items,
                         int32_t *__restrict__ bad) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_ids) return;
    MfItem it{0, 1, 0, 0.0f, {0, 0, 0}};
    const int32_t t = ids[i];
    if (t < 0 || t >= n_tmpl) {
        atomicOr(bad, 1);
    } else if (klo[t] < 1 || klo[t] < k0[t] || khi[t] > half - 1) {
        atomicOr(bad, 2);
    } else {
        it.base = offset[t] - k0[t];
        it.lo = klo[t];
        it.hi = khi[t];
        it.sc = r2scale[t];
    }
    items[i] = it;
}

// 16 x COLS threads; 1024 threads per CU, i.e. 4 waves per SIMD (caps VGPRs at 128).
template <typename ST, int COLS>
__global__ __launch_bounds__(16 * COLS, 64 / COLS) void mf_pass_a(
    const float2 *__restrict__ dspec, const typename ST::elem *__restrict__ spectra,
    const MfItem *__restrict__ items, int32_t id0, int32_t N1, const float2 *__restrict__ tw512,
    const float2 *__restrict__ twlo, const float2 *__restrict__ twhi, float2 *__restrict__ Y) {
    constexpr int LSTRIDE = pa_lds_stride<COLS>();
    __shared__ float2 lds[16 * LSTRIDE];
    const int tb = blockIdx.y;
    const MfItem it = items[id0 + tb];
    const int c = threadIdx.x % COLS;
    const int l = threadIdx.x / COLS;
    const int k1 = blockIdx.x * COLS + c;
    const int64_t base = it.base;
    const int lo = it.lo, hi = it.hi;

    // All 32 band loads are issued before any product uses them: a use right after each
    // band-tested load would make the wavefront wait for every row in turn.  The stored template
    // elements are kept raw inside the band tests and unpacked after them (an unpack inside a
    // test would wait there for its load).
    float2 dd[16], x[16];
    typename ST::elem te[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const int k = k1 + N1 * (l + 16 * j);
        dd[j] = float2{0.0f, 0.0f};
        te[j] = ST::zero();
        if (k >= lo && k <= hi) {
            dd[j] = dspec[k];
            te[j] = spectra[base + k];
        }
    }
    if constexpr (ST::bytes == 4) {
        // An empty asm that takes each raw element as an operand pins it after the load loop, so
        // the compiler cannot fold the conversion into the band test (where it would wait).
#pragma unroll
        for (int j = 0; j < 16; ++j) asm volatile("" : "+v"(te[j]));
    }
#pragma unroll
    for (int j = 0; j < 16; ++j) x[j] = cmulc(dd[j], ST::unpack(te[j]));
    float2 *Yt = Y + (size_t)tb * 512 * (size_t)N1;
    // Twiddles: W_512^{k2} = W_512^l W_32^j; the W_32^j are compile-time constants applied
    // before the radix-16 DFT over j, and the common factor W_512^l is merged after it with
    // W_256^{l a}.  W_256^{l a} and the four-step W_N^{k1 m2} (m2 = 2(a + 16 b) + r) advance by
    // short recurrences from table values, at most 15 products each (relative error ~1e-6,
    // far below the SNR tolerance).
    const float2 w512l = tw512[l];
    const float2 w256l = tw512[2 * l];
    const int ju = 32 * k1;  // < N
    const float2 ustep = cmul(twhi[ju >> 10], twlo[ju & 1023]);  // W_N^{32 k1}
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        float2 v[16];
        if (r) {
            // cos(2 pi j / 32), j = 0..8
            constexpr float C32[9] = {1.0f, 0.98078528040323044913f, 0.92387953251128675613f,
                                      0.83146961230254523708f, 0.70710678118654752440f, 0.55557023301960222474f,
                                      0.38268343236508977173f, 0.19509032201612826785f, 0.0f};
            v[0] = x[0];
            v[8] = float2{-x[8].y, x[8].x};  // x W_32^8 = i x
#pragma unroll
            for (int j = 1; j < 16; ++j) {
                if (j == 8) continue;
                const float cj = j <= 8 ? C32[j] : -C32[16 - j];
                const float sj = j <= 8 ? C32[8 - j] : C32[j - 8];
                v[j] = cmul(x[j], float2{cj, sj});
            }
        } else {
#pragma unroll
            for (int j = 0; j < 16; ++j) v[j] = x[j];
        }
        dft16<1>(v);  // v[a] = sum_j x[l + 16 j] W_32^{r j} W_16^{j a}
        if (r) {
            float2 wa = w512l;  // W_512^l W_256^{l a}
#pragma unroll
            for (int a = 0; a < 16; ++a) {
                v[a] = cmul(v[a], wa);
                wa = cmul(wa, w256l);
            }
        } else {
            float2 wa = w256l;  // W_256^{l a}
#pragma unroll
            for (int a = 1; a < 16; ++a) {
                v[a] = cmul(v[a], wa);
                wa = cmul(wa, w256l);
            }
        }
        if (r) __syncthreads();
#pragma unroll
        for (int a = 0; a < 16; ++a) lds[l * LSTRIDE + a * COLS + c] = v[a];
        __syncthreads();
        const int a = l;
        float2 w[16];
#pragma unroll
        for (int l2 = 0; l2 < 16; ++l2) w[l2] = lds[l2 * LSTRIDE + a * COLS + c];
        dft16<1>(w);  // w[b] = 256-point output a + 16 b
        const int j0 = k1 * (2 * a + r);  // < N
        float2 tw = cmul(twhi[j0 >> 10], twlo[j0 & 1023]);
#pragma unroll
        for (int b = 0; b < 16; ++b) {
            const int m2 = 2 * (a + 16 * b) + r;
            Yt[(size_t)m2 * N1 + k1] = cmul(w[b], tw);
            tw = cmul(tw, ustep);
        }
    }
}

// Radix schedule of pass B: first radix 16, then R2 and R3 (1 = absent).
template <int N1> struct PassBPlan;
template <> struct PassBPlan<16> { static constexpr int R2 = 1, R3 = 1; };
template <> struct PassBPlan<32> { static constexpr int R2 = 2, R3 = 1; };
template <> struct PassBPlan<64> { static constexpr int R2 = 4, R3 = 1; };
template <> struct PassBPlan<128> { static constexpr int R2 = 8, R3 = 1; };
template <> struct PassBPlan<256> { static constexpr int R2 = 16, R3 = 1; };
template <> struct PassBPlan<512> { static constexpr int R2 = 16, R3 = 2; };
template <> struct PassBPlan<1024> { static constexpr int R2 = 16, R3 = 4; };
template <> struct PassBPlan<2048> { static constexpr int R2 = 16, R3 = 8; };

// Output index of register e after a pass with radix R at sub-transform size Ns.
template <int LPR, int R, int Ns>
__host__ __device__ constexpr int pass_out_index(int ln, int e) {
    const int b = e / R, r = e % R;
    const int j = ln + LPR * b;
    return (j / Ns) * Ns * R + (j % Ns) + r * Ns;
}

// Placement of row element i in LDS.  The first pass writes 16 consecutive elements per lane
// (a 128-byte lane stride), which unmapped puts the lanes of a wavefront on the same banks.
// Measured on gfx950 (SQ_LDS_BANK_CONFLICT of single-pattern probes): an 8-byte read is served
// 32 lanes at a time and is conflict-free when those lanes hit distinct (element mod 32)
// slots; an 8-byte write is served 16 consecutive lanes at a time and is conflict-free when
// they hit distinct (element mod 16) slots.  Rows of >= 512 elements XOR bits 4-7 of the
// index into bits 0-3 (no padding): the first pass's 16 lanes then write 16 distinct slots,
// and every other access still reads or writes whole 16-element blocks.  Shorter rows take
// one pad element per 16.  Both were checked conflict-free for every pass of every plan and
// tile with a model of those rules.
template <int N1> __host__ __device__ constexpr int lds_map(int i) {
    if constexpr (N1 >= 512) return i ^ ((i >> 4) & 15);
    else return i + (i >> 4);
}
template <int N1> constexpr int lds_row_len() { return N1 >= 512 ? N1 : N1 + N1 / 16; }

// Every row index a pass touches is a lane part and a register part in disjoint bits (the lane
// number below LPR, the register's offsets above it), and lds_map is linear in such a split: an
// XOR map for rows of >= 512 elements, i + i/16 on disjoint bits otherwise.  So the byte address
// is one per-lane value combined with a compile-time constant per register -- one XOR, or an
// add that folds into the instruction's offset -- instead of the whole swizzle per access.
template <int N1> __device__ __forceinline__ uint32_t lds_combine(uint32_t lane_b, uint32_t reg_b) {
    if constexpr (N1 >= 512) return lane_b ^ reg_b;  // the row offset lies above the in-row bits
    else return lane_b + reg_b;
}

template <int N1, int LPR, int R, int Ns>
__device__ __forceinline__ void lds_write_pass(char *lds_b, uint32_t row_b, const float2 *v, int ln) {
    const uint32_t lane_b = row_b + 8u * (uint32_t)lds_map<N1>(pass_out_index<LPR, R, Ns>(ln, 0));
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const uint32_t reg_b = 8u * (uint32_t)lds_map<N1>(pass_out_index<LPR, R, Ns>(0, e));
        *reinterpret_cast<float2 *>(lds_b + lds_combine<N1>(lane_b, reg_b)) = v[e];
    }
}

// Reads the inputs of a radix-R pass at sub-transform size Ns from LDS: butterfly j = ln + LPR b
// takes row[j + r N1/R], multiplied by W_N1^{k r S} (S = N1 / (Ns R), k = j mod Ns), and runs the
// radix-R DFT.  The twiddles are the powers of one preloaded base per b, base[b] = W_N1^{k S},
// formed by at most R - 2 products: no table load waits behind the LDS barrier.
template <int N1, int LPR, int R, int Ns>
__device__ __forceinline__ void lds_read_pass_pow(float2 *v, const char *lds_b, uint32_t row_b, int ln,
                                                  const float2 *base) {
    const uint32_t lane_b = row_b + 8u * (uint32_t)lds_map<N1>(ln);
#pragma unroll
    for (int b = 0; b < 16 / R; ++b) {
        float2 w = base[b];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint32_t reg_b = 8u * (uint32_t)lds_map<N1>(LPR * b + r * (N1 / R));
            float2 x = *reinterpret_cast<const float2 *>(lds_b + lds_combine<N1>(lane_b, reg_b));
            if (r == 1) x = cmul(x, w);
            if (r > 1) {
                w = cmul(w, base[b]);
                x = cmul(x, w);
            }
            v[b * R + r] = x;
        }
        dft<R, 1>(v + b * R);
    }
}

// Table entries W_N1^{k S}, k = (ln + LPR b) mod Ns, S = N1 / (Ns R), for every b of a pass.
template <int N1, int LPR, int R, int Ns>
__device__ __forceinline__ void pass_bases(float2 *base, int ln, const float2 *tw) {
#pragma unroll
    for (int b = 0; b < 16 / R; ++b) base[b] = tw[((ln + LPR * b) % Ns) * (N1 / (Ns * R))];
}

template <int N1, int PBT, bool WRITE_Z>
__global__ __launch_bounds__(PBT) void mf_pass_b(const float2 *__restrict__ Y, const MfItem *__restrict__ items,
                                                 int32_t id0, float thr2, const float2 *__restrict__ twN1,
                                                 hs_candidate *__restrict__ cand,
                                                 unsigned long long *__restrict__ counter, int64_t cap,
                                                 int64_t spill_cap, float2 *__restrict__ zout) {
    constexpr int LPR = N1 / 16;    // lanes per row
    static_assert(PBT % LPR == 0 && PBT >= LPR && PBT <= 256, "pass-B tile: whole rows, at most 256 threads");
    constexpr int RPB = PBT / LPR;  // rows per block
    constexpr int R2 = PassBPlan<N1>::R2, R3 = PassBPlan<N1>::R3;
    constexpr int ROW = lds_row_len<N1>();
    constexpr int LDS_N = N1 > 16 ? RPB * ROW : 1024;
    __shared__ float2 lds[LDS_N];
    __shared__ unsigned int s_count;
    __shared__ unsigned long long s_base, s_spill;
    if (threadIdx.x == 0) s_count = 0;
    const int tb = blockIdx.y;
    const int lr = threadIdx.x / LPR;
    const int ln = threadIdx.x % LPR;
    const int m2 = blockIdx.x * RPB + lr;
    const float2 *src = Y + ((size_t)tb * 512 + m2) * (size_t)N1;

    const float sc = items[id0 + tb].sc;
    float2 v[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) v[r] = src[ln + r * LPR];
    float2 base2[R2 > 1 ? 16 / R2 : 1], base3[R3 > 1 ? 16 / R3 : 1];
    if constexpr (R2 > 1) pass_bases<N1, LPR, R2, 16>(base2, ln, twN1);
    if constexpr (R3 > 1) pass_bases<N1, LPR, R3, 16 * R2>(base3, ln, twN1);
    dft16<1>(v);
    char *lds_b = reinterpret_cast<char *>(lds);
    const uint32_t row_b = 8u * (uint32_t)(N1 > 16 ? lr * ROW : 0);
    if constexpr (R2 > 1) {
        lds_write_pass<N1, LPR, 16, 1>(lds_b, row_b, v, ln);
        __syncthreads();
        lds_read_pass_pow<N1, LPR, R2, 16>(v, lds_b, row_b, ln, base2);
    }
    if constexpr (R3 > 1) {
        __syncthreads();
        lds_write_pass<N1, LPR, R2, 16>(lds_b, row_b, v, ln);
        __syncthreads();
        lds_read_pass_pow<N1, LPR, R3, 16 * R2>(v, lds_b, row_b, ln, base3);
    }
    constexpr int RL = R3 > 1 ? R3 : (R2 > 1 ? R2 : 16);
    constexpr int NsL = R3 > 1 ? 16 * R2 : (R2 > 1 ? 16 : 1);

    if constexpr (WRITE_Z) {
        const float zs = sqrtf(sc);
        float2 *zt = zout + (size_t)(id0 + tb) * 512 * (size_t)N1;
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const int m1 = pass_out_index<LPR, RL, NsL>(ln, e);
            zt[m2 + 512 * m1] = float2{v[e].x * zs, v[e].y * zs};
        }
    } else {
        // Candidates are staged in LDS (the transform buffer, free after the last pass): each
        // wavefront reserves slots with one LDS atomic per ballot, then the workgroup reserves
        // its block of one of MF_STRIPES candidate lists with a single atomic and writes it out
        // contiguously (striping keeps same-address atomics from serialising across the GPU;
        // the lists are concatenated after the last batch; records past a list's capacity go to
        // the shared spill list).  Slots beyond the staging capacity (only near very loud
        // signals) go straight to the lists, one atomic per lane.
        constexpr int STAGE = LDS_N / 2;  // hs_candidate = 2 float2
        hs_candidate *stage = reinterpret_cast<hs_candidate *>(lds);
        const int stripe = (int)((blockIdx.y * gridDim.x + blockIdx.x) & (MF_STRIPES - 1));
        const int lane = __lane_id();
        const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
        __syncthreads();
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const float2 z = v[e];
            const float r2 = (z.x * z.x + z.y * z.y) * sc;
            const bool p = r2 >= thr2;
            const unsigned long long mask = __ballot(p);
            if (mask) {
                const int leader = __ffsll((long long)mask) - 1;
                unsigned int b0 = 0;
                if (lane == leader) b0 = atomicAdd(&s_count, (unsigned int)__popcll(mask));
                b0 = __shfl(b0, leader);
                if (p) {
                    const unsigned int slot = b0 + (unsigned int)__popcll(mask & below);
                    const int m1 = pass_out_index<LPR, RL, NsL>(ln, e);
                    hs_candidate o;
                    o.tpos = id0 + tb;
                    o.m = m2 + 512 * m1;
                    o.rho2 = r2;
                    o.phase = atan2f(z.y, z.x);
                    if (slot < (unsigned int)STAGE) {
                        stage[slot] = o;
                    } else {
                        const unsigned long long idx = atomicAdd(&counter[stripe], 1ull);
                        mf_store_one(cand, counter, stripe, cap, spill_cap, idx, o);
                    }
                }
            }
        }
        __syncthreads();
        const unsigned int k = s_count < (unsigned int)STAGE ? s_count : (unsigned int)STAGE;
        if (threadIdx.x == 0) {
            const unsigned long long b = k ? atomicAdd(&counter[stripe], (unsigned long long)k) : 0ull;
            // records with reservation index >= cap spill; reserve them in one step
            const unsigned long long first_over = b > (unsigned long long)cap ? b : (unsigned long long)cap;
            const unsigned long long over = (b + k > (unsigned long long)cap) ? b + k - first_over : 0ull;
            s_base = b;
            s_spill = over ? atomicAdd(&counter[MF_STRIPES], over) : 0ull;
        }
        __syncthreads();
        const unsigned long long first_over = s_base > (unsigned long long)cap ? s_base : (unsigned long long)cap;
        for (unsigned int i = threadIdx.x; i < k; i += PBT) {
            const unsigned long long idx = s_base + i;
            if (idx < (unsigned long long)cap) {
                cand[(size_t)stripe * cap + idx] = stage[i];
            } else {
                const unsigned long long j = s_spill + (idx - first_over);
                if (j < (unsigned long long)spill_cap) cand[(size_t)MF_STRIPES * cap + j] = stage[i];
            }
        }
    }
}

// Pass-B threads per workgroup for rows of N1 points: the context's tile, widened to one row.
static int pass_b_threads(const hs_ctx *ctx, int N1) {
    const int t = ctx->mf_pb_threads;
    return t < N1 / 16 ? N1 / 16 : t;
}

template <int N1, bool WRITE_Z>
static void launch_pass_b_n(hs_ctx *ctx, int pbt, int tb, const float2 *Y, const MfItem *items, int32_t id0,
                            float thr2, const float2 *twN1, hs_candidate *cand, unsigned long long *counter,
                            int64_t cap, int64_t spill_cap, float2 *zout) {
    constexpr int LPR = N1 / 16;
    const dim3 grid((unsigned)(512 * LPR / pbt), (unsigned)tb);  // 512 rows / rows per workgroup
    if constexpr (LPR <= 64)
        if (pbt == 64) {
            hipLaunchKernelGGL((mf_pass_b<N1, 64, WRITE_Z>), grid, dim3(64), 0, ctx->stream, Y, items, id0, thr2,
                               twN1, cand, counter, cap, spill_cap, zout);
            return;
        }
    if constexpr (LPR <= 128)
        if (pbt == 128) {
            hipLaunchKernelGGL((mf_pass_b<N1, 128, WRITE_Z>), grid, dim3(128), 0, ctx->stream, Y, items, id0, thr2,
                               twN1, cand, counter, cap, spill_cap, zout);
            return;
        }
    hipLaunchKernelGGL((mf_pass_b<N1, 256, WRITE_Z>), grid, dim3(256), 0, ctx->stream, Y, items, id0, thr2, twN1,
                       cand, counter, cap, spill_cap, zout);
}

template <bool WRITE_Z>
static int launch_pass_b(hs_ctx *ctx, int N1, int tb, const float2 *Y, const MfItem *items, int32_t id0, float thr2,
                         const float2 *twN1, hs_candidate *cand, unsigned long long *counter, int64_t cap,
                         int64_t spill_cap, float2 *zout) {
    const int pbt = pass_b_threads(ctx, N1);
#define HS_PB(NN)                                                                                          \
    case NN:                                                                                               \
        launch_pass_b_n<NN, WRITE_Z>(ctx, pbt, tb, Y, items, id0, thr2, twN1, cand, counter, cap, spill_cap, \
                                     zout);                                                                \
        break;
    switch (N1) {
        HS_PB(16) HS_PB(32) HS_PB(64) HS_PB(128) HS_PB(256) HS_PB(512) HS_PB(1024) HS_PB(2048)
    default: return set_error(HS_EINVAL, "matched filter: unsupported N1 %d", N1);
    }
#undef HS_PB
    HS_HIP(hipGetLastError());
    return HS_OK;
}

template <int COLS>
static int launch_pass_a(hs_ctx *ctx, const hs_bank *bank, const float2 *d, const MfItem *items, int32_t id0,
                         int32_t tb, int N1, const float2 *tw512, const float2 *twlo, const float2 *twhi, float2 *Y) {
    const dim3 ga((unsigned)(N1 / COLS), (unsigned)tb), gt(16 * COLS);
    switch (bank->dtype) {
    case HS_F32:
        hipLaunchKernelGGL((mf_pass_a<StoreF32, COLS>), ga, gt, 0, ctx->stream, d,
                           static_cast<const float2 *>(bank->spectra), items, id0, N1, tw512, twlo, twhi, Y);
        break;
    case HS_BF16:
        hipLaunchKernelGGL((mf_pass_a<StoreBF16, COLS>), ga, gt, 0, ctx->stream, d,
                           static_cast<const uint32_t *>(bank->spectra), items, id0, N1, tw512, twlo, twhi, Y);
        break;
    default:
        hipLaunchKernelGGL((mf_pass_a<StoreF16, COLS>), ga, gt, 0, ctx->stream, d,
                           static_cast<const uint32_t *>(bank->spectra), items, id0, N1, tw512, twlo, twhi, Y);
        break;
    }
    HS_HIP(hipGetLastError());
    return HS_OK;
}

// ---------------------------------------------------------------------------------------------
// Fixed scratch of hs_matched_filter_noalloc.  Each device holds its own copy of this array for
// the life of the process; host code reaches it only through the address hipGetSymbolAddress
// returns for that device (the array's name is a host-side stand-in, not a device address).
// Every allocation-free call on a device shares it, so such calls on one device must not overlap.
// ---------------------------------------------------------------------------------------------
static constexpr size_t MF_NOALLOC_BYTES = size_t(64) << 20;
static_assert(MF_NOALLOC_BYTES == (size_t)HS_MF_NOALLOC_SCRATCH_BYTES, "header and library disagree");
static __device__ __align__(256) char scratch[MF_NOALLOC_BYTES];
static constexpr int MF_MAX_DEVICES = 64;
static char *g_scratch_dev[MF_MAX_DEVICES];
static std::mutex g_scratch_mu;

// Looks up this device's copy of the fixed scratch, once per device; `device` must be current.
int mf_noalloc_setup(int device) {
    if (device < 0 || device >= MF_MAX_DEVICES) return HS_OK;  // the allocation-free call then reports it
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_dev[device]) return HS_OK;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr)
        return set_error(HS_EDEVICE, "fixed matched-filter scratch: hipGetSymbolAddress failed on device %d: %s",
                         device, hipGetErrorString(e));
    g_scratch_dev[device] = static_cast<char *>(p);
    return HS_OK;
}

static char *noalloc_scratch(int device) {
    if (device < 0 || device >= MF_MAX_DEVICES) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return g_scratch_dev[device];
}

// The four twiddle tables the passes read, written into the fixed scratch (the arena path takes
// them from the context's tables): table t holds exp(+2 pi i j / 2^lg[t]) for j < count[t],
// from a float64 sincospi of the exact dyadic argument 2 j / 2^lg, rounded once to float32.
struct MfTwSpec {
    int32_t off[4], count[4], lg[4];
};

__global__ __launch_bounds__(256) void mf_twiddle_fill(float2 *__restrict__ out, MfTwSpec sp) {
    const int t = blockIdx.y;
    for (int j = blockIdx.x * 256 + threadIdx.x; j < sp.count[t]; j += gridDim.x * 256) {
        double s, c;
        sincospi(2.0 * (double)j / (double)(int64_t(1) << sp.lg[t]), &s, &c);
        out[sp.off[t] + j] = float2{(float)c, (float)s};
    }
}

// Carves 256-byte aligned pieces out of the fixed scratch, in order.
struct FixedCarver {
    char *base;
    size_t used = 0;
    template <typename T>
    void add(T **p, size_t count) {
        *p = reinterpret_cast<T *>(base + used);
        used += (count * sizeof(T) + 255) & ~size_t(255);
    }
};

template <bool WRITE_Z>
static int run_mf(hs_ctx *ctx, const void *spec, int64_t n, double fs, const hs_bank *bank, const int32_t *ids,
                  int32_t n_ids, float thr, hs_candidate *cand, int64_t cap, int64_t *n_cand, float2 *zout,
                  char *fixed = nullptr) {
    HS_REQUIRE(ctx && spec && bank && (ids || n_ids == 0), "matched filter: null argument");
    HS_REQUIRE(is_pow2(n) && n >= 8192 && n <= (int64_t(1) << 20),
               "matched filter: n must be a power of two in [2^13, 2^20] (got %lld)", (long long)n);
    HS_REQUIRE(bank->n == n, "matched filter: bank prepared for n=%lld, called with n=%lld", (long long)bank->n,
               (long long)n);
    HS_REQUIRE(bank->fs == fs, "matched filter: bank prepared for fs=%g, called with fs=%g", bank->fs, fs);
    HS_REQUIRE(bank->offset && bank->k0 && bank->k_lo && bank->k_hi && bank->spectra && bank->rho2_scale,
               "matched filter: bank has a null pointer");
    HS_REQUIRE(bank->dtype == HS_F32 || bank->dtype == HS_BF16 || bank->dtype == HS_F16,
               "matched filter: bad bank dtype");
    HS_REQUIRE(n_ids >= 0, "matched filter: negative n_ids");
    if (!WRITE_Z) HS_REQUIRE(cand && n_cand && cap >= 0, "matched filter: bad candidate output");
    else HS_REQUIRE(zout != nullptr, "snr series: null output");
    HS_HIP(hipSetDevice(ctx->device));
    if (!WRITE_Z) *n_cand = 0;
    if (n_ids == 0) return HS_OK;

    const int log2N = ilog2(n);
    const int N1 = (int)(n / 512);
    const int pa_cols = ctx->mf_pa_cols < N1 ? ctx->mf_pa_cols : N1;  // 16, 32 or 64 (N1 >= 16)
    const size_t per_tmpl = (size_t)n * sizeof(float2);
    int64_t tb_max = (int64_t)(ctx->mf_batch_bytes / per_tmpl);
    if (tb_max < 1) tb_max = 1;
    if (tb_max > 65535) tb_max = 65535;
    if (tb_max > n_ids) tb_max = n_ids;

    // Striped candidate lists: MF_STRIPES lists sharing the caller's capacity equally plus a spill
    // list as large as the whole capacity, so every distribution of up to `cap` candidates fits.
    const int64_t stripe_cap = WRITE_Z ? 0 : cap / MF_STRIPES;
    const int64_t spill_cap = WRITE_Z ? 0 : cap;
    const float2 *tw512, *twlo, *twhi, *twN1;
    float2 *Y;
    unsigned long long *counter;
    hs_candidate *sbuf;
    int32_t *bad;
    MfItem *items;
    if (!fixed) {
        HS_TRY(twiddles_f32(ctx, 9, &tw512));
        HS_TRY(twiddles_f32(ctx, log2N, &twlo));
        HS_TRY(twiddles_f32(ctx, log2N - 10, &twhi));
        HS_TRY(twiddles_f32(ctx, ilog2(N1), &twN1));
        Carver cv;
        cv.add(&Y, (size_t)tb_max * n);
        cv.add(&counter, MF_STRIPES + 1);
        cv.add(&sbuf, (size_t)MF_STRIPES * stripe_cap + spill_cap + 1);
        cv.add(&bad, 1);
        cv.add(&items, (size_t)n_ids);
        HS_TRY(cv.commit(ctx));
    } else {
        // pass A reads entries j < 1024 of the length-n table and all n/1024 of the coarse one
        MfTwSpec sp;
        const int cnt[4] = {512, 1024, (int)(n >> 10), N1}, lg[4] = {9, log2N, log2N - 10, ilog2(N1)};
        int off = 0;
        for (int t = 0; t < 4; ++t) {
            sp.off[t] = off;
            sp.count[t] = cnt[t];
            sp.lg[t] = lg[t];
            off += cnt[t];
        }
        HS_REQUIRE(cap <= (int64_t)(MF_NOALLOC_BYTES / sizeof(hs_candidate)) &&
                       n_ids <= (int32_t)(MF_NOALLOC_BYTES / sizeof(MfItem)),
                   "hs_matched_filter_noalloc: capacity %lld or %d templates exceed the fixed scratch (%zu bytes)",
                   (long long)cap, (int)n_ids, MF_NOALLOC_BYTES);
        FixedCarver fc{fixed};
        float2 *tw;
        fc.add(&tw, (size_t)off);
        fc.add(&counter, MF_STRIPES + 1);
        fc.add(&sbuf, (size_t)MF_STRIPES * stripe_cap + spill_cap + 1);
        fc.add(&bad, 1);
        fc.add(&items, (size_t)n_ids);
        const size_t one = (per_tmpl + 255) & ~size_t(255);
        HS_REQUIRE(fc.used + one <= MF_NOALLOC_BYTES,
                   "hs_matched_filter_noalloc: n=%lld, %d templates and capacity %lld need %zu bytes of scratch "
                   "(with one template's %zu-byte intermediate); the fixed scratch holds %zu",
                   (long long)n, (int)n_ids, (long long)cap, fc.used + one, per_tmpl, MF_NOALLOC_BYTES);
        const int64_t room = (int64_t)((MF_NOALLOC_BYTES - fc.used) / per_tmpl);
        if (tb_max > room) tb_max = room;
        fc.add(&Y, (size_t)tb_max * n);
        hipLaunchKernelGGL(mf_twiddle_fill, dim3(4, 4), dim3(256), 0, ctx->stream, tw, sp);
        HS_HIP(hipGetLastError());
        tw512 = tw + sp.off[0];
        twlo = tw + sp.off[1];
        twhi = tw + sp.off[2];
        twN1 = tw + sp.off[3];
    }
    HS_TRY(fill_u64(ctx, reinterpret_cast<uint64_t *>(counter), MF_STRIPES + 1, 0));
    HS_TRY(fill_u32(ctx, reinterpret_cast<uint32_t *>(bad), 1, 0));
    hipLaunchKernelGGL(mf_items, dim3((unsigned)cdiv(n_ids, 256)), dim3(256), 0, ctx->stream, ids, n_ids,
                       bank->n_tmpl, bank->offset, bank->k0, bank->k_lo, bank->k_hi, bank->rho2_scale, n / 2, items,
                       bad);
    HS_HIP(hipGetLastError());

    const float thr2 = thr * thr;
    for (int64_t id0 = 0; id0 < n_ids; id0 += tb_max) {
        const int32_t tb = (int32_t)((n_ids - id0) < tb_max ? (n_ids - id0) : tb_max);
        const float2 *d = static_cast<const float2 *>(spec);
        if (pa_cols == 64) HS_TRY((launch_pass_a<64>(ctx, bank, d, items, (int32_t)id0, tb, N1, tw512, twlo, twhi, Y)));
        else if (pa_cols == 32) HS_TRY((launch_pass_a<32>(ctx, bank, d, items, (int32_t)id0, tb, N1, tw512, twlo, twhi, Y)));
        else HS_TRY((launch_pass_a<16>(ctx, bank, d, items, (int32_t)id0, tb, N1, tw512, twlo, twhi, Y)));
        HS_TRY(launch_pass_b<WRITE_Z>(ctx, N1, tb, Y, items, (int32_t)id0, thr2, twN1, sbuf, counter, stripe_cap,
                                      spill_cap, zout));
    }
    if (!WRITE_Z && cap > 0) {
        hipLaunchKernelGGL(mf_compact, dim3(16, MF_STRIPES + 1), dim3(256), 0, ctx->stream, sbuf, counter,
                           stripe_cap, spill_cap, cand, cap);
        HS_HIP(hipGetLastError());
    }
    unsigned long long hc[MF_STRIPES + 1];
    int32_t hbad = 0;
    if (!fixed) {
        HS_TRY(read_back2(ctx, counter, hc, sizeof(hc), bad, &hbad, sizeof(hbad)));
    } else {  // no pinned staging (it is allocated on first use): copy straight to the host values
        HS_HIP(hipMemcpyAsync(hc, counter, sizeof(hc), hipMemcpyDeviceToHost, ctx->stream));
        HS_HIP(hipMemcpyAsync(&hbad, bad, sizeof(hbad), hipMemcpyDeviceToHost, ctx->stream));
        HS_HIP(hipStreamSynchronize(ctx->stream));
    }
    HS_REQUIRE(hbad == 0, "matched filter: template id out of range or bank band outside [1, n/2-1] (code %d)",
               hbad);
    if (!WRITE_Z) {
        unsigned long long total = 0;
        for (int s = 0; s < MF_STRIPES; ++s) total += hc[s];
        *n_cand = (int64_t)total;
        if ((int64_t)total > cap)
            return set_error(HS_EOVERFLOW, "matched filter: %llu candidates exceed capacity %lld", total,
                             (long long)cap);
    }
    return HS_OK;
}

}  // namespace hs

using namespace hs;

extern "C" int hs_matched_filter(hs_ctx *ctx, const void *spec, int64_t n, double fs, const hs_bank *bank,
                                 const int32_t *tmpl_ids, int32_t n_ids, float thr, hs_candidate *cand, int64_t cap,
                                 int64_t *n_cand) {
    return run_mf<false>(ctx, spec, n, fs, bank, tmpl_ids, n_ids, thr, cand, cap, n_cand, nullptr);
}

extern "C" int hs_matched_filter_noalloc(hs_ctx *ctx, const void *spec, int64_t n, double fs,
                                         const hs_bank *bank, const int32_t *tmpl_ids, int32_t n_ids, float thr,
                                         hs_candidate *cand, int64_t cap, int64_t *n_cand) {
    HS_REQUIRE(ctx, "hs_matched_filter_noalloc: null context");
    char *fixed = noalloc_scratch(ctx->device);
    HS_REQUIRE(fixed, "hs_matched_filter_noalloc: no fixed scratch on device %d (set up by hs_create; "
               "devices 0..%d)", ctx->device, MF_MAX_DEVICES - 1);
    return run_mf<false>(ctx, spec, n, fs, bank, tmpl_ids, n_ids, thr, cand, cap, n_cand, nullptr, fixed);
}

extern "C" int hs_snr_series(hs_ctx *ctx, const void *spec, int64_t n, double fs, const hs_bank *bank,
                             const int32_t *tmpl_ids, int32_t n_ids, void *z_out) {
    return run_mf<true>(ctx, spec, n, fs, bank, tmpl_ids, n_ids, 0.0f, nullptr, 0, nullptr,
                        static_cast<float2 *>(z_out));
}
