// Internal declarations shared by the libhs translation units (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <map>
#include <string>
#include <vector>

#include "../../include/hs.h"

namespace hs {

// ---------------------------------------------------------------------------------------------
// Errors: a thread-local message plus a status code; nothing is thrown across the ABI.
// ---------------------------------------------------------------------------------------------
int set_error(int status, const char *fmt, ...);

#define HS_HIP(expr)                                                                          \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return ::hs::set_error(HS_EDEVICE, "%s failed: %s (%s:%d)", #expr,                \
                                   hipGetErrorString(e_), __FILE__, __LINE__);                \
    } while (0)

#define HS_REQUIRE(cond, ...)                                                                 \
    do {                                                                                      \
        if (!(cond)) return ::hs::set_error(HS_EINVAL, __VA_ARGS__);                          \
    } while (0)

#define HS_TRY(expr)                                                                          \
    do {                                                                                      \
        int s_ = (expr);                                                                      \
        if (s_ != HS_OK) return s_;                                                           \
    } while (0)

inline bool is_pow2(int64_t x) { return x > 0 && (x & (x - 1)) == 0; }
inline int ilog2(int64_t x) { int l = 0; while ((int64_t(1) << l) < x) ++l; return l; }
inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Twiddle table on the device: tab[j] = exp(+2 pi i j / len), j = 0..len-1.
struct Twiddles {
    void *f32 = nullptr;  // float2 [len]
    void *f64 = nullptr;  // double2 [len]
    double hann_sumsq = -1.0;  // sum of squared periodic Hann weights of length len (set on first use)
};

}  // namespace hs

// ---------------------------------------------------------------------------------------------
// Context
// ---------------------------------------------------------------------------------------------
struct hs_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    // Scratch arena (device), grown on demand; carved per call.
    char *arena = nullptr;
    size_t arena_bytes = 0;
    // Pinned host staging for small read-backs.
    char *pinned = nullptr;
    size_t pinned_bytes = 0;
    // Twiddle tables keyed by log2(length).
    std::map<int, hs::Twiddles> tw;
    // Matched-filter batch budget for the pass-A/pass-B intermediate (bytes).
    size_t mf_batch_bytes = size_t(128) << 20;
    int mf_pb_threads = 128;  // matched-filter pass-B workgroup size (64, 128 or 256)
    int mf_pa_cols = 64;      // matched-filter pass-A columns per workgroup (16, 32 or 64)
};

namespace hs {

// Looks up the current device's copy of the allocation-free matched filter's fixed scratch
// (once per device; called by hs_create with that device current).
int mf_noalloc_setup(int device);
// Ensure the arena holds at least `bytes`; synchronises the stream before growing.
int arena_reserve(hs_ctx *ctx, size_t bytes);
// Ensure the pinned host staging holds at least `bytes`.
int pinned_reserve(hs_ctx *ctx, size_t bytes);
// Device twiddle table exp(+2 pi i j / 2^log2len) in float32 or float64 (built on first use).
int twiddles_f32(hs_ctx *ctx, int log2len, const float2 **out);
int twiddles_f64(hs_ctx *ctx, int log2len, const double2 **out);
// Sum over j < 2^log2len of (0.5 - 0.5 cos(2 pi j / len))^2 from the same float64 cosines as the
// float64 twiddle table, computed once per length and kept in the context.
double hann_sumsq(hs_ctx *ctx, int log2len);

// Carves aligned sub-buffers out of the arena for one call.
struct Carver {
    size_t used = 0;
    std::vector<std::pair<void **, size_t>> reqs;
    template <typename T>
    void add(T **p, size_t count) {
        reqs.push_back({reinterpret_cast<void **>(p), count * sizeof(T)});
    }
    int commit(hs_ctx *ctx) {
        size_t total = 0;
        for (auto &r : reqs) total += (r.second + 255) & ~size_t(255);
        HS_TRY(arena_reserve(ctx, total));
        size_t off = 0;
        for (auto &r : reqs) {
            *r.first = ctx->arena + off;
            off += (r.second + 255) & ~size_t(255);
        }
        used = total;
        return HS_OK;
    }
};

// Exclusive prefix sum of `n` uint32 counts into uint64 offsets out[0..n] (out[n] = total).
// `tmp` must hold scan_tmp_elems(n) uint64 values.
size_t scan_tmp_elems(int64_t n);
int exclusive_scan_u32(hs_ctx *ctx, const uint32_t *in, int64_t n, uint64_t *out, uint64_t *tmp);
// Fill helpers (kernels, so they may be captured in a graph).
int fill_u32(hs_ctx *ctx, uint32_t *p, int64_t n, uint32_t v);
int fill_u64(hs_ctx *ctx, uint64_t *p, int64_t n, uint64_t v);
// Copy a small device value back to the host and synchronise.
int read_back(hs_ctx *ctx, const void *dev, void *host, size_t bytes);
// Two small device values back to the host with one synchronisation.
int read_back2(hs_ctx *ctx, const void *dev0, void *host0, size_t bytes0, const void *dev1, void *host1,
               size_t bytes1);

// Batched complex FFT of `batch` contiguous sequences of length 2^log2len, Stockham,
// in global memory.  sign = -1 forward, +1 inverse (unnormalised).  The result lands in
// either `a` or `b`; *result points to it.
int fft_c2c_f32(hs_ctx *ctx, float2 *a, float2 *b, int log2len, int64_t batch, int sign,
                float2 **result);
int fft_c2c_f64(hs_ctx *ctx, double2 *a, double2 *b, int log2len, int64_t batch, int sign,
                double2 **result);

}  // namespace hs
