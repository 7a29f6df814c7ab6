// Context lifetime, errors, scratch arena, twiddle tables, prefix sums, fills and the
// generic batched Stockham FFT used for the (once-per-segment) data transforms.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>

#include "dft.h"
#include "hs_internal.h"

namespace hs {

static thread_local char g_err[1024] = "";

int set_error(int status, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return status;
}

int arena_reserve(hs_ctx *ctx, size_t bytes) {
    if (bytes <= ctx->arena_bytes) return HS_OK;
    // Growth keeps the current contents (copied to the front of the new arena), so a call may
    // carve more buffers after earlier ones are filled, as long as it re-carves them in the
    // same order.
    size_t want = bytes + bytes / 4 + (size_t(1) << 20);
    char *fresh = nullptr;
    if (hipMalloc(reinterpret_cast<void **>(&fresh), want) != hipSuccess) {
        (void)hipGetLastError();
        return set_error(HS_ENOMEM, "scratch allocation of %zu bytes failed", want);
    }
    if (ctx->arena) {
        HS_HIP(hipMemcpyAsync(fresh, ctx->arena, ctx->arena_bytes, hipMemcpyDeviceToDevice, ctx->stream));
        HS_HIP(hipStreamSynchronize(ctx->stream));
        HS_HIP(hipFree(ctx->arena));
    }
    ctx->arena = fresh;
    ctx->arena_bytes = want;
    return HS_OK;
}

int pinned_reserve(hs_ctx *ctx, size_t bytes) {
    if (bytes <= ctx->pinned_bytes) return HS_OK;
    HS_HIP(hipStreamSynchronize(ctx->stream));
    if (ctx->pinned) HS_HIP(hipHostFree(ctx->pinned));
    ctx->pinned = nullptr;
    ctx->pinned_bytes = 0;
    size_t want = bytes < 4096 ? 4096 : bytes;
    if (hipHostMalloc(reinterpret_cast<void **>(&ctx->pinned), want, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        ctx->pinned = nullptr;
        return set_error(HS_ENOMEM, "pinned host allocation of %zu bytes failed", want);
    }
    ctx->pinned_bytes = want;
    return HS_OK;
}

int read_back(hs_ctx *ctx, const void *dev, void *host, size_t bytes) {
    HS_TRY(pinned_reserve(ctx, bytes));
    HS_HIP(hipMemcpyAsync(ctx->pinned, dev, bytes, hipMemcpyDeviceToHost, ctx->stream));
    HS_HIP(hipStreamSynchronize(ctx->stream));
    std::memcpy(host, ctx->pinned, bytes);
    return HS_OK;
}

int read_back2(hs_ctx *ctx, const void *dev0, void *host0, size_t bytes0, const void *dev1, void *host1,
               size_t bytes1) {
    const size_t o1 = (bytes0 + 15) & ~size_t(15);
    HS_TRY(pinned_reserve(ctx, o1 + bytes1));
    char *pin = static_cast<char *>(ctx->pinned);
    HS_HIP(hipMemcpyAsync(pin, dev0, bytes0, hipMemcpyDeviceToHost, ctx->stream));
    HS_HIP(hipMemcpyAsync(pin + o1, dev1, bytes1, hipMemcpyDeviceToHost, ctx->stream));
    HS_HIP(hipStreamSynchronize(ctx->stream));
    std::memcpy(host0, pin, bytes0);
    std::memcpy(host1, pin + o1, bytes1);
    return HS_OK;
}

// exp(+2 pi i j / len) evaluated in extended precision on the host and rounded once.
static void host_twiddles(int log2len, std::vector<long double> &re, std::vector<long double> &im) {
    const int64_t len = int64_t(1) << log2len;
    re.resize(len);
    im.resize(len);
    const long double two_pi = 6.283185307179586476925286766559005768L;
    for (int64_t j = 0; j < len; ++j) {
        long double a = two_pi * (long double)j / (long double)len;
        re[j] = cosl(a);
        im[j] = sinl(a);
    }
}

double hann_sumsq(hs_ctx *ctx, int log2len) {
    Twiddles &t = ctx->tw[log2len];
    if (t.hann_sumsq < 0.0) {
        std::vector<long double> re, im;
        host_twiddles(log2len, re, im);
        double acc = 0.0;
        for (size_t j = 0; j < re.size(); ++j) {
            const double w = 0.5 - 0.5 * (double)re[j];
            acc += w * w;
        }
        t.hann_sumsq = acc;
    }
    return t.hann_sumsq;
}

int twiddles_f32(hs_ctx *ctx, int log2len, const float2 **out) {
    Twiddles &t = ctx->tw[log2len];
    if (!t.f32) {
        std::vector<long double> re, im;
        host_twiddles(log2len, re, im);
        std::vector<float2> h(re.size());
        for (size_t j = 0; j < re.size(); ++j) h[j] = float2{(float)re[j], (float)im[j]};
        HS_HIP(hipMalloc(&t.f32, h.size() * sizeof(float2)));
        HS_HIP(hipMemcpy(t.f32, h.data(), h.size() * sizeof(float2), hipMemcpyHostToDevice));
    }
    *out = static_cast<const float2 *>(t.f32);
    return HS_OK;
}

int twiddles_f64(hs_ctx *ctx, int log2len, const double2 **out) {
    Twiddles &t = ctx->tw[log2len];
    if (!t.f64) {
        std::vector<long double> re, im;
        host_twiddles(log2len, re, im);
        std::vector<double2> h(re.size());
        for (size_t j = 0; j < re.size(); ++j) h[j] = double2{(double)re[j], (double)im[j]};
        HS_HIP(hipMalloc(&t.f64, h.size() * sizeof(double2)));
        HS_HIP(hipMemcpy(t.f64, h.data(), h.size() * sizeof(double2), hipMemcpyHostToDevice));
    }
    *out = static_cast<const double2 *>(t.f64);
    return HS_OK;
}

// ---------------------------------------------------------------------------------------------
// Fills
// ---------------------------------------------------------------------------------------------
template <typename T>
__global__ void fill_kernel(T *p, int64_t n, T v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

static unsigned grid_for(int64_t n, int threads) {
    int64_t g = cdiv(n, threads);
    if (g > 65536) g = 65536;
    if (g < 1) g = 1;
    return (unsigned)g;
}

int fill_u32(hs_ctx *ctx, uint32_t *p, int64_t n, uint32_t v) {
    if (n <= 0) return HS_OK;
    hipLaunchKernelGGL(fill_kernel<uint32_t>, dim3(grid_for(n, 256)), dim3(256), 0, ctx->stream, p, n, v);
    HS_HIP(hipGetLastError());
    return HS_OK;
}

int fill_u64(hs_ctx *ctx, uint64_t *p, int64_t n, uint64_t v) {
    if (n <= 0) return HS_OK;
    hipLaunchKernelGGL(fill_kernel<uint64_t>, dim3(grid_for(n, 256)), dim3(256), 0, ctx->stream, p, n, v);
    HS_HIP(hipGetLastError());
    return HS_OK;
}

// ---------------------------------------------------------------------------------------------
// Exclusive prefix sum (three phases: tile sums, scan of tile sums, tile scans + offsets).
// Tile = 1024 elements (256 threads x 4).
// ---------------------------------------------------------------------------------------------
static constexpr int SCAN_TILE = 1024;

__device__ __forceinline__ uint64_t block_excl_scan_256(uint64_t v, uint64_t *sh, uint64_t *total) {
    // Hillis-Steele over 256 threads in shared memory (deterministic).
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
        uint64_t add = t >= o ? sh[t - o] : 0;
        __syncthreads();
        sh[t] += add;
        __syncthreads();
    }
    uint64_t incl = sh[t];
    if (total) *total = sh[255];
    __syncthreads();
    return incl - v;
}

__global__ __launch_bounds__(256) void scan_tile_sums(const uint32_t *in, int64_t n, uint64_t *sums) {
    __shared__ uint64_t sh[256];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
    uint64_t s = 0;
    for (int e = 0; e < 4; ++e) {
        int64_t i = base + threadIdx.x * 4 + e;
        if (i < n) s += in[i];
    }
    uint64_t tot;
    block_excl_scan_256(s, sh, &tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

__global__ __launch_bounds__(256) void scan_sums_inplace(uint64_t *sums, int64_t nt, uint64_t *grand) {
    __shared__ uint64_t sh[256];
    uint64_t carry = 0;
    for (int64_t b0 = 0; b0 < nt; b0 += 256) {
        int64_t i = b0 + threadIdx.x;
        uint64_t v = i < nt ? sums[i] : 0;
        uint64_t tot;
        uint64_t ex = block_excl_scan_256(v, sh, &tot);
        if (i < nt) sums[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) *grand = carry;
}

__global__ __launch_bounds__(256) void scan_tiles_apply(const uint32_t *in, int64_t n, const uint64_t *sums,
                                                        uint64_t *out) {
    __shared__ uint64_t sh[256];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
    uint32_t v[4];
    uint64_t s = 0;
    for (int e = 0; e < 4; ++e) {
        int64_t i = base + threadIdx.x * 4 + e;
        v[e] = i < n ? in[i] : 0;
        s += v[e];
    }
    uint64_t ex = block_excl_scan_256(s, sh, nullptr) + sums[blockIdx.x];
    for (int e = 0; e < 4; ++e) {
        int64_t i = base + threadIdx.x * 4 + e;
        if (i < n) out[i] = ex;
        ex += v[e];
    }
}

size_t scan_tmp_elems(int64_t n) { return (size_t)cdiv(n > 0 ? n : 1, SCAN_TILE) + 1; }

int exclusive_scan_u32(hs_ctx *ctx, const uint32_t *in, int64_t n, uint64_t *out, uint64_t *tmp) {
    if (n <= 0) {
        hipLaunchKernelGGL(fill_kernel<uint64_t>, dim3(1), dim3(64), 0, ctx->stream, out, (int64_t)1,
                           (uint64_t)0);
        HS_HIP(hipGetLastError());
        return HS_OK;
    }
    const int64_t nt = cdiv(n, SCAN_TILE);
    HS_REQUIRE(nt < (int64_t(1) << 31), "scan of %lld elements too large", (long long)n);
    hipLaunchKernelGGL(scan_tile_sums, dim3((unsigned)nt), dim3(256), 0, ctx->stream, in, n, tmp);
    hipLaunchKernelGGL(scan_sums_inplace, dim3(1), dim3(256), 0, ctx->stream, tmp, nt, out + n);
    hipLaunchKernelGGL(scan_tiles_apply, dim3((unsigned)nt), dim3(256), 0, ctx->stream, in, n, tmp, out);
    HS_HIP(hipGetLastError());
    return HS_OK;
}

// ---------------------------------------------------------------------------------------------
// Batched Stockham FFT in global memory (radix 16 passes, one radix 2/4/8 remainder pass).
// Pass with radix R and current sub-transform size Ns: butterfly j (0..L/R-1) reads
// in[j + r L/R], multiplies by W_{Ns R}^{(j mod Ns) r}, does a radix-R DFT and writes
// out[(j / Ns) Ns R + j mod Ns + r Ns].  After all passes the output is in natural order.
// ---------------------------------------------------------------------------------------------
template <typename T, int R, int S>
__global__ __launch_bounds__(256) void stockham_pass(const T *__restrict__ in, T *__restrict__ out,
                                                     int log2len, int64_t Ns, int64_t batch,
                                                     const T *__restrict__ tw) {
    const int64_t L = int64_t(1) << log2len;
    const int64_t per = L / R;
    const int64_t gid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (gid >= per * batch) return;
    const int64_t b = gid / per;
    const int64_t j = gid - b * per;
    const T *src = in + b * L;
    T *dst = out + b * L;
    T v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = src[j + r * per];
    const int64_t k = j % Ns;
    if (Ns > 1) {
        const int64_t stride = L / (Ns * R);
#pragma unroll
        for (int r = 1; r < R; ++r) {
            T w = tw[k * r * stride];
            if (S < 0) w.y = -w.y;
            v[r] = cmul(v[r], w);
        }
    }
    dft<R, S>(v);
    const int64_t base = (j / Ns) * Ns * R + k;
#pragma unroll
    for (int r = 0; r < R; ++r) dst[base + r * Ns] = v[r];
}

template <typename T, int S>
static int run_pass(hs_ctx *ctx, int R, const T *in, T *out, int log2len, int64_t Ns, int64_t batch,
                    const T *tw) {
    const int64_t L = int64_t(1) << log2len;
    const int64_t work = (L / R) * batch;
    const unsigned grid = (unsigned)cdiv(work, 256);
    switch (R) {
    case 2: hipLaunchKernelGGL((stockham_pass<T, 2, S>), dim3(grid), dim3(256), 0, ctx->stream, in, out, log2len, Ns, batch, tw); break;
    case 4: hipLaunchKernelGGL((stockham_pass<T, 4, S>), dim3(grid), dim3(256), 0, ctx->stream, in, out, log2len, Ns, batch, tw); break;
    case 8: hipLaunchKernelGGL((stockham_pass<T, 8, S>), dim3(grid), dim3(256), 0, ctx->stream, in, out, log2len, Ns, batch, tw); break;
    default: hipLaunchKernelGGL((stockham_pass<T, 16, S>), dim3(grid), dim3(256), 0, ctx->stream, in, out, log2len, Ns, batch, tw); break;
    }
    HS_HIP(hipGetLastError());
    return HS_OK;
}

template <typename T, int S>
static int fft_run(hs_ctx *ctx, T *a, T *b, int log2len, int64_t batch, const T *tw, T **result) {
    T *src = a, *dst = b;
    int rem = log2len;
    int64_t Ns = 1;
    while (rem > 0) {
        int lr = rem >= 4 ? 4 : rem;
        HS_TRY((run_pass<T, S>(ctx, 1 << lr, src, dst, log2len, Ns, batch, tw)));
        Ns <<= lr;
        rem -= lr;
        T *t = src;
        src = dst;
        dst = t;
    }
    *result = src;
    return HS_OK;
}

int fft_c2c_f32(hs_ctx *ctx, float2 *a, float2 *b, int log2len, int64_t batch, int sign, float2 **result) {
    const float2 *tw;
    HS_TRY(twiddles_f32(ctx, log2len, &tw));
    if (sign < 0) return fft_run<float2, -1>(ctx, a, b, log2len, batch, tw, result);
    return fft_run<float2, 1>(ctx, a, b, log2len, batch, tw, result);
}

int fft_c2c_f64(hs_ctx *ctx, double2 *a, double2 *b, int log2len, int64_t batch, int sign, double2 **result) {
    const double2 *tw;
    HS_TRY(twiddles_f64(ctx, log2len, &tw));
    if (sign < 0) return fft_run<double2, -1>(ctx, a, b, log2len, batch, tw, result);
    return fft_run<double2, 1>(ctx, a, b, log2len, batch, tw, result);
}

}  // namespace hs

// ---------------------------------------------------------------------------------------------
// ABI: context
// ---------------------------------------------------------------------------------------------
extern "C" {

const char *hs_last_error(void) { return hs::g_err; }

int hs_abi_version(void) { return 10; }

int hs_set_mf_batch_bytes(hs_ctx *ctx, int64_t bytes) {
    HS_REQUIRE(ctx, "hs_set_mf_batch_bytes: null context");
    HS_REQUIRE(bytes >= (int64_t(1) << 20) && bytes <= (int64_t(1) << 36),
               "hs_set_mf_batch_bytes: %lld bytes outside [1 MiB, 64 GiB]", (long long)bytes);
    ctx->mf_batch_bytes = (size_t)bytes;
    return HS_OK;
}

int64_t hs_get_mf_batch_bytes(const hs_ctx *ctx) { return ctx ? (int64_t)ctx->mf_batch_bytes : 0; }

int hs_set_mf_tile(hs_ctx *ctx, int32_t pass_b_threads) {
    HS_REQUIRE(ctx, "hs_set_mf_tile: null context");
    HS_REQUIRE(pass_b_threads == 64 || pass_b_threads == 128 || pass_b_threads == 256,
               "hs_set_mf_tile: pass-B workgroup of %d threads (64, 128 or 256)", (int)pass_b_threads);
    ctx->mf_pb_threads = pass_b_threads;
    return HS_OK;
}

int32_t hs_get_mf_tile(const hs_ctx *ctx) { return ctx ? ctx->mf_pb_threads : 0; }

int hs_set_mf_pa_cols(hs_ctx *ctx, int32_t cols) {
    HS_REQUIRE(ctx, "hs_set_mf_pa_cols: null context");
    HS_REQUIRE(cols == 16 || cols == 32 || cols == 64, "hs_set_mf_pa_cols: %d columns (16, 32 or 64)", (int)cols);
    ctx->mf_pa_cols = cols;
    return HS_OK;
}

int32_t hs_get_mf_pa_cols(const hs_ctx *ctx) { return ctx ? ctx->mf_pa_cols : 0; }

int hs_create(hs_ctx **ctx, int device, void *hip_stream) {
    if (!ctx) return hs::set_error(HS_EINVAL, "hs_create: ctx is NULL");
    *ctx = nullptr;
    int n_dev = 0;
    HS_HIP(hipGetDeviceCount(&n_dev));
    HS_REQUIRE(device >= 0 && device < n_dev, "hs_create: device %d out of range (%d devices)", device, n_dev);
    HS_HIP(hipSetDevice(device));
    HS_TRY(hs::mf_noalloc_setup(device));
    hs_ctx *c = new (std::nothrow) hs_ctx();
    if (!c) return hs::set_error(HS_ENOMEM, "hs_create: out of host memory");
    c->device = device;
    c->stream = static_cast<hipStream_t>(hip_stream);
    if (const char *s = std::getenv("HS_MF_BATCH_MB")) {
        // a whole number of MiB in the range hs_set_mf_batch_bytes accepts; anything else is ignored
        char *end = nullptr;
        const long v = std::strtol(s, &end, 10);
        if (end != s && *end == 0 && v >= 1 && v <= (long(1) << 16)) c->mf_batch_bytes = size_t(v) << 20;
    }
    *ctx = c;
    hs::g_err[0] = 0;
    return HS_OK;
}

int hs_destroy(hs_ctx *ctx) {
    if (!ctx) return HS_OK;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    if (ctx->arena) (void)hipFree(ctx->arena);
    if (ctx->pinned) (void)hipHostFree(ctx->pinned);
    for (auto &kv : ctx->tw) {
        if (kv.second.f32) (void)hipFree(kv.second.f32);
        if (kv.second.f64) (void)hipFree(kv.second.f64);
    }
    delete ctx;
    return HS_OK;
}

}  // extern "C"
