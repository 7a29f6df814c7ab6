// Learned follow-up proposer: coincidence features, a 16-128-128-128-64 MLP (inference, one
// training step with backpropagation and Adam) and the top-probability cell selection.
//
// This is an addition on top of the stage-1 follow-up of Sec. III: the neighbourhood of a followed
// coarse template is split into 64 (relative chirp-mass, mass-ratio) cells and only the cells the
// MLP ranks as likely are re-filtered (hs_followup_cells applies the masks).  The features use the
// re-weighted SNRs and the per-bin chi-square terms of Eq. (4)'s test.
//
// The network is tiny (43,456 parameters; batches of at most a few thousand coincidences), so
// every layer is a plain FP32 VALU kernel: a workgroup stages 8 samples in LDS and each thread
// produces one output unit for all 8, reading its weight column (coalesced across the workgroup)
// from L2.  Every sum runs in a fixed order, so training is deterministic.  Matrix cores would
// not shorten the wall time of launches this small.
#include <cmath>

#include "hs_internal.h"

namespace hs {

static constexpr int MLP_F = HS_MLP_FEATURES;
static constexpr int MLP_H = 128;
static constexpr int MLP_C = HS_MLP_CELLS;
static constexpr int MLP_S = 8;     // samples per workgroup in the layer kernels
static constexpr int MLP_NORM = 2 * MLP_F;

// Offsets (floats) of the layers in the model vector; gradients use the same layout minus MLP_NORM.
static constexpr int64_t W1 = MLP_NORM, B1 = W1 + MLP_F * MLP_H;
static constexpr int64_t W2 = B1 + MLP_H, B2 = W2 + MLP_H * MLP_H;
static constexpr int64_t W3 = B2 + MLP_H, B3 = W3 + MLP_H * MLP_H;
static constexpr int64_t W4 = B3 + MLP_H, B4 = W4 + MLP_H * MLP_C;
static_assert(B4 + MLP_C == HS_MLP_MODEL, "model layout");
static_assert(HS_MLP_MODEL - MLP_NORM == HS_MLP_PARAMS, "parameter count");

// ---------------------------------------------------------------------------------------------
// Features
// ---------------------------------------------------------------------------------------------
__device__ __forceinline__ int64_t floor_div(int64_t a, int64_t b) {
    int64_t q = a / b;
    if ((a % b != 0) && ((a < 0) != (b < 0))) --q;
    return q;
}

// Index of the trigger with key (seg, tmpl, tick) in an array sorted by that key, or -1.
__device__ int64_t find_trigger(const hs_trigger *__restrict__ tr, int64_t n, int64_t seg, int32_t tmpl,
                                int64_t tick) {
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        const int64_t mid = lo + (hi - lo) / 2;
        const hs_trigger r = tr[mid];
        const bool less = (r.seg < seg) || (r.seg == seg && (r.tmpl < tmpl || (r.tmpl == tmpl && r.tick < tick)));
        if (less) lo = mid + 1;
        else hi = mid;
    }
    if (lo < n && tr[lo].seg == seg && tr[lo].tmpl == tmpl && tr[lo].tick == tick) return lo;
    return -1;
}

__global__ void features_kernel(const hs_coinc *__restrict__ c, int64_t n_c, const hs_trigger *__restrict__ th,
                                int64_t n_h, const float *__restrict__ chi_h, const float *__restrict__ bins_h,
                                const hs_trigger *__restrict__ tl, int64_t n_l, const float *__restrict__ chi_l,
                                const float *__restrict__ bins_l, int64_t seg_ticks,
                                const double *__restrict__ cmc, const double *__restrict__ cq, int32_t n_coarse,
                                int64_t step, int64_t wrap, int64_t tps, float *__restrict__ out,
                                int32_t *__restrict__ bad) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n_c) return;
    const hs_coinc x = c[i];
    float *f = out + i * MLP_F;
    if (x.tmpl < 0 || x.tmpl >= n_coarse) {
        atomicOr(bad, 1);
        for (int q = 0; q < MLP_F; ++q) f[q] = 0.0f;
        return;
    }
    const int64_t a = find_trigger(th, n_h, floor_div(x.tick_h, seg_ticks), x.tmpl, x.tick_h);
    const int64_t b = find_trigger(tl, n_l, floor_div(x.tick_l, seg_ticks), x.tmpl, x.tick_l);
    if (a < 0 || b < 0) {
        atomicOr(bad, 2);
        for (int q = 0; q < MLP_F; ++q) f[q] = 0.0f;
        return;
    }
    constexpr int P = 8;
    const double norm = 2.0 * (2.0 * P - 2.0) / P;
    f[0] = (float)(double)x.snr_h;
    f[1] = (float)(double)x.snr_l;
    f[2] = (float)(double)x.snr_c;
    f[3] = (float)(((double)chi_h[a] + (double)chi_l[b]) / 2.0);
#pragma unroll
    for (int l = 0; l < P; ++l) f[4 + l] = (float)(((double)bins_h[a * P + l] + (double)bins_l[b * P + l]) / norm);
    f[12] = (float)cmc[x.tmpl];
    f[13] = (float)cq[x.tmpl];
    int64_t d = x.tick_h - x.tick_l - (int64_t)x.slide * step;
    int64_t r = (d + wrap / 2) % wrap;
    if (r < 0) r += wrap;
    f[14] = (float)((double)(r - wrap / 2) / (double)tps);
    const double pi = 3.141592653589793;  // the float64 nearest pi
    double dp = remainder((double)th[a].phase - (double)tl[b].phase, 2.0 * pi);
    if (dp == -pi) dp = pi;
    f[15] = (float)dp;
}

// ---------------------------------------------------------------------------------------------
// MLP layers
// ---------------------------------------------------------------------------------------------
// out[s][j] = act(b[j] + sum_k in[s][k] W[k][j]); with NORM the input is (x - mu) * inv_std
// (and is stored to h0 when h0 != nullptr).
template <int K, int J, bool NORM, bool RELU>
__global__ __launch_bounds__(J) void mlp_fwd(const float *__restrict__ in, int64_t n, const float *__restrict__ norm,
                                             const float *__restrict__ W, const float *__restrict__ bias,
                                             float *__restrict__ h0, float *__restrict__ out) {
    __shared__ float xs[MLP_S][K];
    const int64_t s0 = (int64_t)blockIdx.x * MLP_S;
    for (int q = threadIdx.x; q < MLP_S * K; q += J) {
        const int s = q / K, k = q % K;
        const int64_t r = s0 + s;
        float v = 0.0f;
        if (r < n) {
            v = in[r * K + k];
            if constexpr (NORM) {
                v = (v - norm[k]) * norm[K + k];
                if (h0) h0[r * K + k] = v;
            }
        }
        xs[s][k] = v;
    }
    __syncthreads();
    const int j = threadIdx.x;
    float acc[MLP_S];
#pragma unroll
    for (int s = 0; s < MLP_S; ++s) acc[s] = bias[j];
    for (int k = 0; k < K; ++k) {
        const float w = W[k * J + j];
#pragma unroll
        for (int s = 0; s < MLP_S; ++s) acc[s] = fmaf(xs[s][k], w, acc[s]);
    }
#pragma unroll
    for (int s = 0; s < MLP_S; ++s)
        if (s0 + s < n) out[(s0 + s) * J + j] = RELU ? fmaxf(acc[s], 0.0f) : acc[s];
}

// dprev[s][k] = (sum_j dz[s][j] W[k][j]) if a[s][k] > 0 else 0   (a: the layer's ReLU input)
template <int K, int J>
__global__ __launch_bounds__(K) void mlp_bwd(const float *__restrict__ dz, int64_t n, const float *__restrict__ W,
                                             const float *__restrict__ a, float *__restrict__ dprev) {
    __shared__ float ds[MLP_S][J];
    const int64_t s0 = (int64_t)blockIdx.x * MLP_S;
    for (int q = threadIdx.x; q < MLP_S * J; q += K) {
        const int s = q / J, j = q % J;
        ds[s][j] = (s0 + s < n) ? dz[(s0 + s) * J + j] : 0.0f;
    }
    __syncthreads();
    const int k = threadIdx.x;
    float acc[MLP_S];
#pragma unroll
    for (int s = 0; s < MLP_S; ++s) acc[s] = 0.0f;
    for (int j = 0; j < J; ++j) {
        const float w = W[k * J + j];
#pragma unroll
        for (int s = 0; s < MLP_S; ++s) acc[s] = fmaf(ds[s][j], w, acc[s]);
    }
#pragma unroll
    for (int s = 0; s < MLP_S; ++s) {
        const int64_t r = s0 + s;
        if (r < n) dprev[r * K + k] = a[r * K + k] > 0.0f ? acc[s] : 0.0f;
    }
}

// gW[k][j] = sum_s a[s][k] dz[s][j];  gb[j] = sum_s dz[s][j]  (rows k = K of the index space)
template <int K, int J>
__global__ __launch_bounds__(256) void mlp_grad_w(const float *__restrict__ a, const float *__restrict__ dz, int64_t n,
                                                  float *__restrict__ gW, float *__restrict__ gb) {
    const int64_t q = blockIdx.x * 256ll + threadIdx.x;
    if (q >= (int64_t)(K + 1) * J) return;
    const int k = (int)(q / J), j = (int)(q % J);
    float acc = 0.0f;
    if (k < K) {
        for (int64_t s = 0; s < n; ++s) acc = fmaf(a[s * K + k], dz[s * J + j], acc);
        gW[k * J + j] = acc;
    } else {
        for (int64_t s = 0; s < n; ++s) acc += dz[s * J + j];
        gb[j] = acc;
    }
}

// Softmax cross-entropy: per-sample loss and dz = (softmax - onehot) / n.
__global__ void mlp_softmax_ce(const float *__restrict__ logits, const int32_t *__restrict__ labels, int64_t n,
                               float inv_n, float *__restrict__ dz, float *__restrict__ loss_i,
                               int32_t *__restrict__ bad) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float *z = logits + i * MLP_C;
    int lab = labels[i];
    if (lab < 0 || lab >= MLP_C) {
        atomicOr(bad, 1);
        lab = 0;
    }
    float mx = z[0];
    for (int c = 1; c < MLP_C; ++c) mx = fmaxf(mx, z[c]);
    float sum = 0.0f;
    for (int c = 0; c < MLP_C; ++c) sum += expf(z[c] - mx);
    loss_i[i] = logf(sum) - (z[lab] - mx);
    const float is = 1.0f / sum;
    for (int c = 0; c < MLP_C; ++c) dz[i * MLP_C + c] = (expf(z[c] - mx) * is - (c == lab ? 1.0f : 0.0f)) * inv_n;
}

// Mean of loss_i in a fixed order (one workgroup, float64 partial sums).
__global__ __launch_bounds__(256) void mlp_mean(const float *__restrict__ v, int64_t n, float *__restrict__ out) {
    __shared__ double red[256];
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) s += (double)v[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = (float)(red[0] / (double)n);
}

// Adam (Kingma & Ba 2015, Algorithm 1); c1 = 1 / (1 - beta1^t), c2 = 1 / (1 - beta2^t).
__global__ void mlp_adam(float *__restrict__ theta, float *__restrict__ m, float *__restrict__ v,
                         const float *__restrict__ g, int64_t np, float lr, float c1, float c2) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= np) return;
    const float gi = g[i];
    const float mi = 0.9f * m[i] + 0.1f * gi;
    const float vi = 0.999f * v[i] + 0.001f * gi * gi;
    m[i] = mi;
    v[i] = vi;
    theta[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + 1e-8f);
}

// Top-probability cell selection: one wavefront per row, lane c holds cell c.  Rows whose
// feature 2 (the network SNR) is below rho_split use p_cum_low.
__global__ __launch_bounds__(256) void mlp_select(const float *__restrict__ logits, const float *__restrict__ x,
                                                  int64_t n, float p_cum, float rho_split, float p_cum_low,
                                                  uint64_t *__restrict__ mask_out) {
    const int64_t i = blockIdx.x * 4ll + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (i >= n) return;  // whole wavefronts leave together
    const float pc = x[i * MLP_F + 2] >= rho_split ? p_cum : p_cum_low;
    const float z = logits[i * MLP_C + lane];
    float mx = z;
    for (int o = 32; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_down(mx, o));
    mx = __shfl(mx, 0);
    const float e = expf(z - mx);
    float sum = e;
    for (int o = 32; o > 0; o >>= 1) sum += __shfl_down(sum, o);
    sum = __shfl(sum, 0);
    const float p = e / sum;
    bool taken = false;
    float acc = 0.0f;
    uint64_t mask = 0;
    for (int it = 0; it < MLP_C; ++it) {
        // the largest untaken probability, lowest lane on ties
        float bv = taken ? -1.0f : p;
        int bl = lane;
        for (int o = 32; o > 0; o >>= 1) {
            const float ov = __shfl_down(bv, o);
            const int ol = __shfl_down(bl, o);
            if (lane + o < 64 && (ov > bv || (ov == bv && ol < bl))) {
                bv = ov;
                bl = ol;
            }
        }
        bv = __shfl(bv, 0);
        bl = __shfl(bl, 0);
        if (lane == bl) taken = true;
        mask |= 1ull << bl;
        acc += bv;
        if (acc >= pc) break;
    }
    if (lane == 0) mask_out[i] = mask;
}

static unsigned blocks(int64_t n, int per) { return (unsigned)cdiv(n, per); }

// Forward pass into caller-provided buffers (h0 may be null).
static int mlp_forward_into(hs_ctx *ctx, const float *model, const float *x, int64_t n, float *h0, float *a1,
                            float *a2, float *a3, float *logits) {
    const unsigned g = blocks(n, MLP_S);
    hipLaunchKernelGGL((mlp_fwd<MLP_F, MLP_H, true, true>), dim3(g), dim3(MLP_H), 0, ctx->stream, x, n, model,
                       model + W1, model + B1, h0, a1);
    hipLaunchKernelGGL((mlp_fwd<MLP_H, MLP_H, false, true>), dim3(g), dim3(MLP_H), 0, ctx->stream, a1, n, model,
                       model + W2, model + B2, nullptr, a2);
    hipLaunchKernelGGL((mlp_fwd<MLP_H, MLP_H, false, true>), dim3(g), dim3(MLP_H), 0, ctx->stream, a2, n, model,
                       model + W3, model + B3, nullptr, a3);
    hipLaunchKernelGGL((mlp_fwd<MLP_H, MLP_C, false, false>), dim3(g), dim3(MLP_C), 0, ctx->stream, a3, n, model,
                       model + W4, model + B4, nullptr, logits);
    HS_HIP(hipGetLastError());
    return HS_OK;
}

}  // namespace hs

using namespace hs;

extern "C" int hs_proposer_features(hs_ctx *ctx, const hs_coinc *c, int64_t n_c, const hs_trigger *trig_h,
                                    int64_t n_h, const float *chisq_h, const float *bins_h,
                                    const hs_trigger *trig_l, int64_t n_l, const float *chisq_l,
                                    const float *bins_l, int32_t chisq_bins, int64_t seg_ticks,
                                    const double *coarse_mchirp, const double *coarse_q, int32_t n_coarse,
                                    int64_t step, int64_t wrap, int64_t ticks_per_second, float *feat_out) {
    HS_REQUIRE(ctx, "hs_proposer_features: null context");
    HS_REQUIRE(n_c >= 0 && n_h >= 0 && n_l >= 0 && n_coarse >= 0, "hs_proposer_features: negative size");
    HS_REQUIRE(chisq_bins == 8, "hs_proposer_features: the features need 8 chi-square bins (got %d)", chisq_bins);
    HS_REQUIRE(seg_ticks > 0 && wrap > 0 && ticks_per_second > 0, "hs_proposer_features: bad time constants");
    if (n_c == 0) return HS_OK;
    HS_REQUIRE(c && trig_h && chisq_h && bins_h && trig_l && chisq_l && bins_l && coarse_mchirp && coarse_q && feat_out,
               "hs_proposer_features: null argument");
    HS_HIP(hipSetDevice(ctx->device));
    int32_t *bad;
    Carver cv;
    cv.add(&bad, 1);
    HS_TRY(cv.commit(ctx));
    HS_TRY(fill_u32(ctx, reinterpret_cast<uint32_t *>(bad), 1, 0));
    hipLaunchKernelGGL(features_kernel, dim3(blocks(n_c, 256)), dim3(256), 0, ctx->stream, c, n_c, trig_h, n_h,
                       chisq_h, bins_h, trig_l, n_l, chisq_l, bins_l, seg_ticks, coarse_mchirp, coarse_q, n_coarse,
                       step, wrap, ticks_per_second, feat_out, bad);
    HS_HIP(hipGetLastError());
    int32_t hbad = 0;
    HS_TRY(read_back(ctx, bad, &hbad, sizeof(hbad)));
    HS_REQUIRE(hbad == 0, "hs_proposer_features: %s",
               (hbad & 1) ? "coincidence template outside [0, n_coarse)" : "coincidence without its trigger");
    return HS_OK;
}

extern "C" int hs_mlp_forward(hs_ctx *ctx, const float *model, const float *x, int64_t n, float *logits_out) {
    HS_REQUIRE(ctx && n >= 0, "hs_mlp_forward: bad argument");
    if (n == 0) return HS_OK;
    HS_REQUIRE(model && x && logits_out, "hs_mlp_forward: null argument");
    HS_REQUIRE(n < (int64_t(1) << 31) / MLP_H, "hs_mlp_forward: batch too large");
    HS_HIP(hipSetDevice(ctx->device));
    float *a1, *a2, *a3;
    Carver cv;
    cv.add(&a1, (size_t)n * MLP_H);
    cv.add(&a2, (size_t)n * MLP_H);
    cv.add(&a3, (size_t)n * MLP_H);
    HS_TRY(cv.commit(ctx));
    return mlp_forward_into(ctx, model, x, n, nullptr, a1, a2, a3, logits_out);
}

extern "C" int hs_mlp_train_step(hs_ctx *ctx, float *model, float *adam_m, float *adam_v, int64_t t, float lr,
                                 const float *x, const int32_t *labels, int64_t n, float *grad_out,
                                 float *loss_out) {
    HS_REQUIRE(ctx && loss_out, "hs_mlp_train_step: null argument");
    HS_REQUIRE(n >= 1 && n < (int64_t(1) << 31) / MLP_H, "hs_mlp_train_step: batch size must be in [1, 2^24)");
    HS_REQUIRE(t >= 1, "hs_mlp_train_step: step t must be >= 1");
    HS_REQUIRE(model && adam_m && adam_v && x && labels, "hs_mlp_train_step: null argument");
    HS_HIP(hipSetDevice(ctx->device));
    float *h0, *a1, *a2, *a3, *logits, *dz4, *d3, *d2, *d1, *loss_i, *loss, *grad;
    int32_t *bad;
    Carver cv;
    cv.add(&h0, (size_t)n * MLP_F);
    cv.add(&a1, (size_t)n * MLP_H);
    cv.add(&a2, (size_t)n * MLP_H);
    cv.add(&a3, (size_t)n * MLP_H);
    cv.add(&logits, (size_t)n * MLP_C);
    cv.add(&dz4, (size_t)n * MLP_C);
    cv.add(&d3, (size_t)n * MLP_H);
    cv.add(&d2, (size_t)n * MLP_H);
    cv.add(&d1, (size_t)n * MLP_H);
    cv.add(&loss_i, (size_t)n);
    cv.add(&loss, 1);
    cv.add(&grad, grad_out ? 1 : (size_t)HS_MLP_PARAMS);
    cv.add(&bad, 1);
    HS_TRY(cv.commit(ctx));
    if (grad_out) grad = grad_out;
    HS_TRY(fill_u32(ctx, reinterpret_cast<uint32_t *>(bad), 1, 0));
    HS_TRY(mlp_forward_into(ctx, model, x, n, h0, a1, a2, a3, logits));
    hipLaunchKernelGGL(mlp_softmax_ce, dim3(blocks(n, 256)), dim3(256), 0, ctx->stream, logits, labels, n,
                       (float)(1.0 / (double)n), dz4, loss_i, bad);
    // gradient offsets follow the model layout without the normalisation block
    float *gW4 = grad + (W4 - MLP_NORM), *gB4 = grad + (B4 - MLP_NORM), *gW3 = grad + (W3 - MLP_NORM),
          *gB3 = grad + (B3 - MLP_NORM), *gW2 = grad + (W2 - MLP_NORM), *gB2 = grad + (B2 - MLP_NORM),
          *gW1 = grad + (W1 - MLP_NORM), *gB1 = grad + (B1 - MLP_NORM);
    const unsigned gs = blocks(n, MLP_S);
    hipLaunchKernelGGL((mlp_grad_w<MLP_H, MLP_C>), dim3(blocks((MLP_H + 1) * MLP_C, 256)), dim3(256), 0, ctx->stream,
                       a3, dz4, n, gW4, gB4);
    hipLaunchKernelGGL((mlp_bwd<MLP_H, MLP_C>), dim3(gs), dim3(MLP_H), 0, ctx->stream, dz4, n, model + W4, a3, d3);
    hipLaunchKernelGGL((mlp_grad_w<MLP_H, MLP_H>), dim3(blocks((MLP_H + 1) * MLP_H, 256)), dim3(256), 0, ctx->stream,
                       a2, d3, n, gW3, gB3);
    hipLaunchKernelGGL((mlp_bwd<MLP_H, MLP_H>), dim3(gs), dim3(MLP_H), 0, ctx->stream, d3, n, model + W3, a2, d2);
    hipLaunchKernelGGL((mlp_grad_w<MLP_H, MLP_H>), dim3(blocks((MLP_H + 1) * MLP_H, 256)), dim3(256), 0, ctx->stream,
                       a1, d2, n, gW2, gB2);
    hipLaunchKernelGGL((mlp_bwd<MLP_H, MLP_H>), dim3(gs), dim3(MLP_H), 0, ctx->stream, d2, n, model + W2, a1, d1);
    hipLaunchKernelGGL((mlp_grad_w<MLP_F, MLP_H>), dim3(blocks((MLP_F + 1) * MLP_H, 256)), dim3(256), 0, ctx->stream,
                       h0, d1, n, gW1, gB1);
    hipLaunchKernelGGL(mlp_mean, dim3(1), dim3(256), 0, ctx->stream, loss_i, n, loss);
    HS_HIP(hipGetLastError());
    int32_t hbad = 0;
    HS_TRY(read_back(ctx, bad, &hbad, sizeof(hbad)));
    HS_REQUIRE(hbad == 0, "hs_mlp_train_step: label outside [0, 64)");
    const double c1 = 1.0 / (1.0 - std::pow(0.9, (double)t));
    const double c2 = 1.0 / (1.0 - std::pow(0.999, (double)t));
    hipLaunchKernelGGL(mlp_adam, dim3(blocks(HS_MLP_PARAMS, 256)), dim3(256), 0, ctx->stream, model + MLP_NORM,
                       adam_m, adam_v, grad, (int64_t)HS_MLP_PARAMS, lr, (float)c1, (float)c2);
    HS_HIP(hipGetLastError());
    HS_TRY(read_back(ctx, loss, loss_out, sizeof(float)));
    return HS_OK;
}

extern "C" int hs_mlp_propose(hs_ctx *ctx, const float *model, const float *x, int64_t n, float p_cum,
                              float rho_split, float p_cum_low, uint64_t *mask_out) {
    HS_REQUIRE(ctx && n >= 0, "hs_mlp_propose: bad argument");
    if (n == 0) return HS_OK;
    HS_REQUIRE(model && x && mask_out, "hs_mlp_propose: null argument");
    HS_REQUIRE(n < (int64_t(1) << 31) / MLP_H, "hs_mlp_propose: batch too large");
    HS_HIP(hipSetDevice(ctx->device));
    float *a1, *a2, *a3, *logits;
    Carver cv;
    cv.add(&a1, (size_t)n * MLP_H);
    cv.add(&a2, (size_t)n * MLP_H);
    cv.add(&a3, (size_t)n * MLP_H);
    cv.add(&logits, (size_t)n * MLP_C);
    HS_TRY(cv.commit(ctx));
    HS_TRY(mlp_forward_into(ctx, model, x, n, nullptr, a1, a2, a3, logits));
    hipLaunchKernelGGL(mlp_select, dim3(blocks(n, 4)), dim3(256), 0, ctx->stream, logits, x, n, p_cum, rho_split,
                       p_cum_low, mask_out);
    HS_HIP(hipGetLastError());
    return HS_OK;
}
