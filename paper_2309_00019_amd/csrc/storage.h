// Template-spectrum storage formats: complex64, or a pair of bf16 / f16 in 32 bits.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace hs {

// load(p, i) = unpack(p[i]); unpack turns a stored element into a complex value; zero() is the
// stored zero.
struct StoreF32 {
    using elem = float2;
    static constexpr int bytes = 8;
    __device__ __forceinline__ static float2 unpack(elem e) { return e; }
    __device__ __forceinline__ static elem zero() { return float2{0.0f, 0.0f}; }
    __device__ __forceinline__ static float2 load(const elem *p, int64_t i) { return p[i]; }
    __device__ __forceinline__ static elem pack(float re, float im) { return float2{re, im}; }
};

// bf16 as the upper 16 bits of a float, round-to-nearest-even on packing.
struct StoreBF16 {
    using elem = uint32_t;  // low half = re, high half = im
    static constexpr int bytes = 4;
    __device__ __forceinline__ static uint32_t to_bf16(float f) {
        uint32_t u = __float_as_uint(f);
        u += 0x7FFFu + ((u >> 16) & 1u);
        return u >> 16;
    }
    __device__ __forceinline__ static float2 unpack(uint32_t u) {
        return float2{__uint_as_float(u << 16), __uint_as_float(u & 0xFFFF0000u)};
    }
    __device__ __forceinline__ static elem zero() { return 0u; }
    __device__ __forceinline__ static float2 load(const elem *p, int64_t i) { return unpack(p[i]); }
    __device__ __forceinline__ static elem pack(float re, float im) {
        return to_bf16(re) | (to_bf16(im) << 16);
    }
};

struct StoreF16 {
    using elem = uint32_t;  // low half = re, high half = im (IEEE binary16)
    static constexpr int bytes = 4;
    __device__ __forceinline__ static elem zero() { return 0u; }
    __device__ __forceinline__ static float2 load(const elem *p, int64_t i) { return unpack(p[i]); }
    __device__ __forceinline__ static float2 unpack(uint32_t u) {
        _Float16 re, im;
        const uint16_t lo = (uint16_t)(u & 0xFFFFu), hi = (uint16_t)(u >> 16);
        __builtin_memcpy(&re, &lo, 2);
        __builtin_memcpy(&im, &hi, 2);
        return float2{(float)re, (float)im};
    }
    __device__ __forceinline__ static elem pack(float re, float im) {
        const _Float16 a = (_Float16)re, b = (_Float16)im;
        uint16_t lo, hi;
        __builtin_memcpy(&lo, &a, 2);
        __builtin_memcpy(&hi, &b, 2);
        return (uint32_t)lo | ((uint32_t)hi << 16);
    }
};

}  // namespace hs
