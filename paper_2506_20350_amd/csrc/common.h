// Shared device/host helpers of the MLFFT library: complex arithmetic on
// float2/double2, bfloat16 conversion, launch checks.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

template<typename C> struct CTraits;
template<> struct CTraits<float2>  { typedef float real; };
template<> struct CTraits<double2> { typedef double real; };

template<typename C> __host__ __device__ __forceinline__ C czero() { C r; r.x = 0; r.y = 0; return r; }
template<typename C, typename T> __host__ __device__ __forceinline__ C cmake(T re, T im) { C r; r.x = re; r.y = im; return r; }

__host__ __device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__host__ __device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__host__ __device__ __forceinline__ float2 cneg(float2 a) { return make_float2(-a.x, -a.y); }
__host__ __device__ __forceinline__ float2 cmuli(float2 a) { return make_float2(-a.y, a.x); }
__host__ __device__ __forceinline__ float2 cmulni(float2 a) { return make_float2(a.y, -a.x); }
__host__ __device__ __forceinline__ float2 cscale(float2 a, float c) { return make_float2(a.x * c, a.y * c); }
__host__ __device__ __forceinline__ float2 cfmar(float2 a, float c, float2 b) { return make_float2(fmaf(a.x, c, b.x), fmaf(a.y, c, b.y)); }
__host__ __device__ __forceinline__ float2 cmulc(float2 a, float wr, float wi) {
    return make_float2(fmaf(a.x, wr, -a.y * wi), fmaf(a.x, wi, a.y * wr));
}
__host__ __device__ __forceinline__ float2 cmul(float2 a, float2 b) { return cmulc(a, b.x, b.y); }
__host__ __device__ __forceinline__ float2 cconjmul(float2 a, float2 b) {   // conj(a) * b
    return make_float2(fmaf(a.x, b.x, a.y * b.y), fmaf(a.x, b.y, -a.y * b.x));
}

__host__ __device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__host__ __device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__host__ __device__ __forceinline__ double2 cneg(double2 a) { return make_double2(-a.x, -a.y); }
__host__ __device__ __forceinline__ double2 cmuli(double2 a) { return make_double2(-a.y, a.x); }
__host__ __device__ __forceinline__ double2 cmulni(double2 a) { return make_double2(a.y, -a.x); }
__host__ __device__ __forceinline__ double2 cscale(double2 a, double c) { return make_double2(a.x * c, a.y * c); }
__host__ __device__ __forceinline__ double2 cfmar(double2 a, double c, double2 b) { return make_double2(fma(a.x, c, b.x), fma(a.y, c, b.y)); }
__host__ __device__ __forceinline__ double2 cmulc(double2 a, double wr, double wi) {
    return make_double2(fma(a.x, wr, -a.y * wi), fma(a.x, wi, a.y * wr));
}
__host__ __device__ __forceinline__ double2 cmul(double2 a, double2 b) { return cmulc(a, b.x, b.y); }
__host__ __device__ __forceinline__ double2 cconjmul(double2 a, double2 b) {
    return make_double2(fma(a.x, b.x, a.y * b.y), fma(a.x, b.y, -a.y * b.x));
}

// Round-to-nearest-even conversion of an IEEE binary32 value to bfloat16 bits.
__host__ __device__ __forceinline__ uint16_t f32_to_bf16_bits(float f) {
    union { float f; uint32_t u; } v; v.f = f;
    if ((v.u & 0x7f800000u) == 0x7f800000u && (v.u & 0x007fffffu)) return (uint16_t)((v.u >> 16) | 0x40);
    uint32_t lsb = (v.u >> 16) & 1u;
    return (uint16_t)((v.u + 0x7fffu + lsb) >> 16);
}
__host__ __device__ __forceinline__ float bf16_bits_to_f32(uint16_t h) {
    union { float f; uint32_t u; } v; v.u = ((uint32_t)h) << 16; return v.f;
}

#define MLFFT_DEV_INLINE __device__ __forceinline__
