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

// Loads and stores through the global address space.  Pointers taken from task
// tables are generic, for which the compiler emits flat memory instructions;
// a flat load counts against the LDS wait counter as well, so every wait for
// an LDS read would also wait for the global loads in flight (a prefetch of the
// next tile, say).  These helpers make the access a global_load / global_store.
#define MLFFT_GLOBAL __attribute__((address_space(1)))
typedef float mlfft_f2v __attribute__((ext_vector_type(2)));
typedef double mlfft_d2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ float2 gload(const float2* p) {
    const mlfft_f2v v = *(const MLFFT_GLOBAL mlfft_f2v*)p;
    return make_float2(v.x, v.y);
}
__device__ __forceinline__ double2 gload(const double2* p) {
    const mlfft_d2v v = *(const MLFFT_GLOBAL mlfft_d2v*)p;
    return make_double2(v.x, v.y);
}
__device__ __forceinline__ void gstore(float2* p, float2 v) { *(MLFFT_GLOBAL mlfft_f2v*)p = mlfft_f2v{v.x, v.y}; }
__device__ __forceinline__ void gstore(double2* p, double2 v) { *(MLFFT_GLOBAL mlfft_d2v*)p = mlfft_d2v{v.x, v.y}; }
__device__ __forceinline__ uint32_t gload(const uint32_t* p) { return *(const MLFFT_GLOBAL uint32_t*)p; }
