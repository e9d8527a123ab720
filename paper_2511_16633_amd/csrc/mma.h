// Matrix-core building blocks shared by the Born contraction kernels: MFMA
// wrappers with their output-row layouts, 16-bit conversions and guarded loads.
#pragma once
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

namespace rb {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef double d4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef _Float16 h8 __attribute__((ext_vector_type(8)));

template <typename T>
struct MM;
// Both 16x16x4 forms read A[i][k] from lane i + 16k and B[k][j] from lane
// j + 16k.  Output element `i` of lane group kk (lanes 16kk..16kk+15, column
// = lane % 16) holds row 4kk + i for f32 but row kk + 4i for f64 (measured).
template <>
struct MM<float> {
    using acc = f4;
    __device__ __forceinline__ static acc mma(float a, float b, acc c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    __device__ __forceinline__ static int out_row(int kk, int i) { return 4 * kk + i; }
};
template <>
struct MM<double> {
    using acc = d4;
    __device__ __forceinline__ static acc mma(double a, double b, acc c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    __device__ __forceinline__ static int out_row(int kk, int i) { return kk + 4 * i; }
};

// 16-bit storage types and their MFMA (16x16x32, 8 k-values per lane).
template <typename S>
struct MM16;
template <>
struct MM16<__hip_bfloat16> {
    using vec = bf8;
    __device__ __forceinline__ static f4 mma(vec a, vec b, f4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
    }
    __device__ __forceinline__ static float to_f(__hip_bfloat16 v) { return __bfloat162float(v); }
    __device__ __forceinline__ static float bits_to_f(unsigned b) { return __uint_as_float((b & 0xffffu) << 16); }
    __device__ __forceinline__ static __bf16 from_f(float v) {
        __hip_bfloat16 b = __float2bfloat16(v);
        return *reinterpret_cast<__bf16 *>(&b);
    }
};
template <>
struct MM16<__half> {
    using vec = h8;
    __device__ __forceinline__ static f4 mma(vec a, vec b, f4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
    }
    __device__ __forceinline__ static float to_f(__half v) { return __half2float(v); }
    __device__ __forceinline__ static float bits_to_f(unsigned b) {
        return (float)__builtin_bit_cast(_Float16, (unsigned short)(b & 0xffffu));
    }
    __device__ __forceinline__ static _Float16 from_f(float v) { return (_Float16)v; }
};

typedef unsigned int u4x32 __attribute__((ext_vector_type(4)));
// sign flip of eight 16-bit floats (bf16 and fp16 keep the sign in bit 15),
// two per 32-bit operation
template <typename V>
__device__ __forceinline__ V neg(V v) {
    u4x32 b = __builtin_bit_cast(u4x32, v);
    b ^= 0x80008000u;
    return __builtin_bit_cast(V, b);
}

template <typename T>
__device__ __forceinline__ T ld(const T *p, bool ok) {
    return ok ? p[0] : T(0);
}

}  // namespace
}  // namespace rb
