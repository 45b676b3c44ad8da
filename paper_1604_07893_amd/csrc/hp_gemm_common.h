// Device-side pieces shared by the MFMA GEMM sources (hp_gemm.hip: FP64,
// FP32 and FP32-storage 16-bit kernels; hp_gemm_h16.hip: kernels on 16-bit
// operands held in memory). Included inside no namespace; everything here is
// in an anonymous namespace, so each source has its own copy.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace hp {
namespace {

typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef float flt4 __attribute__((ext_vector_type(4)));

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Hardware hands consecutive workgroups to the 8 XCDs in turn; renumber so
// each XCD receives one contiguous range of tile indices (its L2 then holds
// the A and B panels those tiles share).
__device__ inline int xcd_contiguous(int b, int nb) {
    const int nx = 8;
    const int q = nb / nx, r = nb % nx;
    const int x = b % nx;
    return x * q + min(x, r) + b / nx;
}

// Grouped tile order: GROUP tile-rows walked column by column.
__device__ inline void tile_of(int t, int tiles_m, int tiles_n, int& tm, int& tn) {
    constexpr int GROUP = 8;
    const int group_size = GROUP * tiles_n;
    const int g = t / group_size;
    const int first = g * GROUP;
    const int gm = min(tiles_m - first, GROUP);
    const int in = t - g * group_size;
    tm = first + in % gm;
    tn = in / gm;
}

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x4 __attribute__((ext_vector_type(4)));
typedef float flt4v __attribute__((ext_vector_type(4)));

template <typename L>
struct Mfma16;
template <>
struct Mfma16<__bf16> {
    typedef bf16x8 frag_t;
    typedef bf16x4 quad_t;
    static __device__ inline flt4 mma(frag_t a, frag_t b, flt4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
    }
};
template <>
struct Mfma16<_Float16> {
    typedef f16x8 frag_t;
    typedef f16x4 quad_t;
    static __device__ inline flt4 mma(frag_t a, frag_t b, flt4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
    }
};


inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

}  // namespace
}  // namespace hp
