// Device helpers shared by the split-precision contraction kernels: the
// 16-bit operand types, the hi/lo split of a pair of FP32 values, the 16-bit
// MFMA of either format and the six products of one reduction step.
#pragma once

#include <hip/hip_runtime.h>

#include "internal.h"

namespace expenc {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// Split two FP32 values into packed (hi, lo) 16-bit pairs.
template <bool BF>
__device__ inline void split_pair(float a, float b, uint32_t &hi, uint32_t &lo) {
  if constexpr (BF) {
    const bf16x2 h = {(__bf16)a, (__bf16)b};
    hi = __builtin_bit_cast(uint32_t, h);
    const float ah = __uint_as_float(hi << 16), bh = __uint_as_float(hi & 0xffff0000u);
    const bf16x2 l = {(__bf16)(a - ah), (__bf16)(b - bh)};
    lo = __builtin_bit_cast(uint32_t, l);
  } else {
    const f16x2 h = {(_Float16)a, (_Float16)b};
    hi = __builtin_bit_cast(uint32_t, h);
    // v - hi in one fused multiply-add that reads the 16-bit half directly
    // (exact: hi is within a factor 2 of v), instead of converting hi back
    // (writing the rounded differences straight into the halves of lo with
    // v_fma_mixlo/mixhi_f16 saves one instruction per pair but measured 1-2 %
    // slower at 1.5 mm)
    float la, lb;
    __asm__("v_fma_mix_f32 %0, -%1, 1.0, %2 op_sel_hi:[1,0,0]" : "=v"(la) : "v"(hi), "v"(a));
    __asm__("v_fma_mix_f32 %0, -%1, 1.0, %2 op_sel:[1,0,0] op_sel_hi:[1,0,0]" : "=v"(lb) : "v"(hi), "v"(b));
    const f16x2 l = {(_Float16)la, (_Float16)lb};
    lo = __builtin_bit_cast(uint32_t, l);
  }
}

// Masks of the bf16 remainder below, (-1, 0) and (0, -1) as packed bf16
// pairs.  They reach the kernels as arguments (scalar registers): written as
// constants, the compiler encodes (-1, 0) as the inline constant -1.0, which
// the dot-product instruction reads as the FP32 pattern 0xbf800000, (0, -1).
struct Bf16Masks {
  uint32_t lo, hi;
};
inline Bf16Masks bf16_masks() { return Bf16Masks{0x0000bf80u, 0xbf800000u}; }

// split_pair with the bf16 remainders v - hi from a two-term bf16 dot
// product, (hi_a, hi_b) . (-1, 0) + a and (hi_a, hi_b) . (0, -1) + b: one
// instruction per value instead of widening hi and subtracting (exact: the
// product is exact and hi is within a factor 2 of v).  Same bits as
// split_pair<true>; fp16 pairs go to split_pair<false>.
template <bool BF>
__device__ inline void split_pair(float a, float b, uint32_t &hi, uint32_t &lo, Bf16Masks mk) {
  if constexpr (BF) {
    const bf16x2 h = {(__bf16)a, (__bf16)b};
    hi = __builtin_bit_cast(uint32_t, h);
    const float la = __builtin_amdgcn_fdot2_f32_bf16(h, __builtin_bit_cast(bf16x2, mk.lo), a, false);
    const float lb = __builtin_amdgcn_fdot2_f32_bf16(h, __builtin_bit_cast(bf16x2, mk.hi), b, false);
    const bf16x2 l = {(__bf16)la, (__bf16)lb};
    lo = __builtin_bit_cast(uint32_t, l);
  } else {
    split_pair<false>(a, b, hi, lo);
  }
}

template <bool BF>
__device__ inline f32x16 mfma16(u32x4 a, u32x4 b, f32x16 c) {
  if constexpr (BF)
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c,
                                                   0, 0, 0);
  else
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, a), __builtin_bit_cast(f16x8, b), c,
                                                  0, 0, 0);
}

// 6 MFMAs of one step for one 32-row block and one 32-column group:
// cos against b1, sin against b2, each as hi*hi + hi*lo + lo*hi.
template <bool BF>
__device__ inline f32x16 step6(const u32x4 (&A)[4], const u32x4 *b, f32x16 acc) {
  acc = mfma16<BF>(A[0], b[0], acc);
  acc = mfma16<BF>(A[0], b[1], acc);
  acc = mfma16<BF>(A[1], b[0], acc);
  acc = mfma16<BF>(A[2], b[2], acc);
  acc = mfma16<BF>(A[2], b[3], acc);
  acc = mfma16<BF>(A[3], b[2], acc);
  return acc;
}

}  // namespace expenc
