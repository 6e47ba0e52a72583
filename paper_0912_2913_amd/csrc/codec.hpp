// Population storage formats.  F64 and F32 store S_i itself.  The *DEV forms
// store the deviation d_i = S_i - R_i from the rest equilibrium R at
// (n_ref, e_ref); the collision then works on deviations in FP32 and the
// rest part never enters the rounding.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rlb {

enum { ST_F64 = 0, ST_F32 = 1, ST_F32DEV = 2, ST_F16DEV = 3, ST_BF16DEV = 4 };

template <int ST>
struct Codec;

template <>
struct Codec<ST_F64> {
  using elem = double;
  using calc = double;
  using lam = double;
  static constexpr bool dev = false;
  __device__ static calc dec(elem v) { return v; }
  __device__ static elem enc(calc v) { return v; }
};

template <>
struct Codec<ST_F32> {
  using elem = float;
  using calc = float;
  using lam = float;
  static constexpr bool dev = false;
  __device__ static calc dec(elem v) { return v; }
  __device__ static elem enc(calc v) { return v; }
};

template <>
struct Codec<ST_F32DEV> {
  using elem = float;
  using calc = float;
  using lam = float;
  static constexpr bool dev = true;
  __device__ static calc dec(elem v) { return v; }
  __device__ static elem enc(calc v) { return v; }
};

template <>
struct Codec<ST_F16DEV> {
  using elem = _Float16;
  using calc = float;
  using lam = float;
  static constexpr bool dev = true;
  __device__ static calc dec(elem v) { return (float)v; }
  // hardware conversion, round-to-nearest-even (the default rounding mode)
  __device__ static elem enc(calc v) { return (_Float16)v; }
};

// bfloat16 = the upper 16 bits of an IEEE binary32.  Encoding rounds to
// nearest, ties to even, on the discarded 16 bits; NaNs stay (quiet) NaNs.
__device__ inline uint16_t f32_to_bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x0040u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

template <>
struct Codec<ST_BF16DEV> {
  using elem = uint16_t;
  using calc = float;
  using lam = float;
  static constexpr bool dev = true;
  __device__ static calc dec(elem v) { return __uint_as_float((uint32_t)v << 16); }
  __device__ static elem enc(calc v) { return f32_to_bf16_rne(v); }
};

}  // namespace rlb
