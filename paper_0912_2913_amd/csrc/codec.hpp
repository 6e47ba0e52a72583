// Population storage formats and the collision's compute type.
//
// F64 and F32 store S_i itself.  The *DEV forms store the deviation
// d_i = S_i - R_i from the rest equilibrium R at (n_ref, e_ref); the collision
// then works on deviations and the rest part never enters the rounding.  The
// compute type TC (double or float) is the type of the moment sums, the
// equilibria and the relaxation; the moment inversion is FP64 in every case.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace rlb {

// Adjoint (lambda) buffers are FP64 for every storage: lambda carries a large
// component along the collision invariants that cancels in every contraction
// with (pre - eq); stored in FP32 its rounding swamps the small remainder.
using LamT = double;

enum { ST_F64 = 0, ST_F32 = 1, ST_F32DEV = 2, ST_F16DEV = 3, ST_BF16DEV = 4 };

template <int ST>
struct Format;

template <>
struct Format<ST_F64> {
  using elem = double;
  static constexpr bool dev = false;
  template <class T>
  __device__ static T dec(elem v) { return (T)v; }
  template <class T>
  __device__ static elem enc(T v) { return (elem)v; }
};

template <>
struct Format<ST_F32> {
  using elem = float;
  static constexpr bool dev = false;
  template <class T>
  __device__ static T dec(elem v) { return (T)v; }
  // one rounding (round to nearest even) from the compute type
  template <class T>
  __device__ static elem enc(T v) { return (elem)v; }
};

template <>
struct Format<ST_F32DEV> : Format<ST_F32> {
  static constexpr bool dev = true;
};

template <>
struct Format<ST_F16DEV> {
  using elem = _Float16;
  static constexpr bool dev = true;
  template <class T>
  __device__ static T dec(elem v) { return (T)(float)v; }
  // hardware conversion, round to nearest even (the default rounding mode);
  // only FP32 compute is paired with this format
  __device__ static elem enc(float v) { return (_Float16)v; }
};

// bfloat16 = the upper 16 bits of an IEEE binary32.  Encoding rounds to
// nearest, ties to even, on the discarded 16 bits (gfx950's conversion
// instruction); NaNs stay quiet NaNs.
template <>
struct Format<ST_BF16DEV> {
  using elem = uint16_t;
  static constexpr bool dev = true;
  template <class T>
  __device__ static T dec(elem v) { return (T)__uint_as_float((uint32_t)v << 16); }
  // only FP32 compute is paired with this format
  __device__ static elem enc(float v) { return __builtin_bit_cast(uint16_t, (__bf16)v); }
};

// Compute-type tag: FP32 equilibria and relaxation, with FP64 moments: the
// sums (E, M, N) accumulated in FP64 and the g equilibrium corrected to them
// (eq_fix in kernels.hpp).
struct f32s {};

template <int ST, class TC>
struct Codec {
  using F = Format<ST>;
  using elem = typename F::elem;
  using calc = std::conditional_t<std::is_same<TC, f32s>::value, float, TC>;
  using sum = std::conditional_t<std::is_same<TC, f32s>::value, double, calc>;  // moment sums
  using lam = LamT;
  static constexpr bool dev = F::dev;
  __device__ static calc dec(elem v) { return F::template dec<calc>(v); }
  __device__ static elem enc(calc v) { return F::enc(v); }
};

}  // namespace rlb
