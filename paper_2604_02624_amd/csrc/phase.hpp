// exp(i 2 pi rev) for phases whose argument must be reduced in double precision.
//
// The phase of the transmission (2 pi (n - n_m) h / lambda) and of the transfer function
// (2 pi z sqrt(q)) reach hundreds of radians, where single precision cannot resolve the
// fraction of a turn.  The turn count is therefore removed in double precision: with
// r = 4 rev, k = nearest integer to r (the quadrant) and x = r - k in [-1/2, 1/2] (exact in
// double), the angle is k pi/2 + x pi/2.  sin and cos of a = x pi/2 in [-pi/4, pi/4] are
// evaluated in single precision by polynomials in a^2 fitted by least squares on 4000
// Chebyshev nodes of the interval (sin: a (s0 + s1 a^2 + s2 a^4 + s3 a^6), max error 2.3e-9;
// cos: c0 + ... + c4 a^8, max error 4.8e-11; about 1 ulp once evaluated in single
// precision), and the quadrant rotates the result.  That is the transmission's evaluation (row
// passes, bound by memory).  The transfer function (column passes, bound by vector instructions)
// reduces to a fraction of a turn instead and takes its sine and cosine from the hardware
// (cis_turns_hw).
#pragma once

#include <hip/hip_runtime.h>

namespace dpx {

constexpr double kHalfPi = 1.57079632679489661923132169163975144;
// the smallest positive normal double: the square root's stand-in argument outside the disc
constexpr double kMinNormalF64 = 2.2250738585072014e-308;

// returns (cos(pi r / 2), sin(pi r / 2)) / DEN for an angle of r quarter turns; 1/DEN is
// folded into the coefficients, so a power-of-two DEN costs nothing and changes no rounding.
// Callers whose argument is a product c x can pass (4 c) x: scaling by 4 is exact, so the bits
// are those of cis_turns(c x) without the multiplication per element.
template <int DEN = 1>
__device__ __forceinline__ float2 cis_quarter_turns(double r) {
  constexpr double sc = 1.0 / static_cast<double>(DEN);
  const double kq = rint(r);
  const float x = static_cast<float>(r - kq);
  const int q = static_cast<int>(kq);
  const float a = x * static_cast<float>(kHalfPi);
  const float a2 = a * a;
  constexpr float s0 = static_cast<float>(sc * 0.9999999967572502);
  constexpr float s1 = static_cast<float>(sc * -0.1666665021134592);
  constexpr float s2 = static_cast<float>(sc * 0.008332015903612005);
  constexpr float s3 = static_cast<float>(sc * -0.0001950176314224722);
  constexpr float c0 = static_cast<float>(sc * 0.9999999999525452);
  constexpr float c1 = static_cast<float>(sc * -0.49999999615145646);
  constexpr float c2 = static_cast<float>(sc * 0.04166661671587216);
  constexpr float c3 = static_cast<float>(sc * -0.0013886618604925212);
  constexpr float c4 = static_cast<float>(sc * 2.4379880306502892e-05);
  const float sp = fmaf(a2, fmaf(a2, fmaf(a2, s3, s2), s1), s0) * a;
  const float cp = fmaf(a2, fmaf(a2, fmaf(a2, fmaf(a2, c4, c3), c2), c1), c0);
  // rotate by q quarter turns: (c, s) -> (-s, c) -> (-c, -s) -> (s, -c)
  const bool odd = (q & 1) != 0;
  const float cs = odd ? sp : cp;
  const float sn = odd ? cp : sp;
  const unsigned flip_c = static_cast<unsigned>((q + 1) & 2) << 30;  // q = 1, 2
  const unsigned flip_s = static_cast<unsigned>(q & 2) << 30;        // q = 2, 3
  return make_float2(__uint_as_float(__float_as_uint(cs) ^ flip_c),
                     __uint_as_float(__float_as_uint(sn) ^ flip_s));
}

// returns (cos(2 pi rev), sin(2 pi rev)) / DEN
template <int DEN = 1>
__device__ __forceinline__ float2 cis_turns(double rev) {
  return cis_quarter_turns<DEN>(4.0 * rev);
}

// returns (cos(2 pi rev), sin(2 pi rev)) / DEN with the turn count removed in double precision
// (k = nearest integer to rev, x = rev - k in [-1/2, 1/2] exact) and the sine and cosine of the
// remaining fraction of a turn taken from the hardware's single-precision v_sin_f32 / v_cos_f32,
// whose argument is in revolutions.  Measured over one turn (2^24 points against double precision)
// their largest error is 1.3e-7 (rms 4.4e-8), against 9.4e-8 (rms 2.6e-8) for the polynomials of
// cis_quarter_turns with their argument rounding; they replace the polynomial evaluation, its
// quadrant rotation and one of the two conversions, which matters in the column passes, whose
// vector instructions bound them.  1/DEN is one multiplication per component (exact for a
// power-of-two DEN).
template <int DEN = 1>
__device__ __forceinline__ float2 cis_turns_hw(double rev) {
  constexpr float sc = static_cast<float>(1.0 / static_cast<double>(DEN));
  const float x = static_cast<float>(rev - rint(rev));
  return make_float2(__builtin_amdgcn_cosf(x) * sc, __builtin_amdgcn_sinf(x) * sc);
}

// sqrt of a positive double to about 1e-14 relative: hardware reciprocal square root
// estimate refined by one Goldschmidt step (s = q y, h = y / 2, r = 1/2 - h s, s += s r).
__device__ __forceinline__ double sqrt_pos(double q) {
  const double y = __builtin_amdgcn_rsq(q);
  const double s = q * y;
  const double h = 0.5 * y;
  const double r = fma(-h, s, 0.5);
  return fma(s, r, s);
}

}  // namespace dpx
