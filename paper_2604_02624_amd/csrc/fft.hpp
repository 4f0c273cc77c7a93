// Register/LDS Stockham FFT for gfx950 wavefronts.
//
// A length-M transform is owned by a group of P = M / E lanes; every lane keeps E complex
// values in registers in the strided layout  lane j0 holds element j0 + P*t, t = 0..E-1.
// Usually a group lies inside one wavefront (P divides 64); the 1600-point transform
// (E = 20, P = 80) spans wavefronts and orders its LDS exchanges with block barriers.
// With this layout every Stockham radix-R stage (R divides E) finds all R inputs of its
// butterflies in the lane's own registers; only the outputs of a non-final stage are
// scattered, so they go through the group's LDS region and come back strided.  The final
// stage writes its outputs exactly where its inputs were, so the transform ends in the same
// strided natural order it started in, with (#stages - 1) LDS round trips.
//
// Forward transforms use exp(-2 pi i k n / M), inverse ones exp(+2 pi i k n / M), both
// unnormalised.  Inter-stage twiddles come from a per-stage table built on the host in double
// precision from exact integer indices (see twiddle_offset) and staged into LDS by each block;
// inverse stages conjugate it.  Twiddles inside a radix-R butterfly are compile-time
// constants.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <type_traits>
#include <utility>
#include <vector>

namespace dpx {

// ------------------------------------------------------------------------------------------
// complex helpers (float2 = interleaved re, im)
// ------------------------------------------------------------------------------------------
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
// The library is built without floating-point contraction (-ffp-contract=off): every fused
// multiply-add is written out (fmaf), so the rounding of each value is fixed by the source and
// the same operands give the same bits in every kernel that inlines this code (every column
// variant, grouped and per-design launches).
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(fmaf(a.x, b.x, -(a.y * b.y)), fmaf(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
__device__ __forceinline__ float2 conjf2(float2 a) { return make_float2(a.x, -a.y); }
// a * conj(b)
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {
  return make_float2(fmaf(a.x, b.x, a.y * b.y), fmaf(a.y, b.x, -(a.x * b.y)));
}
// multiply by -i (forward quarter turn) / +i
__device__ __forceinline__ float2 mul_negi(float2 a) { return make_float2(a.y, -a.x); }
__device__ __forceinline__ float2 mul_posi(float2 a) { return make_float2(-a.y, a.x); }

// ------------------------------------------------------------------------------------------
// compile-time helpers
// ------------------------------------------------------------------------------------------
template <int I, int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (I < N) {
    f(std::integral_constant<int, I>{});
    static_for<I + 1, N>(f);
  }
}

// sin / cos of 2 pi num / den by a Taylor series on the angle reduced to (-pi, pi]
constexpr double kPi = 3.14159265358979323846264338327950288;
constexpr double taylor_sin(double x) {
  double term = x, sum = x;
  for (int k = 1; k < 40; ++k) {
    term *= -x * x / ((2.0 * k) * (2.0 * k + 1.0));
    sum += term;
  }
  return sum;
}
constexpr double taylor_cos(double x) {
  double term = 1.0, sum = 1.0;
  for (int k = 1; k < 40; ++k) {
    term *= -x * x / ((2.0 * k - 1.0) * (2.0 * k));
    sum += term;
  }
  return sum;
}
constexpr double reduced_angle(int num, int den) {
  int m = ((num % den) + den) % den;
  if (2 * m > den) m -= den;
  return 2.0 * kPi * static_cast<double>(m) / static_cast<double>(den);
}
constexpr double cos2pi(int num, int den) { return taylor_cos(reduced_angle(num, den)); }
constexpr double sin2pi(int num, int den) { return taylor_sin(reduced_angle(num, den)); }

// first factor A of a composite radix R = A * B (even whenever R is, so zero pruning passes on)
constexpr int first_factor(int r) {
  if (r == 8) return 2;
  if (r % 4 == 0) return 4;
  if (r % 2 == 0) return 2;
  if (r % 3 == 0) return 3;
  return r;
}

// v * W_R^e with W_R = exp(-2 pi i / R) (forward) or exp(+2 pi i / R) (inverse); e known at
// compile time, multiples of pi/4 are special-cased.
template <int R, int E, bool INV>
__device__ __forceinline__ float2 twc(float2 v) {
  constexpr int e = ((E % R) + R) % R;
  if constexpr (e == 0) {
    return v;
  } else if constexpr ((8 * e) % R == 0) {
    constexpr int oct = (8 * e) / R;  // angle = oct * pi / 4 (clockwise for forward)
    constexpr float h = 0.70710678118654752440f;
    // forward: multiply by exp(-i oct pi/4); inverse: exp(+i oct pi/4)
    constexpr int o = INV ? (8 - oct) % 8 : oct;
    if constexpr (o == 2) return mul_negi(v);
    else if constexpr (o == 4) return make_float2(-v.x, -v.y);
    else if constexpr (o == 6) return mul_posi(v);
    else if constexpr (o == 1) return make_float2((v.x + v.y) * h, (v.y - v.x) * h);
    else if constexpr (o == 3) return make_float2((v.y - v.x) * h, -(v.x + v.y) * h);
    else if constexpr (o == 5) return make_float2(-(v.x + v.y) * h, (v.x - v.y) * h);
    else return make_float2((v.x - v.y) * h, (v.x + v.y) * h);  // o == 7
  } else {
    constexpr float c = static_cast<float>(cos2pi(e, R));
    constexpr float s = static_cast<float>(INV ? sin2pi(e, R) : -sin2pi(e, R));
    return make_float2(fmaf(v.x, c, -(v.y * s)), fmaf(v.x, s, v.y * c));
  }
}

// W_R^E is an odd multiple of pi/4, i.e. (+-1 +- i) / sqrt(2)
template <int R, int E>
constexpr bool odd_octant() {
  constexpr int e = ((E % R) + R) % R;
  return e != 0 && (8 * e) % R == 0 && ((8 * e) / R) % 2 == 1;
}

// sqrt(2) v W_R^E for an odd octant: the rotation without its 1/sqrt(2), which the consumer
// applies inside its own fused multiply-adds
template <int R, int E, bool INV>
__device__ __forceinline__ float2 twc_octant_unscaled(float2 v) {
  constexpr int e = ((E % R) + R) % R;
  constexpr int oct = (8 * e) / R;
  constexpr int o = INV ? (8 - oct) % 8 : oct;
  static_assert(o % 2 == 1, "odd octants only");
  if constexpr (o == 1) return make_float2(v.x + v.y, v.y - v.x);
  else if constexpr (o == 3) return make_float2(v.y - v.x, -(v.x + v.y));
  else if constexpr (o == 5) return make_float2(-(v.x + v.y), v.x - v.y);
  else return make_float2(v.x - v.y, v.x + v.y);  // o == 7
}

// s x + y per component
__device__ __forceinline__ float2 cfma(float s, float2 x, float2 y) {
  return make_float2(fmaf(s, x.x, y.x), fmaf(s, x.y, y.y));
}

// ------------------------------------------------------------------------------------------
// radix-R DFT on R registers, natural order in and out.  HALF: inputs R/2..R-1 are zero and
// are not read (zero-padded first stage).
// ------------------------------------------------------------------------------------------
template <int R, bool INV, bool HALF>
struct DFT;

template <bool INV, bool HALF>
struct DFT<2, INV, HALF> {
  static __device__ __forceinline__ void run(float2* v) {
    if constexpr (HALF) {
      v[1] = v[0];
    } else {
      float2 a = v[0], b = v[1];
      v[0] = cadd(a, b);
      v[1] = csub(a, b);
    }
  }
};

template <bool INV, bool HALF>
struct DFT<3, INV, HALF> {
  static_assert(!HALF, "radix-3 stages are never zero-pruned");
  static __device__ __forceinline__ void run(float2* v) {
    constexpr float c = -0.5f;
    constexpr float s = INV ? 0.86602540378443864676f : -0.86602540378443864676f;
    float2 a = v[0], b = v[1], d = v[2];
    float2 sum = cadd(b, d), dif = csub(b, d);
    float2 m = make_float2(fmaf(c, sum.x, a.x), fmaf(c, sum.y, a.y));
    // m +- i s (b - d)
    v[0] = cadd(a, sum);
    v[1] = make_float2(fmaf(-s, dif.y, m.x), fmaf(s, dif.x, m.y));
    v[2] = make_float2(fmaf(s, dif.y, m.x), fmaf(-s, dif.x, m.y));
  }
};

// 5-point DFT: with t1 = b + e, t2 = c + d, t3 = b - e, t4 = c - d and W = exp(-+2 pi i / 5)
//   X0 = a + t1 + t2,  X1,4 = a + c1 t1 + c2 t2 -+ i (s1 t3 + s2 t4),
//   X2,3 = a + c2 t1 + c1 t2 -+ i (s2 t3 - s1 t4)
// (c_k = cos(2 pi k / 5), s_k = sin(2 pi k / 5); the upper sign for the forward transform).
template <bool INV, bool HALF>
struct DFT<5, INV, HALF> {
  static_assert(!HALF, "radix-5 stages are never zero-pruned");
  static __device__ __forceinline__ void run(float2* v) {
    constexpr float c1 = 0.30901699437494742410f, c2 = -0.80901699437494742410f;
    constexpr float s1 = INV ? -0.95105651629515357212f : 0.95105651629515357212f;
    constexpr float s2 = INV ? -0.58778525229247312917f : 0.58778525229247312917f;
    const float2 a = v[0];
    const float2 t1 = cadd(v[1], v[4]), t2 = cadd(v[2], v[3]);
    const float2 t3 = csub(v[1], v[4]), t4 = csub(v[2], v[3]);
    const float2 m1 = cfma(c1, t1, cfma(c2, t2, a));
    const float2 m2 = cfma(c2, t1, cfma(c1, t2, a));
    const float2 n1 = cfma(s1, t3, cscale(t4, s2));
    const float2 n2 = cfma(s2, t3, cscale(t4, -s1));
    v[0] = cadd(a, cadd(t1, t2));
    // m -+ i n: (m.x +- n.y, m.y -+ n.x)
    v[1] = make_float2(m1.x + n1.y, m1.y - n1.x);
    v[4] = make_float2(m1.x - n1.y, m1.y + n1.x);
    v[2] = make_float2(m2.x + n2.y, m2.y - n2.x);
    v[3] = make_float2(m2.x - n2.y, m2.y + n2.x);
  }
};

template <bool INV, bool HALF>
struct DFT<4, INV, HALF> {
  static __device__ __forceinline__ void run(float2* v) {
    if constexpr (HALF) {
      float2 a = v[0], b = v[1];
      float2 ib = INV ? mul_posi(b) : mul_negi(b);
      v[0] = cadd(a, b);
      v[2] = csub(a, b);
      v[1] = cadd(a, ib);
      v[3] = csub(a, ib);
    } else {
      float2 a = v[0], b = v[1], c = v[2], d = v[3];
      float2 s0 = cadd(a, c), d0 = csub(a, c), s1 = cadd(b, d), d1 = csub(b, d);
      float2 id1 = INV ? mul_posi(d1) : mul_negi(d1);
      v[0] = cadd(s0, s1);
      v[2] = csub(s0, s1);
      v[1] = cadd(d0, id1);
      v[3] = csub(d0, id1);
    }
  }
};

// 4-point DFT whose inputs 1..3 carry a pending factor 1/sqrt(2) where bit n of SM is set
// (they come from odd-octant twiddles): the factor is folded into the butterfly's additions.
template <bool INV, int SM>
struct DFT4Scaled {
  static_assert((SM & 1) == 0, "input 0 is never scaled");
  static __device__ __forceinline__ void run(float2* v) {
    constexpr float h = 0.70710678118654752440f;
    constexpr bool fb = (SM & 2) != 0, fc = (SM & 4) != 0, fd = (SM & 8) != 0;
    const float2 a = v[0], b = v[1], c = v[2], d = v[3];
    float2 s0, d0, s1, d1;
    if constexpr (fc) {
      s0 = cfma(h, c, a);
      d0 = cfma(-h, c, a);
    } else {
      s0 = cadd(a, c);
      d0 = csub(a, c);
    }
    if constexpr (fb && !fd) {
      s1 = cfma(h, b, d);
      d1 = cfma(h, b, make_float2(-d.x, -d.y));
    } else if constexpr (fd && !fb) {
      s1 = cfma(h, d, b);
      d1 = cfma(-h, d, b);
    } else {  // both scaled (the sums keep the factor) or neither
      s1 = cadd(b, d);
      d1 = csub(b, d);
    }
    const float2 id1 = INV ? mul_posi(d1) : mul_negi(d1);
    if constexpr (fb && fd) {
      v[0] = cfma(h, s1, s0);
      v[2] = cfma(-h, s1, s0);
      v[1] = cfma(h, id1, d0);
      v[3] = cfma(-h, id1, d0);
    } else {
      v[0] = cadd(s0, s1);
      v[2] = csub(s0, s1);
      v[1] = cadd(d0, id1);
      v[3] = csub(d0, id1);
    }
  }
};

// Composite R = A * B:  n = B n1 + n2,  k = k1 + A k2.
//   Y[n2][k1] = DFT_A over n1 of x[B n1 + n2];  Y *= W_R^(n2 k1);  X[k1 + A k2] = DFT_B over n2.
// Zero inputs x[n >= R/2] are exactly the n1 >= A/2 terms, so HALF passes to the A-point DFTs.
template <int R, bool INV, bool HALF>
struct DFT {
  static constexpr int A = first_factor(R);
  static constexpr int B = R / A;
  static_assert(A > 1 && A < R, "unsupported radix");
  static_assert(!HALF || A % 2 == 0, "zero pruning needs an even first factor");
  static __device__ __forceinline__ void run(float2* v) {
    float2 y[R];
    static_for<0, B>([&](auto n2c) {
      constexpr int n2 = decltype(n2c)::value;
      float2 t[A];
      static_for<0, A>([&](auto n1c) {
        constexpr int n1 = decltype(n1c)::value;
        if constexpr (!HALF || n1 < A / 2) t[n1] = v[B * n1 + n2];
      });
      DFT<A, INV, HALF>::run(t);
      static_for<0, A>([&](auto k1c) {
        constexpr int k1 = decltype(k1c)::value;
        // with B = 4 the 1/sqrt(2) of odd-octant twiddles is left to the 4-point butterfly
        if constexpr (B == 4 && odd_octant<R, n2 * k1>())
          y[n2 * A + k1] = twc_octant_unscaled<R, n2 * k1, INV>(t[k1]);
        else
          y[n2 * A + k1] = twc<R, n2 * k1, INV>(t[k1]);
      });
    });
    static_for<0, A>([&](auto k1c) {
      constexpr int k1 = decltype(k1c)::value;
      float2 t[B];
      static_for<0, B>([&](auto n2c) {
        constexpr int n2 = decltype(n2c)::value;
        t[n2] = y[n2 * A + k1];
      });
      if constexpr (B == 4) {
        constexpr int SM = (odd_octant<R, 1 * k1>() ? 2 : 0) | (odd_octant<R, 2 * k1>() ? 4 : 0) |
                           (odd_octant<R, 3 * k1>() ? 8 : 0);
        DFT4Scaled<INV, SM>::run(t);
      } else {
        DFT<B, INV, false>::run(t);
      }
      static_for<0, B>([&](auto k2c) {
        constexpr int k2 = decltype(k2c)::value;
        v[k1 + A * k2] = t[k2];
      });
    });
  }
};

// ------------------------------------------------------------------------------------------
// radix plans: E registers per lane, radices of each stage (all divide E)
// ------------------------------------------------------------------------------------------
// SH: the exchange index i is stored at i + (i >> SH) (one padding slot every 2^SH entries),
// RX / CX: extra slots between the exchange regions of neighbouring transforms in the row /
// column kernels.  First chosen with a bank model of 64 four-byte banks serving 32 lanes per
// cycle.  Measured on gfx950 (bank-conflict counters of probes/lds_bank_probe.hip, which
// writes and reads one lane-address pattern at a time), 8-byte writes follow another model:
// 16 lanes per cycle over 32 four-byte banks, so a quarter-wavefront's 32 dwords must fall on
// distinct banks (stride-2 writes take twice the cycles, stride-16 ones 16 times), while
// 8-byte reads of the same patterns show almost no conflicts.  The plans of 128 to 1024
// points are chosen with that model (the exchanges of the row and column kernels and the
// column kernels' staging);
// 512 keeps SH = 4, with which its column kernels that evaluate H per element stay at 128
// registers (SH = 3, conflict-free in its exchanges too, takes them to 144-150).
template <int M>
struct Plan;
template <> struct Plan<64>   { static constexpr int E = 16, NST = 2, SH = 4, RX = 0, CX = 0;  static constexpr int R[4] = {16, 4, 0, 0}; };
template <> struct Plan<96>   { static constexpr int E = 24, NST = 3, SH = 6, RX = 1, CX = 1;  static constexpr int R[4] = {3, 8, 4, 0}; };
template <> struct Plan<128>  { static constexpr int E = 16, NST = 2, SH = 3, RX = 1, CX = 1;  static constexpr int R[4] = {16, 8, 0, 0}; };
template <> struct Plan<192>  { static constexpr int E = 12, NST = 3, SH = 2, RX = 0, CX = 2;  static constexpr int R[4] = {12, 4, 4, 0}; };
template <> struct Plan<256>  { static constexpr int E = 16, NST = 2, SH = 4, RX = 0, CX = 2;  static constexpr int R[4] = {16, 16, 0, 0}; };
template <> struct Plan<384>  { static constexpr int E = 12, NST = 4, SH = 2, RX = 0, CX = 2;  static constexpr int R[4] = {12, 4, 4, 2}; };
template <> struct Plan<512>  { static constexpr int E = 16, NST = 3, SH = 4, RX = 16, CX = 2; static constexpr int R[4] = {8, 8, 8, 0}; };
template <> struct Plan<1024> { static constexpr int E = 16, NST = 3, SH = 4, RX = 0, CX = 4;  static constexpr int R[4] = {8, 8, 16, 0}; };
template <> struct Plan<1600> { static constexpr int E = 20, NST = 3, SH = 4, RX = 0, CX = 0;  static constexpr int R[4] = {20, 20, 4, 0}; };

// Radix plans: plan 0 of every length is Plan<M>::R; the lengths of the large workloads have
// alternatives with the same registers per lane (so the same lanes, blocks and LDS regions),
// chosen per pass by the autotuner.  Transforms of different radix plans round differently but
// compute the same DFT.  At 1024, 8 x 8 x 16 is the built-in plan: on the large workload it runs
// the column and row passes about 1 % faster than 16 x 16 x 4 (plan 1) and 2 % faster than
// 4 x 16 x 16 (plan 2).
template <int M, int V>
struct Radix {
  static_assert(V == 0, "no such radix plan");
  static constexpr int NST = Plan<M>::NST;
  static constexpr int R[4] = {Plan<M>::R[0], Plan<M>::R[1], Plan<M>::R[2], Plan<M>::R[3]};
};
template <> struct Radix<512, 1>  { static constexpr int NST = 3; static constexpr int R[4] = {16, 16, 2, 0}; };
template <> struct Radix<512, 2>  { static constexpr int NST = 3; static constexpr int R[4] = {4, 8, 16, 0}; };
template <> struct Radix<1024, 1> { static constexpr int NST = 3; static constexpr int R[4] = {16, 16, 4, 0}; };
template <> struct Radix<1024, 2> { static constexpr int NST = 3; static constexpr int R[4] = {4, 16, 16, 0}; };
// number of radix plans of a length
constexpr int radix_plans(int M) { return (M == 512 || M == 1024) ? 3 : 1; }

// Block padding of the exchanges of a plan: where A[s] > 0, the exchange after stage s stores
// index i at i + (i / A[s]) B[s] (B[s] padding slots after every A[s] entries) instead of the
// shift padding of Plan::SH; REGION then is the exchange region of every transform and SKEW the
// offset of the staged column rows of tile column c, SKEW (c / 2) slots into its region.  A[s]
// is a multiple of both P and the span NS R of the stage's butterflies, so every lane's writes
// and reads stay a lane base plus compile-time offsets.  Both plans are chosen with the
// measured write model above.  For the 1600-point transform (20 20 4), whose 80-lane groups
// span wavefronts, the 16 lanes of a write cycle store stage 0's outputs 20 entries apart
// (4 distinct bank pairs without padding): one slot after every 80 entries separates them;
// stage 1 takes 4 slots after every 400; 1622-slot regions put the staged rows of the eight
// tile columns on distinct banks.  At 1024 = 8 8 16, the 16 lanes of one write cycle hold
// only the NS = 8 twiddle columns k of stage 1, so each output's writes of two 64-entry groups
// fell on the same banks (2-way): 8 slots after every 64 move the second group by 16 banks.  Stage 0 takes the shift padding
// with SH = 4, which is conflict-free for its writes.  The region, 1146 slots (2 mod 4, so
// that the staged rows of the eight tile columns fall on distinct banks), keeps two column
// blocks of 8 columns, 81.5 KB each with the twiddle table, within a CU's 160 KB.
template <int M>
struct XPad {
  static constexpr int A[4] = {0, 0, 0, 0};
  static constexpr int B[4] = {0, 0, 0, 0};
  static constexpr int REGION = 0;
  static constexpr int SKEW = 0;
  static constexpr bool ROWS = true;  // the row passes use it too
};
template <> struct XPad<1024> {
  static constexpr int A[4] = {0, 64, 0, 0};
  static constexpr int B[4] = {0, 8, 0, 0};
  static constexpr int REGION = 1146;
  static constexpr int SKEW = 0;
  // the row passes keep the shift padding: they run at the HBM rate, and the block padding's
  // lane bases would take their forward middle pass over 128 registers
  static constexpr bool ROWS = false;
};
template <> struct XPad<1600> {
  static constexpr int A[4] = {80, 400, 0, 0};
  static constexpr int B[4] = {1, 4, 0, 0};
  static constexpr int REGION = 1622;
  static constexpr int SKEW = 0;
  static constexpr bool ROWS = true;
};

template <int M>
struct Geo {
  static constexpr int E = Plan<M>::E;
  static constexpr int P = M / E;  // lanes per transform
  static constexpr int ROW_REGION = (XPad<M>::REGION > 0 && XPad<M>::ROWS) ? XPad<M>::REGION
                                                                            : M + (M >> Plan<M>::SH) + Plan<M>::RX;
  static constexpr int COL_REGION = XPad<M>::REGION > 0 ? XPad<M>::REGION : M + (M >> Plan<M>::SH) + Plan<M>::CX;
  // the lanes of one transform lie in one wavefront
  static constexpr bool WAVE_LOCAL = P <= 64 && 64 % P == 0;
  static_assert(WAVE_LOCAL || P % 16 == 0, "a group spanning wavefronts is a whole number of 16-lane rows");
};

// Per-stage twiddle table: stage s (radix R, NS = product of the earlier radices, s >= 1)
// stores W_{NS R}^{r k} = exp(-2 pi i r k / (NS R)) at twiddle_offset(s) + (r - 1) NS + k for
// r = 1..R-1, k = 0..NS-1, so that the lanes of one butterfly row read consecutive entries.
template <int M, int V = 0>
constexpr int twiddle_offset(int stage) {
  int off = 0, ns = 1;
  for (int s = 0; s < stage; ++s) {
    if (s > 0) off += (Radix<M, V>::R[s] - 1) * ns;
    ns *= Radix<M, V>::R[s];
  }
  return off;
}
template <int M, int V = 0>
constexpr int twiddle_count() { return twiddle_offset<M, V>(Radix<M, V>::NST); }

// The table of radix plan V of length M, built on the host in double precision from exact
// integer indices: W_L^(r k) with the exponent reduced mod L before the angle is formed.
template <int M, int V>
inline void twiddle_table_host(std::vector<float2>& out) {
  out.assign(twiddle_count<M, V>() > 0 ? twiddle_count<M, V>() : 1, make_float2(1.f, 0.f));
  int ns = Radix<M, V>::R[0];
  for (int st = 1; st < Radix<M, V>::NST; ++st) {
    const int R = Radix<M, V>::R[st];
    const int L = ns * R;
    const int off = twiddle_offset<M, V>(st);
    for (int r = 1; r < R; ++r)
      for (int k = 0; k < ns; ++k) {
        const double ang = 6.283185307179586476925286766559 * static_cast<double>((r * k) % L) /
                           static_cast<double>(L);
        out[off + (r - 1) * ns + k] = make_float2(static_cast<float>(std::cos(ang)),
                                                  static_cast<float>(-std::sin(ang)));
      }
    ns = L;
  }
}

template <int M>
__device__ __forceinline__ int lds_slot(int i) {
  return i + (i >> Plan<M>::SH);
}

// Copies the per-stage twiddle table from global memory into LDS (caller synchronises).
template <int M, int V = 0>
__device__ __forceinline__ void stage_twiddles(float2* __restrict__ dst, const float2* __restrict__ src,
                                               int tid, int nthreads) {
  for (int i = tid; i < twiddle_count<M, V>(); i += nthreads) dst[i] = src[i];
}

// LDS ordering between the lanes of one transform.  A transform never spans more than one
// wavefront, and a wavefront's LDS instructions execute in program order, so a wave-level
// fence + barrier orders the scattered writes before the strided reads.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// LDS ordering between the lanes of one transform of length M: the wave-level fence when the
// group lies in one wavefront, a block barrier otherwise (every thread of the block runs every
// transform, so the barrier is reached uniformly).
template <int M>
__device__ __forceinline__ void group_sync() {
  if constexpr (Geo<M>::WAVE_LOCAL)
    wave_sync();
  else
    __syncthreads();
}

constexpr bool divides_or_multiple(int a, int b) { return a % b == 0 || b % a == 0; }

// One Stockham stage: radix R, NS = product of the radices of the earlier stages.
// Exchange addresses are padded (lds_slot).  When NS and NS*R are both divisors or multiples
// of the padding period 2^SH, the padded address of output r splits exactly into a per-lane
// base plus a compile-time offset, and the reads j0 + P t split the same way when P is a
// multiple of 2^SH; the other stages compute the padded address directly.
template <int M, int V, int ST, int R, int NS, bool LAST, bool INV, bool HALF, int CST = -1, bool BP = true>
__device__ __forceinline__ void stockham_stage(float2 (&reg)[Geo<M>::E], float2* __restrict__ lds,
                                               int j0, const float2* __restrict__ tw,
                                               const float2* treg = nullptr) {
  constexpr int E = Geo<M>::E;
  constexpr int P = Geo<M>::P;
  constexpr int S = E / R;
  constexpr int SH = Plan<M>::SH;
  constexpr int S2 = 1 << SH;
  constexpr bool LIN_W = divides_or_multiple(NS, S2) && divides_or_multiple(NS * R, S2);
  constexpr bool LIN_R = (P % S2 == 0);
  constexpr int XA = (V == 0 && BP) ? XPad<M>::A[ST] : 0;  // BP: the plan's block padding
  constexpr int XB = (V == 0 && BP) ? XPad<M>::B[ST] : 0;
  static_assert(E % R == 0, "radix must divide the registers per lane");
  static_assert(XA == 0 || LAST || (XA % P == 0 && XA % (NS * R) == 0), "block padding must keep lanes linear");
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const int j = j0 + P * s;
    const int k = (NS > 1) ? (j % NS) : 0;
    float2 v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = reg[s + r * S];
    if constexpr (NS > 1) {
      constexpr int OFF = twiddle_offset<M, V>(ST);
#pragma unroll
      for (int r = 1; r < R; ++r) {
        // stage CST: the lane's R - 1 twiddles are held in registers (treg), the same for all s
        const float2 w = (ST == CST) ? treg[r - 1] : tw[OFF + (r - 1) * NS + k];
        v[r] = INV ? cmulc(v[r], w) : cmul(v[r], w);
      }
    }
    DFT<R, INV, HALF>::run(v);
    if constexpr (LAST) {
#pragma unroll
      for (int r = 0; r < R; ++r) reg[s + r * S] = v[r];
    } else {
      const int b0 = (j / NS) * NS * R;
      if constexpr (XA > 0) {
        // b0 + k + r NS stays inside one padding block (XA is a multiple of NS R)
        const int lane_base = b0 + k + (b0 / XA) * XB;
#pragma unroll
        for (int r = 0; r < R; ++r) lds[lane_base + r * NS] = v[r];
      } else if constexpr (LIN_W) {
        const int lane_base = b0 + (b0 >> SH) + k + (k >> SH);
#pragma unroll
        for (int r = 0; r < R; ++r) lds[lane_base + r * NS + ((r * NS) >> SH)] = v[r];
      } else {
#pragma unroll
        for (int r = 0; r < R; ++r) lds[lds_slot<M>(b0 + k + r * NS)] = v[r];
      }
    }
  }
  if constexpr (!LAST) {
    group_sync<M>();
    if constexpr (XA > 0) {
      // j0 + P t: j0 < P and XA is a multiple of P, so the block is that of P t
#pragma unroll
      for (int t = 0; t < E; ++t) reg[t] = lds[j0 + P * t + ((P * t) / XA) * XB];
    } else if constexpr (LIN_R) {
      const int rb = j0 + (j0 >> SH);
#pragma unroll
      for (int t = 0; t < E; ++t) reg[t] = lds[rb + P * t + ((P * t) >> SH)];
    } else {
#pragma unroll
      for (int t = 0; t < E; ++t) reg[t] = lds[lds_slot<M>(j0 + P * t)];
    }
    group_sync<M>();
  }
}

template <int M, int V, int ST, int NS, bool INV, bool HALF, int CST = -1, bool BP = true>
__device__ __forceinline__ void fft_stages(float2 (&reg)[Geo<M>::E], float2* __restrict__ lds, int j0,
                                           const float2* __restrict__ tw, const float2* treg = nullptr) {
  if constexpr (ST < Radix<M, V>::NST) {
    constexpr int R = Radix<M, V>::R[ST];
    constexpr bool LAST = (ST + 1 == Radix<M, V>::NST);
    stockham_stage<M, V, ST, R, NS, LAST, INV, HALF && ST == 0, CST, BP>(reg, lds, j0, tw, treg);
    fft_stages<M, V, ST + 1, NS * R, INV, false, CST, BP>(reg, lds, j0, tw, treg);
  }
}

// The stage whose twiddles a caller may hold in registers: stage 1, when its twiddle index
// k = j mod NS is the same for every butterfly of a lane (NS divides P), it needs at most
// seven values (radix 8) and one transform fills a wavefront (P = 64; with two per wavefront,
// as at 512, the column kernels have no room for the registers and spill); -1 when no stage
// qualifies.
template <int M, int V>
constexpr int register_twiddle_stage() {
  return (Radix<M, V>::NST >= 3 && Radix<M, V>::R[1] <= 8 && Geo<M>::P == 64 &&
          Geo<M>::P % Radix<M, V>::R[0] == 0) ? 1 : -1;
}
template <int M, int V>
struct RegTwiddles {
  static constexpr int STAGE = register_twiddle_stage<M, V>();
  static constexpr int N = STAGE < 0 ? 1 : Radix<M, V>::R[1] - 1;  // registers (1 when unused)
};

// Loads the lane's twiddles of that stage from the table (in LDS) into treg.
template <int M, int V>
__device__ __forceinline__ void load_register_twiddles(float2* treg, const float2* __restrict__ tw,
                                                       int j0) {
  if constexpr (RegTwiddles<M, V>::STAGE >= 0) {
    constexpr int NS = Radix<M, V>::R[0];
    constexpr int OFF = twiddle_offset<M, V>(1);
#pragma unroll
    for (int r = 1; r < Radix<M, V>::R[1]; ++r) treg[r - 1] = tw[OFF + (r - 1) * NS + j0 % NS];
  }
}

// Full length-M transform of the group's registers with radix plan V.  HALF: elements
// M/2..M-1 are zero (zero-padded input); only used when the first radix is even.  tw: the
// plan's per-stage twiddle table (in LDS).
template <int M, bool INV, bool HALF, int V = 0, bool BP = true>
__device__ __forceinline__ void fft(float2 (&reg)[Geo<M>::E], float2* __restrict__ lds, int j0,
                                    const float2* __restrict__ tw) {
  constexpr bool H = HALF && (Radix<M, V>::R[0] % 2 == 0);
  if constexpr (HALF && !H) {
#pragma unroll
    for (int t = Geo<M>::E / 2; t < Geo<M>::E; ++t) reg[t] = make_float2(0.f, 0.f);
  }
  fft_stages<M, V, 0, 1, INV, H, -1, BP>(reg, lds, j0, tw);
}

// The same transform with the twiddles of register_twiddle_stage() taken from treg (loaded by
// load_register_twiddles) instead of the table: the same values, so the same bits.
template <int M, bool INV, bool HALF, int V = 0>
__device__ __forceinline__ void fft_treg(float2 (&reg)[Geo<M>::E], float2* __restrict__ lds, int j0,
                                         const float2* __restrict__ tw,
                                         const float2* treg) {
  constexpr bool H = HALF && (Radix<M, V>::R[0] % 2 == 0);
  if constexpr (HALF && !H) {
#pragma unroll
    for (int t = Geo<M>::E / 2; t < Geo<M>::E; ++t) reg[t] = make_float2(0.f, 0.f);
  }
  fft_stages<M, V, 0, 1, INV, H, RegTwiddles<M, V>::STAGE>(reg, lds, j0, tw, treg);
}

// fft_treg when TREG, else fft (treg unused).
template <int M, bool INV, bool HALF, int V, bool TREG>
__device__ __forceinline__ void fft_sel(float2 (&reg)[Geo<M>::E], float2* __restrict__ lds, int j0,
                                        const float2* __restrict__ tw, const float2* treg) {
  if constexpr (TREG) fft_treg<M, INV, HALF, V>(reg, lds, j0, tw, treg);
  else fft<M, INV, HALF, V>(reg, lds, j0, tw);
}

}  // namespace dpx
